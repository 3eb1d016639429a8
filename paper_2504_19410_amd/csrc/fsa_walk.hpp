// Work walks of the persistent pass kernels: which work items each
// workgroup of a grid visits, in what order.  Plain C++ with host/device
// qualifiers, so that the CPU tests can check that every mode visits every
// item exactly once.
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#else
#define __host__
#define __device__
#define __forceinline__ inline
#endif

namespace fsa {

// The work items one workgroup visits, in order: first, first + stride, ...
// below last (uniform over the group).
//   Default: a contiguous chunk per workgroup.
//   XCD (for tiles whose rows are narrower than a 128-byte cache line, so
// that neighbouring tiles share lines): the dispatcher deals workgroups to
// the 8 XCDs in turn (workgroup g runs on XCD g mod 8), and each XCD has its
// own L2.  Each XCD takes a contiguous eighth of the items, which its
// workgroups visit side by side (workgroup g, the s-th of its XCD, takes
// items s, s + G/8, ... of that eighth): neighbouring tiles are in flight at
// the same time under one L2, so a shared line is read from memory once
// instead of once per tile.
//   PAIR (same case): the two tiles 2j and 2j + 1, which share every 128-byte
// line they touch when a tile row is 64 bytes, go to two workgroups of one
// XCD (g and g + 8) that run side by side, each stepping two items at a time
// through the pair chunk of the two; the pairs take contiguous chunks like
// the default, so only two workgroups ever read one line at once.
enum WalkMode { kWalkChunk = 0, kWalkXcd = 1, kWalkPair = 2 };
struct Walk {
    int first, last, stride;
    // the walk of workgroup g of a grid of G workgroups over `items` items
    template <int MODE>
    __host__ __device__ __forceinline__ static Walk make(int items, int G, int g) {
        if (MODE == kWalkPair && G >= 16 && (G & 15) == 0) {
            const int pairs = (items + 1) >> 1, np = G >> 1;
            const int x = g & 7, s = g >> 3, q = s >> 1, b = s & 1;
            const int c = (pairs + np - 1) / np, pg = q * 8 + x;
            const int lo = 2 * pg * c + b, hi = 2 * (pg * c + c);
            return Walk{lo, hi < items ? hi : items, 2};
        }
        if (MODE == kWalkXcd && G >= 8 && (G & 7) == 0) {
            const int per = (items + 7) / 8, x = g & 7, s = g >> 3;
            const int lo = x * per, hi = lo + per < items ? lo + per : items;
            return Walk{lo + s, hi, G >> 3};
        }
        const int c = (items + G - 1) / G;
        const int first = g * c;
        return Walk{first, first + c < items ? first + c : items, 1};
    }
};

}  // namespace fsa
