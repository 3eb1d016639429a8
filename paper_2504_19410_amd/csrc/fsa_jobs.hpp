// fsa_jobs.hpp -- descriptors of one problem's share of a pass (host and device).
#pragma once

namespace fsa {

// Pointers are device addresses; complex arrays are interleaved (re, im).
struct JobR2c {   // pass A: rho rows (n_outer * n_inner of N_last reals) -> X
    const void* rho;
    void* out;
    int n_outer, n_inner;
};
struct JobC2r {   // pass E: X -> phi rows
    const void* in;
    void* phi;
    int n_outer, n_inner;
    const void* add = nullptr;  // if set: phi += alpha * add (same layout as phi)
    double alpha = 0.0;
};
struct JobT {     // passes B and D (3D): X1[i0][p2][i1] <-> X2[p2][p1][i0]
    const void* in;
    void* out;
    int N0, H;
    int p2_lo, p2_n;  // the bins p2 in [p2_lo, p2_lo + p2_n) this job covers
};
struct JobConv {  // pass C: pencils of X2 (3D) or X (2D), in place
    void* data;
    const void* tensor;
    int n_pencils, P1, N1;  // n_pencils = P1 * (bins covered)
    int p2_lo;              // first bin p2 covered (0 in 2D)
};

enum class Pass { R2C = 0, FWD_T = 1, CONV = 2, INV_T = 3, C2R = 4 };

}  // namespace fsa
