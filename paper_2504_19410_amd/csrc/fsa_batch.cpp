// fsa_batch.cpp -- batched evaluation of independent problems.
#include <hip/hip_runtime.h>

#include "fsa_internal.hpp"

namespace fsa {
void set_last_error(const char* msg);
hipError_t apply_plan(const fsa_plan_s* pl, const void* rho, void* phi, void* ws, hipStream_t st,
                      hipEvent_t const* events);
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

extern "C" {

fsa_status fsa_batch_workspace_bytes(int n, const fsa_plan* plans, size_t* bytes) {
    if (n < 0 || (n > 0 && !plans) || !bytes) {
        fsa::set_last_error("fsa_batch_workspace_bytes: bad arguments");
        return FSA_EINVAL;
    }
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) {
            fsa::set_last_error("fsa_batch_workspace_bytes: null plan");
            return FSA_EINVAL;
        }
        total += align256(plans[i]->ws_bytes);
    }
    *bytes = total;
    return FSA_OK;
}

fsa_status fsa_apply_batched(int n, const fsa_plan* plans, const void* const* rho,
                             void* const* phi, void* workspace, size_t workspace_bytes,
                             void* stream) {
    size_t need = 0;
    fsa_status s = fsa_batch_workspace_bytes(n, plans, &need);
    if (s != FSA_OK) return s;
    if (n > 0 && (!rho || !phi || !workspace)) {
        fsa::set_last_error("fsa_apply_batched: null array");
        return FSA_EINVAL;
    }
    if (workspace_bytes < need) {
        fsa::set_last_error("fsa_apply_batched: workspace too small");
        return FSA_EINVAL;
    }
    char* ws = (char*)workspace;
    for (int i = 0; i < n; ++i) {
        if (!plans[i]->built) {
            fsa::set_last_error("fsa_apply_batched: tensor not built");
            return FSA_ESTATE;
        }
        hipError_t e = fsa::apply_plan(plans[i], rho[i], phi[i], ws, (hipStream_t)stream, nullptr);
        if (e != hipSuccess) {
            fsa::set_last_error(hipGetErrorString(e));
            return FSA_EDEVICE;
        }
        ws += align256(plans[i]->ws_bytes);
    }
    return FSA_OK;
}

}  // extern "C"
