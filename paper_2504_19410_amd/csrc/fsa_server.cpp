// fsa_server.cpp -- served variant (continuous batching with HBM-budget
// admission).  Placeholder entry points until the scheduler lands.
#include "fsa_internal.hpp"

namespace fsa {
void set_last_error(const char* msg);
}

static fsa_status unsupported(const char* what) {
    fsa::set_last_error(what);
    return FSA_EUNSUPPORTED;
}

extern "C" {
fsa_status fsa_server_create(size_t, int, int, fsa_server*) {
    return unsupported("fsa_server_create: not available in this build");
}
fsa_status fsa_server_submit(fsa_server, const fsa_kernel*, int, const double*, const int64_t*,
                             fsa_precision, const void*, void*, uint64_t*) {
    return unsupported("fsa_server_submit: not available in this build");
}
fsa_status fsa_server_poll(fsa_server, uint64_t, int*, fsa_status*) {
    return unsupported("fsa_server_poll: not available in this build");
}
fsa_status fsa_server_wait(fsa_server, uint64_t, fsa_status*) {
    return unsupported("fsa_server_wait: not available in this build");
}
fsa_status fsa_server_cancel(fsa_server, uint64_t) {
    return unsupported("fsa_server_cancel: not available in this build");
}
fsa_status fsa_server_stats(fsa_server, fsa_stats*) {
    return unsupported("fsa_server_stats: not available in this build");
}
fsa_status fsa_server_destroy(fsa_server) {
    return unsupported("fsa_server_destroy: not available in this build");
}
}
