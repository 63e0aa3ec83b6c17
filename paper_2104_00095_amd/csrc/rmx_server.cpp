// Serving loop: placeholder until the scheduler lands.
#include "rmx.h"

extern "C" {
int rmx_server_create(int, size_t, int32_t, rmx_server** out) {
    if (out) *out = nullptr;
    return RMX_E_ARG;
}
int rmx_server_register(rmx_server*, const rmx_grid*, const rmx_solid*, int32_t, int64_t*) {
    return RMX_E_ARG;
}
int rmx_server_field(rmx_server*, int64_t, int32_t, double**, int8_t**) { return RMX_E_ARG; }
int rmx_server_submit(rmx_server*, int64_t, const rmx_options*, int64_t*) { return RMX_E_ARG; }
int rmx_server_wait(rmx_server*, int64_t, rmx_solid_stats*, double*) { return RMX_E_ARG; }
int rmx_server_release(rmx_server*, int64_t) { return RMX_E_ARG; }
int rmx_server_usage(rmx_server*, size_t*, size_t*) { return RMX_E_ARG; }
int rmx_server_destroy(rmx_server*) { return RMX_E_ARG; }
}
