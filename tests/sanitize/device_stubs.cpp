// Stand-ins for the device-side entry points of libsvbatch.so, so that the
// host runtime (validation, noise expansion, pass planning, the C ABI's
// argument and state checks) links and runs under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU. Every stand-in
// reports that no device is there; none is reached by the planner.
#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

extern "C" {
hipError_t svb_launch_init(const void *, int, int, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t svb_launch_restart(const void *, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t svb_launch_exec(const void *, int, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t svb_exec_occupancy(int, int, int, int, int, int, int *blocks) { *blocks = 0; return hipErrorNoDevice; }
size_t svb_exec_lds_bytes(int tile_q, int amp_bytes, int, int nbuf, int)
{
    return ((size_t)amp_bytes << tile_q) * (size_t)nbuf;
}
hipError_t svb_counts(const uint64_t *, int64_t, void *, size_t, uint64_t *, uint64_t *, uint32_t *,
                      uint32_t *, hipStream_t)
{
    return hipErrorNoDevice;
}
size_t svb_counts_temp_bytes(int64_t n) { return (size_t)n * 8; }
hipError_t svb_noalloc_scratch(void **, uint64_t *) { return hipErrorNoDevice; }
hipError_t svb_graph_nodes(const void *, int, int, int, void **, unsigned *, void **, unsigned *,
                           unsigned *, size_t *)
{
    return hipErrorNoDevice;
}
hipError_t svb_plain_run(int, const void *, const void *, int, const void *, const void *, const double *,
                         int, uint64_t, uint64_t, uint64_t, void *, uint64_t *, uint64_t *, double *, int,
                         double *, void *, double, double, hipStream_t)
{
    return hipErrorNoDevice;
}
}
