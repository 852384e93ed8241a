// The persistent executor with complex64 fused one-qubit micro-ops on the
// matrix cores (v_mfma_f32_4x4x1f32), for register groups on two register
// sets. Built as its own translation unit from the executor's source, so
// the default executor's code object is unchanged by it.
#define SVB_MFMA_UNIT 1
#include "kernels.hip"

namespace svb {
template __global__ void exec_kernel_mfma<float, 4>(ExecParams);
template __global__ void exec_kernel_mfma<float, 8>(ExecParams);
template __global__ void exec_kernel_mfma<float, 16>(ExecParams);
template __global__ void exec_kernel_mfma<float, 32>(ExecParams);
}  // namespace svb
