// Bit-count histogram of the per-shot classical registers (the result of a
// multi-shot run, Sec. III-B): device radix sort of the 64-bit registers,
// then run-length encoding into (key, count) pairs in ascending key order.
#include <hip/hip_runtime.h>
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_run_length_encode.hpp>

#include <algorithm>
#include <cstdint>

extern "C" {

size_t svb_counts_temp_bytes(int64_t n)
{
    size_t a = 0, b = 0;
    const unsigned N = (unsigned)n;
    if (rocprim::radix_sort_keys(nullptr, a, (const uint64_t *)nullptr, (uint64_t *)nullptr, N) !=
        hipSuccess)
        a = 64u << 20;
    if (rocprim::run_length_encode(nullptr, b, (const uint64_t *)nullptr, N, (uint64_t *)nullptr,
                                   (uint32_t *)nullptr, (uint32_t *)nullptr) != hipSuccess)
        b = 64u << 20;
    return std::max(a, b) + 256;
}

hipError_t svb_counts(const uint64_t *memory, int64_t n, void *temp, size_t temp_bytes,
                      uint64_t *keys_sorted, uint64_t *uniq, uint32_t *cnt, uint32_t *n_uniq,
                      hipStream_t st)
{
    const unsigned N = (unsigned)n;
    size_t tb = temp_bytes;
    hipError_t e = rocprim::radix_sort_keys(temp, tb, memory, keys_sorted, N, 0, 64, st);
    if (e != hipSuccess) return e;
    tb = temp_bytes;
    return rocprim::run_length_encode(temp, tb, keys_sorted, N, uniq, cnt, n_uniq, st);
}

}  // extern "C"
