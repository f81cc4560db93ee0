// k_copy.hip -- the reference stream of the benchmark: a plain device copy with
// one 16-byte nontemporal load and store per thread.  Nothing of the method runs
// here; its rate is the achievable HBM bandwidth the push is measured against.
#include <stdint.h>

#include "pcpic_internal.h"
#include "push_common.h"

namespace pcpic {

__global__ __launch_bounds__(64) void k_copy16(const dvec2 *__restrict__ src, dvec2 *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t n16, hipStream_t stream)
{
    const int64_t blocks = (n16 + 63) / 64;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(64), 0, stream, (const dvec2 *)src, (dvec2 *)dst, n16);
    return hipGetLastError();
}

}  // namespace pcpic
