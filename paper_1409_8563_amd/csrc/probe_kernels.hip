// Achievable-bandwidth probe: a plain device-to-device copy written for
// gfx950 (16-byte accesses, U independent loads in flight per thread, a grid
// sized by the compute units).  It measures the HBM ceiling that a streaming
// kernel of this library can reach on the device at hand, against which the
// stencil kernels' read-once/write-once traffic is compared.
#include "pr.h"
#include "pr_internal.h"

namespace pr {
namespace {

#define PR_GLOBAL __attribute__((address_space(1)))

using u32x4 = unsigned int __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;

// Thread t copies the 16-byte words t, t + S, t + 2S, ... (S = all threads),
// U of them per trip with every load issued before the first store.
template <int U, bool NT>
__global__ void __launch_bounds__(kProbeThreads)
    copy_probe_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * kProbeThreads;
    size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
    const PR_GLOBAL u32x4 *s = (const PR_GLOBAL u32x4 *)src;
    PR_GLOBAL u32x4 *d = (PR_GLOBAL u32x4 *)dst;
    for (; i + (size_t)(U - 1) * stride < n16; i += (size_t)U * stride) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (NT) v[u] = __builtin_nontemporal_load(&s[i + u * stride]);
            else v[u] = s[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (NT) __builtin_nontemporal_store(v[u], &d[i + u * stride]);
            else d[i + u * stride] = v[u];
        }
    }
    for (; i < n16; i += stride) d[i] = s[i];
}

}  // namespace

hipError_t launch_copy_probe(int variant, const void *src, void *dst, size_t bytes, int blocks, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    const dim3 grid(blocks), block(kProbeThreads);
    const u32x4 *a = (const u32x4 *)src;
    u32x4 *b = (u32x4 *)dst;
    switch (variant) {
    case 0: hipLaunchKernelGGL((copy_probe_kernel<4, false>), grid, block, 0, s, a, b, n16); break;
    case 1: hipLaunchKernelGGL((copy_probe_kernel<4, true>), grid, block, 0, s, a, b, n16); break;
    case 2: hipLaunchKernelGGL((copy_probe_kernel<8, false>), grid, block, 0, s, a, b, n16); break;
    default: hipLaunchKernelGGL((copy_probe_kernel<1, false>), grid, block, 0, s, a, b, n16); break;
    }
    return hipGetLastError();
}

}  // namespace pr
