// Grid transfers of the coarsened coarse propagator: restriction of a fine
// field to the grid coarsened by 2 in every direction (injection) and
// interpolation back (linear, or the 4-point cubic midpoint rule).  A coarser
// spatial mesh for G is the cheaper-G option of the speedup discussion
// (Section 2.2.2); the paper fixes no transfer operators.
//
// Items are ItemDesc entries: src0 -> dst, nx/ny/nz the FINE grid.  A launch
// covers a table of items (blockIdx.y = item) with grid-stride loops.
#include "pr.h"
#include "pr_internal.h"

namespace pr {
namespace {

#define PR_GLOBAL __attribute__((address_space(1)))

constexpr int kXferThreads = 256;
constexpr int kXferBlocksX = 1024;

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__global__ void __launch_bounds__(kXferThreads) restrict_kernel(const ItemDesc *__restrict__ items)
{
    const ItemDesc &it = items[blockIdx.y];
    const int nx = it.nx, ny = it.ny;
    const int cx = nx / 2, cy = ny / 2, cz = it.nz / 2;
    const int64_t nc = (int64_t)cx * cy * cz;
    const PR_GLOBAL T *src = (const PR_GLOBAL T *)it.src0;
    PR_GLOBAL T *dst = (PR_GLOBAL T *)it.dst;
    for (int64_t i = (int64_t)blockIdx.x * kXferThreads + threadIdx.x; i < nc;
         i += (int64_t)gridDim.x * kXferThreads) {
        const int x = (int)(i % cx);
        const int64_t r = i / cx;
        const int y = (int)(r % cy);
        const int z = (int)(r / cy);
        dst[i] = src[((int64_t)(2 * z) * ny + 2 * y) * nx + 2 * x];
    }
}

// Taps of fine index i on a coarse axis of nc points: even i copies point
// i/2; odd i uses its two coarse neighbours (ORDER 1: 1/2, 1/2) or four
// (ORDER 3: -1/16, 9/16, 9/16, -1/16), indices periodic.
template <int ORDER, typename T>
__device__ __forceinline__ int taps(int i, int nc, int (&idx)[4], T (&w)[4])
{
    if ((i & 1) == 0) {
        idx[0] = i >> 1;
        w[0] = (T)1;
        return 1;
    }
    const int m = (i - 1) >> 1;
    if constexpr (ORDER == 1) {
        idx[0] = m;
        idx[1] = wrapc(m + 1, nc);
        w[0] = (T)0.5;
        w[1] = (T)0.5;
        return 2;
    } else {
        idx[0] = wrapc(m - 1, nc);
        idx[1] = m;
        idx[2] = wrapc(m + 1, nc);
        idx[3] = wrapc(m + 2, nc);
        w[0] = (T)(-1.0 / 16.0);
        w[1] = (T)(9.0 / 16.0);
        w[2] = (T)(9.0 / 16.0);
        w[3] = (T)(-1.0 / 16.0);
        return 4;
    }
}

// Tensor-product interpolation: terms (wz*wy*wx) * value, z taps outermost,
// then y, then x, added in that order (the weight products are exact).
template <typename T, int ORDER>
__global__ void __launch_bounds__(kXferThreads) prolong_kernel(const ItemDesc *__restrict__ items)
{
    const ItemDesc &it = items[blockIdx.y];
    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const int64_t n = (int64_t)nx * ny * nz;
    const PR_GLOBAL T *src = (const PR_GLOBAL T *)it.src0;
    PR_GLOBAL T *dst = (PR_GLOBAL T *)it.dst;
    for (int64_t i = (int64_t)blockIdx.x * kXferThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kXferThreads) {
        const int x = (int)(i % nx);
        const int64_t r = i / nx;
        const int y = (int)(r % ny);
        const int z = (int)(r / ny);
        int iz[4], iy[4], ix[4];
        T wz[4], wy[4], wx[4];
        const int tz = taps<ORDER>(z, cz, iz, wz);
        const int ty = taps<ORDER>(y, cy, iy, wy);
        const int tx = taps<ORDER>(x, cx, ix, wx);
        T acc = (T)0;
        for (int c = 0; c < tz; ++c)
            for (int b = 0; b < ty; ++b) {
                const PR_GLOBAL T *row = src + ((int64_t)iz[c] * cy + iy[b]) * cx;
                const T wzy = wz[c] * wy[b];
                for (int a = 0; a < tx; ++a) acc = acc + (wzy * wx[a]) * row[ix[a]];
            }
        dst[i] = acc;
    }
}

dim3 xfer_grid(int nitems) { return dim3(kXferBlocksX, (unsigned)nitems); }

}  // namespace

hipError_t launch_restrict(int dtype, const ItemDesc *items, int nitems, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (dtype == PR_FP64)
        hipLaunchKernelGGL((restrict_kernel<double>), xfer_grid(nitems), dim3(kXferThreads), 0, s, items);
    else
        hipLaunchKernelGGL((restrict_kernel<float>), xfer_grid(nitems), dim3(kXferThreads), 0, s, items);
    return hipGetLastError();
}

hipError_t launch_prolong(int dtype, int order, const ItemDesc *items, int nitems, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (dtype == PR_FP64) {
        if (order == 3)
            hipLaunchKernelGGL((prolong_kernel<double, 3>), xfer_grid(nitems), dim3(kXferThreads), 0, s, items);
        else
            hipLaunchKernelGGL((prolong_kernel<double, 1>), xfer_grid(nitems), dim3(kXferThreads), 0, s, items);
    } else {
        if (order == 3)
            hipLaunchKernelGGL((prolong_kernel<float, 3>), xfer_grid(nitems), dim3(kXferThreads), 0, s, items);
        else
            hipLaunchKernelGGL((prolong_kernel<float, 1>), xfer_grid(nitems), dim3(kXferThreads), 0, s, items);
    }
    return hipGetLastError();
}

}  // namespace pr
