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

// Interpolation, one thread per coarse cell (x, y, z): it writes the 8 fine
// points (2x+px, 2y+py, 2z+pz), px, py, pz in {0, 1}.  Per direction an even
// fine index copies the coarse point, an odd one takes coarse offsets 0, 1
// with weights 1/2, 1/2 (ORDER 1) or offsets -1, 0, 1, 2 with -1/16, 9/16,
// 9/16, -1/16 (ORDER 3), periodic.  A fine value is the tensor-product sum
// of the terms (wz*wy*wx) * value, z taps outermost, then y, then x, added
// in that order (the weight products are exact).
template <int ORDER>
struct Taps;
template <>
struct Taps<1> {
    static constexpr int lo = 0, n = 2;   // coarse offsets lo .. lo+n-1 around the cell
    template <typename T>
    __device__ static constexpr T w(int k) { return (T)0.5; }
};
template <>
struct Taps<3> {
    static constexpr int lo = -1, n = 4;
    template <typename T>
    __device__ static constexpr T w(int k) { return (k == 0 || k == 3) ? (T)(-1.0 / 16.0) : (T)(9.0 / 16.0); }
};

template <typename T, int ORDER>
__global__ void __launch_bounds__(kXferThreads) prolong_kernel(const ItemDesc *__restrict__ items)
{
    using TP = Taps<ORDER>;
    constexpr int NO = TP::n;
    const ItemDesc &it = items[blockIdx.y];
    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const int64_t nc = (int64_t)cx * cy * cz;
    const PR_GLOBAL T *src = (const PR_GLOBAL T *)it.src0;
    PR_GLOBAL T *dst = (PR_GLOBAL T *)it.dst;
    for (int64_t i = (int64_t)blockIdx.x * kXferThreads + threadIdx.x; i < nc;
         i += (int64_t)gridDim.x * kXferThreads) {
        const int x = (int)(i % cx);
        const int64_t r = i / cx;
        const int y = (int)(r % cy);
        const int z = (int)(r / cy);
        int ox[NO], oy[NO], oz[NO];
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            ox[k] = wrapc(x + TP::lo + k, cx);
            oy[k] = wrapc(y + TP::lo + k, cy);
            oz[k] = wrapc(z + TP::lo + k, cz);
        }
        T v[NO][NO][NO];
#pragma unroll
        for (int c = 0; c < NO; ++c)
#pragma unroll
            for (int b = 0; b < NO; ++b) {
                const PR_GLOBAL T *row = src + ((int64_t)oz[c] * cy + oy[b]) * cx;
#pragma unroll
                for (int a = 0; a < NO; ++a) v[c][b][a] = row[ox[a]];
            }
        constexpr int E = -TP::lo;   // offset index of the cell's own coarse point
        T out[2][2][2];
#pragma unroll
        for (int pz = 0; pz < 2; ++pz)
#pragma unroll
            for (int py = 0; py < 2; ++py)
#pragma unroll
                for (int px = 0; px < 2; ++px) {
                    const int nzt = pz ? NO : 1, nyt = py ? NO : 1, nxt = px ? NO : 1;
                    T acc = (T)0;
#pragma unroll
                    for (int c = 0; c < nzt; ++c)
#pragma unroll
                        for (int b = 0; b < nyt; ++b) {
                            const T wz = pz ? TP::template w<T>(c) : (T)1;
                            const T wy = py ? TP::template w<T>(b) : (T)1;
                            const T wzy = wz * wy;
#pragma unroll
                            for (int a = 0; a < nxt; ++a) {
                                const T wx = px ? TP::template w<T>(a) : (T)1;
                                acc = acc + (wzy * wx) * v[pz ? c : E][py ? b : E][px ? a : E];
                            }
                        }
                    out[pz][py][px] = acc;
                }
#pragma unroll
        for (int pz = 0; pz < 2; ++pz)
#pragma unroll
            for (int py = 0; py < 2; ++py) {
                PR_GLOBAL T *row = dst + ((int64_t)(2 * z + pz) * ny + (2 * y + py)) * nx + 2 * x;
                row[0] = out[pz][py][0];
                row[1] = out[pz][py][1];
            }
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
