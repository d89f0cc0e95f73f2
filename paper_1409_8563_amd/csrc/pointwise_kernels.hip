// Pointwise kernels: the Parareal correction (FP64), dtype casts and the
// deterministic two-pass defect norms (Section 2.2, eq. parareal; Section
// 2.2.3, eq. defect and the consecutive-iterate monitor).
//
// Reductions use a fixed grid (kNormBlocks blocks per item, grid-stride
// loop), a fixed butterfly inside each wavefront, a fixed order across the
// wavefronts of a block, and a one-block final pass over the partials in
// index order: results do not depend on timing or launch order.
#include "pr_internal.h"

namespace pr {
namespace {

#define PR_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const PR_GLOBAL T *G(const void *p)
{
    return (const PR_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ PR_GLOBAL T *Gw(void *p)
{
    return (PR_GLOBAL T *)p;
}

struct PointArgs {
    const PointItem *table;  // device table, or nullptr to use `inl`
    PointItem inl;           // single inline item
};

__device__ __forceinline__ void load_item(const PointArgs &a, int i, PointItem &it)
{
    if (a.table) it = a.table[i];
    else it = a.inl;
}

struct Acc4 {
    double mx, mr, sx, sr;
};

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

// Maximum that propagates NaN (fmax drops it): a field holding a NaN must
// give a NaN maximum, so that a defect norm or the early-stop test cannot
// report a small value for it.  Order independent like fmax: the result is
// NaN if either operand is NaN, else the larger one.
__device__ __forceinline__ double nmax(double m, double v) { return (v != v || v > m) ? v : m; }

// Deterministic block reduction of (max, max, sum, sum); result valid in thread 0.
__device__ __forceinline__ Acc4 block_reduce(Acc4 a)
{
    __shared__ double red[kNormThreads / 64][4];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        a.mx = nmax(a.mx, shfl_xor_d(a.mx, m));
        a.mr = nmax(a.mr, shfl_xor_d(a.mr, m));
        a.sx = a.sx + shfl_xor_d(a.sx, m);
        a.sr = a.sr + shfl_xor_d(a.sr, m);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[wv][0] = a.mx;
        red[wv][1] = a.mr;
        red[wv][2] = a.sx;
        red[wv][3] = a.sr;
    }
    __syncthreads();
    Acc4 r{0.0, 0.0, 0.0, 0.0};
    if (threadIdx.x == 0) {
        for (int w = 0; w < kNormThreads / 64; ++w) {
            r.mx = nmax(r.mx, red[w][0]);
            r.mr = nmax(r.mr, red[w][1]);
            r.sx = r.sx + red[w][2];
            r.sr = r.sr + red[w][3];
        }
    }
    return r;
}

template <typename T>
__global__ void __launch_bounds__(kNormThreads) pointwise_kernel(PointArgs args, int op, int with_partials)
{
    PointItem it;
    load_item(args, (int)blockIdx.y, it);
    const int64_t n = it.npts;
    const int64_t stride = (int64_t)gridDim.x * kNormThreads;
    Acc4 acc{0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kNormThreads + threadIdx.x; i < n; i += stride) {
        double u;
        if (op == kOpCorrect) {
            const double f = (double)G<T>(it.a)[i];
            const double gn = (double)G<T>(it.b)[i];
            const double go = (double)G<T>(it.c)[i];
            u = f + (gn - go);
        } else if (op == kOpAssign) {
            u = (double)G<T>(it.a)[i];
        } else {
            u = G<double>(it.a)[i];
        }
        if (with_partials) {
            const double d = u - G<double>(it.u)[i];
            acc.mx = nmax(acc.mx, fabs(d));
            acc.mr = nmax(acc.mr, fabs(u));
            acc.sx += d * d;
            acc.sr += u * u;
        }
        if (it.u) Gw<double>(it.u)[i] = u;
        if (it.ulo) Gw<T>(it.ulo)[i] = (T)u;
    }
    if (with_partials) {
        const Acc4 r = block_reduce(acc);
        if (threadIdx.x == 0) {
            double *p = it.partials + (size_t)blockIdx.x * 4;
            p[0] = r.mx;
            p[1] = r.mr;
            p[2] = r.sx;
            p[3] = r.sr;
        }
    }
}

template <typename TX, typename TR>
__global__ void __launch_bounds__(kNormThreads) defect_partials_kernel(PointArgs args)
{
    PointItem it;
    load_item(args, (int)blockIdx.y, it);
    const int64_t n = it.npts;
    const int64_t stride = (int64_t)gridDim.x * kNormThreads;
    Acc4 acc{0.0, 0.0, 0.0, 0.0};
    const PR_GLOBAL TX *x = G<TX>(it.a);
    const PR_GLOBAL TR *r = G<TR>(it.b);
    for (int64_t i = (int64_t)blockIdx.x * kNormThreads + threadIdx.x; i < n; i += stride) {
        const double rv = (double)r[i];
        const double d = (double)x[i] - rv;
        acc.mx = nmax(acc.mx, fabs(d));
        acc.mr = nmax(acc.mr, fabs(rv));
        acc.sx += d * d;
        acc.sr += rv * rv;
    }
    const Acc4 res = block_reduce(acc);
    if (threadIdx.x == 0) {
        double *p = it.partials + (size_t)blockIdx.x * 4;
        p[0] = res.mx;
        p[1] = res.mr;
        p[2] = res.sx;
        p[3] = res.sr;
    }
}

// One block per item: reduce the kNormBlocks partials in index order.
__global__ void __launch_bounds__(kNormThreads) defect_final_kernel(PointArgs args)
{
    PointItem it;
    load_item(args, (int)blockIdx.x, it);
    Acc4 acc{0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < kNormBlocks; b += kNormThreads) {
        const double *p = it.partials + (size_t)b * 4;
        acc.mx = nmax(acc.mx, p[0]);
        acc.mr = nmax(acc.mr, p[1]);
        acc.sx += p[2];
        acc.sr += p[3];
    }
    const Acc4 r = block_reduce(acc);
    if (threadIdx.x == 0) {
        it.out4[0] = r.mx;
        it.out4[1] = r.mr;
        it.out4[2] = r.sx;
        it.out4[3] = r.sr;
    }
}

constexpr int kWriteBatch = 16;
struct ItemBatch {
    ItemDesc v[kWriteBatch];
    int n;
};
struct PointBatch {
    PointItem v[kWriteBatch * 2];
    int n;
};

__global__ void write_items_kernel(ItemBatch b, ItemDesc *dst)
{
    const int i = (int)threadIdx.x;
    if (i < b.n) dst[i] = b.v[i];
}

__global__ void write_points_kernel(PointBatch b, PointItem *dst)
{
    const int i = (int)threadIdx.x;
    if (i < b.n) dst[i] = b.v[i];
}

}  // namespace

hipError_t launch_pointwise(int op, int sweep_dtype, const PointItem *items, int nitems, bool with_partials,
                            hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    PointArgs a{};
    a.table = items;
    const dim3 grid(kNormBlocks, nitems);
    if (sweep_dtype == 2)
        hipLaunchKernelGGL(pointwise_kernel<double>, grid, dim3(kNormThreads), 0, s, a, op, with_partials ? 1 : 0);
    else
        hipLaunchKernelGGL(pointwise_kernel<float>, grid, dim3(kNormThreads), 0, s, a, op, with_partials ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_pointwise_inline(int op, int sweep_dtype, const PointItem &item, hipStream_t s)
{
    PointArgs a{};
    a.table = nullptr;
    a.inl = item;
    const dim3 grid(kNormBlocks, 1);
    if (sweep_dtype == 2)
        hipLaunchKernelGGL(pointwise_kernel<double>, grid, dim3(kNormThreads), 0, s, a, op, 0);
    else
        hipLaunchKernelGGL(pointwise_kernel<float>, grid, dim3(kNormThreads), 0, s, a, op, 0);
    return hipGetLastError();
}

hipError_t launch_defect_partials(int xd, int rd, const PointItem *items, int nitems, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    PointArgs a{};
    a.table = items;
    const dim3 grid(kNormBlocks, nitems);
    if (xd == 2 && rd == 2)
        hipLaunchKernelGGL((defect_partials_kernel<double, double>), grid, dim3(kNormThreads), 0, s, a);
    else if (xd == 2 && rd == 1)
        hipLaunchKernelGGL((defect_partials_kernel<double, float>), grid, dim3(kNormThreads), 0, s, a);
    else if (xd == 1 && rd == 2)
        hipLaunchKernelGGL((defect_partials_kernel<float, double>), grid, dim3(kNormThreads), 0, s, a);
    else
        hipLaunchKernelGGL((defect_partials_kernel<float, float>), grid, dim3(kNormThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_defect_final(const PointItem *items, int nitems, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    PointArgs a{};
    a.table = items;
    hipLaunchKernelGGL(defect_final_kernel, dim3(nitems), dim3(kNormThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_write_items(const ItemDesc *host_items, int n, ItemDesc *dev_table, hipStream_t s)
{
    for (int off = 0; off < n; off += kWriteBatch) {
        ItemBatch b{};
        b.n = (n - off) < kWriteBatch ? (n - off) : kWriteBatch;
        for (int i = 0; i < b.n; ++i) b.v[i] = host_items[off + i];
        hipLaunchKernelGGL(write_items_kernel, dim3(1), dim3(64), 0, s, b, dev_table + off);
    }
    return hipGetLastError();
}

hipError_t launch_write_points(const PointItem *host_items, int n, PointItem *dev_table, hipStream_t s)
{
    for (int off = 0; off < n; off += 2 * kWriteBatch) {
        PointBatch b{};
        b.n = (n - off) < 2 * kWriteBatch ? (n - off) : 2 * kWriteBatch;
        for (int i = 0; i < b.n; ++i) b.v[i] = host_items[off + i];
        hipLaunchKernelGGL(write_points_kernel, dim3(1), dim3(64), 0, s, b, dev_table + off);
    }
    return hipGetLastError();
}

}  // namespace pr
