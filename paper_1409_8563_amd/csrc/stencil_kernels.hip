// Stencil kernels of the fine propagator F (classical RK4, centered stencils)
// and the coarse propagator G (forward Euler, upwind advection) for gfx950.
//
// Fused kernels march along z.  A block owns an x-y tile extended by a halo
// of (stages x stencil radius) points in x and y, and walks the whole z range
// of its chunk plane by plane.  Every stage of the step (four RK4 stages, or
// S Euler steps) is evaluated on the fly, lagging its predecessor by one
// stencil radius in z: stage inputs live in per-thread register rings of z
// planes, and the current plane of each stage input is exchanged through
// LDS for the in-plane neighbours.  One step therefore costs one read and one
// write of the field in HBM; the halo is recomputed redundantly.
//
// Per-point arithmetic is fixed by `apply()` (operand order and explicit
// fused multiply-adds) and shared with the unfused reference kernels, so
// every kernel variant, tile shape and launch order yields bitwise identical
// fields.
#include "pr_internal.h"

#include <mutex>
#include <utility>

namespace pr {
namespace {

template <int N>
using ic = std::integral_constant<int, N>;

template <typename T, int N>
struct alignas(sizeof(T) * N) Vec {
    T v[N];
};

// Global-memory accesses through address space 1: the compiler then emits
// global_load/global_store, whose completion is tracked by vmcnt alone, so
// waiting for LDS traffic does not also wait for the prefetched plane (flat
// accesses count against both counters).
#define PR_GLOBAL __attribute__((address_space(1)))

template <typename T, int N>
using ExtVec = T __attribute__((ext_vector_type(N)));

template <typename V>
struct VecTraits;
template <typename T, int N>
struct VecTraits<Vec<T, N>> {
    using E = ExtVec<T, N>;
    static constexpr int n = N;
};

template <typename V>
__device__ __forceinline__ V gld(const void *p)
{
    using E = typename VecTraits<V>::E;
    const E e = *(const PR_GLOBAL E *)p;
    V v;
#pragma unroll
    for (int i = 0; i < VecTraits<V>::n; ++i) v.v[i] = e[i];
    return v;
}

template <typename V>
__device__ __forceinline__ void gst(void *p, const V &v)
{
    using E = typename VecTraits<V>::E;
    E e;
#pragma unroll
    for (int i = 0; i < VecTraits<V>::n; ++i) e[i] = v.v[i];
    *(PR_GLOBAL E *)p = e;
}

// Store with the non-temporal hint: the output of a step is not read again
// by this launch, so it need not displace the input planes (which the
// neighbouring tiles re-read for their halos) from the caches.
template <typename V>
__device__ __forceinline__ void gst_nt(void *p, const V &v)
{
    using E = typename VecTraits<V>::E;
    E e;
#pragma unroll
    for (int i = 0; i < VecTraits<V>::n; ++i) e[i] = v.v[i];
    __builtin_nontemporal_store(e, (PR_GLOBAL E *)p);
}

__device__ __forceinline__ int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Blocks are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous range of logical blocks so that neighbouring tiles (which read
// each other's halos) share an L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int find_item(const ItemDesc *__restrict__ items, int nitems, int lb)
{
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].block_begin <= lb) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double nu_at(const ItemDesc &it, double t)
{
    return it.nu0 * (1.0 + it.nu_amp * sin(it.nu_omega * t));
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Stencil weights of one stage: centre, and for every axis d the weights of
// the points at -k and +k (k = 1..R).
template <typename T, int R>
struct Wts {
    T c;
    T m[3][R];
    T p[3][R];
};

// Fine operator L = nu Lap - a.grad, centered differences of order 2R.
template <typename T, int R>
__device__ __forceinline__ Wts<T, R> fine_weights(const ItemDesc &it, double nu)
{
    Wts<T, R> w;
    double c = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double dif = nu * it.inv_h2[d];
        const double adv = it.a_over_h[d];
        if constexpr (R == 1) {
            w.m[d][0] = (T)(dif + 0.5 * adv);
            w.p[d][0] = (T)(dif - 0.5 * adv);
            c += -2.0 * dif;
        } else {
            w.m[d][0] = (T)(dif * (16.0 / 12.0) + adv * (8.0 / 12.0));
            w.p[d][0] = (T)(dif * (16.0 / 12.0) - adv * (8.0 / 12.0));
            w.m[d][1] = (T)(-dif * (1.0 / 12.0) - adv * (1.0 / 12.0));
            w.p[d][1] = (T)(-dif * (1.0 / 12.0) + adv * (1.0 / 12.0));
            c += -dif * (30.0 / 12.0);
        }
    }
    w.c = (T)c;
    return w;
}

// Coarse operator of Algorithm 2: nu * 7-point Laplacian, minus first-order
// upwind advection (backward difference for a_d > 0, forward otherwise).
template <typename T>
__device__ __forceinline__ Wts<T, 1> coarse_weights(const ItemDesc &it, double nu)
{
    Wts<T, 1> w;
    double c = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double dif = nu * it.inv_h2[d];
        const double adv = it.a_over_h[d];
        double m = dif, p = dif;
        c += -2.0 * dif;
        if (adv > 0.0) {
            c -= adv;
            m += adv;
        } else {
            c += adv;
            p -= adv;
        }
        w.m[d][0] = (T)m;
        w.p[d][0] = (T)p;
    }
    w.c = (T)c;
    return w;
}

// The one definition of a stencil application: centre product, then per axis
// x, y, z and per distance k the -k and +k neighbours, each a fused
// multiply-add.  Every kernel evaluates S through this function.
template <typename T, int R>
__device__ __forceinline__ T apply(const Wts<T, R> &w, T cen, const T (&mn)[3][R], const T (&pn)[3][R])
{
    T s = w.c * cen;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            s = fmaT(w.m[d][k], mn[d][k], s);
            s = fmaT(w.p[d][k], pn[d][k], s);
        }
    }
    return s;
}

// Wave-uniform values (weights computed from the step time) are moved to
// scalar registers; VOP3 FMAs take one scalar operand, which frees VGPRs.
__device__ __forceinline__ float uni(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double uni(double x)
{
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, int R>
__device__ __forceinline__ Wts<T, R> uni(const Wts<T, R> &w)
{
    Wts<T, R> o;
    o.c = uni(w.c);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            o.m[d][k] = uni(w.m[d][k]);
            o.p[d][k] = uni(w.p[d][k]);
        }
    return o;
}

template <typename T>
struct RK4Consts {
    T c1, c2, c3, b1, b2, b3, b4;
};

template <typename T>
__device__ __forceinline__ RK4Consts<T> rk4_consts(double dt)
{
    RK4Consts<T> k;
    k.c1 = (T)(0.5 * dt);
    k.c2 = (T)(0.5 * dt);
    k.c3 = (T)dt;
    k.b1 = (T)(dt / 6.0);
    k.b2 = (T)(dt / 3.0);
    k.b3 = (T)(dt / 3.0);
    k.b4 = (T)(dt / 6.0);
    return k;
}

// Step j reads the field written by step j-1 and writes dst for the last step.
template <typename T>
__device__ __forceinline__ void pingpong(const ItemDesc &it, int j, int n, const T *&src, T *&dst)
{
    src = (j == 0) ? (const T *)it.src0 : ((((n - j) & 1) == 0) ? (const T *)it.dst : (const T *)it.tmp);
    dst = ((((n - 1 - j) & 1) == 0) ? (T *)it.dst : (T *)it.tmp);
}

template <int L>
__host__ __device__ constexpr int slot(int m, int off)
{
    return ((m - off) % L + L) % L;
}

// ---------------------------------------------------------------------------
// Fused RK4 step.  Tile of EX x EY threads-points (BXT x BY threads, each
// owning NXP consecutive x and NY consecutive y), output TX x TY, halo 4R.
// ---------------------------------------------------------------------------
template <typename T, int R, int NXP, int NY, int BXT, int BY>
__global__ void __launch_bounds__(BXT *BY)
    rk4_step_fused(const ItemDesc *__restrict__ items, int nitems, int jstep)
{
    constexpr int H = 4 * R;
    constexpr int EX = BXT * NXP, EY = BY * NY;
    constexpr int TX = EX - 2 * H, TY = EY - 2 * H;
    constexpr int L = 3 * R + 1;                       // z-ring length
    constexpr int CO = ((R + NXP - 1) / NXP) * NXP;    // LDS column offset (aligned halo)
    constexpr int LX = EX + 2 * CO + (sizeof(T) == 8 ? 2 : 4);
    constexpr int LY = EY + 2 * R;
    static_assert(TX > 0 && TY > 0, "tile too small for the halo");
    __shared__ __align__(16) T lds[2][LY][LX];

    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    if (jstep >= it.nsteps) return;
    const int local = lb - it.block_begin;
    if (local < 0 || local >= it.nblocks) return;

    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int txt = local % it.tiles_x;
    const int rest = local / it.tiles_x;
    const int tyt = rest % it.tiles_y;
    const int zc = rest / it.tiles_y;
    const int x0 = txt * TX, y0 = tyt * TY;
    const int z0 = zc * it.tz;
    const int zend = min(z0 + it.tz, nz);

    const T *src;
    T *dst;
    pingpong<T>(it, jstep, it.nsteps, src, dst);

    const int tid = (int)threadIdx.x;
    const int txi = tid % BXT, tyi = tid / BXT;
    const int cx0 = txi * NXP, ry0 = tyi * NY;
    const int gx0 = wrapi(x0 - H + cx0, nx);
    int rowoff[NY];
    bool yok[NY];
#pragma unroll
    for (int iy = 0; iy < NY; ++iy) {
        const int ry = ry0 + iy;
        rowoff[iy] = wrapi(y0 - H + ry, ny) * nx + gx0;
        yok[iy] = (ry >= H) && (ry < H + TY) && (y0 + ry - H < ny);
    }
    const bool xok = (cx0 >= H) && (cx0 < H + TX) && (x0 + cx0 - H < nx);
    const int nxy = nx * ny;

    // stage times and weights
    const double dt = it.dt;
    const double t = (double)(it.step0 + jstep) * dt;
    const double nu1 = nu_at(it, t);
    const double nu2 = it.frozen ? nu1 : nu_at(it, t + 0.5 * dt);
    const double nu4 = it.frozen ? nu1 : nu_at(it, t + dt);
    const Wts<T, R> w1 = uni(fine_weights<T, R>(it, nu1));
    const Wts<T, R> w2 = uni(fine_weights<T, R>(it, nu2));
    const Wts<T, R> w4 = uni(fine_weights<T, R>(it, nu4));
    RK4Consts<T> kc = rk4_consts<T>(dt);
    kc.c1 = uni(kc.c1);
    kc.c2 = uni(kc.c2);
    kc.c3 = uni(kc.c3);
    kc.b1 = uni(kc.b1);
    kc.b2 = uni(kc.b2);
    kc.b3 = uni(kc.b3);
    kc.b4 = uni(kc.b4);

    T ur[L][NY][NXP], y1[L][NY][NXP], y2[L][NY][NXP], y3[L][NY][NXP], ac[L][NY][NXP];
    T pf[NY][NXP];

    auto load_plane = [&](int p) {
        const T *base = src + (size_t)wrapi(p, nz) * nxy;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            const Vec<T, NXP> v = gld<Vec<T, NXP>>(base + rowoff[iy]);
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) pf[iy][ix] = v.v[ix];
        }
    };

    // Evaluate S = L(f)(plane at offset OFF from p) for the thread's points,
    // f given by its z-ring `in`; uses LDS buffer BUF.
    auto stage = [&](auto Mc, auto OFFc, auto BUFc, T(&in)[L][NY][NXP], const Wts<T, R> &w, bool active,
                     T(&S)[NY][NXP]) {
        constexpr int M = decltype(Mc)::value;
        constexpr int OFF = decltype(OFFc)::value;
        constexpr int B = decltype(BUFc)::value;
        constexpr int sc = slot<L>(M, OFF);
        if (active) {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) {
                Vec<T, NXP> v;
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) v.v[ix] = in[sc][iy][ix];
                *reinterpret_cast<Vec<T, NXP> *>(&lds[B][R + ry0 + iy][CO + cx0]) = v;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) {
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    T mn[3][R], pn[3][R];
#pragma unroll
                    for (int k = 1; k <= R; ++k) {
                        mn[0][k - 1] = (ix - k >= 0) ? in[sc][iy][ix - k] : lds[B][R + ry0 + iy][CO + cx0 + ix - k];
                        pn[0][k - 1] = (ix + k < NXP) ? in[sc][iy][ix + k] : lds[B][R + ry0 + iy][CO + cx0 + ix + k];
                        mn[1][k - 1] = (iy - k >= 0) ? in[sc][iy - k][ix] : lds[B][R + ry0 + iy - k][CO + cx0 + ix];
                        pn[1][k - 1] = (iy + k < NY) ? in[sc][iy + k][ix] : lds[B][R + ry0 + iy + k][CO + cx0 + ix];
                        mn[2][k - 1] = in[slot<L>(M, OFF + k)][iy][ix];   // plane q - k
                        pn[2][k - 1] = in[slot<L>(M, OFF - k)][iy][ix];   // plane q + k
                    }
                    S[iy][ix] = apply<T, R>(w, in[sc][iy][ix], mn, pn);
                }
            }
        }
    };

    auto body = [&](auto Mc, int p) {
        constexpr int M = decltype(Mc)::value;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy)
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) ur[slot<L>(M, 0)][iy][ix] = pf[iy][ix];
        load_plane(p + 1);

        T S[NY][NXP];
        // stage 1 at plane p - R
        const bool a1 = p >= z0 - 2 * R;
        stage(Mc, ic<R>{}, ic<0>{}, ur, w1, a1, S);
        if (a1) {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, R)][iy][ix];
                    y1[slot<L>(M, R)][iy][ix] = fmaT(kc.c1, S[iy][ix], u);
                    ac[slot<L>(M, R)][iy][ix] = fmaT(kc.b1, S[iy][ix], u);
                }
        }
        // stage 2 at plane p - 2R
        const bool a2 = p >= z0;
        stage(Mc, ic<2 * R>{}, ic<1>{}, y1, w2, a2, S);
        if (a2) {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 2 * R)][iy][ix];
                    y2[slot<L>(M, 2 * R)][iy][ix] = fmaT(kc.c2, S[iy][ix], u);
                    ac[slot<L>(M, 2 * R)][iy][ix] = fmaT(kc.b2, S[iy][ix], ac[slot<L>(M, 2 * R)][iy][ix]);
                }
        }
        // stage 3 at plane p - 3R
        const bool a3 = p >= z0 + 2 * R;
        stage(Mc, ic<3 * R>{}, ic<0>{}, y2, w2, a3, S);
        if (a3) {
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 3 * R)][iy][ix];
                    y3[slot<L>(M, 3 * R)][iy][ix] = fmaT(kc.c3, S[iy][ix], u);
                    ac[slot<L>(M, 3 * R)][iy][ix] = fmaT(kc.b3, S[iy][ix], ac[slot<L>(M, 3 * R)][iy][ix]);
                }
        }
        // stage 4 at plane p - 4R, result stored
        const bool a4 = p >= z0 + 4 * R;
        stage(Mc, ic<4 * R>{}, ic<1>{}, y3, w4, a4, S);
        const int q = p - 4 * R;
        if (a4 && q < zend && xok) {
            T *obase = dst + (size_t)q * nxy;
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) {
                if (yok[iy]) {
                    Vec<T, NXP> v;
#pragma unroll
                    for (int ix = 0; ix < NXP; ++ix)
                        v.v[ix] = fmaT(kc.b4, S[iy][ix], ac[slot<L>(M, 4 * R)][iy][ix]);
                    gst<Vec<T, NXP>>(obase + rowoff[iy], v);
                }
            }
        }
    };

    const int pstart = z0 - 4 * R;
    const int niter = (zend - z0) + 8 * R;
    load_plane(pstart);
    for (int pb = 0; pb < niter; pb += L) {
        [&]<int... Ms>(std::integer_sequence<int, Ms...>) {
            (body(ic<Ms>{}, pstart + pb + Ms), ...);
        }(std::make_integer_sequence<int, L>{});
    }
}

// ---------------------------------------------------------------------------
// Fused RK4 step with one barrier per z plane (radius-1 stencils).  Every
// stage writes its *output* plane to LDS; the next stage reads it one
// iteration later, when it is that stage's centre plane.  Two LDS slots per
// stage output alternate between iterations, so a single barrier at the top
// of each iteration separates the writes of iteration p-1 from the reads of
// iteration p and the reads of p-1 from the writes of p.  In-plane
// neighbours are read as aligned NXP-vectors (whole neighbour groups), which
// keeps lanes on consecutive LDS addresses.
// ---------------------------------------------------------------------------
template <typename T, int NXP, int NY, int BXT, int BY, int PD>
__global__ void __launch_bounds__(BXT *BY)
    rk4_step_fused1b(const ItemDesc *__restrict__ items, int nitems, int jstep)
{
    static_assert(4 % PD == 0, "prefetch depth must divide the unroll");
    constexpr int R = 1;
    constexpr int H = 4;
    constexpr int EX = BXT * NXP, EY = BY * NY;
    constexpr int TX = EX - 2 * H, TY = EY - 2 * H;
    constexpr int L = 4;                                   // z-ring length (even: LDS slot = phase parity)
    constexpr int CO = NXP;                                // halo columns in LDS, one aligned group
    constexpr int LX = EX + 2 * CO + (sizeof(T) == 8 ? 2 : 4);
    constexpr int LY = EY + 2;
    static_assert(TX > 0 && TY > 0, "tile too small for the halo");
    __shared__ __align__(16) T lds[4][2][LY][LX];          // [stage input 0..3][slot][row][col]

    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    if (jstep >= it.nsteps) return;
    const int local = lb - it.block_begin;
    if (local < 0 || local >= it.nblocks) return;

    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int txt = local % it.tiles_x;
    const int rest = local / it.tiles_x;
    const int tyt = rest % it.tiles_y;
    const int zc = rest / it.tiles_y;
    const int x0 = txt * TX, y0 = tyt * TY;
    const int z0 = zc * it.tz;
    const int zend = min(z0 + it.tz, nz);

    const T *src;
    T *dst;
    pingpong<T>(it, jstep, it.nsteps, src, dst);

    const int tid = (int)threadIdx.x;
    const int txi = tid % BXT, tyi = tid / BXT;
    const int cx0 = txi * NXP, ry0 = tyi * NY;
    const int gx0 = wrapi(x0 - H + cx0, nx);
    int rowoff[NY];
    bool yok[NY];
#pragma unroll
    for (int iy = 0; iy < NY; ++iy) {
        const int ry = ry0 + iy;
        rowoff[iy] = wrapi(y0 - H + ry, ny) * nx + gx0;
        yok[iy] = (ry >= H) && (ry < H + TY) && (y0 + ry - H < ny);
    }
    const bool xok = (cx0 >= H) && (cx0 < H + TX) && (x0 + cx0 - H < nx);
    const int nxy = nx * ny;

    const double dt = it.dt;
    const double t = (double)(it.step0 + jstep) * dt;
    const double nu1 = nu_at(it, t);
    const double nu2 = it.frozen ? nu1 : nu_at(it, t + 0.5 * dt);
    const double nu4 = it.frozen ? nu1 : nu_at(it, t + dt);
    const Wts<T, R> w1 = uni(fine_weights<T, R>(it, nu1));
    const Wts<T, R> w2 = uni(fine_weights<T, R>(it, nu2));
    const Wts<T, R> w4 = uni(fine_weights<T, R>(it, nu4));
    RK4Consts<T> kc = rk4_consts<T>(dt);
    kc.c1 = uni(kc.c1);
    kc.c2 = uni(kc.c2);
    kc.c3 = uni(kc.c3);
    kc.b1 = uni(kc.b1);
    kc.b2 = uni(kc.b2);
    kc.b3 = uni(kc.b3);
    kc.b4 = uni(kc.b4);

    T ur[L][NY][NXP], y1[L][NY][NXP], y2[L][NY][NXP], y3[L][NY][NXP], ac[L][NY][NXP];
    T pf[PD][NY][NXP];   // planes p .. p+PD-1 in flight (prefetch ring)

    auto load_plane = [&](int p, T(&dstp)[NY][NXP]) {
        const T *base = src + (size_t)wrapi(p, nz) * nxy;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            const Vec<T, NXP> v = gld<Vec<T, NXP>>(base + rowoff[iy]);
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) dstp[iy][ix] = v.v[ix];
        }
    };

    // write this thread's values of a plane to LDS buffer B, slot SL
    auto put = [&](auto Bc, auto SLc, const T(&v)[NY][NXP]) {
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            Vec<T, NXP> w;
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) w.v[ix] = v[iy][ix];
            *reinterpret_cast<Vec<T, NXP> *>(&lds[B][SL][1 + ry0 + iy][CO + cx0]) = w;
        }
    };

    // S = L(f)(plane q) for the thread's points.  Centre and z neighbours
    // from the ring `in` (slots SC, SC_M = plane q-1, SC_P = plane q+1),
    // in-plane neighbours from LDS buffer B, slot SL.
    auto stencil = [&](auto Bc, auto SLc, const T(&in)[L][NY][NXP], auto SCc, auto SCMc, auto SCPc,
                       const Wts<T, R> &w, T(&S)[NY][NXP]) {
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
        constexpr int SC = decltype(SCc)::value;
        constexpr int SCM = decltype(SCMc)::value;
        constexpr int SCP = decltype(SCPc)::value;
        Vec<T, NXP> up, dn;
        up = *reinterpret_cast<const Vec<T, NXP> *>(&lds[B][SL][ry0][CO + cx0]);
        dn = *reinterpret_cast<const Vec<T, NXP> *>(&lds[B][SL][1 + ry0 + NY][CO + cx0]);
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            const Vec<T, NXP> lf = *reinterpret_cast<const Vec<T, NXP> *>(&lds[B][SL][1 + ry0 + iy][CO + cx0 - NXP]);
            const Vec<T, NXP> rt = *reinterpret_cast<const Vec<T, NXP> *>(&lds[B][SL][1 + ry0 + iy][CO + cx0 + NXP]);
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) {
                T mn[3][1], pn[3][1];
                mn[0][0] = (ix >= 1) ? in[SC][iy][ix - 1] : lf.v[NXP - 1];
                pn[0][0] = (ix + 1 < NXP) ? in[SC][iy][ix + 1] : rt.v[0];
                mn[1][0] = (iy >= 1) ? in[SC][iy - 1][ix] : up.v[ix];
                pn[1][0] = (iy + 1 < NY) ? in[SC][iy + 1][ix] : dn.v[ix];
                mn[2][0] = in[SCM][iy][ix];
                pn[2][0] = in[SCP][iy][ix];
                S[iy][ix] = apply<T, 1>(w, in[SC][iy][ix], mn, pn);
            }
        }
    };

    auto body = [&](auto Mc, int p) {
        constexpr int M = decltype(Mc)::value;
        constexpr int WS = M & 1;        // slot written in this iteration
        constexpr int RS = (M + 1) & 1;  // slot written in the previous iteration
        __syncthreads();
#pragma unroll
        for (int iy = 0; iy < NY; ++iy)
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) ur[slot<L>(M, 0)][iy][ix] = pf[M % PD][iy][ix];
        load_plane(p + PD, pf[M % PD]);
        put(ic<0>{}, ic<WS>{}, ur[slot<L>(M, 0)]);

        T S[NY][NXP];
        // stage 1 at plane p - 1
        if (p >= z0 - 2) {
            stencil(ic<0>{}, ic<RS>{}, ur, ic<slot<L>(M, 1)>{}, ic<slot<L>(M, 2)>{}, ic<slot<L>(M, 0)>{}, w1, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 1)][iy][ix];
                    y1[slot<L>(M, 1)][iy][ix] = fmaT(kc.c1, S[iy][ix], u);
                    ac[slot<L>(M, 1)][iy][ix] = fmaT(kc.b1, S[iy][ix], u);
                }
            put(ic<1>{}, ic<WS>{}, y1[slot<L>(M, 1)]);
        }
        // stage 2 at plane p - 2
        if (p >= z0) {
            stencil(ic<1>{}, ic<RS>{}, y1, ic<slot<L>(M, 2)>{}, ic<slot<L>(M, 3)>{}, ic<slot<L>(M, 1)>{}, w2, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 2)][iy][ix];
                    y2[slot<L>(M, 2)][iy][ix] = fmaT(kc.c2, S[iy][ix], u);
                    ac[slot<L>(M, 2)][iy][ix] = fmaT(kc.b2, S[iy][ix], ac[slot<L>(M, 2)][iy][ix]);
                }
            put(ic<2>{}, ic<WS>{}, y2[slot<L>(M, 2)]);
        }
        // stage 3 at plane p - 3
        if (p >= z0 + 2) {
            stencil(ic<2>{}, ic<RS>{}, y2, ic<slot<L>(M, 3)>{}, ic<slot<L>(M, 4)>{}, ic<slot<L>(M, 2)>{}, w2, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 3)][iy][ix];
                    y3[slot<L>(M, 3)][iy][ix] = fmaT(kc.c3, S[iy][ix], u);
                    ac[slot<L>(M, 3)][iy][ix] = fmaT(kc.b3, S[iy][ix], ac[slot<L>(M, 3)][iy][ix]);
                }
            put(ic<3>{}, ic<WS>{}, y3[slot<L>(M, 3)]);
        }
        // stage 4 at plane p - 4, stored
        const int q = p - 4;
        if (p >= z0 + 4 && q < zend) {
            stencil(ic<3>{}, ic<RS>{}, y3, ic<slot<L>(M, 4)>{}, ic<slot<L>(M, 5)>{}, ic<slot<L>(M, 3)>{}, w4, S);
            if (xok) {
                T *obase = dst + (size_t)q * nxy;
#pragma unroll
                for (int iy = 0; iy < NY; ++iy) {
                    if (yok[iy]) {
                        Vec<T, NXP> v;
#pragma unroll
                        for (int ix = 0; ix < NXP; ++ix)
                            v.v[ix] = fmaT(kc.b4, S[iy][ix], ac[slot<L>(M, 4)][iy][ix]);
                        gst<Vec<T, NXP>>(obase + rowoff[iy], v);
                    }
                }
            }
        }
    };

    const int pstart = z0 - 4;
    const int niter = (zend - z0) + 8;
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(pstart + d, pf[d]);
    for (int pb = 0; pb < niter; pb += L) {
        [&]<int... Ms>(std::integer_sequence<int, Ms...>) {
            (body(ic<Ms>{}, pstart + pb + Ms), ...);
        }(std::make_integer_sequence<int, L>{});
    }
}

// ---------------------------------------------------------------------------
// Fused RK4 step over whole x rows (radius-1 stencils, n_x = 64 * NXP).
//
// Lane l of a wavefront holds x = l*NXP .. l*NXP + NXP-1 of NY consecutive
// rows, so a wavefront covers complete periodic rows: the x neighbours of a
// point are the lane's own values and, at the ends of its group, the values
// of lanes l-1 and l+1 (mod 64), moved across the wavefront with DPP
// rotations (every source lane exists, so the bound control is moot).  No
// x halo exists and no LDS traffic is spent on x.  In y the
// block holds EY = NW*NY rows (output TY = EY - 8: a halo of 4 rows per side
// for the four stages); y neighbours inside a wavefront's rows come from
// registers, and each wavefront exchanges only its first and last row with
// its neighbours through LDS.  A wavefront skips a stage once all its rows
// lie within s rows of the tile edge, where stage s can no longer feed an
// output point.  z pipeline, prefetch ring and one-barrier LDS double
// buffering as in rk4_step_fused1b.
// ---------------------------------------------------------------------------
constexpr int kDppWaveRor1 = 0x13C;  // lane l receives the value of lane (l - 1) mod 64
constexpr int kDppWaveRol1 = 0x134;  // lane l receives the value of lane (l + 1) mod 64
// rotations inside each row of 16 lanes (lane l, row base b = l & ~15):
constexpr int kDppRowRor1 = 0x121;   // lane l receives lane b + (l - 1) mod 16
constexpr int kDppRowRor15 = 0x12F;  // lane l receives lane b + (l + 1) mod 16

// N consecutive elements of a row moved in the widest aligned pieces: four
// or two elements when N is a multiple of that (the start is then aligned to
// the piece, since it is a multiple of N elements into a 16-byte aligned
// row), single elements otherwise.
template <int N>
constexpr int piece_of() { return N % 4 == 0 ? 4 : (N % 2 == 0 ? 2 : 1); }

template <typename T, int N>
__device__ __forceinline__ void gld_row(const T *p, T (&d)[N])
{
    constexpr int C = piece_of<N>();
#pragma unroll
    for (int k = 0; k < N / C; ++k) {
        if constexpr (C == 1) {
            d[k] = *(const PR_GLOBAL T *)(p + k);
        } else {
            const ExtVec<T, C> e = *(const PR_GLOBAL ExtVec<T, C> *)(p + k * C);
#pragma unroll
            for (int i = 0; i < C; ++i) d[k * C + i] = e[i];
        }
    }
}
template <typename T, int N>
__device__ __forceinline__ void gst_nt_row(T *p, const T (&v)[N])
{
    constexpr int C = piece_of<N>();
#pragma unroll
    for (int k = 0; k < N / C; ++k) {
        if constexpr (C == 1) {
            __builtin_nontemporal_store(v[k], (PR_GLOBAL T *)(p + k));
        } else {
            ExtVec<T, C> e;
#pragma unroll
            for (int i = 0; i < C; ++i) e[i] = v[k * C + i];
            __builtin_nontemporal_store(e, (PR_GLOBAL ExtVec<T, C> *)(p + k * C));
        }
    }
}
template <typename T, int N>
__device__ __forceinline__ void lds_st_row(T *p, const T (&v)[N])
{
    constexpr int C = piece_of<N>();
#pragma unroll
    for (int k = 0; k < N / C; ++k) {
        Vec<T, C> e;
#pragma unroll
        for (int i = 0; i < C; ++i) e.v[i] = v[k * C + i];
        *reinterpret_cast<Vec<T, C> *>(p + k * C) = e;
    }
}
template <typename T, int N>
__device__ __forceinline__ void lds_ld_row(const T *p, T (&d)[N])
{
    constexpr int C = piece_of<N>();
#pragma unroll
    for (int k = 0; k < N / C; ++k) {
        const Vec<T, C> e = *reinterpret_cast<const Vec<T, C> *>(p + k * C);
#pragma unroll
        for (int i = 0; i < C; ++i) d[k * C + i] = e.v[i];
    }
}

template <int CTRL>
__device__ __forceinline__ float wave_rot(float v)
{
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double wave_rot(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, int NXP, int NY, int NW, int PD, int SEG, int XT = 0>
__global__ void __launch_bounds__(64 * NW)
    rk4_step_rows(const ItemDesc *__restrict__ items, int nitems, int jstep)
{
    static_assert(4 % PD == 0, "prefetch depth must divide the unroll");
    static_assert(SEG == 64 || SEG == 16, "a grid row spans a wavefront or a 16-lane DPP row");
    static_assert(!XT || SEG == 64, "x tiles span a wavefront");
    constexpr int R = 1;
    constexpr int H = 4;
    constexpr int RG = 64 / SEG;          // grid rows side by side in a wavefront
    constexpr int NVW = NW * RG;          // row groups of the block
    constexpr int NX = SEG * NXP;         // x extent of a row group (the whole row unless XT)
    constexpr int HX = XT ? H : 0;        // x halo of an x tile
    constexpr int TXT = NX - 2 * HX;      // output columns of an x tile
    constexpr int EY = NVW * NY, TY = EY - 2 * H;
    constexpr int L = 4;                  // z-ring length (even: LDS slot = phase parity)
    constexpr int NE = NY == 1 ? 1 : 2;   // exchanged rows per row group: first, last
    static_assert(TY > 0, "tile too small for the halo");
    __shared__ __align__(16) T lds[4][2][NVW][NE][NX];   // [stage input][slot][row group][edge][x]

    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    if (jstep >= it.nsteps || (!XT && it.nx != NX)) return;
    const int local = lb - it.block_begin;
    if (local < 0 || local >= it.nblocks) return;

    const int nx = XT ? it.nx : NX, ny = it.ny, nz = it.nz;
    int txt = 0, rest = local;
    if constexpr (XT) {
        txt = local % it.tiles_x;
        rest = local / it.tiles_x;
    }
    const int tyt = rest % it.tiles_y;
    const int zc = rest / it.tiles_y;
    const int x0 = txt * TXT;
    const int y0 = tyt * TY;
    const int z0 = zc * it.tz;
    const int zend = min(z0 + it.tz, nz);

    const T *src;
    T *dst;
    pingpong<T>(it, jstep, it.nsteps, src, dst);

    const int lane = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int vw = wv * RG + lane / SEG;          // row group (the wavefront itself for SEG = 64)
    const int wup = vw > 0 ? vw - 1 : 0;          // clamped: row group 0 never uses its upper neighbour
    const int wdn = vw < NVW - 1 ? vw + 1 : NVW - 1;
    const int ry0 = vw * NY;
    const int cx0 = (lane % SEG) * NXP;
    int rowoff[NY];
    bool rowout[NY];
#pragma unroll
    for (int iy = 0; iy < NY; ++iy) {
        const int ry = ry0 + iy;
        rowoff[iy] = wrapi(y0 - H + ry, ny) * nx + (XT ? 0 : cx0);
        rowout[iy] = (ry >= H) && (ry < H + TY) && (y0 + ry - H < ny);
    }
    // x tiles: the lane's columns, wrapped onto the periodic row, and which
    // of them are outputs of this tile (inside the halo, and not past n_x in
    // the last, ragged tile).  A row group's lanes hold consecutive columns,
    // so the rotated-in x neighbours are right except at the two ends of the
    // wavefront, whose errors reach at most one column further per stage:
    // four stages stay inside the 4-column halo.
    int colx[XT ? NXP : 1];
    bool colout[XT ? NXP : 1];
    if constexpr (XT) {
#pragma unroll
        for (int ix = 0; ix < NXP; ++ix) {
            const int c = cx0 + ix;
            colx[ix] = wrapi(x0 - HX + c, nx);
            colout[ix] = (c >= HX) && (c < HX + TXT) && (x0 + c - HX < nx);
        }
    }
    const int nxy = nx * ny;
    // stage s (1..4) can feed an output point only on rows s .. EY-1-s; a
    // wavefront runs a stage if any of its rows needs it
    const int wr0 = wv * RG * NY;
    auto wave_active = [&](int s) { return wr0 + RG * NY - 1 >= s && wr0 < EY - s; };
    const bool act1 = wave_active(1), act2 = wave_active(2), act3 = wave_active(3), act4 = wave_active(4);

    const double dt = it.dt;
    const double t = (double)(it.step0 + jstep) * dt;
    const double nu1 = nu_at(it, t);
    const double nu2 = it.frozen ? nu1 : nu_at(it, t + 0.5 * dt);
    const double nu4 = it.frozen ? nu1 : nu_at(it, t + dt);
    const Wts<T, R> w1 = uni(fine_weights<T, R>(it, nu1));
    const Wts<T, R> w2 = uni(fine_weights<T, R>(it, nu2));
    const Wts<T, R> w4 = uni(fine_weights<T, R>(it, nu4));
    RK4Consts<T> kc = rk4_consts<T>(dt);
    kc.c1 = uni(kc.c1);
    kc.c2 = uni(kc.c2);
    kc.c3 = uni(kc.c3);
    kc.b1 = uni(kc.b1);
    kc.b2 = uni(kc.b2);
    kc.b3 = uni(kc.b3);
    kc.b4 = uni(kc.b4);

    T ur[L][NY][NXP], y1[L][NY][NXP], y2[L][NY][NXP], y3[L][NY][NXP], ac[L][NY][NXP];
    T pf[PD][NY][NXP];

    auto load_plane = [&](int p, T(&dstp)[NY][NXP]) {
        const T *base = src + (size_t)wrapi(p, nz) * nxy;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            if constexpr (XT) {
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) dstp[iy][ix] = *(const PR_GLOBAL T *)(base + rowoff[iy] + colx[ix]);
            } else {
                gld_row<T, NXP>(base + rowoff[iy], dstp[iy]);
            }
        }
    };

    // first and last row of this row group's values of a plane -> LDS
    auto put = [&](auto Bc, auto SLc, const T(&v)[NY][NXP]) {
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
        lds_st_row<T, NXP>(&lds[B][SL][vw][0][cx0], v[0]);
        if constexpr (NE == 2) lds_st_row<T, NXP>(&lds[B][SL][vw][1][cx0], v[NY - 1]);
    };

    // rows above and below this row group of a plane of stage input B, slot SL
    struct Nb {
        T up[NXP], dn[NXP];
    };
    auto fetch = [&](auto Bc, auto SLc) {
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
        Nb nb;
        lds_ld_row<T, NXP>(&lds[B][SL][wup][NE - 1][cx0], nb.up);
        lds_ld_row<T, NXP>(&lds[B][SL][wdn][0][cx0], nb.dn);
        return nb;
    };

    // S = L(f)(plane q) on this wavefront's rows.  Centre and z neighbours
    // from the ring `in` (slots SC, SCM = plane q-1, SCP = plane q+1); the
    // rows above and below the wavefront from `nb`.
    auto stencil = [&](const Nb &nb, const T(&in)[L][NY][NXP], auto SCc, auto SCMc, auto SCPc, const Wts<T, R> &w,
                       T(&S)[NY][NXP]) {
        constexpr int SC = decltype(SCc)::value;
        constexpr int SCM = decltype(SCMc)::value;
        constexpr int SCP = decltype(SCPc)::value;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            const T left = wave_rot<SEG == 64 ? kDppWaveRor1 : kDppRowRor1>(in[SC][iy][NXP - 1]);
            const T right = wave_rot<SEG == 64 ? kDppWaveRol1 : kDppRowRor15>(in[SC][iy][0]);
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) {
                T mn[3][1], pn[3][1];
                mn[0][0] = (ix >= 1) ? in[SC][iy][ix - 1] : left;
                pn[0][0] = (ix + 1 < NXP) ? in[SC][iy][ix + 1] : right;
                mn[1][0] = (iy >= 1) ? in[SC][iy - 1][ix] : nb.up[ix];
                pn[1][0] = (iy + 1 < NY) ? in[SC][iy + 1][ix] : nb.dn[ix];
                mn[2][0] = in[SCM][iy][ix];
                pn[2][0] = in[SCP][iy][ix];
                S[iy][ix] = apply<T, 1>(w, in[SC][iy][ix], mn, pn);
            }
        }
    };

    // FAST: a wavefront that computes all four stages, after the pipeline
    // fill (every stage active): straight-line code, only the store guarded.
    auto body = [&](auto Mc, auto FASTc, int p) __attribute__((always_inline)) {
        constexpr int M = decltype(Mc)::value;
        constexpr bool FAST = decltype(FASTc)::value;
        constexpr int WS = M & 1;        // slot written in this iteration
        constexpr int RS = (M + 1) & 1;  // slot written in the previous iteration
        __syncthreads();
#pragma unroll
        for (int iy = 0; iy < NY; ++iy)
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) ur[slot<L>(M, 0)][iy][ix] = pf[M % PD][iy][ix];
        load_plane(p + PD, pf[M % PD]);
        put(ic<0>{}, ic<WS>{}, ur[slot<L>(M, 0)]);

        // the four stage updates, each reading its in-plane neighbour rows nb
        auto st1 = [&](const Nb &nb) __attribute__((always_inline)) {
            T S[NY][NXP];
            stencil(nb, ur, ic<slot<L>(M, 1)>{}, ic<slot<L>(M, 2)>{}, ic<slot<L>(M, 0)>{}, w1, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 1)][iy][ix];
                    y1[slot<L>(M, 1)][iy][ix] = fmaT(kc.c1, S[iy][ix], u);
                    ac[slot<L>(M, 1)][iy][ix] = fmaT(kc.b1, S[iy][ix], u);
                }
            put(ic<1>{}, ic<WS>{}, y1[slot<L>(M, 1)]);
        };
        auto st2 = [&](const Nb &nb) __attribute__((always_inline)) {
            T S[NY][NXP];
            stencil(nb, y1, ic<slot<L>(M, 2)>{}, ic<slot<L>(M, 3)>{}, ic<slot<L>(M, 1)>{}, w2, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 2)][iy][ix];
                    y2[slot<L>(M, 2)][iy][ix] = fmaT(kc.c2, S[iy][ix], u);
                    ac[slot<L>(M, 2)][iy][ix] = fmaT(kc.b2, S[iy][ix], ac[slot<L>(M, 2)][iy][ix]);
                }
            put(ic<2>{}, ic<WS>{}, y2[slot<L>(M, 2)]);
        };
        auto st3 = [&](const Nb &nb) __attribute__((always_inline)) {
            T S[NY][NXP];
            stencil(nb, y2, ic<slot<L>(M, 3)>{}, ic<slot<L>(M, 4)>{}, ic<slot<L>(M, 2)>{}, w2, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 3)][iy][ix];
                    y3[slot<L>(M, 3)][iy][ix] = fmaT(kc.c3, S[iy][ix], u);
                    ac[slot<L>(M, 3)][iy][ix] = fmaT(kc.b3, S[iy][ix], ac[slot<L>(M, 3)][iy][ix]);
                }
            put(ic<3>{}, ic<WS>{}, y3[slot<L>(M, 3)]);
        };
        auto st4 = [&](const Nb &nb, int q) __attribute__((always_inline)) {
            T S[NY][NXP];
            stencil(nb, y3, ic<slot<L>(M, 4)>{}, ic<slot<L>(M, 5)>{}, ic<slot<L>(M, 3)>{}, w4, S);
            T *obase = dst + (size_t)q * nxy;
#pragma unroll
            for (int iy = 0; iy < NY; ++iy) {
                if (rowout[iy]) {
                    T v[NXP];
#pragma unroll
                    for (int ix = 0; ix < NXP; ++ix) v[ix] = fmaT(kc.b4, S[iy][ix], ac[slot<L>(M, 4)][iy][ix]);
                    if constexpr (XT) {
#pragma unroll
                        for (int ix = 0; ix < NXP; ++ix)
                            if (colout[ix])
                                __builtin_nontemporal_store(v[ix], (PR_GLOBAL T *)(obase + rowoff[iy] + colx[ix]));
                    } else {
                        gst_nt_row<T, NXP>(obase + rowoff[iy], v);
                    }
                }
            }
        };
        const int q = p - 4;
        if constexpr (FAST) {
            st1(fetch(ic<0>{}, ic<RS>{}));
            st2(fetch(ic<1>{}, ic<RS>{}));
            st3(fetch(ic<2>{}, ic<RS>{}));
            if (q < zend) st4(fetch(ic<3>{}, ic<RS>{}), q);
        } else {
            if (act1 && p >= z0 - 2) st1(fetch(ic<0>{}, ic<RS>{}));   // stage 1 at plane p - 1
            if (act2 && p >= z0) st2(fetch(ic<1>{}, ic<RS>{}));       // stage 2 at plane p - 2
            if (act3 && p >= z0 + 2) st3(fetch(ic<2>{}, ic<RS>{}));   // stage 3 at plane p - 3
            if (act4 && p >= z0 + 4 && q < zend) st4(fetch(ic<3>{}, ic<RS>{}), q);   // stage 4, stored
        }
    };

    const int pstart = z0 - 4;
    const int niter = (zend - z0) + 8;
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(pstart + d, pf[d]);
    // trips of L iterations; the first two contain the pipeline fill (stage s
    // starts at iteration 2s - 2 of the chunk), later ones have every stage
    // active.  Both loops execute one barrier per iteration and the same
    // number of trips, so wavefronts on either path meet at every barrier.
    auto trip = [&](int pb, auto FASTc) __attribute__((always_inline)) {
        [&]<int... Ms>(std::integer_sequence<int, Ms...>) {
            (body(ic<Ms>{}, FASTc, pstart + pb + Ms), ...);
        }(std::make_integer_sequence<int, L>{});
    };
    if (act4) {
        // with two wavefronts per SIMD, the wavefronts that run all four
        // stages issue first; the partner wavefront (fewer stages) fills in
        if constexpr (NW <= 8) __builtin_amdgcn_s_setprio(1);
        int pb = 0;
        for (; pb < niter && pb < 2 * L; pb += L) trip(pb, std::false_type{});
        for (; pb < niter; pb += L) trip(pb, std::true_type{});
    } else {
        for (int pb = 0; pb < niter; pb += L) trip(pb, std::false_type{});
    }
}
// ---------------------------------------------------------------------------
// Half of an RK4 step over whole x rows for stencils of radius R (R <= NXP),
// two stages per launch.  Four fused stages of a radius-2 stencil need a
// halo of 8 rows and 8 planes per side, whose register rings do not fit one
// CU; two fused stages need a halo of 4, the same as four radius-1 stages.
//   HALF 0: stages 1 and 2 from u; writes y2 = u + c2 k2 and the partial sum
//           a2 = (u + b1 k1) + b2 k2 to the item's scratch fields 0 and 1.
//   HALF 1: stages 3 and 4 from y2 (stencil input), u and a2 (pointwise);
//           writes the step's output.
// The per-point arithmetic is that of the fused kernels (same apply(), same
// fused multiply-adds in the same order), so the result is bitwise the same.
// Layout as rk4_step_rows with one row per lane (NY = 1): every row of the
// stage inputs is exchanged through LDS.  Stage s of the half evaluates plane
// p - sR in iteration p; the plane that stage s + 1 reads in iteration p + 1
// was computed in iteration p - 1, so every LDS put happens at the top of
// the iteration, into the slot of this iteration's parity, and one barrier
// per plane orders the puts before the reads of the next iteration.
// ---------------------------------------------------------------------------
template <typename T, int R, int NXP, int NW, int PD, int HALF, int XT = 0>
__global__ void __launch_bounds__(64 * NW)
    rk4_half_rows(const ItemDesc *__restrict__ items, int nitems, int jstep)
{
    static_assert(R >= 2 && R <= NXP, "radius 2..NXP: x neighbours in the adjacent lanes, and the plane that "
                                      "stage B reads next was computed an iteration earlier");
    constexpr int H = 2 * R;              // halo of two stages (rows and planes per side)
    constexpr int NX = 64 * NXP;          // x extent of a wavefront (the whole row unless XT)
    constexpr int HX = XT ? H : 0;        // x halo of an x tile
    constexpr int TXT = NX - 2 * HX;      // output columns of an x tile
    constexpr int EY = NW, TY = EY - 2 * H;
    constexpr int L = 6;                  // z-ring length: even, >= 2R + 1
    static_assert(L >= 2 * R + 1 && L % 2 == 0 && L % PD == 0, "ring length");
    static_assert(TY > 0, "tile too small for the halo");
    __shared__ __align__(16) T lds[2][2][NW][NX];   // [stage input][slot][wavefront = row][x]

    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    if (jstep >= it.nsteps || (!XT && it.nx != NX)) return;
    const int local = lb - it.block_begin;
    if (local < 0 || local >= it.nblocks) return;

    const int nx = XT ? it.nx : NX, ny = it.ny, nz = it.nz;
    int txt = 0, rest = local;
    if constexpr (XT) {
        txt = local % it.tiles_x;
        rest = local / it.tiles_x;
    }
    const int tyt = rest % it.tiles_y;
    const int zc = rest / it.tiles_y;
    const int x0 = txt * TXT;
    const int y0 = tyt * TY;
    const int z0 = zc * it.tz;
    const int zend = min(z0 + it.tz, nz);
    const int nxy = nx * ny;
    const size_t npts = (size_t)nxy * nz;

    const T *src;
    T *dst;
    pingpong<T>(it, jstep, it.nsteps, src, dst);
    T *const scr_y = (T *)it.scratch;           // y2 (stage 2 output)
    T *const scr_a = (T *)it.scratch + npts;    // a2 (partial RK4 sum after stage 2)

    const int lane = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);   // = tile row
    const int cx0 = lane * NXP;
    const int rowoff = wrapi(y0 - H + wv, ny) * nx + (XT ? 0 : cx0);
    const bool rowout = (wv >= H) && (wv < H + TY) && (y0 + wv - H < ny);
    // x tiles, as in rk4_step_rows (two radius-R stages reach 2R columns
    // into the halo)
    int colx[XT ? NXP : 1];
    bool colout[XT ? NXP : 1];
    if constexpr (XT) {
#pragma unroll
        for (int ix = 0; ix < NXP; ++ix) {
            const int c = cx0 + ix;
            colx[ix] = wrapi(x0 - HX + c, nx);
            colout[ix] = (c >= HX) && (c < HX + TXT) && (x0 + c - HX < nx);
        }
    }
    // stage s of the half can feed an output point only on rows sR .. EY-1-sR
    const bool act1 = wv >= R && wv < EY - R, act2 = wv >= 2 * R && wv < EY - 2 * R;
    int wn[2][R];   // wavefronts holding rows wv -/+ k (clamped; only active stages read them)
#pragma unroll
    for (int k = 0; k < R; ++k) {
        wn[0][k] = max(wv - k - 1, 0);
        wn[1][k] = min(wv + k + 1, NW - 1);
    }

    const double dt = it.dt;
    const double t = (double)(it.step0 + jstep) * dt;
    const double nu1 = nu_at(it, t);
    const double nu2 = it.frozen ? nu1 : nu_at(it, t + 0.5 * dt);
    const double nu4 = it.frozen ? nu1 : nu_at(it, t + dt);
    const Wts<T, R> wA = uni(fine_weights<T, R>(it, HALF == 0 ? nu1 : nu2));
    const Wts<T, R> wB = uni(fine_weights<T, R>(it, HALF == 0 ? nu2 : nu4));
    RK4Consts<T> kc = rk4_consts<T>(dt);
    // stage constants of this half: y = u + cA S_A, a = fma(bA, S_A, a'), then bB for S_B
    const T cA = uni(HALF == 0 ? kc.c1 : kc.c3);
    const T bA = uni(HALF == 0 ? kc.b1 : kc.b3);
    const T cB = uni(kc.c2);
    const T bB = uni(HALF == 0 ? kc.b2 : kc.b4);

    // rings: in = stencil input of stage A (u, or y2), mid = output of stage A
    // (y1, or y3), acc = partial sums after stage A; for HALF 1 also u and a2
    T in[L][NXP], mid[L][NXP], acc[L][NXP];
    T pin[PD][NXP];
    // HALF 1 only: u and a2 of the plane stage A evaluates, loaded one
    // iteration ahead (double buffered by iteration parity)
    T pu[2][NXP], pa[2][NXP];

    const T *in_src = HALF == 0 ? src : scr_y;
    auto load_plane = [&](const T *base, int pz, T(&d)[NXP]) {
        const T *row = base + (size_t)wrapi(pz, nz) * nxy + rowoff;
        if constexpr (XT) {
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) d[ix] = *(const PR_GLOBAL T *)(row + colx[ix]);
        } else {
            const Vec<T, NXP> v = gld<Vec<T, NXP>>(row);
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) d[ix] = v.v[ix];
        }
    };
    auto put = [&](auto Bc, auto SLc, const T(&v)[NXP]) {
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
        Vec<T, NXP> a;
#pragma unroll
        for (int ix = 0; ix < NXP; ++ix) a.v[ix] = v[ix];
        *reinterpret_cast<Vec<T, NXP> *>(&lds[B][SL][wv][cx0]) = a;
    };
    struct Nb {
        Vec<T, NXP> m[R], p[R];   // rows wv-k-1 and wv+k+1
    };
    auto fetch = [&](auto Bc, auto SLc) {
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
        Nb nb;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            nb.m[k] = *reinterpret_cast<const Vec<T, NXP> *>(&lds[B][SL][wn[0][k]][cx0]);
            nb.p[k] = *reinterpret_cast<const Vec<T, NXP> *>(&lds[B][SL][wn[1][k]][cx0]);
        }
        return nb;
    };
    // S = L(f) at the plane in ring slot SC; z neighbours at slots SC -/+ k
    auto stencil = [&](const Nb &nb, const T(&f)[L][NXP], auto SCc, const Wts<T, R> &w, T(&S)[NXP]) {
        constexpr int SC = decltype(SCc)::value;
        T left[NXP], right[NXP];   // the values of lanes l-1 and l+1 (mod 64)
#pragma unroll
        for (int ix = 0; ix < NXP; ++ix) {
            left[ix] = wave_rot<kDppWaveRor1>(f[SC][ix]);
            right[ix] = wave_rot<kDppWaveRol1>(f[SC][ix]);
        }
#pragma unroll
        for (int ix = 0; ix < NXP; ++ix) {
            T mn[3][R], pn[3][R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int im = ix - k - 1, ip = ix + k + 1;
                mn[0][k] = im >= 0 ? f[SC][im] : left[NXP + im];
                pn[0][k] = ip < NXP ? f[SC][ip] : right[ip - NXP];
                mn[1][k] = nb.m[k].v[ix];
                pn[1][k] = nb.p[k].v[ix];
                mn[2][k] = f[(SC - k - 1 + 2 * L) % L][ix];
                pn[2][k] = f[(SC + k + 1) % L][ix];
            }
            S[ix] = apply<T, R>(w, f[SC][ix], mn, pn);
        }
    };

    auto body = [&](auto Mc, auto FASTc, int p) __attribute__((always_inline)) {
        constexpr int M = decltype(Mc)::value;
        constexpr bool FAST = decltype(FASTc)::value;
        constexpr int WS = M & 1, RS = (M + 1) & 1;
        constexpr int S0 = slot<L>(M, 0);          // plane p
        constexpr int SA = slot<L>(M, R);          // plane p - R: stage A's centre
        constexpr int SB = slot<L>(M, 2 * R);      // plane p - 2R: stage B's centre
        __syncthreads();
#pragma unroll
        for (int ix = 0; ix < NXP; ++ix) in[S0][ix] = pin[M % PD][ix];
        load_plane(in_src, p + PD, pin[M % PD]);
        if constexpr (HALF == 1) {
            // u and a2 at plane p + 1 - R, for stage A of the next iteration
            load_plane(src, p + 1 - R, pu[M & 1]);
            load_plane(scr_a, p + 1 - R, pa[M & 1]);
        }
        // planes read by the stages of iteration p + 1: input plane p + 1 - R
        // (loaded in iteration p + 1 - R) and stage A's output plane p + 1 - 2R
        // (computed in iteration p + 1 - R)
        put(ic<0>{}, ic<WS>{}, in[slot<L>(M, R - 1)]);
        if (FAST || act1) put(ic<1>{}, ic<WS>{}, mid[slot<L>(M, 2 * R - 1)]);

        auto stA = [&]() __attribute__((always_inline)) {
            T S[NXP];
            stencil(fetch(ic<0>{}, ic<RS>{}), in, ic<SA>{}, wA, S);
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) {
                if constexpr (HALF == 0) {
                    const T u = in[SA][ix];
                    mid[SA][ix] = fmaT(cA, S[ix], u);
                    acc[SA][ix] = fmaT(bA, S[ix], u);
                } else {
                    mid[SA][ix] = fmaT(cA, S[ix], pu[(M + 1) & 1][ix]);
                    acc[SA][ix] = fmaT(bA, S[ix], pa[(M + 1) & 1][ix]);
                }
            }
        };
        auto stB = [&](int q) __attribute__((always_inline)) {
            T S[NXP];
            stencil(fetch(ic<1>{}, ic<RS>{}), mid, ic<SB>{}, wB, S);
            if (rowout && q < zend) {
                const size_t off = (size_t)q * nxy + rowoff;
                if constexpr (HALF == 0) {
                    Vec<T, NXP> vy, va;
#pragma unroll
                    for (int ix = 0; ix < NXP; ++ix) {
                        vy.v[ix] = fmaT(cB, S[ix], in[SB][ix]);
                        va.v[ix] = fmaT(bB, S[ix], acc[SB][ix]);
                    }
                    if constexpr (XT) {
#pragma unroll
                        for (int ix = 0; ix < NXP; ++ix)
                            if (colout[ix]) {
                                *(PR_GLOBAL T *)(scr_y + off + colx[ix]) = vy.v[ix];
                                *(PR_GLOBAL T *)(scr_a + off + colx[ix]) = va.v[ix];
                            }
                    } else {
                        gst<Vec<T, NXP>>(scr_y + off, vy);
                        gst<Vec<T, NXP>>(scr_a + off, va);
                    }
                } else {
                    Vec<T, NXP> v;
#pragma unroll
                    for (int ix = 0; ix < NXP; ++ix) v.v[ix] = fmaT(bB, S[ix], acc[SB][ix]);
                    if constexpr (XT) {
#pragma unroll
                        for (int ix = 0; ix < NXP; ++ix)
                            if (colout[ix]) __builtin_nontemporal_store(v.v[ix], (PR_GLOBAL T *)(dst + off + colx[ix]));
                    } else {
                        gst_nt<Vec<T, NXP>>(dst + off, v);
                    }
                }
            }
        };
        const int q = p - 2 * R;
        if constexpr (FAST) {
            stA();
            stB(q);
        } else {
            if (act1 && p >= z0) stA();               // stage A at plane p - R >= z0 - R
            if (act2 && p >= z0 + 2 * R) stB(q);      // stage B at plane p - 2R >= z0
        }
    };

    const int pstart = z0 - H;
    const int niter = (zend - z0) + 2 * H;
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(in_src, pstart + d, pin[d]);
    auto trip = [&](int pb, auto FASTc) __attribute__((always_inline)) {
        [&]<int... Ms>(std::integer_sequence<int, Ms...>) {
            (body(ic<Ms>{}, FASTc, pstart + pb + Ms), ...);
        }(std::make_integer_sequence<int, L>{});
    };
    // stage B starts at iteration 2H (p = z0 + 2R); trips from iteration 2L on
    // have both stages active for the wavefronts that compute both
    if (act2) {
        int pb = 0;
        for (; pb < niter && pb < 2 * L; pb += L) trip(pb, std::false_type{});
        for (; pb < niter; pb += L) trip(pb, std::true_type{});
    } else {
        for (int pb = 0; pb < niter; pb += L) trip(pb, std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// Fused RK4 step for stencils of radius R with one barrier per z plane.
// Stage s evaluates plane p - sR in iteration p.  Each of the four stage
// inputs has two LDS slots, chosen by iteration parity; in iteration p input
// B (0..3) puts the plane that stage B+1 evaluates in iteration p+1, namely
// p + 1 - (B+1)R.  For R >= 2 that plane was computed an iteration earlier,
// so every put happens at the top of the iteration; for R = 1 it is the plane
// just computed, put right after its stage.  One barrier per iteration orders
// the puts of iteration p-1 before the reads of p, and the reads of p-1
// before the puts of p.  In-plane neighbours at distance k <= R come from the
// thread's own registers inside its NXP x NY group, else from LDS; z
// neighbours from the register rings.
// ---------------------------------------------------------------------------
template <typename T, int R, int NXP, int NY, int BXT, int BY, int PD>
__global__ void __launch_bounds__(BXT *BY)
    rk4_step_fused1r(const ItemDesc *__restrict__ items, int nitems, int jstep)
{
    constexpr int H = 4 * R;
    constexpr int EX = BXT * NXP, EY = BY * NY;
    constexpr int TX = EX - 2 * H, TY = EY - 2 * H;
    constexpr int L = (3 * R + 2) / 2 * 2;                 // z-ring length >= 3R+1, even
    static_assert(L % PD == 0, "prefetch depth must divide the unroll");
    constexpr int CO = ((R + NXP - 1) / NXP) * NXP;        // halo columns in LDS, whole groups
    constexpr int LX = EX + 2 * CO + (sizeof(T) == 8 ? 2 : 4);
    constexpr int LY = EY + 2 * R;
    static_assert(TX > 0 && TY > 0, "tile too small for the halo");
    __shared__ __align__(16) T lds[4][2][LY][LX];          // [stage input][slot][row][col]

    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    if (jstep >= it.nsteps) return;
    const int local = lb - it.block_begin;
    if (local < 0 || local >= it.nblocks) return;

    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int txt = local % it.tiles_x;
    const int rest = local / it.tiles_x;
    const int tyt = rest % it.tiles_y;
    const int zc = rest / it.tiles_y;
    const int x0 = txt * TX, y0 = tyt * TY;
    const int z0 = zc * it.tz;
    const int zend = min(z0 + it.tz, nz);

    const T *src;
    T *dst;
    pingpong<T>(it, jstep, it.nsteps, src, dst);

    const int tid = (int)threadIdx.x;
    const int txi = tid % BXT, tyi = tid / BXT;
    const int cx0 = txi * NXP, ry0 = tyi * NY;
    const int gx0 = wrapi(x0 - H + cx0, nx);
    int rowoff[NY];
    bool yok[NY];
#pragma unroll
    for (int iy = 0; iy < NY; ++iy) {
        const int ry = ry0 + iy;
        rowoff[iy] = wrapi(y0 - H + ry, ny) * nx + gx0;
        yok[iy] = (ry >= H) && (ry < H + TY) && (y0 + ry - H < ny);
    }
    const bool xok = (cx0 >= H) && (cx0 < H + TX) && (x0 + cx0 - H < nx);
    const int nxy = nx * ny;

    const double dt = it.dt;
    const double t = (double)(it.step0 + jstep) * dt;
    const double nu1 = nu_at(it, t);
    const double nu2 = it.frozen ? nu1 : nu_at(it, t + 0.5 * dt);
    const double nu4 = it.frozen ? nu1 : nu_at(it, t + dt);
    const Wts<T, R> w1 = uni(fine_weights<T, R>(it, nu1));
    const Wts<T, R> w2 = uni(fine_weights<T, R>(it, nu2));
    const Wts<T, R> w4 = uni(fine_weights<T, R>(it, nu4));
    RK4Consts<T> kc = rk4_consts<T>(dt);
    kc.c1 = uni(kc.c1);
    kc.c2 = uni(kc.c2);
    kc.c3 = uni(kc.c3);
    kc.b1 = uni(kc.b1);
    kc.b2 = uni(kc.b2);
    kc.b3 = uni(kc.b3);
    kc.b4 = uni(kc.b4);

    T ur[L][NY][NXP], y1[L][NY][NXP], y2[L][NY][NXP], y3[L][NY][NXP], ac[L][NY][NXP];
    T pf[PD][NY][NXP];   // planes in flight (prefetch ring)

    auto load_plane = [&](int p, T(&dstp)[NY][NXP]) {
        const T *base = src + (size_t)wrapi(p, nz) * nxy;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            const Vec<T, NXP> v = gld<Vec<T, NXP>>(base + rowoff[iy]);
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) dstp[iy][ix] = v.v[ix];
        }
    };

    // ring slot SC of `v` -> LDS input B, slot SL
    auto put = [&](auto Bc, auto SLc, auto SCc, const T(&v)[L][NY][NXP]) {
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
        constexpr int SC = decltype(SCc)::value;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            Vec<T, NXP> w;
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) w.v[ix] = v[SC][iy][ix];
            *reinterpret_cast<Vec<T, NXP> *>(&lds[B][SL][R + ry0 + iy][CO + cx0]) = w;
        }
    };

    // S = L(f)(plane p - OFF) for the thread's points; `in` is the ring of f,
    // the in-plane neighbours outside the thread's group come from LDS input
    // B, slot SL
    auto stencil = [&](auto Mc, auto OFFc, auto Bc, auto SLc, const T(&in)[L][NY][NXP], const Wts<T, R> &w,
                       T(&S)[NY][NXP]) {
        constexpr int M = decltype(Mc)::value;
        constexpr int OFF = decltype(OFFc)::value;
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
        constexpr int sc = slot<L>(M, OFF);
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) {
                T mn[3][R], pn[3][R];
#pragma unroll
                for (int k = 1; k <= R; ++k) {
                    mn[0][k - 1] = (ix - k >= 0) ? in[sc][iy][ix - k] : lds[B][SL][R + ry0 + iy][CO + cx0 + ix - k];
                    pn[0][k - 1] = (ix + k < NXP) ? in[sc][iy][ix + k] : lds[B][SL][R + ry0 + iy][CO + cx0 + ix + k];
                    mn[1][k - 1] = (iy - k >= 0) ? in[sc][iy - k][ix] : lds[B][SL][R + ry0 + iy - k][CO + cx0 + ix];
                    pn[1][k - 1] = (iy + k < NY) ? in[sc][iy + k][ix] : lds[B][SL][R + ry0 + iy + k][CO + cx0 + ix];
                    mn[2][k - 1] = in[slot<L>(M, OFF + k)][iy][ix];   // plane q - k
                    pn[2][k - 1] = in[slot<L>(M, OFF - k)][iy][ix];   // plane q + k
                }
                S[iy][ix] = apply<T, R>(w, in[sc][iy][ix], mn, pn);
            }
        }
    };

    auto body = [&](auto Mc, int p) {
        constexpr int M = decltype(Mc)::value;
        constexpr int WS = M & 1;        // slot written in this iteration
        constexpr int RS = (M + 1) & 1;  // slot written in the previous iteration
        __syncthreads();
#pragma unroll
        for (int iy = 0; iy < NY; ++iy)
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) ur[slot<L>(M, 0)][iy][ix] = pf[M % PD][iy][ix];
        load_plane(p + PD, pf[M % PD]);
        put(ic<0>{}, ic<WS>{}, ic<slot<L>(M, R - 1)>{}, ur);   // plane p + 1 - R
        if constexpr (R >= 2) {
            put(ic<1>{}, ic<WS>{}, ic<slot<L>(M, 2 * R - 1)>{}, y1);
            put(ic<2>{}, ic<WS>{}, ic<slot<L>(M, 3 * R - 1)>{}, y2);
            put(ic<3>{}, ic<WS>{}, ic<slot<L>(M, 4 * R - 1)>{}, y3);
        }

        T S[NY][NXP];
        // stage 1 at plane p - R
        if (p >= z0 - 2 * R) {
            stencil(Mc, ic<R>{}, ic<0>{}, ic<RS>{}, ur, w1, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, R)][iy][ix];
                    y1[slot<L>(M, R)][iy][ix] = fmaT(kc.c1, S[iy][ix], u);
                    ac[slot<L>(M, R)][iy][ix] = fmaT(kc.b1, S[iy][ix], u);
                }
        }
        if constexpr (R == 1) put(ic<1>{}, ic<WS>{}, ic<slot<L>(M, 1)>{}, y1);
        // stage 2 at plane p - 2R
        if (p >= z0) {
            stencil(Mc, ic<2 * R>{}, ic<1>{}, ic<RS>{}, y1, w2, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 2 * R)][iy][ix];
                    y2[slot<L>(M, 2 * R)][iy][ix] = fmaT(kc.c2, S[iy][ix], u);
                    ac[slot<L>(M, 2 * R)][iy][ix] = fmaT(kc.b2, S[iy][ix], ac[slot<L>(M, 2 * R)][iy][ix]);
                }
        }
        if constexpr (R == 1) put(ic<2>{}, ic<WS>{}, ic<slot<L>(M, 2)>{}, y2);
        // stage 3 at plane p - 3R
        if (p >= z0 + 2 * R) {
            stencil(Mc, ic<3 * R>{}, ic<2>{}, ic<RS>{}, y2, w2, S);
#pragma unroll
            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) {
                    const T u = ur[slot<L>(M, 3 * R)][iy][ix];
                    y3[slot<L>(M, 3 * R)][iy][ix] = fmaT(kc.c3, S[iy][ix], u);
                    ac[slot<L>(M, 3 * R)][iy][ix] = fmaT(kc.b3, S[iy][ix], ac[slot<L>(M, 3 * R)][iy][ix]);
                }
        }
        if constexpr (R == 1) put(ic<3>{}, ic<WS>{}, ic<slot<L>(M, 3)>{}, y3);
        // stage 4 at plane p - 4R, stored
        const int q = p - 4 * R;
        if (p >= z0 + 4 * R && q < zend) {
            stencil(Mc, ic<4 * R>{}, ic<3>{}, ic<RS>{}, y3, w4, S);
            if (xok) {
                T *obase = dst + (size_t)q * nxy;
#pragma unroll
                for (int iy = 0; iy < NY; ++iy) {
                    if (yok[iy]) {
                        Vec<T, NXP> v;
#pragma unroll
                        for (int ix = 0; ix < NXP; ++ix)
                            v.v[ix] = fmaT(kc.b4, S[iy][ix], ac[slot<L>(M, 4 * R)][iy][ix]);
                        gst<Vec<T, NXP>>(obase + rowoff[iy], v);
                    }
                }
            }
        }
    };

    const int pstart = z0 - 4 * R;
    const int niter = (zend - z0) + 8 * R;
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(pstart + d, pf[d]);
    for (int pb = 0; pb < niter; pb += L) {
        [&]<int... Ms>(std::integer_sequence<int, Ms...>) {
            (body(ic<Ms>{}, pstart + pb + Ms), ...);
        }(std::make_integer_sequence<int, L>{});
    }
}

// ---------------------------------------------------------------------------
// Fused forward Euler chunk with one barrier per z plane (same scheme as
// rk4_step_fused1b: stage outputs go to LDS and are read one iteration later).
// ---------------------------------------------------------------------------
template <typename T, int S, int NXP, int NY, int BXT, int BY, int PD>
__global__ void __launch_bounds__(BXT *BY)
    euler_chunk_fused1b(const ItemDesc *__restrict__ items, int nitems, int chunk)
{
    static_assert(6 % PD == 0, "prefetch depth must divide the unroll");
    constexpr int H = S;
    constexpr int EX = BXT * NXP, EY = BY * NY;
    constexpr int TX = EX - 2 * H, TY = EY - 2 * H;
    constexpr int L = 3;                                   // z-ring length
    constexpr int U = 6;                                   // unroll: ring phase and LDS slot parity
    constexpr int CO = NXP;
    constexpr int LX = EX + 2 * CO + (sizeof(T) == 8 ? 2 : 4);
    constexpr int LY = EY + 2;
    static_assert(TX > 0 && TY > 0, "tile too small for the halo");
    __shared__ __align__(16) T lds[S][2][LY][LX];

    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    const int nchunks = (it.nsteps + S - 1) / S;
    if (chunk >= nchunks) return;
    const int local = lb - it.block_begin;
    if (local < 0 || local >= it.nblocks) return;

    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int txt = local % it.tiles_x;
    const int rest = local / it.tiles_x;
    const int tyt = rest % it.tiles_y;
    const int zc = rest / it.tiles_y;
    const int x0 = txt * TX, y0 = tyt * TY;
    const int z0 = zc * it.tz;
    const int zend = min(z0 + it.tz, nz);

    const T *src;
    T *dst;
    pingpong<T>(it, chunk, nchunks, src, dst);

    const int tid = (int)threadIdx.x;
    const int txi = tid % BXT, tyi = tid / BXT;
    const int cx0 = txi * NXP, ry0 = tyi * NY;
    const int gx0 = wrapi(x0 - H + cx0, nx);
    int rowoff[NY];
    bool yok[NY];
#pragma unroll
    for (int iy = 0; iy < NY; ++iy) {
        const int ry = ry0 + iy;
        rowoff[iy] = wrapi(y0 - H + ry, ny) * nx + gx0;
        yok[iy] = (ry >= H) && (ry < H + TY) && (y0 + ry - H < ny);
    }
    const bool xok = (cx0 >= H) && (cx0 < H + TX) && (x0 + cx0 - H < nx);
    const int nxy = nx * ny;

    Wts<T, 1> w[S];
    T dts[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t j = (int64_t)chunk * S + s;
        const bool act = j < it.nsteps;
        const double nu = nu_at(it, (double)(it.step0 + j) * it.dt);
        w[s] = uni(coarse_weights<T>(it, nu));
        dts[s] = uni(act ? (T)it.dt : (T)0);
    }

    T f[S][L][NY][NXP];
    T pf[PD][NY][NXP];

    auto load_plane = [&](int p, T(&dstp)[NY][NXP]) {
        const T *base = src + (size_t)wrapi(p, nz) * nxy;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            const Vec<T, NXP> v = gld<Vec<T, NXP>>(base + rowoff[iy]);
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) dstp[iy][ix] = v.v[ix];
        }
    };

    auto body = [&](auto Mc, int p) {
        constexpr int M = decltype(Mc)::value;
        constexpr int WS = M & 1, RS = (M + 1) & 1;
        __syncthreads();
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            Vec<T, NXP> wv;
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) {
                f[0][slot<L>(M, 0)][iy][ix] = pf[M % PD][iy][ix];
                wv.v[ix] = pf[M % PD][iy][ix];
            }
            *reinterpret_cast<Vec<T, NXP> *>(&lds[0][WS][1 + ry0 + iy][CO + cx0]) = wv;
        }
        load_plane(p + PD, pf[M % PD]);

        [&]<int... Ss>(std::integer_sequence<int, Ss...>) {
            (
                [&] {
                    constexpr int s = Ss + 1;          // stage s computes plane p - s from f[s-1]
                    constexpr int sc = slot<L>(M, s);
                    if (p >= z0 - S + 2 * s && p < zend + S) {
                        const Vec<T, NXP> up = *reinterpret_cast<const Vec<T, NXP> *>(&lds[s - 1][RS][ry0][CO + cx0]);
                        const Vec<T, NXP> dn =
                            *reinterpret_cast<const Vec<T, NXP> *>(&lds[s - 1][RS][1 + ry0 + NY][CO + cx0]);
                        T res[NY][NXP];
#pragma unroll
                        for (int iy = 0; iy < NY; ++iy) {
                            const Vec<T, NXP> lf =
                                *reinterpret_cast<const Vec<T, NXP> *>(&lds[s - 1][RS][1 + ry0 + iy][CO + cx0 - NXP]);
                            const Vec<T, NXP> rt =
                                *reinterpret_cast<const Vec<T, NXP> *>(&lds[s - 1][RS][1 + ry0 + iy][CO + cx0 + NXP]);
#pragma unroll
                            for (int ix = 0; ix < NXP; ++ix) {
                                T mn[3][1], pn[3][1];
                                mn[0][0] = (ix >= 1) ? f[s - 1][sc][iy][ix - 1] : lf.v[NXP - 1];
                                pn[0][0] = (ix + 1 < NXP) ? f[s - 1][sc][iy][ix + 1] : rt.v[0];
                                mn[1][0] = (iy >= 1) ? f[s - 1][sc][iy - 1][ix] : up.v[ix];
                                pn[1][0] = (iy + 1 < NY) ? f[s - 1][sc][iy + 1][ix] : dn.v[ix];
                                mn[2][0] = f[s - 1][slot<L>(M, s + 1)][iy][ix];
                                pn[2][0] = f[s - 1][slot<L>(M, s - 1)][iy][ix];
                                const T cen = f[s - 1][sc][iy][ix];
                                const T Sv = apply<T, 1>(w[s - 1], cen, mn, pn);
                                res[iy][ix] = fmaT(dts[s - 1], Sv, cen);
                            }
                        }
                        if constexpr (s < S) {
#pragma unroll
                            for (int iy = 0; iy < NY; ++iy) {
                                Vec<T, NXP> wv;
#pragma unroll
                                for (int ix = 0; ix < NXP; ++ix) {
                                    f[s][slot<L>(M, s)][iy][ix] = res[iy][ix];
                                    wv.v[ix] = res[iy][ix];
                                }
                                *reinterpret_cast<Vec<T, NXP> *>(&lds[s][WS][1 + ry0 + iy][CO + cx0]) = wv;
                            }
                        } else {
                            const int q = p - S;
                            if (xok) {
                                T *obase = dst + (size_t)q * nxy;
#pragma unroll
                                for (int iy = 0; iy < NY; ++iy) {
                                    if (yok[iy]) {
                                        Vec<T, NXP> v;
#pragma unroll
                                        for (int ix = 0; ix < NXP; ++ix) v.v[ix] = res[iy][ix];
                                        gst<Vec<T, NXP>>(obase + rowoff[iy], v);
                                    }
                                }
                            }
                        }
                    }
                }(),
                ...);
        }(std::make_integer_sequence<int, S>{});
    };

    const int pstart = z0 - S;
    const int niter = (zend - z0) + 2 * S;
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(pstart + d, pf[d]);
    for (int pb = 0; pb < niter; pb += U) {
        [&]<int... Ms>(std::integer_sequence<int, Ms...>) {
            (body(ic<Ms>{}, pstart + pb + Ms), ...);
        }(std::make_integer_sequence<int, U>{});
    }
}

// ---------------------------------------------------------------------------
// S fused Euler steps of G over whole x rows (n_x = 64 * NXP): the layout of
// rk4_step_rows (x neighbours by wavefront rotation, y-edge rows through
// LDS, y halo of S rows per side, stages skipped per wavefront near the tile
// edge) with the z pipeline of euler_chunk_fused1b.
// ---------------------------------------------------------------------------
template <typename T, int S, int NXP, int NY, int NW, int PD, int XT = 0>
__global__ void __launch_bounds__(64 * NW)
    euler_chunk_rows(const ItemDesc *__restrict__ items, int nitems, int chunk)
{
    static_assert(6 % PD == 0, "prefetch depth must divide the unroll");
    constexpr int H = S;
    constexpr int NX = 64 * NXP;          // x extent of a wavefront (the whole row unless XT)
    constexpr int HX = XT ? H : 0;        // x halo of an x tile
    constexpr int TXT = NX - 2 * HX;      // output columns of an x tile
    constexpr int EY = NW * NY, TY = EY - 2 * H;
    constexpr int L = 3;                  // z-ring length
    constexpr int U = 6;                  // unroll: ring phase and LDS slot parity
    constexpr int NE = NY == 1 ? 1 : 2;   // exchanged rows per wavefront: first, last
    static_assert(TY > 0, "tile too small for the halo");
    __shared__ __align__(16) T lds[S][2][NW][NE][NX];   // [stage input][slot][wavefront][edge][x]

    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    const int nchunks = (it.nsteps + S - 1) / S;
    if (chunk >= nchunks || (!XT && it.nx != NX)) return;
    const int local = lb - it.block_begin;
    if (local < 0 || local >= it.nblocks) return;

    const int nx = XT ? it.nx : NX, ny = it.ny, nz = it.nz;
    int txt = 0, rest = local;
    if constexpr (XT) {
        txt = local % it.tiles_x;
        rest = local / it.tiles_x;
    }
    const int tyt = rest % it.tiles_y;
    const int zc = rest / it.tiles_y;
    const int x0 = txt * TXT;
    const int y0 = tyt * TY;
    const int z0 = zc * it.tz;
    const int zend = min(z0 + it.tz, nz);

    const T *src;
    T *dst;
    pingpong<T>(it, chunk, nchunks, src, dst);

    const int lane = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int wup = wv > 0 ? wv - 1 : 0;
    const int wdn = wv < NW - 1 ? wv + 1 : NW - 1;
    const int ry0 = wv * NY;
    const int cx0 = lane * NXP;
    int rowoff[NY];
    bool rowout[NY];
#pragma unroll
    for (int iy = 0; iy < NY; ++iy) {
        const int ry = ry0 + iy;
        rowoff[iy] = wrapi(y0 - H + ry, ny) * nx + (XT ? 0 : cx0);
        rowout[iy] = (ry >= H) && (ry < H + TY) && (y0 + ry - H < ny);
    }
    // x tiles: as in rk4_step_rows (S steps reach S columns into the halo)
    int colx[XT ? NXP : 1];
    bool colout[XT ? NXP : 1];
    if constexpr (XT) {
#pragma unroll
        for (int ix = 0; ix < NXP; ++ix) {
            const int c = cx0 + ix;
            colx[ix] = wrapi(x0 - HX + c, nx);
            colout[ix] = (c >= HX) && (c < HX + TXT) && (x0 + c - HX < nx);
        }
    }
    const int nxy = nx * ny;

    Wts<T, 1> w[S];
    T dts[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t j = (int64_t)chunk * S + s;
        const bool act = j < it.nsteps;
        const double nu = nu_at(it, (double)(it.step0 + j) * it.dt);
        w[s] = uni(coarse_weights<T>(it, nu));
        dts[s] = uni(act ? (T)it.dt : (T)0);
    }

    T f[S][L][NY][NXP];
    T pf[PD][NY][NXP];

    auto load_plane = [&](int p, T(&dstp)[NY][NXP]) {
        const T *base = src + (size_t)wrapi(p, nz) * nxy;
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
            if constexpr (XT) {
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) dstp[iy][ix] = *(const PR_GLOBAL T *)(base + rowoff[iy] + colx[ix]);
            } else {
                const Vec<T, NXP> v = gld<Vec<T, NXP>>(base + rowoff[iy]);
#pragma unroll
                for (int ix = 0; ix < NXP; ++ix) dstp[iy][ix] = v.v[ix];
            }
        }
    };

    auto put = [&](auto Bc, auto SLc, const T(&v)[NY][NXP]) {
        constexpr int B = decltype(Bc)::value;
        constexpr int SL = decltype(SLc)::value;
        Vec<T, NXP> a;
#pragma unroll
        for (int ix = 0; ix < NXP; ++ix) a.v[ix] = v[0][ix];
        *reinterpret_cast<Vec<T, NXP> *>(&lds[B][SL][wv][0][cx0]) = a;
        if constexpr (NE == 2) {
            Vec<T, NXP> b;
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) b.v[ix] = v[NY - 1][ix];
            *reinterpret_cast<Vec<T, NXP> *>(&lds[B][SL][wv][1][cx0]) = b;
        }
    };

    // FAST: a wavefront that computes every stage, after the pipeline fill:
    // straight-line code, only the final store guarded
    auto body = [&](auto Mc, auto FASTc, int p) __attribute__((always_inline)) {
        constexpr int M = decltype(Mc)::value;
        constexpr bool FAST = decltype(FASTc)::value;
        constexpr int WS = M & 1, RS = (M + 1) & 1;
        __syncthreads();
#pragma unroll
        for (int iy = 0; iy < NY; ++iy)
#pragma unroll
            for (int ix = 0; ix < NXP; ++ix) f[0][slot<L>(M, 0)][iy][ix] = pf[M % PD][iy][ix];
        put(ic<0>{}, ic<WS>{}, f[0][slot<L>(M, 0)]);
        load_plane(p + PD, pf[M % PD]);

        [&]<int... Ss>(std::integer_sequence<int, Ss...>) {
            (
                [&] {
                    constexpr int s = Ss + 1;          // stage s computes plane p - s from f[s-1]
                    constexpr int sc = slot<L>(M, s);
                    const bool wact = ry0 + NY - 1 >= s && ry0 < EY - s;
                    if (FAST || (wact && p >= z0 - S + 2 * s && p < zend + S)) {
                        const Vec<T, NXP> up =
                            *reinterpret_cast<const Vec<T, NXP> *>(&lds[s - 1][RS][wup][NE - 1][cx0]);
                        const Vec<T, NXP> dn = *reinterpret_cast<const Vec<T, NXP> *>(&lds[s - 1][RS][wdn][0][cx0]);
                        T res[NY][NXP];
#pragma unroll
                        for (int iy = 0; iy < NY; ++iy) {
                            const T left = wave_rot<kDppWaveRor1>(f[s - 1][sc][iy][NXP - 1]);
                            const T right = wave_rot<kDppWaveRol1>(f[s - 1][sc][iy][0]);
#pragma unroll
                            for (int ix = 0; ix < NXP; ++ix) {
                                T mn[3][1], pn[3][1];
                                mn[0][0] = (ix >= 1) ? f[s - 1][sc][iy][ix - 1] : left;
                                pn[0][0] = (ix + 1 < NXP) ? f[s - 1][sc][iy][ix + 1] : right;
                                mn[1][0] = (iy >= 1) ? f[s - 1][sc][iy - 1][ix] : up.v[ix];
                                pn[1][0] = (iy + 1 < NY) ? f[s - 1][sc][iy + 1][ix] : dn.v[ix];
                                mn[2][0] = f[s - 1][slot<L>(M, s + 1)][iy][ix];
                                pn[2][0] = f[s - 1][slot<L>(M, s - 1)][iy][ix];
                                const T cen = f[s - 1][sc][iy][ix];
                                const T Sv = apply<T, 1>(w[s - 1], cen, mn, pn);
                                res[iy][ix] = fmaT(dts[s - 1], Sv, cen);
                            }
                        }
                        if constexpr (s < S) {
#pragma unroll
                            for (int iy = 0; iy < NY; ++iy)
#pragma unroll
                                for (int ix = 0; ix < NXP; ++ix) f[s][slot<L>(M, s)][iy][ix] = res[iy][ix];
                            put(ic<s>{}, ic<WS>{}, res);
                        } else if (!FAST || p < zend + S) {
                            T *obase = dst + (size_t)(p - S) * nxy;
#pragma unroll
                            for (int iy = 0; iy < NY; ++iy) {
                                if (rowout[iy]) {
                                    if constexpr (XT) {
#pragma unroll
                                        for (int ix = 0; ix < NXP; ++ix)
                                            if (colout[ix]) *(PR_GLOBAL T *)(obase + rowoff[iy] + colx[ix]) = res[iy][ix];
                                    } else {
                                        Vec<T, NXP> v;
#pragma unroll
                                        for (int ix = 0; ix < NXP; ++ix) v.v[ix] = res[iy][ix];
                                        gst<Vec<T, NXP>>(obase + rowoff[iy], v);
                                    }
                                }
                            }
                        }
                    }
                }(),
                ...);
        }(std::make_integer_sequence<int, S>{});
    };

    const int pstart = z0 - S;
    const int niter = (zend - z0) + 2 * S;
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(pstart + d, pf[d]);
    // trips of U iterations; stage s starts at iteration 2s - S of the chunk
    // pipeline, so trips from pb >= 2S on have every stage active.  Both
    // loops run one barrier per iteration and the same number of trips.
    auto trip = [&](int pb, auto FASTc) __attribute__((always_inline)) {
        [&]<int... Ms>(std::integer_sequence<int, Ms...>) {
            (body(ic<Ms>{}, FASTc, pstart + pb + Ms), ...);
        }(std::make_integer_sequence<int, U>{});
    };
    constexpr int kFastFrom = ((2 * S + U - 1) / U) * U;
    if (ry0 + NY - 1 >= S && ry0 < EY - S) {
        int pb = 0;
        for (; pb < niter && pb < kFastFrom; pb += U) trip(pb, std::false_type{});
        for (; pb < niter; pb += U) trip(pb, std::true_type{});
    } else {
        for (int pb = 0; pb < niter; pb += U) trip(pb, std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// Unfused reference kernels: one thread per point, neighbours read from
// global memory.  RK4 runs as four stage launches through three scratch
// fields [Ya | Yb | Acc]; Euler as one launch per step.
// ---------------------------------------------------------------------------
template <typename T, int R>
__device__ __forceinline__ void gather(const T *f, int x, int y, int z, int nx, int ny, int nz, T &cen,
                                       T (&mn)[3][R], T (&pn)[3][R])
{
    const int nxy = nx * ny;
    const PR_GLOBAL T *g = (const PR_GLOBAL T *)f;
    cen = g[(size_t)z * nxy + y * nx + x];
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        mn[0][k - 1] = g[(size_t)z * nxy + y * nx + wrapi(x - k, nx)];
        pn[0][k - 1] = g[(size_t)z * nxy + y * nx + wrapi(x + k, nx)];
        mn[1][k - 1] = g[(size_t)z * nxy + wrapi(y - k, ny) * nx + x];
        pn[1][k - 1] = g[(size_t)z * nxy + wrapi(y + k, ny) * nx + x];
        mn[2][k - 1] = g[(size_t)wrapi(z - k, nz) * nxy + y * nx + x];
        pn[2][k - 1] = g[(size_t)wrapi(z + k, nz) * nxy + y * nx + x];
    }
}

constexpr int kRefThreads = 256;

template <typename T, int R>
__global__ void __launch_bounds__(kRefThreads)
    rk4_stage_ref(const ItemDesc *__restrict__ items, int nitems, int jstep, int stagei)
{
    const int lb = (int)blockIdx.x;
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    if (jstep >= it.nsteps) return;
    const int local = lb - it.block_begin;
    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int64_t npts = (int64_t)nx * ny * nz;
    const int64_t idx = (int64_t)local * kRefThreads + threadIdx.x;
    if (idx >= npts) return;
    const int x = (int)(idx % nx), y = (int)((idx / nx) % ny), z = (int)(idx / ((int64_t)nx * ny));

    const T *src0;
    T *dst0;
    pingpong<T>(it, jstep, it.nsteps, src0, dst0);
    const PR_GLOBAL T *src = (const PR_GLOBAL T *)src0;
    PR_GLOBAL T *dst = (PR_GLOBAL T *)dst0;
    PR_GLOBAL T *Ya = (PR_GLOBAL T *)it.scratch;
    PR_GLOBAL T *Yb = Ya + npts;
    PR_GLOBAL T *Ac = Yb + npts;

    const double dt = it.dt;
    const double t = (double)(it.step0 + jstep) * dt;
    const double nu1 = nu_at(it, t);
    const double nu2 = it.frozen ? nu1 : nu_at(it, t + 0.5 * dt);
    const double nu4 = it.frozen ? nu1 : nu_at(it, t + dt);
    const RK4Consts<T> kc = rk4_consts<T>(dt);

    T cen, mn[3][R], pn[3][R];
    if (stagei == 1) {
        const Wts<T, R> w = fine_weights<T, R>(it, nu1);
        gather<T, R>(src0, x, y, z, nx, ny, nz, cen, mn, pn);
        const T S = apply<T, R>(w, cen, mn, pn);
        Ya[idx] = fmaT(kc.c1, S, cen);
        Ac[idx] = fmaT(kc.b1, S, cen);
    } else if (stagei == 2) {
        const Wts<T, R> w = fine_weights<T, R>(it, nu2);
        gather<T, R>((const T *)Ya, x, y, z, nx, ny, nz, cen, mn, pn);
        const T S = apply<T, R>(w, cen, mn, pn);
        Yb[idx] = fmaT(kc.c2, S, src[idx]);
        Ac[idx] = fmaT(kc.b2, S, Ac[idx]);
    } else if (stagei == 3) {
        const Wts<T, R> w = fine_weights<T, R>(it, nu2);
        gather<T, R>((const T *)Yb, x, y, z, nx, ny, nz, cen, mn, pn);
        const T S = apply<T, R>(w, cen, mn, pn);
        Ya[idx] = fmaT(kc.c3, S, src[idx]);
        Ac[idx] = fmaT(kc.b3, S, Ac[idx]);
    } else {
        const Wts<T, R> w = fine_weights<T, R>(it, nu4);
        gather<T, R>((const T *)Ya, x, y, z, nx, ny, nz, cen, mn, pn);
        const T S = apply<T, R>(w, cen, mn, pn);
        dst[idx] = fmaT(kc.b4, S, Ac[idx]);
    }
}

template <typename T>
__global__ void __launch_bounds__(kRefThreads)
    euler_step_ref(const ItemDesc *__restrict__ items, int nitems, int jstep)
{
    const int lb = (int)blockIdx.x;
    const ItemDesc &it = items[find_item(items, nitems, lb)];
    if (jstep >= it.nsteps) return;
    const int local = lb - it.block_begin;
    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int64_t npts = (int64_t)nx * ny * nz;
    const int64_t idx = (int64_t)local * kRefThreads + threadIdx.x;
    if (idx >= npts) return;
    const int x = (int)(idx % nx), y = (int)((idx / nx) % ny), z = (int)(idx / ((int64_t)nx * ny));
    const T *src;
    T *dst;
    pingpong<T>(it, jstep, it.nsteps, src, dst);
    const double nu = nu_at(it, (double)(it.step0 + jstep) * it.dt);
    const Wts<T, 1> w = coarse_weights<T>(it, nu);
    T cen, mn[3][1], pn[3][1];
    gather<T, 1>(src, x, y, z, nx, ny, nz, cen, mn, pn);
    const T S = apply<T, 1>(w, cen, mn, pn);
    ((PR_GLOBAL T *)dst)[idx] = fmaT((T)it.dt, S, cen);
}

// ---------------------------------------------------------------------------
// Variant registry
// ---------------------------------------------------------------------------
// A launch function launches its kernel, or with occ != nullptr only stores
// the kernel's resident blocks per compute unit in *occ.
using FineLaunch = void (*)(const ItemDesc *, int, int, int, hipStream_t, int *);
using CoarseLaunch = void (*)(const ItemDesc *, int, int, int, hipStream_t, int *);

template <typename K>
void occupancy_of(K kernel, int threads, int *occ)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1) n = 1;
    *occ = n;
}

template <typename T, int R, int NXP, int NY, int BXT, int BY>
void fine_launch(const ItemDesc *items, int nitems, int nblocks, int jstep, hipStream_t s, int *occ)
{
    if (occ) return occupancy_of((rk4_step_fused<T, R, NXP, NY, BXT, BY>), BXT * BY, occ);
    hipLaunchKernelGGL((rk4_step_fused<T, R, NXP, NY, BXT, BY>), dim3(nblocks), dim3(BXT * BY), 0, s, items,
                       nitems, jstep);
}

template <typename T, int NXP, int NY, int BXT, int BY, int PD>
void fine_launch_1b(const ItemDesc *items, int nitems, int nblocks, int jstep, hipStream_t s, int *occ)
{
    if (occ) return occupancy_of((rk4_step_fused1b<T, NXP, NY, BXT, BY, PD>), BXT * BY, occ);
    hipLaunchKernelGGL((rk4_step_fused1b<T, NXP, NY, BXT, BY, PD>), dim3(nblocks), dim3(BXT * BY), 0, s, items,
                       nitems, jstep);
}

template <typename T, int S, int NXP, int NY, int BXT, int BY, int PD>
void coarse_launch_1b(const ItemDesc *items, int nitems, int nblocks, int chunk, hipStream_t s, int *occ)
{
    if (occ) return occupancy_of((euler_chunk_fused1b<T, S, NXP, NY, BXT, BY, PD>), BXT * BY, occ);
    hipLaunchKernelGGL((euler_chunk_fused1b<T, S, NXP, NY, BXT, BY, PD>), dim3(nblocks), dim3(BXT * BY), 0, s, items,
                       nitems, chunk);
}

struct FineEntry {
    VariantInfo info;
    FineLaunch fn;
};
struct CoarseEntry {
    VariantInfo info;
    CoarseLaunch fn;
};

#define FINE_V(T, DT, R, NXP, NY, BXT, BY, NAME)                                                          \
    FineEntry{VariantInfo{NAME, DT, 2 * R, BXT * NXP - 8 * R, BY * NY - 8 * R, NXP, BXT * BY, 1},       \
              &fine_launch<T, R, NXP, NY, BXT, BY>}
#define FINE_1B(T, DT, NXP, NY, BXT, BY, PD, NAME)                                                       \
    FineEntry{VariantInfo{NAME, DT, 2, BXT * NXP - 8, BY * NY - 8, NXP, BXT * BY, 1},                  \
              &fine_launch_1b<T, NXP, NY, BXT, BY, PD>}
template <typename T, int NXP, int NY, int NW, int PD, int SEG, int XT = 0>
void fine_launch_rows(const ItemDesc *items, int nitems, int nblocks, int jstep, hipStream_t s, int *occ)
{
    if (occ) return occupancy_of((rk4_step_rows<T, NXP, NY, NW, PD, SEG, XT>), 64 * NW, occ);
    hipLaunchKernelGGL((rk4_step_rows<T, NXP, NY, NW, PD, SEG, XT>), dim3(nblocks), dim3(64 * NW), 0, s, items, nitems,
                       jstep);
}
#define FINE_ROWS(T, DT, NXP, NY, NW, PD, NAME)                                                          \
    FineEntry{VariantInfo{NAME, DT, 2, 64 * NXP, NW * NY - 8, NXP, 64 * NW, 1, 64 * NXP},              \
              &fine_launch_rows<T, NXP, NY, NW, PD, 64>}
// x tiles of 64*NXP columns (output 64*NXP - 8) over rows of any length
#define FINE_ROWSX(T, DT, NXP, NY, NW, PD, NAME)                                                         \
    FineEntry{VariantInfo{NAME, DT, 2, 64 * NXP - 8, NW * NY - 8, 1, 64 * NW, 1, 0},                    \
              &fine_launch_rows<T, NXP, NY, NW, PD, 64, 1>}
// grid rows of 16 lanes, four side by side in a wavefront
#define FINE_ROWS16(T, DT, NXP, NY, NW, PD, NAME)                                                        \
    FineEntry{VariantInfo{NAME, DT, 2, 16 * NXP, 4 * NW * NY - 8, NXP, 64 * NW, 1, 16 * NXP},          \
              &fine_launch_rows<T, NXP, NY, NW, PD, 16>}
template <typename T, int R, int NXP, int NY, int BXT, int BY, int PD>
void fine_launch_1r(const ItemDesc *items, int nitems, int nblocks, int jstep, hipStream_t s, int *occ)
{
    if (occ) return occupancy_of((rk4_step_fused1r<T, R, NXP, NY, BXT, BY, PD>), BXT * BY, occ);
    hipLaunchKernelGGL((rk4_step_fused1r<T, R, NXP, NY, BXT, BY, PD>), dim3(nblocks), dim3(BXT * BY), 0, s, items,
                       nitems, jstep);
}
#define FINE_1R(T, DT, R, NXP, NY, BXT, BY, PD, NAME)                                                    \
    FineEntry{VariantInfo{NAME, DT, 2 * R, BXT * NXP - 8 * R, BY * NY - 8 * R, NXP, BXT * BY, 1},       \
              &fine_launch_1r<T, R, NXP, NY, BXT, BY, PD>}
// Two launches per step (stages 1-2, then 3-4) through the item's scratch
// fields; the occupancy is that of the fuller half.
template <typename T, int R, int NXP, int NW, int PD, int XT = 0>
void fine_launch_half_rows(const ItemDesc *items, int nitems, int nblocks, int jstep, hipStream_t s, int *occ)
{
    if (occ) {
        int a = 1, b = 1;
        occupancy_of((rk4_half_rows<T, R, NXP, NW, PD, 0, XT>), 64 * NW, &a);
        occupancy_of((rk4_half_rows<T, R, NXP, NW, PD, 1, XT>), 64 * NW, &b);
        *occ = a < b ? a : b;
        return;
    }
    hipLaunchKernelGGL((rk4_half_rows<T, R, NXP, NW, PD, 0, XT>), dim3(nblocks), dim3(64 * NW), 0, s, items, nitems,
                       jstep);
    hipLaunchKernelGGL((rk4_half_rows<T, R, NXP, NW, PD, 1, XT>), dim3(nblocks), dim3(64 * NW), 0, s, items, nitems,
                       jstep);
}
#define FINE_HALF_ROWS(T, DT, R, NXP, NW, PD, NAME)                                                      \
    FineEntry{VariantInfo{NAME, DT, 2 * R, 64 * NXP, NW - 4 * R, NXP, 64 * NW, 1, 64 * NXP, 2},        \
              &fine_launch_half_rows<T, R, NXP, NW, PD>}
// the same over x tiles of 64*NXP columns (output 64*NXP - 4R) on rows of any length
#define FINE_HALF_ROWSX(T, DT, R, NXP, NW, PD, NAME)                                                     \
    FineEntry{VariantInfo{NAME, DT, 2 * R, 64 * NXP - 4 * R, NW - 4 * R, 1, 64 * NW, 1, 0, 2},         \
              &fine_launch_half_rows<T, R, NXP, NW, PD, 1>}
template <typename T, int S, int NXP, int NY, int NW, int PD, int XT = 0>
void coarse_launch_rows(const ItemDesc *items, int nitems, int nblocks, int chunk, hipStream_t s, int *occ)
{
    if (occ) return occupancy_of((euler_chunk_rows<T, S, NXP, NY, NW, PD, XT>), 64 * NW, occ);
    hipLaunchKernelGGL((euler_chunk_rows<T, S, NXP, NY, NW, PD, XT>), dim3(nblocks), dim3(64 * NW), 0, s, items,
                       nitems, chunk);
}
#define COARSE_ROWS(T, DT, S, NXP, NY, NW, PD, NAME)                                                     \
    CoarseEntry{VariantInfo{NAME, DT, 0, 64 * NXP, NW * NY - 2 * S, NXP, 64 * NW, S, 64 * NXP},         \
                &coarse_launch_rows<T, S, NXP, NY, NW, PD>}
// x tiles of 64*NXP columns (output 64*NXP - 2S) over rows of any length
#define COARSE_ROWSX(T, DT, S, NXP, NY, NW, PD, NAME)                                                    \
    CoarseEntry{VariantInfo{NAME, DT, 0, 64 * NXP - 2 * S, NW * NY - 2 * S, 1, 64 * NW, S, 0},          \
                &coarse_launch_rows<T, S, NXP, NY, NW, PD, 1>}
#define COARSE_1B(T, DT, S, NXP, NY, BXT, BY, PD, NAME)                                                   \
    CoarseEntry{VariantInfo{NAME, DT, 0, BXT * NXP - 2 * S, BY * NY - 2 * S, NXP, BXT * BY, S},          \
                &coarse_launch_1b<T, S, NXP, NY, BXT, BY, PD>}

// index 0 and 1 are reserved (automatic, unfused reference)
const FineEntry kFine[] = {
    // first fused form (four barriers per plane), fourth order
    FINE_V(float, 1, 2, 1, 2, 48, 16, "rk4_f32_o4_t32x16_p1x2"),
    // one barrier per plane, any radius
    FINE_1R(float, 1, 2, 2, 2, 24, 16, 2, "rk4r_f32_o4_t32x16_p2x2_d2"),
    // one barrier per plane, radius 1, 2-D tiles
    FINE_1B(float, 1, 2, 2, 36, 20, 2, "rk4b_f32_t64x32_p2x2_d2"),
    FINE_1B(float, 1, 2, 2, 28, 16, 2, "rk4b_f32_t48x24_p2x2_d2"),
    FINE_1B(float, 1, 2, 2, 28, 20, 2, "rk4b_f32_t48x32_p2x2_d2"),
    FINE_1B(float, 1, 2, 2, 36, 16, 2, "rk4b_f32_t64x24_p2x2_d2"),
    // whole rows, radius 1 (a grid row spans a wavefront, or a 16-lane DPP row: rk4s_)
    FINE_ROWS(double, 2, 2, 1, 16, 2, "rk4w_f64_x128_y8_p2x1_w16"),
    FINE_ROWS(double, 2, 1, 2, 8, 2, "rk4w_f64_x64_y8_p1x2_w8"),
    FINE_ROWS(double, 2, 1, 2, 12, 2, "rk4w_f64_x64_y16_p1x2_w12"),
    FINE_ROWS(float, 1, 4, 2, 8, 2, "rk4w_f32_x256_y8_p4x2_w8"),
    FINE_ROWS(float, 1, 2, 2, 8, 2, "rk4w_f32_x128_y8_p2x2_w8"),
    FINE_ROWS(float, 1, 2, 2, 12, 2, "rk4w_f32_x128_y16_p2x2_w12"),
    FINE_ROWS16(float, 1, 6, 1, 8, 2, "rk4s_f32_x96_y24_p6x1_w8"),
    FINE_ROWS16(float, 1, 3, 1, 8, 2, "rk4s_f32_x48_y24_p3x1_w8"),
    FINE_ROWS16(double, 2, 3, 1, 8, 2, "rk4s_f64_x48_y24_p3x1_w8"),
    FINE_ROWS16(double, 2, 2, 1, 10, 2, "rk4s_f64_x32_y32_p2x1_w10"),
    FINE_ROWS16(float, 1, 4, 1, 8, 2, "rk4s_f32_x64_y24_p4x1_w8"),
    FINE_ROWS16(float, 1, 4, 1, 12, 2, "rk4s_f32_x64_y40_p4x1_w12"),
    FINE_ROWS16(float, 1, 2, 1, 10, 2, "rk4s_f32_x32_y32_p2x1_w10"),
    // x tiles of 64 columns (56 outputs) wrapped onto rows of any length
    FINE_ROWSX(float, 1, 1, 3, 16, 2, "rk4x_f32_t56x40_p1x3_w16"),
    FINE_ROWSX(double, 2, 1, 2, 8, 2, "rk4x_f64_t56x8_p1x2_w8"),
    FINE_ROWSX(double, 2, 1, 3, 8, 2, "rk4x_f64_t56x16_p1x3_w8"),
    // whole rows, radius 2, two launches of two stages
    FINE_HALF_ROWS(double, 2, 2, 2, 16, 1, "rk4h_f64_o4_x128_y8_p2_w16_d1"),
    FINE_HALF_ROWS(float, 1, 2, 2, 16, 2, "rk4h_f32_o4_x128_y8_p2_w16"),
    FINE_HALF_ROWSX(double, 2, 2, 2, 16, 1, "rk4hx_f64_o4_t120x8_p2_w16_d1"),
};

const CoarseEntry kCoarse[] = {
    // one barrier per plane, 2-D tiles (S Euler steps per launch)
    COARSE_1B(double, 2, 4, 2, 2, 20, 20, 2, "euler4b_f64_t32x32_p2x2_d2"),
    COARSE_1B(double, 2, 4, 1, 4, 40, 10, 2, "euler4b_f64_t32x32_p1x4_d2"),
    COARSE_1B(double, 2, 2, 2, 2, 18, 18, 2, "euler2b_f64_t32x32_p2x2_d2"),
    COARSE_1B(float, 1, 4, 2, 2, 20, 20, 2, "euler4b_f32_t32x32_p2x2_d2"),
    COARSE_1B(float, 1, 4, 1, 4, 40, 10, 2, "euler4b_f32_t32x32_p1x4_d2"),
    COARSE_1B(float, 1, 8, 2, 2, 24, 16, 2, "euler8b_f32_t32x16_p2x2_d2"),
    // whole rows
    COARSE_ROWS(double, 2, 4, 2, 1, 16, 2, "euler4w_f64_x128_y8_p2x1_w16"),
    COARSE_ROWS(double, 2, 2, 2, 1, 16, 2, "euler2w_f64_x128_y12_p2x1_w16"),
    COARSE_ROWS(double, 2, 4, 1, 1, 16, 2, "euler4w_f64_x64_y8_p1x1_w16"),
    COARSE_ROWS(float, 1, 4, 4, 1, 16, 2, "euler4w_f32_x256_y8_p4x1_w16"),
    COARSE_ROWS(float, 1, 4, 2, 1, 16, 2, "euler4w_f32_x128_y8_p2x1_w16"),
    // x tiles of 64 columns (56 outputs) wrapped onto rows of any length
    COARSE_ROWSX(double, 2, 4, 1, 2, 16, 2, "euler4x_f64_t56x24_p1x2_w16"),
    COARSE_ROWSX(float, 1, 4, 1, 2, 16, 2, "euler4x_f32_t56x24_p1x2_w16"),
    COARSE_ROWSX(float, 1, 4, 1, 3, 16, 2, "euler4x_f32_t56x40_p1x3_w16"),
};

constexpr int kNumFine = (int)(sizeof(kFine) / sizeof(kFine[0]));
constexpr int kNumCoarse = (int)(sizeof(kCoarse) / sizeof(kCoarse[0]));

}  // namespace

int fine_variant_count() { return kNumFine + 2; }
int coarse_variant_count() { return kNumCoarse + 2; }

const VariantInfo *fine_variant(int v)
{
    if (v < 2 || v >= kNumFine + 2) return nullptr;
    return &kFine[v - 2].info;
}

const VariantInfo *coarse_variant(int v)
{
    if (v < 2 || v >= kNumCoarse + 2) return nullptr;
    return &kCoarse[v - 2].info;
}

// Resident blocks per compute unit of a fused variant on the current device
// (queried once per variant; 1 for anything else).
int fine_occupancy(int v)
{
    static std::mutex mu;
    static int cache[kNumFine] = {};
    if (v < 2 || v >= kNumFine + 2) return 1;
    std::lock_guard<std::mutex> lk(mu);
    int &c = cache[v - 2];
    if (c == 0) kFine[v - 2].fn(nullptr, 0, 0, 0, nullptr, &c);
    return c;
}

int coarse_occupancy(int v)
{
    static std::mutex mu;
    static int cache[kNumCoarse] = {};
    if (v < 2 || v >= kNumCoarse + 2) return 1;
    std::lock_guard<std::mutex> lk(mu);
    int &c = cache[v - 2];
    if (c == 0) kCoarse[v - 2].fn(nullptr, 0, 0, 0, nullptr, &c);
    return c;
}

hipError_t launch_fine_step(int variant, int dtype, int order, const ItemDesc *items, int nitems, int nblocks,
                            int jstep, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (variant == 1) {
        for (int st = 1; st <= 4; ++st) {
            if (dtype == 2) {
                if (order == 4)
                    hipLaunchKernelGGL((rk4_stage_ref<double, 2>), dim3(nblocks), dim3(kRefThreads), 0, s, items,
                                       nitems, jstep, st);
                else
                    hipLaunchKernelGGL((rk4_stage_ref<double, 1>), dim3(nblocks), dim3(kRefThreads), 0, s, items,
                                       nitems, jstep, st);
            } else {
                if (order == 4)
                    hipLaunchKernelGGL((rk4_stage_ref<float, 2>), dim3(nblocks), dim3(kRefThreads), 0, s, items,
                                       nitems, jstep, st);
                else
                    hipLaunchKernelGGL((rk4_stage_ref<float, 1>), dim3(nblocks), dim3(kRefThreads), 0, s, items,
                                       nitems, jstep, st);
            }
        }
        return hipGetLastError();
    }
    if (variant < 2 || variant >= kNumFine + 2) return hipErrorInvalidValue;
    kFine[variant - 2].fn(items, nitems, nblocks, jstep, s, nullptr);
    return hipGetLastError();
}

hipError_t launch_coarse_chunk(int variant, int dtype, const ItemDesc *items, int nitems, int nblocks, int chunk,
                               hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (variant == 1) {
        if (dtype == 2)
            hipLaunchKernelGGL((euler_step_ref<double>), dim3(nblocks), dim3(kRefThreads), 0, s, items, nitems, chunk);
        else
            hipLaunchKernelGGL((euler_step_ref<float>), dim3(nblocks), dim3(kRefThreads), 0, s, items, nitems, chunk);
        return hipGetLastError();
    }
    if (variant < 2 || variant >= kNumCoarse + 2) return hipErrorInvalidValue;
    kCoarse[variant - 2].fn(items, nitems, nblocks, chunk, s, nullptr);
    return hipGetLastError();
}

}  // namespace pr
