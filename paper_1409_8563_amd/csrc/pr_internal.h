// Internal declarations shared by the HIP kernels and the host runtime of the
// Parareal-over-stencils library (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pr {

// One field advanced by a sweep ("item"): a time slice of one problem
// instance.  Tables of items live in device memory and are read with uniform
// (scalar) loads by every block of a launch.
struct ItemDesc {
    const void *src0;     // input field (read by the first step/chunk)
    void *dst;            // output of the last step/chunk
    void *tmp;            // ping-pong partner of dst (unused when one launch suffices)
    void *scratch;        // 3 fields of stage storage (unfused reference kernels, two-launch RK4 steps)
    int64_t step0;        // global index of the first step
    int32_t nsteps;       // steps of this sweep
    int32_t nx, ny, nz;
    int32_t tiles_x, tiles_y, zchunks, tz;
    int32_t block_begin;  // first logical block of this item in a launch
    int32_t nblocks;      // blocks of this item in a launch
    double dt;            // step size
    double nu0, nu_amp, nu_omega;
    double inv_h2[3];     // 1/h_d^2
    double a_over_h[3];   // a_d/h_d
    int32_t frozen;       // RK4: nu(t_j) in all stages
    int32_t pad_;
};

// One pointwise item (correction, casts, norms): npts contiguous values.
struct PointItem {
    const void *a;        // f_new (correction) / x (norms) / source (casts)
    const void *b;        // g_new / ref
    const void *c;        // g_old
    double *u;            // FP64 output (correction), or nullptr
    void *ulo;            // sweep-dtype copy of u, or nullptr
    double *partials;     // [nbp][4] block partials, or nullptr
    double *out4;         // final 4 norms (defect_final), or nullptr
    int64_t npts;
};

constexpr int kNormBlocks = 512;   // blocks per item of the deterministic reductions
constexpr int kNormThreads = 512;

// ---- launch wrappers (kernels.hip) ----------------------------------------
// Fine RK4, one step per launch, over the first `nitems` items of `items`
// (device table).  variant >= 2 selects a fused tile configuration; 1 = the
// unfused reference (four stage launches).
hipError_t launch_fine_step(int variant, int dtype, int order, const ItemDesc *items, int nitems,
                            int nblocks, int jstep, hipStream_t s);
// Coarse Euler: chunk `chunk` of S steps (S = steps_per_launch of the variant).
hipError_t launch_coarse_chunk(int variant, int dtype, const ItemDesc *items, int nitems, int nblocks,
                               int chunk, hipStream_t s);

// Fused-variant metadata used by the host to lay out tiles.
struct VariantInfo {
    const char *name;
    int dtype;            // PR_FP32 / PR_FP64
    int order;            // fine: 2/4 ; coarse: 0
    int tx, ty;           // output tile
    int nxp;              // x points per thread (nx must be a multiple)
    int threads;
    int steps;            // coarse: Euler steps fused per launch
    int rowx = 0;         // nonzero: whole-row kernel, n_x must equal rowx (= tx, one tile in x)
    int scratch = 0;      // fields of per-item scratch (ItemDesc::scratch) the kernel uses
};
int fine_variant_count();
const VariantInfo *fine_variant(int v);      // v >= 2
int coarse_variant_count();
const VariantInfo *coarse_variant(int v);    // v >= 2
int fine_occupancy(int v);                   // resident blocks per compute unit (1 if v < 2)
int coarse_occupancy(int v);

// Grid transfers of the coarsened G over tables of ItemDesc (src0 -> dst,
// nx/ny/nz of the fine grid): injection to the grid coarsened by 2, and
// interpolation of order 1 or 3 back to the fine grid.
hipError_t launch_restrict(int dtype, const ItemDesc *items, int nitems, hipStream_t s);
hipError_t launch_prolong(int dtype, int order, const ItemDesc *items, int nitems, hipStream_t s);

// Pointwise kernels over tables of PointItem (blockIdx.y = item).
enum PointOp { kOpCorrect = 0, kOpAssign = 1, kOpCopy64 = 2 };
//   kOpCorrect: u = a + (b - c) in FP64 (a, b, c of sweep dtype); ulo = (T)u;
//               partials of (u - previous u) if requested
//   kOpAssign : u = (double)a; ulo = a
//   kOpCopy64 : u = a (a is FP64); ulo = (T)a
hipError_t launch_pointwise(int op, int sweep_dtype, const PointItem *items, int nitems, bool with_partials,
                            hipStream_t s);
hipError_t launch_pointwise_inline(int op, int sweep_dtype, const PointItem &item, hipStream_t s);
hipError_t launch_defect_partials(int xd, int rd, const PointItem *items, int nitems, hipStream_t s);
hipError_t launch_defect_final(const PointItem *items, int nitems, hipStream_t s);
// Achievable-bandwidth probe: copy `bytes` (multiple of 16) with `blocks`
// blocks; variant 0: 4 loads in flight per thread, 1: the same with
// non-temporal accesses, 2: 8 in flight, 3: 1 in flight.
hipError_t launch_copy_probe(int variant, const void *src, void *dst, size_t bytes, int blocks, hipStream_t s);
// Copy host descriptor arrays into device tables through kernel arguments
// (stream ordered and safe to record in a graph).
hipError_t launch_write_items(const ItemDesc *host_items, int n, ItemDesc *dev_table, hipStream_t s);
hipError_t launch_write_points(const PointItem *host_items, int n, PointItem *dev_table, hipStream_t s);

}  // namespace pr
