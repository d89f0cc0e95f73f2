/*
 * pr.h -- C ABI of the MI355X (gfx950) Parareal-over-stencils library.
 *
 * The library advances the 3D periodic advection-diffusion equation
 *     u_t + a . grad(u) = nu(t) Lap(u),   nu(t) = nu0 (1 + nu_amp sin(nu_omega t))
 * (arXiv 1409.8563, Section 3, eq. adv_diff_eq) with
 *   F  the fine propagator: classical RK4 with centered stencils of order 2
 *      (7-point) or 4 (13-point)              (Section 2.3, fine propagation; Section 3.1)
 *   G  the coarse propagator: forward Euler, first-order upwind advection and
 *      second-order centered diffusion        (Section 2.3, Algorithm 2)
 * and Parareal U^{k+1}_{n+1} = G(U^{k+1}_n) + F(U^k_n) - G(U^k_n)
 *                                              (Section 2.2, eq. parareal; Algorithm 1)
 *
 * Conventions shared by every entry point
 *   Grid     vertex based and periodic on [0,1)^3: x_i = i/n_x, h_d = 1/n_d.
 *   Layout   a field is n_x*n_y*n_z contiguous values, x fastest:
 *            u[(z*n_y + y)*n_x + x].  A batch of fields is contiguous,
 *            field b starting at element b*n_x*n_y*n_z.
 *   Memory   every `void*`/`double*` data argument is a DEVICE pointer unless
 *            stated otherwise; the caller owns all memory, including
 *            workspaces.  The library never frees caller memory.
 *   Streams  `stream` is a hipStream_t passed as void* (NULL = the null
 *            stream).  Entry points other than pr_parareal_solve are
 *            asynchronous on that stream.
 *   Time     fine step j of a run on [0,T] starts at t_j = j*T/nt_fine; time
 *            slice n covers global fine steps n*Nf .. n*Nf+Nf-1 with
 *            Nf = nt_fine/P (Section 2.1: integer step counts per slice).
 *            Coarse steps likewise with nt_coarse and Nc = nt_coarse/P.
 *            RK4 stages use nu at t_j, t_j+dt/2, t_j+dt/2, t_j+dt, or nu(t_j)
 *            for all four stages with PR_NU_FROZEN; Euler steps use nu(T_j).
 *   Errors   functions return PR_OK (0) or a negative status; no exception
 *            crosses the ABI.  All argument validation happens before any
 *            device work.  pr_last_error() returns a thread-local message for
 *            the last failing call.  The library can be loaded and every
 *            validation path exercised without a GPU; device work then fails
 *            with PR_EDEVICE.
 */
#ifndef PR_H
#define PR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PR_OK            0
#define PR_EINVAL       -1  /* invalid argument (sizes, counts, pointers, aliasing) */
#define PR_EUNSTABLE    -2  /* explicit step outside its stability bound (see pr_check_stability) */
#define PR_ENOMEM       -3  /* workspace smaller than the queried size */
#define PR_EDEVICE      -4  /* HIP runtime failure or no device */
#define PR_EUNSUPPORTED -5  /* valid request the library does not implement */
#define PR_ENONFINITE   -6  /* a defect norm became NaN or Inf during a solve */

/* dtypes of fields */
#define PR_FP32 1
#define PR_FP64 2

/* precision modes of a plan */
#define PR_MODE_FP64      0   /* sweeps, correction and norms in FP64 */
#define PR_MODE_MIXED     1   /* FP32 sweeps; FP64 correction, U and norms */
#define PR_MODE_PER_SLICE 16  /* OR-able: launch F slice by slice instead of batched */
#define PR_MODE_GRAPH     32  /* OR-able: record the solve once in a HIP graph and replay it */
#define PR_MODE_TIMED     64  /* OR-able: time the F and G phases with HIP events (eager launches) */
/* OR-able: the pipelined schedule of Section 2.2.1 on one device.  The slices
 * are cut into consecutive slice groups; F of group g in iteration k starts as
 * soon as iteration k-1's coarse chain has corrected every slice of g, on
 * streams owned by the plan, while the chain goes on with later groups on the
 * solve's stream, and iteration k's chain enters group g once that F is done.
 * Results are bitwise those of the phase-by-phase schedule.  Not with
 * PR_MODE_PER_SLICE or PR_EARLY_STOP (which reads each iteration's norms on
 * the host before the next F may start). */
#define PR_MODE_PIPELINED 128
/* slice groups of PR_MODE_PIPELINED (1..255; 0 or absent: 2), OR-ed into mode */
#define PR_MODE_PIPELINE_GROUPS(g) ((int32_t)(g) << 16)

/* problem flags */
#define PR_NU_FROZEN      1u  /* nu(t_j) for all RK4 stages of step j */
#define PR_ALLOW_UNSTABLE 2u  /* skip the stability guard */
#define PR_EARLY_STOP     4u  /* stop when max|U^{k+1}_P - U^k_P| <= tol * max|U^{k+1}_P| */
#define PR_SKIP_CONVERGED 8u  /* do not recompute slices n < k in iteration k (bitwise identical result) */
#define PR_COARSEN_G      16u /* plans: G runs on the grid coarsened by 2 per direction (every n_d even,
                                 n_d/2 >= 3): injection, the Euler steps with h = 2/n, interpolation back
                                 (Section 2.2.2 names a coarser mesh for G; the transfers are a reading) */
#define PR_CUBIC_INTERP   32u /* with PR_COARSEN_G: cubic (4-point) instead of linear interpolation */

/* One problem instance: the paper's problem statement (Section 2.1, Section 3). */
typedef struct pr_problem {
    int32_t  n[3];          /* n_x, n_y, n_z; each >= 3 (>= 5 for fine_order 4) */
    double   a[3];          /* advection velocity (the paper's c) */
    double   nu0;           /* nu(t) = nu0 * (1 + nu_amp * sin(nu_omega * t)), nu > 0 required */
    double   nu_amp;
    double   nu_omega;
    double   T;             /* final time, > 0 */
    int32_t  P;             /* number of time slices N_p, >= 1 */
    int32_t  nt_fine;       /* fine steps on [0,T]; multiple of P */
    int32_t  nt_coarse;     /* coarse steps on [0,T]; multiple of P */
    int32_t  K;             /* Parareal iterations, 0 <= K <= P (K = 0 returns the coarse guess) */
    int32_t  fine_order;    /* 2 or 4 */
    uint32_t flags;         /* PR_NU_FROZEN | PR_ALLOW_UNSTABLE | PR_EARLY_STOP | PR_SKIP_CONVERGED |
                               PR_COARSEN_G | PR_CUBIC_INTERP */
    double   tol;           /* early-stop threshold (PR_EARLY_STOP) */
} pr_problem;

/* Opaque solve plan: validated problems, workspace layout, descriptor tables,
 * optionally a recorded HIP graph. */
typedef struct pr_plan pr_plan;

/* Thread-local description of the last non-OK status (never NULL). */
const char *pr_last_error(void);

/* Library version string (static storage). */
const char *pr_version(void);

/*
 * pr_check_stability -- stability margins of the explicit steppers.
 *   fine_margin   <- max |R(dt * mu)| of the RK4 amplification polynomial
 *                    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 over the stencil
 *                    symbols mu = nu * sD(theta) + sA(theta) of 48 sampled
 *                    wavenumbers per axis (endpoints 0 and pi included) and
 *                    nu in {nu_min, nu_max}; <= 1 is stable
 *   coarse_margin <- max_t Dt * (sum_d |a_d|/h_d + 2 nu(t) sum_d 1/h_d^2); forward
 *                    Euler with upwind advection keeps every Fourier mode's
 *                    amplification in the unit disc iff this is <= 1.
 * Either output pointer (HOST) may be NULL.  Returns PR_EUNSTABLE if a margin
 * exceeds 1, PR_EINVAL for an invalid problem, PR_OK otherwise.  No device work.
 */
int pr_check_stability(const pr_problem *prob, double *fine_margin, double *coarse_margin);

/*
 * pr_fine_sweep -- F: nsteps RK4 steps on `batch` fields at once (Section 2.3,
 * fine propagation; eq. fine applied step by step).
 *   dtype      PR_FP32 or PR_FP64: storage and arithmetic type of u_in/u_out
 *   u_in       batch fields (read only), 16-byte aligned
 *   u_out      batch fields, 16-byte aligned; must not overlap u_in
 *   step0      HOST array [batch]: global fine step index of each field's
 *              first step (slice n starts at n*Nf)
 *   nsteps     >= 0 (0 copies u_in to u_out)
 *   ws         device workspace of at least pr_sweep_workspace_bytes(...) bytes
 * Asynchronous on `stream`.  prob->P, K and nt_coarse are not used here;
 * prob->nt_fine and T define dt.
 */
int pr_fine_sweep(const pr_problem *prob, int32_t dtype, int32_t batch, const void *u_in, void *u_out,
                  const int64_t *step0, int32_t nsteps, void *ws, size_t ws_bytes, void *stream);

/*
 * pr_coarse_sweep -- G: nsteps forward Euler steps of Algorithm 2 (upwind
 * advection chosen by the sign of a_d, a_d = 0 takes the downwind branch whose
 * term vanishes), arguments as pr_fine_sweep; step0 counts coarse steps.
 */
int pr_coarse_sweep(const pr_problem *prob, int32_t dtype, int32_t batch, const void *u_in, void *u_out,
                    const int64_t *step0, int32_t nsteps, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes needed by pr_fine_sweep / pr_coarse_sweep for these sizes. */
size_t pr_sweep_workspace_bytes(const pr_problem *prob, int32_t dtype, int32_t batch);

/*
 * Grid transfers of the coarsened G (PR_COARSEN_G), on `batch` contiguous
 * fields; prob gives the FINE grid (every n_d even, n_d/2 >= 3), dtype is
 * PR_FP32 or PR_FP64 for input and output.
 *   pr_restrict  u_coarse[(z*ny/2 + y)*nx/2 + x] = u_fine at (2x, 2y, 2z)
 *                (injection); u_coarse holds batch * npts/8 values
 *   pr_prolong   u_fine from u_coarse: per direction an even index copies
 *                coarse point i/2, an odd index takes 1/2, 1/2 of its two
 *                coarse neighbours (order 1) or -1/16, 9/16, 9/16, -1/16 of
 *                four (order 3), periodic; the 3-D value is the tensor
 *                product, summed z taps outermost, then y, then x
 *   ws           workspace of pr_transfer_workspace_bytes(batch) bytes
 * The coarse sweep in between is pr_coarse_sweep on the problem with n/2.
 */
size_t pr_transfer_workspace_bytes(int32_t batch);
int pr_restrict(const pr_problem *prob, int32_t dtype, int32_t batch, const void *u_fine, void *u_coarse,
                void *ws, size_t ws_bytes, void *stream);
int pr_prolong(const pr_problem *prob, int32_t dtype, int32_t order, int32_t batch, const void *u_coarse,
               void *u_fine, void *ws, size_t ws_bytes, void *stream);

/*
 * pr_parareal_update -- the correction of eq. parareal / Algorithm 1 evaluated
 * in FP64 as  u_out = f_new + (g_new - g_old)  for npts*batch values.
 *   sweep_dtype  dtype of f_new, g_new, g_old (PR_FP32 or PR_FP64)
 *   u_out        FP64 result
 *   u_out_lo     optional copy of u_out rounded to sweep_dtype (may be NULL)
 * With g_new == g_old elementwise the result equals f_new exactly.
 */
int pr_parareal_update(int64_t npts, int32_t batch, int32_t sweep_dtype, const void *f_new,
                       const void *g_new, const void *g_old, double *u_out, void *u_out_lo, void *stream);

/*
 * pr_defect_norm -- for each of `batch` field pairs (x_b, r_b) of npts values,
 * out4[b] = { max|x-r|, max|r|, sum (x-r)^2, sum r^2 } in FP64 (Section 2.2.3,
 * eq. defect is out4[0]/out4[1]).  Deterministic: fixed partition and fixed
 * reduction order, independent of timing.  xd/rd: PR_FP32 or PR_FP64.
 *   out4  DEVICE array [batch][4] doubles
 *   ws    workspace of at least pr_defect_workspace_bytes(batch) bytes
 */
int pr_defect_norm(int64_t npts, int32_t batch, int32_t xd, const void *x, int32_t rd, const void *ref,
                   double *out4, void *ws, size_t ws_bytes, void *stream);
size_t pr_defect_workspace_bytes(int32_t batch);

/*
 * pr_defect_norm_static -- pr_defect_norm without a workspace argument and
 * without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and determinism as pr_defect_norm
 * (bitwise the same out4; same kernels).  Its descriptor table and block
 * partials live in a library-owned device array of
 * pr_defect_static_scratch_bytes() bytes (about 1 MiB), one per GPU, held
 * until the process ends; it serves at most PR_DEFECT_STATIC_MAX_BATCH field
 * pairs per call (larger batch: PR_EINVAL, nothing launched).  Every call on
 * one GPU shares that GPU's array: calls whose work overlaps on one GPU (on
 * different streams, or from several threads) race and must be ordered by
 * the caller.  Nothing in the array needs clearing between calls (every
 * partial is written before it is read).
 */
#define PR_DEFECT_STATIC_MAX_BATCH 64
int pr_defect_norm_static(int64_t npts, int32_t batch, int32_t xd, const void *x, int32_t rd, const void *ref,
                          double *out4, void *stream);
size_t pr_defect_static_scratch_bytes(void);

/*
 * pr_copy_probe -- achievable HBM bandwidth of a plain streaming kernel of
 * this library: copies `bytes` (a positive multiple of 16; src and dst
 * 16-byte aligned, not overlapping) from src to dst with 16-byte accesses,
 * on blocks_per_cu (1..64, 0 = 8) blocks of 256 threads per compute unit.
 * variant 0: four 16-byte loads in flight per thread, 1: the same with
 * non-temporal loads and stores, 2: eight in flight, 3: one.  It is the
 * measured ceiling of a kernel that reads once and writes once, beside the
 * device's nominal peak.  Asynchronous on `stream`.
 */
int pr_copy_probe(const void *src, void *dst, size_t bytes, int32_t variant, int32_t blocks_per_cu, void *stream);

/*
 * Plans and the full solve (Algorithm 1 with all slices of all instances on
 * one device; the slices are a batch dimension of F).
 *   probs   HOST array [ninst] of problems (each with its own grid, a, nu,
 *           step counts and P; K and flags must be equal across instances)
 *   mode    PR_MODE_FP64 or PR_MODE_MIXED, optionally | PR_MODE_PER_SLICE,
 *           | PR_MODE_GRAPH, | PR_MODE_TIMED, | PR_MODE_PIPELINED (with
 *           | PR_MODE_PIPELINE_GROUPS(g))
 *   ws      device workspace of pr_plan_workspace_bytes(probs, ninst, mode)
 *           bytes; owned by the caller, must outlive the plan
 * pr_plan_create validates everything (including stability unless
 * PR_ALLOW_UNSTABLE) and performs no kernel launch.  Each instance takes the
 * F variant chosen for its own grid (tuned, else built-in, at the batch of
 * all slices of the instances with that grid); instances with the same
 * choice form a launch group, and every fine step is one launch per group.
 * With several groups, the groups' launches of an F phase run concurrently
 * on streams owned by the plan, forked from and joined back to the solve's
 * stream.  G uses one variant for all instances.
 */
size_t pr_plan_workspace_bytes(const pr_problem *probs, int32_t ninst, int32_t mode);
int pr_plan_create(const pr_problem *probs, int32_t ninst, int32_t mode, void *ws, size_t ws_bytes,
                   pr_plan **out);
void pr_plan_destroy(pr_plan *plan);

/*
 * pr_parareal_solve -- run K iterations (or fewer with PR_EARLY_STOP).
 *   u0    HOST array [ninst] of DEVICE pointers to FP64 initial fields
 *   uT    HOST array [ninst] of DEVICE pointers receiving U^K_P (FP64)
 *   ref   HOST array [ninst] of DEVICE pointers to FP64 reference fields at
 *         T (e.g. the serial fine solution) for d^k, or NULL
 *   log   HOST array [ninst][K][12] or NULL; row k of instance i:
 *          [0..3]  {max|dU|, max|U|, sum dU^2, sum U^2} for dU = U^{k+1}_P - U^k_P
 *          [4..7]  the same over all slices n = 1..P (max of max, sum of sums)
 *          [8..11] {max|U^{k+1}_P - ref|, max|ref|, sum (.)^2, sum ref^2} (zeros if ref is NULL)
 * Blocking: returns after the results are in uT.  Returns PR_ENONFINITE if a
 * logged norm is not finite.
 */
int pr_parareal_solve(pr_plan *plan, const double *const *u0, double *const *uT, const double *const *ref,
                      double *log, void *stream);

/* Iterations performed by the last solve (< K only with PR_EARLY_STOP). */
int pr_plan_iterations(const pr_plan *plan);

/* Kernel variants the plan launches for F and G (HOST outputs, may be NULL);
 * for F, the variant of the group with the most fine grid-point updates.
 * Names via pr_kernel_variant_name. */
int pr_plan_kernel_variants(const pr_plan *plan, int32_t *fine_variant, int32_t *coarse_variant);

/* The plan's F launch groups: *count (HOST) receives the number of groups;
 * the first min(count, max) entries of variant, blocks_per_cu (0: default
 * layout) and instances (instances in the group) are filled, in the order
 * of the groups' first instance.  The arrays may be NULL when max is 0. */
int pr_plan_fine_groups(const pr_plan *plan, int32_t max, int32_t *count, int32_t *variant,
                        int32_t *blocks_per_cu, int32_t *instances);

/*
 * pr_plan_timings -- phase times of the last solve of a PR_MODE_TIMED plan
 * (HOST out[6]): {F ms, G-chain ms (coarse sweeps and corrections), start-up
 * coarse ms, number of fused F step launches, number of G launches, total ms}.
 * F time is measured from before the first to after the last step launch of
 * each iteration, so it includes launch gaps.  Under PR_MODE_PIPELINED the
 * phases overlap: F time sums, over iterations and slice groups, the span of
 * the group's step launches on the F streams, and G-chain time sums, per
 * iteration, the span from the chain's entry into the first slice group to
 * its end.
 */
int pr_plan_timings(const pr_plan *plan, double *out6);

/*
 * pr_plan_slice_state -- DEVICE pointer to the FP64 state U_n (n = 0..P) of
 * instance `inst` inside the plan workspace, valid after a solve until the
 * next one (the current iterate at every slice boundary).
 */
int pr_plan_slice_state(const pr_plan *plan, int32_t inst, int32_t n, const double **out);

/*
 * Kernel variant selection (testing and tuning).  0 = automatic choice
 * (autotuned table, else built-in default); 1 = unfused reference kernels
 * (one launch per RK4 stage / Euler step); >= 2 index the fused variants
 * listed by pr_kernel_variant_name.  Per process, not thread-safe with
 * concurrent launches.
 */
int pr_set_kernel_variant(int32_t fine_variant, int32_t coarse_variant);
int pr_kernel_variant_count(int32_t which /* 0 fine, 1 coarse */);
const char *pr_kernel_variant_name(int32_t which, int32_t variant);
/* Properties of a fused variant (HOST outputs, any may be NULL): field dtype,
 * fine stencil order (0 for coarse), output tile, x points per thread (n_x
 * must be a multiple), Euler steps fused per launch (1 for fine), and the
 * exact n_x a whole-row variant requires (0: any multiple of nxp). */
int pr_kernel_variant_info(int32_t which, int32_t variant, int32_t *dtype, int32_t *order, int32_t *tile_x,
                           int32_t *tile_y, int32_t *nxp, int32_t *steps, int32_t *nx_exact);

/* Variant a sweep of this problem, dtype and batch would launch for F
 * (which = 0) or G (which = 1) -- tuned, forced or built-in default (HOST
 * output).  No device work. */
int pr_sweep_kernel_variant(const pr_problem *prob, int32_t dtype, int32_t batch, int32_t which, int32_t *variant);

/*
 * pr_autotune -- time the fused variants of F (which = 0) or G (which = 1)
 * for this problem and batch on the device, each with z chunks sized for the
 * kernel's resident blocks per compute unit (reported as 0) and for 1, 2
 * and 4 blocks per compute unit, and remember the fastest pair for (grid,
 * dtype, fine_order, batch); sweeps of that shape then use it (the entry of
 * their batch, else any tuned batch of the shape).  Scratch buffers come
 * from `ws` (pr_autotune_workspace_bytes).  Blocking.  best_variant (HOST,
 * may be NULL) receives the variant.  Results do not depend on the choice.
 */
size_t pr_autotune_workspace_bytes(const pr_problem *prob, int32_t dtype, int32_t batch);
int pr_autotune(const pr_problem *prob, int32_t dtype, int32_t batch, int32_t which, void *ws,
                size_t ws_bytes, void *stream, int32_t *best_variant);

/*
 * pr_plan_autotune -- tune the plan's own launches: for each F launch group,
 * every fused variant of F that applies to all its instances, with z chunks
 * sized as in pr_autotune (0: resident blocks, or 1, 2, 4 blocks per compute
 * unit), timed on the group's F
 * launch over all its slices; likewise G (one variant for all instances) on
 * the coarse chain's launch.  The plan keeps the fastest (a recorded graph
 * is re-recorded at the next solve).  Overwrites the slice states in the
 * workspace (the next solve starts from u0 anyway); blocking.  Outputs
 * (HOST, may be NULL): the choice of the group with the most fine work and
 * of G, variant and blocks per compute unit.  Results of later solves are
 * bitwise the same as before.
 */
int pr_plan_autotune(pr_plan *plan, void *stream, int32_t *fine_variant, int32_t *fine_blocks_per_cu,
                     int32_t *coarse_variant, int32_t *coarse_blocks_per_cu);

/*
 * Persisted autotune table.  The choices of pr_autotune and pr_plan_autotune
 * are kept per (device architecture, F or G, grid, dtype, fine order, batch)
 * with the variant stored by name; plan creation and sweeps look them up for
 * the current device's architecture only.
 *   pr_autotune_save   write the table as JSON to `path` (HOST string)
 *   pr_autotune_load   merge the entries of such a file into the table;
 *                      entries naming a variant the library lacks are skipped;
 *                      *loaded (HOST, may be NULL) receives the number merged
 *   pr_autotune_clear  empty the table
 * If the environment variable PR_AUTOTUNE_CACHE names a file, that file is
 * loaded before the first lookup and rewritten after every tuning call.
 * Errors: PR_EINVAL for a NULL path, an unreadable or unwritable file, or a
 * file that is not such a table.  No device work.
 */
int pr_autotune_save(const char *path);
int pr_autotune_load(const char *path, int32_t *loaded);
int pr_autotune_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* PR_H */
