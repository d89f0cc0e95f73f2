/*
 * Plain serial FP64 CPU oracle for Parareal over 3D advection-diffusion
 * stencils.  TEST INFRASTRUCTURE ONLY: it is called by the test suite, by the
 * smoke check and by the benchmark's CPU-baseline leg, never by the product
 * path.  It shares no code, header or table with the GPU library.
 *
 * What it computes, with the passage each part follows:
 *   - the IVP u_t = f(u, t) split into P time slices  (Section 2.1, eq. ivp)
 *   - the benchmark PDE u_t + a.grad u = nu(t) Lap u on the periodic unit
 *     cube with nu(t) = nu0 (1 + amp sin(omega t))     (Section 3, eq. adv_diff_eq)
 *   - the 7-point Laplacian                            (Section 2.3, the Laplacian formula)
 *   - coarse propagator G: forward Euler, first-order upwind advection,
 *     second-order centered diffusion                  (Section 2.3, Algorithm 2)
 *   - fine propagator F: classical RK4 with centered differences; order 2
 *     (7-point) or order 4 (13-point, Section 3.1)     (Section 2.3, the fine-propagation item)
 *   - Parareal iteration                               (Section 2.2, eq. parareal; Algorithm 1)
 *   - optionally G on a spatially coarsened mesh with restriction and
 *     interpolation                                    (Section 2.2.2, speedup-bound discussion)
 *   - norms of the defect                              (Section 2.2.3, eq. defect)
 *
 * Readings taken where the paper is silent:
 *   - grid points x_i = i/n, periodic, h_d = 1/n_d, storage u[(z*ny + y)*nx + x];
 *   - RK4 stage times t, t+dt/2, t+dt/2, t+dt (or all t with nu_frozen);
 *   - fine step j of the whole run starts at t = j*dt (slice n, local step i:
 *     j = n*Nf + i), coarse step j at t = j*Dt;
 *   - second-order centered advection (u_{+1} - u_{-1})/(2h); fourth-order
 *     stencils are the textbook central differences;
 *   - the Euler loop of Algorithm 2 performs Nc steps (its loop bound counts
 *     Nc + 1);
 *   - the correction is evaluated as F + (G_new - G_old);
 *   - upwind for a_d == 0 takes the "else" branch (the term vanishes);
 *   - coarsened G: injection restriction, linear or cubic Lagrange
 *     interpolation, the Euler steps of Algorithm 2 on the grid with h = 2/n.
 *
 * Floating point: IEEE binary64, round to nearest, built with
 * -O2 -ffp-contract=off and no fast-math.  Loops over z may run under OpenMP;
 * every output point is computed by the same operations whatever the thread
 * count, and all reductions are serial, so results do not depend on it.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    int32_t order;        /* fine stencil order: 2 or 4 */
    double ax, ay, az;    /* advection velocity */
    double nu0, nu_amp, nu_omega;
    double T;
    int32_t P;            /* number of time slices */
    int32_t nt_fine;      /* fine steps on [0, T] */
    int32_t nt_coarse;    /* coarse steps on [0, T] */
    int32_t nu_frozen;    /* 1: nu(t_j) for all four RK4 stages */
    int32_t coarsen;      /* 1: G runs on the grid coarsened by 2 in every direction */
    int32_t interp_order; /* coarse -> fine interpolation: 1 (linear) or 3 (cubic) */
} or_prob;

/* Threads the z loops run on (1 without OpenMP). */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the z loops (results do not depend on it). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static long npts_of(const or_prob *p) { return (long)p->nx * p->ny * p->nz; }

static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

double or_nu(const or_prob *p, double t)
{
    return p->nu0 * (1.0 + p->nu_amp * sin(p->nu_omega * t));
}

/* Fine right-hand side L(u) = nu * Lap(u) - a.grad(u), centered differences of
 * order 2 (radius 1) or 4 (radius 2). */
void or_fine_rhs(const or_prob *p, double nu, const double *u, double *out)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const double hx = 1.0 / nx, hy = 1.0 / ny, hz = 1.0 / nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                const long c = ((long)z * ny + y) * nx + x;
                double lap, adv;
                if (p->order == 4) {
                    const double xm2 = u[((long)z * ny + y) * nx + wrap(x - 2, nx)];
                    const double xm1 = u[((long)z * ny + y) * nx + wrap(x - 1, nx)];
                    const double xp1 = u[((long)z * ny + y) * nx + wrap(x + 1, nx)];
                    const double xp2 = u[((long)z * ny + y) * nx + wrap(x + 2, nx)];
                    const double ym2 = u[((long)z * ny + wrap(y - 2, ny)) * nx + x];
                    const double ym1 = u[((long)z * ny + wrap(y - 1, ny)) * nx + x];
                    const double yp1 = u[((long)z * ny + wrap(y + 1, ny)) * nx + x];
                    const double yp2 = u[((long)z * ny + wrap(y + 2, ny)) * nx + x];
                    const double zm2 = u[((long)wrap(z - 2, nz) * ny + y) * nx + x];
                    const double zm1 = u[((long)wrap(z - 1, nz) * ny + y) * nx + x];
                    const double zp1 = u[((long)wrap(z + 1, nz) * ny + y) * nx + x];
                    const double zp2 = u[((long)wrap(z + 2, nz) * ny + y) * nx + x];
                    const double uc = u[c];
                    lap = (-xp2 + 16.0 * xp1 - 30.0 * uc + 16.0 * xm1 - xm2) / (12.0 * hx * hx)
                        + (-yp2 + 16.0 * yp1 - 30.0 * uc + 16.0 * ym1 - ym2) / (12.0 * hy * hy)
                        + (-zp2 + 16.0 * zp1 - 30.0 * uc + 16.0 * zm1 - zm2) / (12.0 * hz * hz);
                    adv = p->ax * (-xp2 + 8.0 * xp1 - 8.0 * xm1 + xm2) / (12.0 * hx)
                        + p->ay * (-yp2 + 8.0 * yp1 - 8.0 * ym1 + ym2) / (12.0 * hy)
                        + p->az * (-zp2 + 8.0 * zp1 - 8.0 * zm1 + zm2) / (12.0 * hz);
                } else {
                    const double xm1 = u[((long)z * ny + y) * nx + wrap(x - 1, nx)];
                    const double xp1 = u[((long)z * ny + y) * nx + wrap(x + 1, nx)];
                    const double ym1 = u[((long)z * ny + wrap(y - 1, ny)) * nx + x];
                    const double yp1 = u[((long)z * ny + wrap(y + 1, ny)) * nx + x];
                    const double zm1 = u[((long)wrap(z - 1, nz) * ny + y) * nx + x];
                    const double zp1 = u[((long)wrap(z + 1, nz) * ny + y) * nx + x];
                    const double uc = u[c];
                    lap = (xp1 + xm1 - 2.0 * uc) / (hx * hx)
                        + (yp1 + ym1 - 2.0 * uc) / (hy * hy)
                        + (zp1 + zm1 - 2.0 * uc) / (hz * hz);
                    adv = p->ax * (xp1 - xm1) / (2.0 * hx)
                        + p->ay * (yp1 - ym1) / (2.0 * hy)
                        + p->az * (zp1 - zm1) / (2.0 * hz);
                }
                out[c] = nu * lap - adv;
            }
        }
    }
}

/* First-order one-sided difference along one axis, taken on the side the
 * flow comes from: the backward difference (u_0 - u_{-1})/h for a positive
 * velocity component, the forward difference (u_{+1} - u_0)/h otherwise
 * (a zero component multiplies the result by zero either way). */
static double upwind_slope(double vel, double um, double u0, double up, double h)
{
    return vel > 0.0 ? (u0 - um) / h : (up - u0) / h;
}

/* Coarse right-hand side (the operator of Algorithm 2): nu times the 7-point
 * Laplacian, minus a.grad(u) where each component of grad(u) is the upwind
 * one-sided difference of its axis.  Assembled axis by axis: for axis d the
 * two neighbours at distance one along d enter both the second difference
 * and the upwind slope. */
void or_coarse_rhs(const or_prob *p, double nu, const double *u, double *out)
{
    const int n[3] = {p->nx, p->ny, p->nz};
    const double vel[3] = {p->ax, p->ay, p->az};
#pragma omp parallel for schedule(static)
    for (int z = 0; z < n[2]; ++z) {
        for (int y = 0; y < n[1]; ++y) {
            for (int x = 0; x < n[0]; ++x) {
                const int at[3] = {x, y, z};
                const double uc = u[((long)z * n[1] + y) * n[0] + x];
                double lap = 0.0, adv = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int lo[3] = {x, y, z}, hi[3] = {x, y, z};
                    lo[d] = wrap(at[d] - 1, n[d]);
                    hi[d] = wrap(at[d] + 1, n[d]);
                    const double um = u[((long)lo[2] * n[1] + lo[1]) * n[0] + lo[0]];
                    const double up = u[((long)hi[2] * n[1] + hi[1]) * n[0] + hi[0]];
                    const double h = 1.0 / n[d];
                    lap += (up + um - 2.0 * uc) / (h * h);
                    adv += vel[d] * upwind_slope(vel[d], um, uc, up, h);
                }
                out[((long)z * n[1] + y) * n[0] + x] = nu * lap - adv;
            }
        }
    }
}

/* One classical RK4 step of the fine method, global step index j.
 * work must hold 5 * npts doubles; u and out may alias. */
void or_rk4_step(const or_prob *p, long j, const double *u, double *out, double *work)
{
    const long n = npts_of(p);
    const double dt = p->T / p->nt_fine;
    const double t = (double)j * dt;
    const double nu1 = or_nu(p, t);
    const double nu2 = p->nu_frozen ? nu1 : or_nu(p, t + 0.5 * dt);
    const double nu4 = p->nu_frozen ? nu1 : or_nu(p, t + dt);
    double *y = work, *k1 = work + n, *k2 = work + 2 * n, *k3 = work + 3 * n, *k4 = work + 4 * n;

    or_fine_rhs(p, nu1, u, k1);
    for (long i = 0; i < n; ++i) y[i] = u[i] + 0.5 * dt * k1[i];
    or_fine_rhs(p, nu2, y, k2);
    for (long i = 0; i < n; ++i) y[i] = u[i] + 0.5 * dt * k2[i];
    or_fine_rhs(p, nu2, y, k3);
    for (long i = 0; i < n; ++i) y[i] = u[i] + dt * k3[i];
    or_fine_rhs(p, nu4, y, k4);
    for (long i = 0; i < n; ++i)
        out[i] = u[i] + dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* One forward Euler step of the coarse method (Algorithm 2), global coarse
 * step index j.  work must hold npts doubles; u and out may alias. */
void or_euler_step(const or_prob *p, long j, const double *u, double *out, double *work)
{
    const long n = npts_of(p);
    const double Dt = p->T / p->nt_coarse;
    const double nu = or_nu(p, (double)j * Dt);
    or_coarse_rhs(p, nu, u, work);
    for (long i = 0; i < n; ++i) out[i] = u[i] + Dt * work[i];
}

/* F over time slice s: Nf = nt_fine / P RK4 steps starting at global step s*Nf. */
void or_fine_prop(const or_prob *p, int s, const double *u, double *out, double *work)
{
    const long n = npts_of(p);
    const int nf = p->nt_fine / p->P;
    memcpy(out, u, (size_t)n * sizeof(double));
    for (int i = 0; i < nf; ++i) or_rk4_step(p, (long)s * nf + i, out, out, work);
}

/* Restriction to the grid coarsened by 2 in every direction, by injection:
 * coarse point (x, y, z) takes the fine value at (2x, 2y, 2z).  Coarsening
 * the spatial mesh of G is the option the paper names for a cheaper coarse
 * propagator (Section 2.2.2, the discussion of the speedup bound); the paper
 * fixes no transfer operators, injection is the simplest one. */
void or_restrict(const or_prob *p, const double *u, double *uc)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    for (int z = 0; z < cz; ++z)
        for (int y = 0; y < cy; ++y)
            for (int x = 0; x < cx; ++x)
                uc[((long)z * cy + y) * cx + x] = u[((long)(2 * z) * ny + 2 * y) * nx + 2 * x];
}

/* One-dimensional interpolation taps from the coarse grid (size nc) to fine
 * index i: an even index copies coarse point i/2; an odd index averages its
 * two coarse neighbours (order 1) or takes the 4-point Lagrange midpoint
 * rule -1/16, 9/16, 9/16, -1/16 (order 3).  Returns the number of taps. */
static int interp_taps(int i, int nc, int order, int *idx, double *w)
{
    if (i % 2 == 0) {
        idx[0] = i / 2;
        w[0] = 1.0;
        return 1;
    }
    const int m = (i - 1) / 2;   /* coarse neighbour on the left */
    if (order == 1) {
        idx[0] = wrap(m, nc);     w[0] = 0.5;
        idx[1] = wrap(m + 1, nc); w[1] = 0.5;
        return 2;
    }
    idx[0] = wrap(m - 1, nc); w[0] = -1.0 / 16.0;
    idx[1] = wrap(m, nc);     w[1] = 9.0 / 16.0;
    idx[2] = wrap(m + 1, nc); w[2] = 9.0 / 16.0;
    idx[3] = wrap(m + 2, nc); w[3] = -1.0 / 16.0;
    return 4;
}

/* Interpolation from the coarsened grid back to the fine grid: the tensor
 * product of the 1-D taps, summed z-tap outermost, then y, then x, each term
 * (wz*wy*wx) * value added in that order. */
void or_prolong(const or_prob *p, int order, const double *uc, double *u)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        int iz[4], iy[4], ix[4];
        double wz[4], wy[4], wx[4];
        const int tz = interp_taps(z, cz, order, iz, wz);
        for (int y = 0; y < ny; ++y) {
            const int ty = interp_taps(y, cy, order, iy, wy);
            for (int x = 0; x < nx; ++x) {
                const int tx = interp_taps(x, cx, order, ix, wx);
                double acc = 0.0;
                for (int c = 0; c < tz; ++c)
                    for (int b = 0; b < ty; ++b)
                        for (int a = 0; a < tx; ++a)
                            acc += (wz[c] * wy[b] * wx[a]) * uc[((long)iz[c] * cy + iy[b]) * cx + ix[a]];
                u[((long)z * ny + y) * nx + x] = acc;
            }
        }
    }
}

/* The problem on the coarsened grid: same physics and time grid, half the
 * points per direction. */
static or_prob coarsened(const or_prob *p)
{
    or_prob q = *p;
    q.nx = p->nx / 2;
    q.ny = p->ny / 2;
    q.nz = p->nz / 2;
    q.coarsen = 0;
    return q;
}

/* G over time slice s: Nc = nt_coarse / P Euler steps starting at global step
 * s*Nc.  With coarsening: restrict, the Nc Euler steps on the coarse grid,
 * interpolate back.  work must hold npts doubles; u and out may alias. */
void or_coarse_prop(const or_prob *p, int s, const double *u, double *out, double *work)
{
    const long n = npts_of(p);
    const int nc = p->nt_coarse / p->P;
    if (p->coarsen) {
        const or_prob q = coarsened(p);
        const long m = npts_of(&q);
        double *uc = work, *wk = work + m;
        or_restrict(p, u, uc);
        for (int i = 0; i < nc; ++i) or_euler_step(&q, (long)s * nc + i, uc, uc, wk);
        or_prolong(p, p->interp_order, uc, out);
        return;
    }
    memcpy(out, u, (size_t)n * sizeof(double));
    for (int i = 0; i < nc; ++i) or_euler_step(p, (long)s * nc + i, out, out, work);
}

/* out4 = { max|x - r|, max|r|, sum (x - r)^2, sum r^2 } in index order. */
void or_norms(long n, const double *x, const double *r, double *out4)
{
    double mx = 0.0, mr = 0.0, sx = 0.0, sr = 0.0;
    for (long i = 0; i < n; ++i) {
        const double d = x[i] - r[i];
        const double ad = fabs(d), ar = fabs(r[i]);
        if (ad > mx) mx = ad;
        if (ar > mr) mr = ar;
        sx += d * d;
        sr += r[i] * r[i];
    }
    out4[0] = mx; out4[1] = mr; out4[2] = sx; out4[3] = sr;
}

/* Serial fine solution u_fine = F_{P-1}(...F_0(u0)) (eq. fine evaluated slice
 * after slice).  If traj is not NULL it receives the state at every slice
 * boundary t_0..t_P, (P+1)*npts doubles. */
int or_serial_fine(const or_prob *p, const double *u0, double *out, double *traj)
{
    const long n = npts_of(p);
    double *work = (double *)malloc((size_t)5 * n * sizeof(double));
    if (!work) return -1;
    memcpy(out, u0, (size_t)n * sizeof(double));
    if (traj) memcpy(traj, u0, (size_t)n * sizeof(double));
    for (int s = 0; s < p->P; ++s) {
        or_fine_prop(p, s, out, out, work);
        if (traj) memcpy(traj + (size_t)(s + 1) * n, out, (size_t)n * sizeof(double));
    }
    free(work);
    return 0;
}

/* Serial coarse solution over all P slices (the start-up guess). */
int or_serial_coarse(const or_prob *p, const double *u0, double *out, double *traj)
{
    const long n = npts_of(p);
    double *work = (double *)malloc((size_t)n * sizeof(double));
    if (!work) return -1;
    memcpy(out, u0, (size_t)n * sizeof(double));
    if (traj) memcpy(traj, u0, (size_t)n * sizeof(double));
    for (int s = 0; s < p->P; ++s) {
        or_coarse_prop(p, s, out, out, work);
        if (traj) memcpy(traj + (size_t)(s + 1) * n, out, (size_t)n * sizeof(double));
    }
    free(work);
    return 0;
}

/*
 * Parareal (eq. parareal, Algorithm 1 run for all slices in turn):
 *   U^0_0 = u0;  U^0_{s+1} = G_s(U^0_s)                      (start-up coarse run)
 *   for k = 0..K-1:
 *     Fh_s = F_s(U^k_s) for every slice s                    (parallel in the paper)
 *     U^{k+1}_0 = u0
 *     for s = 0..P-1:  Gn = G_s(U^{k+1}_s)
 *                      U^{k+1}_{s+1} = Fh_s + (Gn - Gold_s);  Gold_s = Gn
 * U receives U^K_0..U^K_P ((P+1)*npts).  If hist is not NULL it receives every
 * iterate U^k_s, k = 0..K, as (K+1)*(P+1)*npts doubles.  If log is not NULL,
 * row k (8 doubles) holds the change between consecutive iterates (the
 * production monitor of Section 2.2.3): entries 0..3 are
 * {max|U^{k+1}_P - U^k_P|, max|U^{k+1}_P|, sum (U^{k+1}_P - U^k_P)^2,
 * sum (U^{k+1}_P)^2}; entries 4..7 the same quantities over all slices
 * s = 1..P (maxima of maxima, sums of sums).
 */
int or_parareal(const or_prob *p, int K, const double *u0, double *U, double *hist, double *log)
{
    const long n = npts_of(p);
    const int P = p->P;
    double *work = (double *)malloc((size_t)5 * n * sizeof(double));
    double *Fh = (double *)malloc((size_t)P * n * sizeof(double));
    double *Gold = (double *)malloc((size_t)P * n * sizeof(double));
    double *Gn = (double *)malloc((size_t)n * sizeof(double));
    double *prev = (double *)malloc((size_t)n * sizeof(double));
    if (!work || !Fh || !Gold || !Gn || !prev) {
        free(work); free(Fh); free(Gold); free(Gn); free(prev);
        return -1;
    }

    memcpy(U, u0, (size_t)n * sizeof(double));
    for (int s = 0; s < P; ++s) {
        or_coarse_prop(p, s, U + (size_t)s * n, U + (size_t)(s + 1) * n, work);
        memcpy(Gold + (size_t)s * n, U + (size_t)(s + 1) * n, (size_t)n * sizeof(double));
    }
    if (hist) memcpy(hist, U, (size_t)(P + 1) * n * sizeof(double));

    for (int k = 0; k < K; ++k) {
        for (int s = 0; s < P; ++s)
            or_fine_prop(p, s, U + (size_t)s * n, Fh + (size_t)s * n, work);
        double agg[4] = {0.0, 0.0, 0.0, 0.0};
        /* U^{k+1}_0 = u0 is already in place */
        for (int s = 0; s < P; ++s) {
            double *Unext = U + (size_t)(s + 1) * n;
            const double *fh = Fh + (size_t)s * n;
            double *go = Gold + (size_t)s * n;
            or_coarse_prop(p, s, U + (size_t)s * n, Gn, work);
            memcpy(prev, Unext, (size_t)n * sizeof(double));
            for (long i = 0; i < n; ++i) {
                Unext[i] = fh[i] + (Gn[i] - go[i]);
                go[i] = Gn[i];
            }
            double nr[4];
            or_norms(n, prev, Unext, nr); /* max|U^k - U^{k+1}|, max|U^{k+1}|, ... */
            if (nr[0] > agg[0]) agg[0] = nr[0];
            if (nr[1] > agg[1]) agg[1] = nr[1];
            agg[2] += nr[2];
            agg[3] += nr[3];
            if (log && s == P - 1) {
                log[(size_t)k * 8 + 0] = nr[0];
                log[(size_t)k * 8 + 1] = nr[1];
                log[(size_t)k * 8 + 2] = nr[2];
                log[(size_t)k * 8 + 3] = nr[3];
            }
        }
        if (log) {
            log[(size_t)k * 8 + 4] = agg[0];
            log[(size_t)k * 8 + 5] = agg[1];
            log[(size_t)k * 8 + 6] = agg[2];
            log[(size_t)k * 8 + 7] = agg[3];
        }
        if (hist) memcpy(hist + (size_t)(k + 1) * (P + 1) * n, U, (size_t)(P + 1) * n * sizeof(double));
    }
    free(work); free(Fh); free(Gold); free(Gn); free(prev);
    return 0;
}

/* Convenience wrappers used by the tests: a single RK4 / Euler step. */
int or_rk4_step_alloc(const or_prob *p, long j, const double *u, double *out)
{
    double *work = (double *)malloc((size_t)5 * npts_of(p) * sizeof(double));
    if (!work) return -1;
    or_rk4_step(p, j, u, out, work);
    free(work);
    return 0;
}

int or_euler_step_alloc(const or_prob *p, long j, const double *u, double *out)
{
    double *work = (double *)malloc((size_t)npts_of(p) * sizeof(double));
    if (!work) return -1;
    or_euler_step(p, j, u, out, work);
    free(work);
    return 0;
}

/* Fine sweep of `nsteps` RK4 steps starting at global step j0 (used for
 * sampled parity checks of single steps and short sweeps). */
int or_fine_steps(const or_prob *p, long j0, int nsteps, const double *u, double *out)
{
    const long n = npts_of(p);
    double *work = (double *)malloc((size_t)5 * n * sizeof(double));
    if (!work) return -1;
    memcpy(out, u, (size_t)n * sizeof(double));
    for (int i = 0; i < nsteps; ++i) or_rk4_step(p, j0 + i, out, out, work);
    free(work);
    return 0;
}

int or_coarse_steps(const or_prob *p, long j0, int nsteps, const double *u, double *out)
{
    const long n = npts_of(p);
    double *work = (double *)malloc((size_t)n * sizeof(double));
    if (!work) return -1;
    memcpy(out, u, (size_t)n * sizeof(double));
    for (int i = 0; i < nsteps; ++i) or_euler_step(p, j0 + i, out, out, work);
    free(work);
    return 0;
}
