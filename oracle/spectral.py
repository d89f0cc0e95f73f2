"""Per-Fourier-mode reference for the Parareal advection-diffusion scheme.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

On a periodic grid every constant-coefficient stencil is diagonalised by the
grid exponentials e_q(x) = exp(2 pi i q.x), q integer.  The discrete scheme
therefore reduces, mode by mode, to scalar complex recurrences:

  * operator symbol mu(t) = nu(t) * sD(q) + sA(q)   (Lap and -a.grad stencils)
  * one RK4 step from t:  R_F = 1 + dt/6 (k1 + 2 k2 + 2 k3 + k4) with
    k1 = mu(t), k2 = mu(t+dt/2)(1 + dt/2 k1), k3 = mu(t+dt/2)(1 + dt/2 k2),
    k4 = mu(t+dt)(1 + dt k3)                               (classical RK4)
  * one Euler step from t: R_G = 1 + Dt mu_G(t)            (Algorithm 2)
  * slice propagators f_s, g_s: products of the step factors over slice s
  * Parareal (eq. parareal) per mode:
        Z^{k+1}_{s+1} = g_s Z^{k+1}_s + f_s Z^k_s - g_s Z^k_s

The grid field is the synthesis sum_q c_q Z_q e_q(x); with G on a coarsened
grid the recurrences couple the 8 aliases of a coarse mode (see below).  This
path shares no
code with oracle.c; agreement of the two pins both.  It also provides the
continuous solution of the PDE (Section 3: u = a(t) u0(x - c t) with
a(t) = exp(-4 pi^2 |kappa|^2 int_0^t nu)) for the discretisation-error checks.
"""
from __future__ import annotations

import math

import numpy as np


def _theta(q, n):
    q = np.asarray(q, dtype=np.float64)
    nn = np.asarray(n, dtype=np.float64)
    return 2.0 * np.pi * q / nn[None, :]


def fine_symbols(q, n, a, order=2):
    """(sD, sA) with mu = nu * sD + sA for the centered fine stencils."""
    th = _theta(q, n)
    nn = np.asarray(n, dtype=np.float64)[None, :]
    aa = np.asarray(a, dtype=np.float64)[None, :]
    if order == 2:
        sD = ((2.0 * np.cos(th) - 2.0) * nn * nn).sum(axis=1)
        sA = -1j * (aa * np.sin(th) * nn).sum(axis=1)
    elif order == 4:
        sD = (((-2.0 * np.cos(2 * th) + 32.0 * np.cos(th) - 30.0) / 12.0) * nn * nn).sum(axis=1)
        sA = -1j * (aa * (8.0 * np.sin(th) - np.sin(2 * th)) / 6.0 * nn).sum(axis=1)
    else:
        raise ValueError(order)
    return sD.astype(np.complex128), sA.astype(np.complex128)


def coarse_symbols(q, n, a):
    """(sD, sA) for Algorithm 2: 7-point diffusion, upwind advection."""
    th = _theta(q, n)
    nn = np.asarray(n, dtype=np.float64)[None, :]
    sD = ((2.0 * np.cos(th) - 2.0) * nn * nn).sum(axis=1).astype(np.complex128)
    sA = np.zeros(th.shape[0], dtype=np.complex128)
    for d in range(3):
        ad = float(a[d])
        if ad > 0.0:
            sA += -ad * (1.0 - np.exp(-1j * th[:, d])) * nn[0, d]
        else:
            sA += -ad * (np.exp(1j * th[:, d]) - 1.0) * nn[0, d]
    return sD, sA


def nu_of(p, t):
    return p.nu0 * (1.0 + p.nu_amp * np.sin(p.nu_omega * t))


def nu_integral(p, t):
    """int_0^t nu(s) ds for nu = nu0 (1 + amp sin(omega s))."""
    if p.nu_omega == 0.0:
        return p.nu0 * (1.0 + p.nu_amp * 0.0) * t
    return p.nu0 * (t + p.nu_amp * (1.0 - math.cos(p.nu_omega * t)) / p.nu_omega)


def rk4_factors(p, q, j0, nsteps, frozen=None):
    """R_F for global fine steps j0..j0+nsteps-1; shape (nsteps, Q)."""
    if frozen is None:
        frozen = bool(int(getattr(p, "flags", 0)) & 1)
    sD, sA = fine_symbols(q, p.n, p.a, p.fine_order)
    dt = p.T / p.nt_fine
    out = np.empty((nsteps, sD.size), dtype=np.complex128)
    for i in range(nsteps):
        t = (j0 + i) * dt
        n1 = nu_of(p, t)
        n2 = n1 if frozen else nu_of(p, t + 0.5 * dt)
        n4 = n1 if frozen else nu_of(p, t + dt)
        m1 = n1 * sD + sA
        m2 = n2 * sD + sA
        m4 = n4 * sD + sA
        k1 = m1
        k2 = m2 * (1.0 + 0.5 * dt * k1)
        k3 = m2 * (1.0 + 0.5 * dt * k2)
        k4 = m4 * (1.0 + dt * k3)
        out[i] = 1.0 + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return out


def euler_factors(p, q, j0, nsteps):
    sD, sA = coarse_symbols(q, p.n, p.a)
    Dt = p.T / p.nt_coarse
    out = np.empty((nsteps, sD.size), dtype=np.complex128)
    for i in range(nsteps):
        out[i] = 1.0 + Dt * (nu_of(p, (j0 + i) * Dt) * sD + sA)
    return out


def _prod_rows(R):
    acc = np.ones(R.shape[1], dtype=np.complex128)
    for r in R:
        acc = acc * r
    return acc


def slice_factors(p, q):
    """(f, g): arrays (P, Q) of the fine / coarse slice propagators per mode."""
    RF = rk4_factors(p, q, 0, p.nt_fine)
    RG = euler_factors(p, q, 0, p.nt_coarse)
    f = np.stack([_prod_rows(RF[s * p.nf:(s + 1) * p.nf]) for s in range(p.P)])
    g = np.stack([_prod_rows(RG[s * p.nc:(s + 1) * p.nc]) for s in range(p.P)])
    return f, g


def parareal_modes(f, g, K):
    """Z[k, s, q] = Parareal iterate k at slice boundary s for unit initial data."""
    P, Q = f.shape
    Z = np.zeros((K + 1, P + 1, Q), dtype=np.complex128)
    Z[0, 0] = 1.0
    for s in range(P):
        Z[0, s + 1] = g[s] * Z[0, s]
    for k in range(K):
        Z[k + 1, 0] = 1.0
        for s in range(P):
            Z[k + 1, s + 1] = g[s] * Z[k + 1, s] + f[s] * Z[k, s] - g[s] * Z[k, s]
    return Z


def expand_modes(modes):
    """Write u0 = sum_m A_m prod_d sin(2 pi kappa_d x_d) as sum_q c_q e_q(x).

    sin(t) = (e^{it} - e^{-it}) / (2i), so each product of three sines is a
    sum over the 8 sign vectors s of (prod s_d) / (2i)^3 e_{s*kappa}."""
    qs, cs = [], []
    for kap, A in zip(modes.kappa, modes.amp):
        for sx in (1, -1):
            for sy in (1, -1):
                for sz in (1, -1):
                    qs.append((sx * kap[0], sy * kap[1], sz * kap[2]))
                    cs.append(A * sx * sy * sz / (2j) ** 3)
    return np.asarray(qs, dtype=np.int64), np.asarray(cs, dtype=np.complex128)


def synth(n, q, coef):
    """Real grid field [z, y, x] of sum_q coef_q e_q(x)."""
    nx, ny, nz = (int(v) for v in n)
    out = np.zeros((nz, ny, nx), dtype=np.complex128)
    ix = np.arange(nx) / nx
    iy = np.arange(ny) / ny
    iz = np.arange(nz) / nz
    for (qx, qy, qz), c in zip(q, coef):
        ex = np.exp(2j * np.pi * qx * ix)
        ey = np.exp(2j * np.pi * qy * iy)
        ez = np.exp(2j * np.pi * qz * iz)
        out += c * (ez[:, None, None] * ey[None, :, None] * ex[None, None, :])
    return out.real.copy()


def synth_fft(n, q, coef):
    """The field of synth(n, q, coef), evaluated with one inverse FFT: the
    coefficients are summed into the DFT bins (q mod n) of the grid, which is
    the same trigonometric sum sampled at x_i = i/n (exact up to rounding)."""
    nx, ny, nz = (int(v) for v in n)
    spec = np.zeros((nz, ny, nx), dtype=np.complex128)
    q = np.asarray(q, dtype=np.int64)
    np.add.at(spec, (q[:, 2] % nz, q[:, 1] % ny, q[:, 0] % nx), np.asarray(coef, dtype=np.complex128))
    return (np.fft.ifftn(spec) * (nx * ny * nz)).real.copy()


def synth_points(n, q, coef, flat_idx):
    """Values of sum_q coef_q e_q at the flat grid indices (z*ny + y)*nx + x."""
    nx, ny, nz = (int(v) for v in n)
    flat_idx = np.asarray(flat_idx, dtype=np.int64)
    x = (flat_idx % nx) / nx
    y = ((flat_idx // nx) % ny) / ny
    z = (flat_idx // (nx * ny)) / nz
    qf = np.asarray(q, dtype=np.float64)
    ph = 2.0 * np.pi * (np.outer(x, qf[:, 0]) + np.outer(y, qf[:, 1]) + np.outer(z, qf[:, 2]))
    return (np.exp(1j * ph) @ np.asarray(coef)).real


class ModalSolution:
    """All Parareal iterates of one problem in modal form."""

    def __init__(self, p, modes, K=None):
        self.p = p
        self.K = p.K if K is None else int(K)
        self.q, self.c = expand_modes(modes)
        self.f, self.g = slice_factors(p, self.q)
        self.Z = parareal_modes(self.f, self.g, self.K)
        # serial fine (and coarse) trajectories at slice boundaries
        P = p.P
        self.fine = np.ones((P + 1, self.q.shape[0]), dtype=np.complex128)
        self.coarse = np.ones((P + 1, self.q.shape[0]), dtype=np.complex128)
        for s in range(P):
            self.fine[s + 1] = self.fine[s] * self.f[s]
            self.coarse[s + 1] = self.coarse[s] * self.g[s]

    def iterate(self, k, s):
        return synth(self.p.n, self.q, self.c * self.Z[k, s])

    def iterate_points(self, k, s, idx):
        return synth_points(self.p.n, self.q, self.c * self.Z[k, s], idx)

    def iterate_fft(self, k, s):
        return synth_fft(self.p.n, self.q, self.c * self.Z[k, s])

    def serial_fine(self, s=None):
        s = self.p.P if s is None else s
        return synth(self.p.n, self.q, self.c * self.fine[s])

    def serial_fine_points(self, idx, s=None):
        s = self.p.P if s is None else s
        return synth_points(self.p.n, self.q, self.c * self.fine[s], idx)

    def serial_fine_fft(self, s=None):
        s = self.p.P if s is None else s
        return synth_fft(self.p.n, self.q, self.c * self.fine[s])

    def serial_coarse(self, s=None):
        s = self.p.P if s is None else s
        return synth(self.p.n, self.q, self.c * self.coarse[s])


# ---------------------------------------------------------------------------
# G on the grid coarsened by 2 per direction (restriction by injection,
# Euler/upwind steps with h = 2/n, interpolation of order 1 or 3).
#
# Injection maps every fine exponential q to the coarse exponential q mod n/2,
# so the 8 aliases q + (n/2) s, s in {0,1}^3, land on the same coarse mode.
# Interpolating a coarse exponential b puts, per direction, the weight
# (1 + c(theta))/2 on the fine exponentials b and b + n/2, with theta = 2 pi m/n
# of that member and c = cos(theta) (linear midpoint average) or
# (9 cos(theta) - cos(3 theta))/8 (4-point cubic midpoint rule).  Each alias
# group is therefore invariant: F acts diagonally, the coarsened G as the
# rank-one map x -> g alpha (sum of x), and Parareal runs on 8-vectors.
# ---------------------------------------------------------------------------

def interp_odd_factor(theta, order):
    """Value of an interpolated exponential at an odd fine index, relative to
    the exponential itself (one direction)."""
    theta = np.asarray(theta, dtype=np.float64)
    if order == 1:
        return np.cos(theta)
    if order == 3:
        return (9.0 * np.cos(theta) - np.cos(3.0 * theta)) / 8.0
    raise ValueError(order)


def alias_groups(q, coef, n):
    """Group fine exponentials by their coarse image.  Returns (members
    [G, 8, 3] wavenumbers in [0, n), bases [G, 3], coefficients [G, 8])."""
    nn = np.asarray([int(v) for v in n], dtype=np.int64)
    half = nn // 2
    qm = np.mod(np.asarray(q, dtype=np.int64), nn[None, :])
    base = np.mod(qm, half[None, :])
    sel = qm // half[None, :]
    slot = sel[:, 0] + 2 * sel[:, 1] + 4 * sel[:, 2]
    keys = {}
    for b in map(tuple, base):
        keys.setdefault(b, len(keys))
    G = len(keys)
    bases = np.zeros((G, 3), dtype=np.int64)
    for b, gi in keys.items():
        bases[gi] = b
    svec = np.array([[m & 1, (m >> 1) & 1, (m >> 2) & 1] for m in range(8)], dtype=np.int64)
    members = bases[:, None, :] + svec[None, :, :] * half[None, None, :]
    C = np.zeros((G, 8), dtype=np.complex128)
    for qi in range(qm.shape[0]):
        C[keys[tuple(base[qi])], slot[qi]] += coef[qi]
    return members, bases, C


def coarsened_slice_factors(p, members, bases, order):
    """(f [P, G, 8], g [P, G], alpha [G, 8]) for the coarsened G."""
    P = p.P
    Gn = members.shape[0]
    RF = rk4_factors(p, members.reshape(-1, 3), 0, p.nt_fine)
    f = np.stack([_prod_rows(RF[s * p.nf:(s + 1) * p.nf]) for s in range(P)]).reshape(P, Gn, 8)
    half = [int(v) // 2 for v in p.n]
    sD, sA = coarse_symbols(bases, half, p.a)
    Dt = p.T / p.nt_coarse
    g = np.ones((P, Gn), dtype=np.complex128)
    for s in range(P):
        for i in range(p.nc):
            j = s * p.nc + i
            g[s] = g[s] * (1.0 + Dt * (nu_of(p, j * Dt) * sD + sA))
    nn = np.asarray([int(v) for v in p.n], dtype=np.float64)
    theta = 2.0 * np.pi * members / nn[None, None, :]
    alpha = np.prod(0.5 * (1.0 + interp_odd_factor(theta, order)), axis=2)
    return f, g, alpha


class CoarsenedModalSolution:
    """All Parareal iterates with the spatially coarsened G, in modal form."""

    def __init__(self, p, modes, order=1, K=None):
        self.p = p
        self.K = p.K if K is None else int(K)
        q, c = expand_modes(modes)
        self.members, self.bases, C = alias_groups(q, c, p.n)
        f, g, alpha = coarsened_slice_factors(p, self.members, self.bases, order)
        P, K = p.P, self.K

        def G(s, x):
            return g[s][:, None] * alpha * x.sum(axis=1)[:, None]

        Z = np.zeros((K + 1, P + 1) + C.shape, dtype=np.complex128)
        Z[0, 0] = C
        for s in range(P):
            Z[0, s + 1] = G(s, Z[0, s])
        for k in range(K):
            Z[k + 1, 0] = C
            for s in range(P):
                Z[k + 1, s + 1] = G(s, Z[k + 1, s]) + f[s] * Z[k, s] - G(s, Z[k, s])
        self.Z = Z
        self.fine = np.zeros((P + 1,) + C.shape, dtype=np.complex128)
        self.fine[0] = C
        for s in range(P):
            self.fine[s + 1] = f[s] * self.fine[s]
        self.q = self.members.reshape(-1, 3)

    def iterate(self, k, s):
        return synth(self.p.n, self.q, self.Z[k, s].reshape(-1))

    def iterate_points(self, k, s, idx):
        return synth_points(self.p.n, self.q, self.Z[k, s].reshape(-1), idx)

    def serial_fine_points(self, idx, s=None):
        s = self.p.P if s is None else s
        return synth_points(self.p.n, self.q, self.fine[s].reshape(-1), idx)


def analytic(p, modes, t):
    """Continuous solution sum_m A_m exp(-4 pi^2 |kappa_m|^2 int nu) prod_d
    sin(2 pi kappa_d (x_d - a_d t)) on the grid (Section 3, eq. sol_form)."""
    nx, ny, nz = (int(v) for v in p.n)
    xs = [np.arange(nx) / nx, np.arange(ny) / ny, np.arange(nz) / nz]
    I = nu_integral(p, t)
    u = np.zeros((nz, ny, nx))
    for kap, A in zip(modes.kappa, modes.amp):
        k2 = float(kap[0] ** 2 + kap[1] ** 2 + kap[2] ** 2)
        dec = math.exp(-4.0 * math.pi ** 2 * k2 * I)
        s = [np.sin(2 * np.pi * kap[d] * (xs[d] - p.a[d] * t)) for d in range(3)]
        u += A * dec * (s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :])
    return u


def analytic_points(p, modes, t, flat_idx):
    nx, ny, nz = (int(v) for v in p.n)
    flat_idx = np.asarray(flat_idx, dtype=np.int64)
    xyz = [(flat_idx % nx) / nx, ((flat_idx // nx) % ny) / ny, (flat_idx // (nx * ny)) / nz]
    I = nu_integral(p, t)
    u = np.zeros(flat_idx.shape)
    for kap, A in zip(modes.kappa, modes.amp):
        k2 = float(kap[0] ** 2 + kap[1] ** 2 + kap[2] ** 2)
        dec = math.exp(-4.0 * math.pi ** 2 * k2 * I)
        term = A * dec
        for d in range(3):
            term = term * np.sin(2 * np.pi * kap[d] * (xyz[d] - p.a[d] * t))
        u += term
    return u
