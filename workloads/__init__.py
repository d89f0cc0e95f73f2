"""Seeded synthetic workloads for the Parareal advection-diffusion solver.

This module is the only code shared by the CPU oracle (``oracle/``) and the
GPU library's tests and benchmarks.  It holds *inputs only*: problem
parameters, seeded Fourier-mode initial data sampled on the grid, and the
coarse step counts chosen from the explicit-Euler stability bound.  None of
the method's arithmetic (stencils, time steppers, the Parareal iteration,
norms) lives here.

Benchmark PDE (Section 3, eq. adv_diff_eq): u_t + a.grad(u) = nu(t) Lap(u) on
the periodic unit cube, nu(t) = nu0 * (1 + amp * sin(omega * t)).  The paper's
single-mode initial value sin(2 pi x) sin(2 pi y) sin(2 pi z) is the special
case M = 1, kappa = (1, 1, 1), A = 1 of the mode sums used here.

Grid points are vertex based, x_i = i / n (periodic), and arrays are stored
x-fastest as ``u[z, y, x]``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED = 1409

# flags shared by name with the C ABI (values fixed by include/pr.h)
NU_FROZEN = 1          # evaluate nu at the start of each RK4 step for all stages
ALLOW_UNSTABLE = 2     # skip the coarse stability guard
EARLY_STOP = 4
SKIP_CONVERGED = 8     # reuse F/G results of slices that have already converged
COARSEN_G = 16         # G on the grid coarsened by 2 per direction (injection, interpolation back)
CUBIC_INTERP = 32      # with COARSEN_G: cubic instead of linear interpolation


@dataclasses.dataclass
class Problem:
    """Parameters of one Parareal problem instance (Section 2.1-2.2, Section 3)."""
    n: tuple                  # (nx, ny, nz)
    a: tuple                  # advection velocity (paper: c)
    nu0: float
    nu_amp: float = 0.5
    nu_omega: float = 0.0     # angular frequency of nu(t)
    T: float = 0.25
    P: int = 4                # time slices N_p
    nt_fine: int = 256        # total fine steps on [0, T]
    nt_coarse: int = 64       # total coarse steps on [0, T]
    K: int = 1                # Parareal iterations
    fine_order: int = 2       # 2: 7-point stencils, 4: 13-point stencils
    flags: int = 0
    tol: float = 0.0

    @property
    def npts(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def nf(self) -> int:
        return self.nt_fine // self.P

    @property
    def nc(self) -> int:
        return self.nt_coarse // self.P


@dataclasses.dataclass
class Modes:
    """u0(x) = sum_m amp[m] * prod_d sin(2 pi kappa[m, d] x_d)."""
    kappa: np.ndarray         # (M, 3) integers, column order (x, y, z)
    amp: np.ndarray           # (M,) float64


def draw_modes(rng: np.random.Generator, m: int, kmax: int) -> Modes:
    kappa = rng.integers(1, kmax + 1, size=(m, 3))
    amp = rng.standard_normal(m)
    return Modes(kappa=np.asarray(kappa, dtype=np.int64), amp=np.asarray(amp, dtype=np.float64))


def single_mode(kappa=(1, 1, 1), amp: float = 1.0) -> Modes:
    return Modes(kappa=np.asarray([kappa], dtype=np.int64), amp=np.asarray([amp], dtype=np.float64))


def synth_u0(n, modes: Modes, dtype=np.float64) -> np.ndarray:
    """Sample the mode sum on the vertex grid; returns a C-contiguous [z, y, x] array."""
    nx, ny, nz = (int(v) for v in n)
    xs = np.arange(nx, dtype=np.float64) / nx
    ys = np.arange(ny, dtype=np.float64) / ny
    zs = np.arange(nz, dtype=np.float64) / nz
    u = np.zeros((nz, ny, nx), dtype=np.float64)
    for (kx, ky, kz), amp in zip(modes.kappa, modes.amp):
        sx = np.sin(2.0 * np.pi * kx * xs)
        sy = np.sin(2.0 * np.pi * ky * ys)
        sz = np.sin(2.0 * np.pi * kz * zs)
        u += amp * (sz[:, None, None] * sy[None, :, None] * sx[None, None, :])
    return np.ascontiguousarray(u, dtype=dtype)


def coarse_bound(n, a, nu_max: float) -> float:
    """Largest |1 - R| scale of forward Euler with upwind advection and the
    7-point Laplacian: dt * (sum_d |a_d| / h_d + 2 nu_max sum_d 1/h_d^2) <= 1
    keeps every Fourier mode's amplification inside the unit disc."""
    return sum(abs(float(a[d])) * n[d] + 2.0 * nu_max * n[d] * n[d] for d in range(3))


def stable_coarse_steps(n, a, nu0, amp, T, multiple: int, margin: float = 0.9,
                        power_of_two: bool = False, minimum: int = 1) -> int:
    b = coarse_bound(n, a, nu0 * (1.0 + abs(amp)))
    need = T * b / margin
    if power_of_two:
        c = max(minimum, multiple)
        while c < need:
            c *= 2
        return c
    c = int(math.ceil(need / multiple)) * multiple
    return max(c, minimum, multiple)


# ---------------------------------------------------------------------------
# The five benchmark workloads.  Coarse counts of the 128^3, 256^3 and 512^3
# cases are raised to the smallest power of two that satisfies the stability
# bound with margin 0.9 (the counts 256 / 512 / 1024 violate it).
# ---------------------------------------------------------------------------

A_DEFAULT = (1.0, 0.5, 0.25)


def _omega(T: float) -> float:
    return 2.0 * math.pi / T


def config(name: str, K: Optional[int] = None):
    """Return ``(problem, modes)`` for a single-instance workload.

    names: 'c1_32_fp64', 'c2_128_fp64', 'c3_256_mixed', 'c5_512_mixed'.
    """
    rng = np.random.default_rng(SEED)
    T = 0.25
    if name == "c1_32_fp64":
        p = Problem(n=(32, 32, 32), a=A_DEFAULT, nu0=0.01, nu_amp=0.5, nu_omega=_omega(T), T=T,
                    P=4, nt_fine=256, nt_coarse=64, K=4)
        modes = draw_modes(rng, 8, 4)
    elif name == "c2_128_fp64":
        p = Problem(n=(128, 128, 128), a=A_DEFAULT, nu0=0.01, nu_amp=0.5, nu_omega=_omega(T), T=T,
                    P=16, nt_fine=2048, nt_coarse=512, K=6)
        modes = draw_modes(rng, 16, 8)
    elif name == "c3_256_mixed":
        p = Problem(n=(256, 256, 256), a=A_DEFAULT, nu0=0.005, nu_amp=0.5, nu_omega=_omega(T), T=T,
                    P=32, nt_fine=4096, nt_coarse=1024, K=6)
        modes = draw_modes(rng, 16, 8)
    elif name == "c5_512_mixed":
        p = Problem(n=(512, 512, 512), a=A_DEFAULT, nu0=0.005, nu_amp=0.5, nu_omega=_omega(T), T=T,
                    P=32, nt_fine=8192, nt_coarse=4096, K=5)
        modes = draw_modes(rng, 32, 16)
    else:
        raise KeyError(name)
    if K is not None:
        p.K = K
    return p, modes


# literal coarse counts of the workload descriptions (rejected by the stability guard)
LITERAL_COARSE = {"c2_128_fp64": 256, "c3_256_mixed": 512, "c5_512_mixed": 1024}

MIXED = {"c1_32_fp64": False, "c2_128_fp64": False, "c3_256_mixed": True, "c5_512_mixed": True}


def batched_config(ninst: int = 64, sizes=(48, 64, 96, 128)):
    """The batched workload: ``ninst`` independent instances of uneven cubic
    size, each with its own a and nu0.  Returns a list of (problem, modes)."""
    rng = np.random.default_rng(SEED)
    ns = rng.choice(np.asarray(sizes), size=ninst)
    a = rng.uniform(0.25, 1.0, size=(ninst, 3))
    nu0 = rng.uniform(0.002, 0.01, size=ninst)
    seeds = np.random.SeedSequence(SEED).spawn(ninst)
    T = 0.25
    out = []
    for i in range(ninst):
        n = int(ns[i])
        ai = tuple(float(v) for v in a[i])
        nui = float(nu0[i])
        ntc = stable_coarse_steps((n, n, n), ai, nui, 0.5, T, multiple=8)
        p = Problem(n=(n, n, n), a=ai, nu0=nui, nu_amp=0.5, nu_omega=_omega(T), T=T,
                    P=8, nt_fine=16 * n, nt_coarse=ntc, K=3)
        modes = draw_modes(np.random.default_rng(seeds[i]), 8, 4)
        out.append((p, modes))
    return out


def paper_setup(omega: float, P: int = 8, K: int = 3, n: int = 128) -> Problem:
    """The paper's benchmark (Section 3.1): 128^3, c = (1,1,1), nu0 = 0.1,
    amplitude nu0/2, T = 0.1, fine dt = T/2^15 with the fourth-order stencils,
    coarse dt = T/2^11."""
    return Problem(n=(n, n, n), a=(1.0, 1.0, 1.0), nu0=0.1, nu_amp=0.5, nu_omega=float(omega),
                   T=0.1, P=P, nt_fine=2 ** 15, nt_coarse=2 ** 11, K=K, fine_order=4)


def small_problem(n=(8, 8, 8), a=A_DEFAULT, nu0=0.02, P=4, nf=6, nc=3, K=2, order=2,
                  omega=None, T=0.1, flags=0) -> Problem:
    """A small problem for tests; step counts are given per slice."""
    om = _omega(T) if omega is None else omega
    return Problem(n=tuple(n), a=tuple(a), nu0=nu0, nu_amp=0.5, nu_omega=om, T=T, P=P,
                   nt_fine=P * nf, nt_coarse=P * nc, K=K, fine_order=order, flags=flags)


def random_field(n, seed: int, dtype=np.float64) -> np.ndarray:
    """A seeded N(0,1) field of shape [nz, ny, nx] (tests of linearity and
    translation equivariance use fields with all Fourier content)."""
    nx, ny, nz = (int(v) for v in n)
    return np.random.default_rng(seed).standard_normal((nz, ny, nx)).astype(dtype)
