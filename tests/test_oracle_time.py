"""Pins of the oracle's time steppers: the textbook closed form of classical
RK4 for autonomous linear systems, its fourth-order convergence with a
time-dependent coefficient against the exact solution of the semi-discrete
mode equation, forward Euler against its definition, and the global step
index of slices.  CPU only."""
import math

import numpy as np
import pytest

import workloads as W
from test_oracle_operators import dense_coarse, dense_fine


@pytest.mark.parametrize("order", [2, 4])
def test_rk4_constant_nu_is_taylor_polynomial(orc, order):
    """For u' = L u with constant L, one classical RK4 step is
    sum_{m<=4} (dt L)^m / m!."""
    n3 = (5, 5, 6) if order == 4 else (4, 5, 3)
    a = (0.7, -0.2, 0.45)
    p = W.Problem(n=n3, a=a, nu0=0.03, nu_amp=0.0, nu_omega=0.0, T=0.02, P=1,
                  nt_fine=5, nt_coarse=1, K=0, fine_order=order)
    dt = p.T / p.nt_fine
    M = dt * dense_fine(n3, a, p.nu0, order)
    R = np.eye(M.shape[0])
    term = np.eye(M.shape[0])
    for m in range(1, 5):
        term = term @ M / m
        R = R + term
    u = W.random_field(n3, 21)
    ref = (R @ u.ravel()).reshape(u.shape)
    got = orc.rk4_step(p, 2, u)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def _mode_exact(p, q, Lfun):
    """Exact solution at T of u' = L(nu(t)) u for u0 = Re e_q, using the
    eigenvalue of the dense operator: lambda(nu) = nu sD + sA."""
    n3 = p.n
    x = np.arange(n3[0]) / n3[0]
    y = np.arange(n3[1]) / n3[1]
    z = np.arange(n3[2]) / n3[2]
    e = (np.exp(2j * np.pi * q[2] * z)[:, None, None] * np.exp(2j * np.pi * q[1] * y)[None, :, None]
         * np.exp(2j * np.pi * q[0] * x)[None, None, :])
    L0 = Lfun(0.0)
    L1 = Lfun(1.0)
    ef = e.ravel()
    sA = (L0 @ ef)[0] / ef[0]
    sD = (L1 @ ef)[0] / ef[0] - sA
    if p.nu_omega == 0.0:
        I = p.nu0 * p.T
    else:
        I = p.nu0 * (p.T + p.nu_amp * (1 - math.cos(p.nu_omega * p.T)) / p.nu_omega)
    return e.real.copy(), (np.exp(sD * I + sA * p.T) * e).real


@pytest.mark.parametrize("order", [2, 4])
def test_rk4_time_dependent_nu_is_fourth_order(orc, order):
    n3 = (4, 5, 6) if order == 2 else (5, 6, 7)
    a = (0.5, 0.25, -0.35)
    q = (1, -1, 2)
    errs = []
    for nt in (8, 16, 32, 64):
        # 2.3 periods of nu on [0, T]: over whole periods the leading error
        # term integrates to zero and the observed order would be five
        p = W.Problem(n=n3, a=a, nu0=0.004, nu_amp=0.5, nu_omega=2 * math.pi * 2.3 / 0.5, T=0.5,
                      P=1, nt_fine=nt, nt_coarse=1, K=0, fine_order=order)
        u0, exact = _mode_exact(p, q, lambda nu: dense_fine(n3, a, nu, order))
        got = orc.fine_steps(p, 0, nt, u0)
        errs.append(np.max(np.abs(got - exact)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(13.0 < r < 19.0 for r in ratios[1:]), (errs, ratios)


def test_rk4_frozen_nu_is_first_order_in_nu_variation(orc):
    """With nu frozen at the step start the scheme is only first-order
    accurate for time-dependent nu (the option used to reproduce the paper's
    fine-solution errors)."""
    n3 = (4, 5, 6)
    a = (0.5, 0.25, -0.35)
    q = (1, -1, 2)
    errs = []
    for nt in (32, 64, 128):
        p = W.Problem(n=n3, a=a, nu0=0.004, nu_amp=0.5, nu_omega=2 * math.pi * 2.3 / 0.5, T=0.5,
                      P=1, nt_fine=nt, nt_coarse=1, K=0, flags=W.NU_FROZEN)
        u0, exact = _mode_exact(p, q, lambda nu: dense_fine(n3, a, nu, 2))
        got = orc.fine_steps(p, 0, nt, u0)
        errs.append(np.max(np.abs(got - exact)))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(1.7 < r < 2.3 for r in ratios), (errs, ratios)


def test_euler_step_definition_and_time_index(orc):
    n3 = (4, 5, 3)
    a = (-0.3, 0.6, 0.2)
    # 10 coarse steps per period of nu: nu(j Dt) differs from nu((j +- 1) Dt)
    p = W.small_problem(n=n3, a=a, nu0=0.02, P=2, nc=5)
    Dt = p.T / p.nt_coarse
    j = 4
    assert len({round(math.sin(p.nu_omega * i * Dt), 12) for i in (j - 1, j, j + 1)}) == 3
    nu = p.nu0 * (1 + p.nu_amp * math.sin(p.nu_omega * j * Dt))
    M = np.eye(np.prod(n3)) + Dt * dense_coarse(n3, a, nu)
    u = W.random_field(n3, 22)
    ref = (M @ u.ravel()).reshape(u.shape)
    got = orc.euler_step(p, j, u)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_euler_convergence_first_order(orc):
    """Forward Euler on a single mode converges at first order in Dt against
    the exact semi-discrete solution."""
    n3 = (4, 5, 6)
    a = (0.5, -0.25, 0.35)
    q = (1, 2, -1)
    errs = []
    for nt in (64, 128, 256):
        p = W.Problem(n=n3, a=a, nu0=0.004, nu_amp=0.5, nu_omega=2 * math.pi / 0.5, T=0.5,
                      P=1, nt_fine=1, nt_coarse=nt, K=0)
        u0, exact = _mode_exact(p, q, lambda nu: dense_coarse(n3, a, nu))
        got = orc.coarse_steps(p, 0, nt, u0)
        errs.append(np.max(np.abs(got - exact)))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(1.8 < r < 2.2 for r in ratios), (errs, ratios)


def test_slices_use_global_step_index(orc):
    """Marching slice by slice equals one uninterrupted run over all fine
    (and coarse) steps, bitwise: slice s starts at global step s * N_f."""
    p = W.small_problem(n=(5, 6, 4), P=3, nf=4, nc=2)
    u0 = W.random_field(p.n, 23)
    assert np.array_equal(orc.serial_fine(p, u0), orc.fine_steps(p, 0, p.nt_fine, u0))
    assert np.array_equal(orc.serial_coarse(p, u0), orc.coarse_steps(p, 0, p.nt_coarse, u0))


def test_norms_definition(orc):
    x = W.random_field((5, 4, 3), 24)
    r = W.random_field((5, 4, 3), 25)
    n = orc.norms(x, r)
    assert n[0] == np.max(np.abs(x - r))
    assert n[1] == np.max(np.abs(r))
    assert abs(n[2] - np.sum((x - r) ** 2)) <= 1e-13 * n[2]
    assert abs(n[3] - np.sum(r ** 2)) <= 1e-13 * n[3]
