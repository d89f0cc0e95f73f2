"""Pins of the oracle's spatially coarsened coarse propagator: G on the grid
coarsened by 2 per direction (restriction by injection, the Euler/upwind
steps of Algorithm 2 with h = 2/n, interpolation of order 1 or 3 back to the
fine grid) -- the cheaper-G option of the speedup discussion (Section 2.2.2).
CPU only."""
import math

import numpy as np
import pytest

import workloads as W


def sin_mode(n, kappa, shift=(0.0, 0.0, 0.0)):
    """prod_d sin(2 pi kappa_d x_d + shift_d) sampled on the vertex grid n."""
    nx, ny, nz = n
    xs = [np.arange(nx) / nx, np.arange(ny) / ny, np.arange(nz) / nz]
    s = [np.sin(2 * np.pi * kappa[d] * xs[d] + shift[d]) for d in range(3)]
    return s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]


def test_restriction_samples_the_coarse_grid(orc):
    """Injection of samples of a smooth function gives its samples on the
    coarsened grid, x_c = i * 2h (any wavenumber, any phase)."""
    n = (12, 10, 14)
    p = W.small_problem(n=n)
    for kap, sh in (((1, 2, 3), (0.3, -0.7, 1.1)), ((5, 4, 6), (0.0, 0.5, 0.25))):
        got = orc.restrict(p, sin_mode(n, kap, sh))
        ref = sin_mode((n[0] // 2, n[1] // 2, n[2] // 2), kap, sh)
        assert np.max(np.abs(got - ref)) <= 1e-14


@pytest.mark.parametrize("order", [1, 3])
def test_interpolation_of_a_mode_closed_form(orc, order):
    """A mode sin(2 pi kappa x) sampled on the coarse grid is interpolated to
    its own fine samples times, per direction with an odd index, cos(theta)
    (linear: the mean of sin at x -/+ h) or (9 cos(theta) - cos(3 theta))/8
    (cubic: -1/16, 9/16, 9/16, -1/16 at x -3h, -h, +h, +3h), theta = 2 pi kappa h."""
    n = (16, 12, 20)
    p = W.small_problem(n=n)
    kap = (3, 2, 4)
    coarse = sin_mode((8, 6, 10), kap)
    got = orc.prolong(p, coarse, order)
    fine = sin_mode(n, kap)
    fac = []
    for d in range(3):
        th = 2 * np.pi * kap[d] / n[d]
        odd = math.cos(th) if order == 1 else (9 * math.cos(th) - math.cos(3 * th)) / 8
        fac.append(np.where(np.arange(n[d]) % 2 == 1, odd, 1.0))
    ref = fine * fac[2][:, None, None] * fac[1][None, :, None] * fac[0][None, None, :]
    assert np.max(np.abs(got - ref)) <= 1e-14


@pytest.mark.parametrize("order", [1, 3])
def test_interpolation_keeps_coarse_points_and_constants(orc, order):
    """Restriction after interpolation is the identity (bitwise), and a
    constant field stays constant (the taps sum to one)."""
    n = (10, 8, 6)
    p = W.small_problem(n=n)
    uc = np.random.default_rng(3).standard_normal((3, 4, 5))
    assert np.array_equal(orc.restrict(p, orc.prolong(p, uc, order)), uc)
    c = orc.prolong(p, np.full((3, 4, 5), 2.5), order)
    assert np.max(np.abs(c - 2.5)) <= 1e-15


@pytest.mark.parametrize("order", [1, 3])
def test_coarsened_parareal_matches_alias_group_model(orc, order):
    """The grid oracle with coarsened G against the independent modal model in
    which F is diagonal and the coarsened G is the rank-one map of each
    8-member alias group: every iterate at every slice boundary."""
    from oracle import spectral as S
    p = W.small_problem(n=(16, 12, 20), a=(0.8, -0.5, 0.3), nu0=0.004, P=4, nf=8, nc=4, K=3,
                        flags=W.COARSEN_G | (W.CUBIC_INTERP if order == 3 else 0))
    modes = W.draw_modes(np.random.default_rng(5), 5, 3)
    u0 = W.synth_u0(p.n, modes)
    _, _, hist = orc.parareal(p, u0, K=p.K, history=True)
    ms = S.CoarsenedModalSolution(p, modes, order=order)
    for k in range(p.K + 1):
        for s in range(p.P + 1):
            ref = ms.iterate(k, s)
            assert orc.rel_l2(hist[k, s], ref) <= 1e-12, (k, s)


def test_coarsened_k_equals_p_is_exact_and_k0_is_coarse_run(orc):
    """K = P reproduces the serial fine solution bitwise whatever G is, and
    K = 0 returns the coarsened coarse run."""
    p = W.small_problem(n=(12, 10, 8), P=3, nf=6, nc=3, K=3, flags=W.COARSEN_G)
    u0 = W.random_field(p.n, 21)
    U, _ = orc.parareal(p, u0, K=p.P)
    assert np.array_equal(U[-1], orc.serial_fine(p, u0))
    U0, _ = orc.parareal(p, u0, K=0)
    assert np.array_equal(U0[-1], orc.serial_coarse(p, u0))
