"""Pins of the oracle's Parareal iteration: exactness invariants, the
closed-form iterate for constant coefficients, agreement with the independent
per-mode reference, and the spatial order of the fine propagator against the
continuous solution.  CPU only."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import spectral as S


def test_k_equals_p_is_serial_fine_bitwise(orc):
    p = W.small_problem(n=(6, 5, 7), P=4, nf=3, nc=2, K=4)
    u0 = W.random_field(p.n, 31)
    U, _ = orc.parareal(p, u0, K=p.P)
    assert np.array_equal(U[-1], orc.serial_fine(p, u0))


def test_converged_prefix_and_coarse_start_bitwise(orc):
    """After iteration k the slices s <= k hold the serial fine solution
    exactly; iterate 0 is the start-up coarse run."""
    p = W.small_problem(n=(5, 6, 4), P=5, nf=3, nc=2)
    u0 = W.random_field(p.n, 32)
    _, _, hist = orc.parareal(p, u0, K=3, history=True)
    _, ftraj = orc.serial_fine(p, u0, trajectory=True)
    _, gtraj = orc.serial_coarse(p, u0, trajectory=True)
    assert np.array_equal(hist[0], gtraj)
    for k in range(4):
        for s in range(k + 1):
            assert np.array_equal(hist[k, s], ftraj[s]), (k, s)
        if k < 3:
            assert not np.array_equal(hist[k, k + 1], ftraj[k + 1])


def test_log_is_inter_iterate_change(orc):
    p = W.small_problem(n=(5, 4, 6), P=3, nf=2, nc=1)
    u0 = W.random_field(p.n, 33)
    _, log, hist = orc.parareal(p, u0, K=2, history=True)
    for k in range(2):
        d = hist[k + 1, -1] - hist[k, -1]
        assert log[k, 0] == np.max(np.abs(d))
        assert log[k, 1] == np.max(np.abs(hist[k + 1, -1]))
        assert abs(log[k, 2] - np.sum(d * d)) <= 1e-12 * log[k, 2]
        dall = hist[k + 1, 1:] - hist[k, 1:]
        assert log[k, 4] == np.max(np.abs(dall))
        assert abs(log[k, 6] - np.sum(dall * dall)) <= 1e-12 * log[k, 6]


def test_binomial_closed_form_constant_coefficients(orc):
    """For a linear autonomous problem (omega = 0) F and G are the same
    commuting operators on every slice and Parareal has the closed form
    U^k_n = sum_{j <= min(k, n)} C(n, j) (F - G)^j G^(n-j) u0."""
    p = W.small_problem(n=(5, 4, 6), P=5, nf=4, nc=2, omega=0.0, a=(0.6, -0.3, 0.8))
    u0 = W.random_field(p.n, 34)
    _, _, hist = orc.parareal(p, u0, K=3, history=True)

    def Fop(v):
        return orc.fine_prop(p, 0, v)

    def Gop(v):
        return orc.coarse_prop(p, 0, v)

    for k in range(4):
        for n in range(p.P + 1):
            acc = np.zeros_like(u0)
            for j in range(min(k, n) + 1):
                w = u0.copy()
                for _ in range(n - j):
                    w = Gop(w)
                for _ in range(j):
                    w = Fop(w) - Gop(w)
                acc += math.comb(n, j) * w
            scale = np.max(np.abs(hist[k, n]))
            assert np.max(np.abs(hist[k, n] - acc)) <= 1e-12 * scale, (k, n)


def _rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def test_spectral_matches_oracle_c1_all_iterates(orc):
    """The 32^3 plain-FP64 workload (P = 4, K = 4), every iterate at every
    slice boundary: grid oracle and per-mode reference agree to 1e-12."""
    p, modes = W.config("c1_32_fp64")
    u0 = W.synth_u0(p.n, modes)
    _, _, hist = orc.parareal(p, u0, K=p.K, history=True)
    ms = S.ModalSolution(p, modes)
    for k in range(p.K + 1):
        for s in range(1, p.P + 1):
            ref = ms.iterate(k, s)
            assert _rel_l2(hist[k, s], ref) <= 1e-12, (k, s)
    assert _rel_l2(orc.serial_fine(p, u0), ms.serial_fine()) <= 1e-12


@pytest.mark.parametrize("order,flags", [(4, 0), (4, W.NU_FROZEN), (2, W.NU_FROZEN)])
def test_spectral_matches_oracle_variants(orc, order, flags):
    rng = np.random.default_rng(35)
    modes = W.draw_modes(rng, 5, 3)
    p = W.small_problem(n=(12, 10, 14), a=(0.9, -0.4, 0.3), nu0=0.01, P=3, nf=5, nc=2, K=2,
                        order=order, flags=flags)
    u0 = W.synth_u0(p.n, modes)
    _, _, hist = orc.parareal(p, u0, K=2, history=True)
    ms = S.ModalSolution(p, modes)
    for k in range(3):
        for s in range(1, p.P + 1):
            assert _rel_l2(hist[k, s], ms.iterate(k, s)) <= 1e-12, (k, s)


def test_spectral_matches_oracle_batched_instance(orc):
    """One instance of the uneven batched workload, reduced to its smallest
    size class and 2 iterations."""
    insts = W.batched_config(64)
    p, modes = next((pp, mm) for pp, mm in insts if pp.n[0] == 48)
    p.K = 1
    u0 = W.synth_u0(p.n, modes)
    U, _ = orc.parareal(p, u0, K=1)
    ms = S.ModalSolution(p, modes, K=1)
    assert _rel_l2(U[-1], ms.iterate(1, p.P)) <= 1e-12


@pytest.mark.parametrize("order,expected", [(2, 4.0), (4, 16.0)])
def test_fine_spatial_order_against_continuous_solution(orc, order, expected):
    """Halving h (with dt proportional to h^2 so that time errors stay
    negligible) divides the error of the serial fine solution by 2^order."""
    modes = W.Modes(kappa=np.array([[1, 2, 1], [2, 1, 1]]), amp=np.array([1.0, -0.5]))
    errs = []
    for n in (16, 32):
        nt = 8 * (n // 16) ** 2 * 8
        p = W.Problem(n=(n, n, n), a=(1.0, 0.5, 0.25), nu0=0.01, nu_amp=0.5,
                      nu_omega=2 * math.pi / 0.05, T=0.05, P=1, nt_fine=nt, nt_coarse=1, K=0,
                      fine_order=order)
        u0 = W.synth_u0(p.n, modes)
        uf = orc.fine_steps(p, 0, nt, u0)
        ex = S.analytic(p, modes, p.T)
        errs.append(np.max(np.abs(uf - ex)) / np.max(np.abs(ex)))
    r = errs[0] / errs[1]
    assert 0.85 * expected < r < 1.15 * expected, (errs, r)


def test_analytic_matches_paper_decay_factor():
    """Single mode sin sin sin with c = 0: the amplitude decays as
    exp(-12 pi^2 int nu) (Section 3, eq. sol_form and the a(t) formula)."""
    p = W.Problem(n=(8, 8, 8), a=(0.0, 0.0, 0.0), nu0=0.1, nu_amp=0.5, nu_omega=100.0, T=0.1)
    m = W.single_mode((1, 1, 1))
    t = 0.1
    u = S.analytic(p, m, t)
    u0 = W.synth_u0(p.n, m)
    integral = 0.1 * t - 0.1 / (2 * 100.0) * (math.cos(100.0 * t) - 1.0)
    fac = math.exp(-12 * math.pi ** 2 * integral)
    assert np.max(np.abs(u - fac * u0)) <= 1e-14


def test_thread_count_does_not_change_results(orc):
    """The oracle's z loops give bitwise the same fields on 1 thread and on
    several (each output point is computed by the same operations), so its
    single- and multi-thread wall times time the same computation."""
    p = W.small_problem(n=(9, 7, 12), P=3, nf=2, nc=2, K=2)
    u0 = W.random_field(p.n, 33)
    default = orc.threads()
    try:
        orc.set_threads(1)
        assert orc.threads() == 1
        U1, log1 = orc.parareal(p, u0)
        orc.set_threads(4)
        U4, log4 = orc.parareal(p, u0)
    finally:
        orc.set_threads(default)
    assert np.array_equal(U1, U4) and np.array_equal(log1, log4)


def test_fft_synthesis_equals_direct_sum():
    """The inverse-FFT evaluation of a trigonometric sum on the grid equals
    the direct sum of its exponentials (wavenumbers of both signs, beyond the
    Nyquist index, and repeated), and the synthesis of the initial modes
    equals the initial field sampled in real arithmetic."""
    rng = np.random.default_rng(5)
    n = (12, 10, 9)
    q = rng.integers(-20, 21, size=(40, 3))
    q[5] = q[4]
    c = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    assert np.allclose(S.synth_fft(n, q, c), S.synth(n, q, c), rtol=0, atol=1e-12)
    p, modes = W.config("c1_32_fp64")
    qq, cc = S.expand_modes(modes)
    u0 = W.synth_u0(p.n, modes)
    assert np.max(np.abs(S.synth_fft(p.n, qq, cc) - u0)) <= 1e-13 * np.max(np.abs(u0))
    ms = S.ModalSolution(p, modes)
    assert np.max(np.abs(ms.iterate_fft(p.K, p.P) - ms.iterate(p.K, p.P))) <= 1e-13
