"""Checks against the numbers the paper prints (tests/golden/paper_values.json,
each entry with its section or table).  CPU only."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import spectral as S
from paper_1409_8563_amd import costmodel as C

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _two_digit_match(value, printed):
    """`printed` is given to two significant digits."""
    return abs(value - printed) <= 0.05 * abs(printed) + 1e-300


def _paper_problem(omega, P=8, K=3, frozen=True):
    p = W.paper_setup(omega, P=P, K=K)
    p.flags = W.NU_FROZEN if frozen else 0
    return p


@pytest.mark.parametrize("omega,key", [(0.0, "omega_0"), (100.0, "omega_100")])
def test_eps_fine_reproduced_with_frozen_nu(omega, key):
    """Fourth-order F, dt = T/2^15, 128^3: relative inf-norm error against the
    continuous solution.  The printed values are met when nu is evaluated at
    the start of each RK4 step for all stages."""
    m = W.single_mode((1, 1, 1))
    p = _paper_problem(omega)
    q, c = S.expand_modes(m)
    zf = np.prod(S.rk4_factors(p, q, 0, p.nt_fine), axis=0)
    uf = S.synth(p.n, q, c * zf)
    ex = S.analytic(p, m, p.T)
    eps = np.max(np.abs(uf - ex)) / np.max(np.abs(ex))
    assert _two_digit_match(eps, GOLD["eps_fine"][key]), eps


def test_eps_fine_classical_stage_times_do_not_give_printed_value():
    """With classical stage times (nu at t, t+dt/2, t+dt) the omega = 100 error
    is about 25x smaller than printed: the paper's F froze nu per step."""
    m = W.single_mode((1, 1, 1))
    p = _paper_problem(100.0, frozen=False)
    q, c = S.expand_modes(m)
    zf = np.prod(S.rk4_factors(p, q, 0, p.nt_fine), axis=0)
    uf = S.synth(p.n, q, c * zf)
    ex = S.analytic(p, m, p.T)
    eps = np.max(np.abs(uf - ex)) / np.max(np.abs(ex))
    assert eps < 0.1 * GOLD["eps_fine"]["omega_100"]


def test_eps_coarse_spectral_both_omega():
    m = W.single_mode((1, 1, 1))
    for omega in (0.0, 100.0):
        p = _paper_problem(omega)
        q, c = S.expand_modes(m)
        zg = np.prod(S.euler_factors(p, q, 0, p.nt_coarse), axis=0)
        ug = S.synth(p.n, q, c * zg)
        ex = S.analytic(p, m, p.T)
        eps = np.max(np.abs(ug - ex)) / np.max(np.abs(ex))
        assert _two_digit_match(eps, GOLD["eps_coarse"]["value"]), (omega, eps)


def test_eps_coarse_grid_oracle_128(orc):
    """The grid oracle's G run serially over all 2^11 coarse steps on 128^3
    (omega = 100) gives the printed coarse error and agrees with the per-mode
    reference."""
    m = W.single_mode((1, 1, 1))
    p = _paper_problem(100.0)
    u0 = W.synth_u0(p.n, m)
    ug = orc.coarse_steps(p, 0, p.nt_coarse, u0)
    ex = S.analytic(p, m, p.T)
    eps = np.max(np.abs(ug - ex)) / np.max(np.abs(ex))
    assert _two_digit_match(eps, GOLD["eps_coarse"]["value"]), eps
    q, c = S.expand_modes(m)
    zg = np.prod(S.euler_factors(p, q, 0, p.nt_coarse), axis=0)
    ref = S.synth(p.n, q, c * zg)
    assert np.sqrt(np.sum((ug - ref) ** 2) / np.sum(ref ** 2)) <= 1e-12


@pytest.mark.parametrize("P", GOLD["parareal_defect_k3"]["P"])
def test_defect_after_three_iterations(P):
    """d^3 is far below eps_fine for omega = 100 and of the order of eps_fine
    for omega = 0 (Section 3.3.1)."""
    m = W.single_mode((1, 1, 1))
    eps = GOLD["eps_fine"]
    for omega, bound in ((100.0, None), (0.0, eps["omega_0"])):
        p = _paper_problem(omega, P=P, K=3)
        ms = S.ModalSolution(p, m)
        uf = ms.serial_fine()
        d3 = np.max(np.abs(ms.iterate(3, P) - uf)) / np.max(np.abs(uf))
        d2 = np.max(np.abs(ms.iterate(2, P) - uf)) / np.max(np.abs(uf))
        if bound is None:
            assert d3 < 0.1 * eps["omega_100"], d3
        else:
            assert 0.1 * bound < d3 < 10 * bound, d3
        assert d3 < d2


@pytest.mark.parametrize("side", ["cpu", "gpu"])
def test_table1_speedup_bound_reproduced(side):
    """eq. speedup with one tau_c/tau_f per backend (fitted on the 128-node
    row) reproduces every S_bound and E_bound entry of Table 1 to its printed
    rounding (|dS| <= 0.08, |dE| <= 0.17 percentage points)."""
    t = GOLD["table1"]
    K, r = t["K"], 1.0 / t["nf_over_nc"]
    rows = t[side]
    tau = C.fit_tau_ratio(rows["nodes"][-1], K, r, rows["S_bound"][-1])
    assert 0.15 < tau < 0.2
    for n, S_b, E_b in zip(rows["nodes"], rows["S_bound"], rows["E_bound"]):
        s = C.speedup_bound(n, K, r, tau)
        assert abs(s - S_b) <= 0.08, (n, s, S_b)
        assert abs(100 * C.efficiency(s, n) - E_b) <= 0.17, (n, s, E_b)
        lim1, lim2 = C.speedup_limits(n, K, r, tau)
        assert s <= lim1 and s <= lim2
        assert abs(C.gamma_bound(n, s) - 1.0 / C.efficiency(s, n)) < 1e-12


def test_cost_model_consistency():
    """S_bound = C_f / C_p with the two cost formulas."""
    for n_p in (4, 16, 128):
        cf = C.cost_serial(n_p, 16 * 8, 1.0)
        cp = C.cost_parareal(n_p, 3, 8, 16 * 8, 0.2, 1.0)
        assert abs(cf / cp - C.speedup_bound(n_p, 3, 8 / (16 * 8), 0.2)) < 1e-12
