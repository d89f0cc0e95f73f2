"""Runtime model of serial time stepping and pipelined Parareal (host-side
reporting only; no GPU work).

  C_f = N_p N_f tau_f                                        (Section 2.1.1, eq. cost_serial)
  C_p = (N_p + K) N_c tau_c + K N_f tau_f                    (Section 2.2.1, eq. cost_parareal)
  S_bound = 1 / ((1 + K/N_p)(N_c/N_f)(tau_c/tau_f) + K/N_p)  (Section 2.2.2, eq. speedup)
  E = S / N_p                                                (Section 2.2.2, eq. efficiency)
  gamma_bound = N_p / S_bound                                (Section 2.2.2, eq. gamma_expected)
"""
from __future__ import annotations


def cost_serial(n_p: int, n_f: int, tau_f: float) -> float:
    return float(n_p) * n_f * tau_f


def cost_parareal(n_p: int, k: int, n_c: int, n_f: int, tau_c: float, tau_f: float) -> float:
    return (n_p + k) * n_c * tau_c + k * n_f * tau_f


def speedup_bound(n_p: int, k: int, nc_over_nf: float, tauc_over_tauf: float) -> float:
    return 1.0 / ((1.0 + k / n_p) * nc_over_nf * tauc_over_tauf + k / n_p)


def speedup_limits(n_p: int, k: int, nc_over_nf: float, tauc_over_tauf: float):
    """The two upper bounds that follow from eq. speedup: N_p/K and
    (N_f/N_c)(tau_f/tau_c)."""
    return n_p / k, 1.0 / (nc_over_nf * tauc_over_tauf)


def efficiency(speedup: float, n_p: int) -> float:
    return speedup / n_p


def gamma_bound(n_p: int, s_bound: float) -> float:
    return n_p / s_bound


def fit_tau_ratio(n_p: int, k: int, nc_over_nf: float, speedup: float) -> float:
    """Invert eq. speedup for tau_c/tau_f given one (N_p, S) pair."""
    return (1.0 / speedup - k / n_p) / ((1.0 + k / n_p) * nc_over_nf)
