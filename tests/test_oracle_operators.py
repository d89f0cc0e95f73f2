"""Pins of the oracle's spatial operators against definitions written out
independently (dense matrices built from periodic shift matrices), special
cases with exact answers, and invariants.  CPU only."""
import numpy as np
import pytest

import workloads as W
from oracle import spectral as S


def shift(n, k):
    """Dense periodic shift: (shift(n,k) @ v)[i] = v[(i + k) mod n]."""
    M = np.zeros((n, n))
    for i in range(n):
        M[i, (i + k) % n] = 1.0
    return M


def axis_op(n3, d, M1):
    """Embed a 1D operator acting along axis d (0=x, 1=y, 2=z) for [z, y, x] storage."""
    nx, ny, nz = n3
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    if d == 0:
        return np.kron(Iz, np.kron(Iy, M1))
    if d == 1:
        return np.kron(Iz, np.kron(M1, Ix))
    return np.kron(M1, np.kron(Iy, Ix))


def dense_fine(n3, a, nu, order):
    L = 0.0
    for d in range(3):
        n = n3[d]
        h = 1.0 / n
        Sp, Sm, Sp2, Sm2, I = shift(n, 1), shift(n, -1), shift(n, 2), shift(n, -2), np.eye(n)
        if order == 2:
            D2 = (Sp + Sm - 2 * I) / h ** 2
            D1 = (Sp - Sm) / (2 * h)
        else:
            D2 = (-Sp2 + 16 * Sp - 30 * I + 16 * Sm - Sm2) / (12 * h ** 2)
            D1 = (-Sp2 + 8 * Sp - 8 * Sm + Sm2) / (12 * h)
        L = L + nu * axis_op(n3, d, D2) - a[d] * axis_op(n3, d, D1)
    return L


def dense_coarse(n3, a, nu):
    L = 0.0
    for d in range(3):
        n = n3[d]
        h = 1.0 / n
        Sp, Sm, I = shift(n, 1), shift(n, -1), np.eye(n)
        D2 = (Sp + Sm - 2 * I) / h ** 2
        up = (I - Sm) / h if a[d] > 0 else (Sp - I) / h
        L = L + nu * axis_op(n3, d, D2) - a[d] * axis_op(n3, d, up)
    return L


GRIDS2 = [(3, 4, 5), (4, 3, 6), (5, 5, 3)]
GRIDS4 = [(5, 6, 7), (7, 5, 6)]
AS = [(1.0, 0.5, 0.25), (-0.7, 0.3, -1.1), (0.0, -0.4, 0.9)]


@pytest.mark.parametrize("n3", GRIDS2)
@pytest.mark.parametrize("a", AS)
def test_fine_rhs_order2_matches_dense(orc, n3, a):
    p = W.small_problem(n=n3, a=a)
    u = W.random_field(n3, 11)
    nu = 0.037
    ref = (dense_fine(n3, a, nu, 2) @ u.ravel()).reshape(u.shape)
    got = orc.fine_rhs(p, nu, u)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n3", GRIDS4)
@pytest.mark.parametrize("a", AS)
def test_fine_rhs_order4_matches_dense(orc, n3, a):
    p = W.small_problem(n=n3, a=a, order=4)
    u = W.random_field(n3, 12)
    nu = 0.021
    ref = (dense_fine(n3, a, nu, 4) @ u.ravel()).reshape(u.shape)
    got = orc.fine_rhs(p, nu, u)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n3", GRIDS2)
@pytest.mark.parametrize("a", AS)
def test_coarse_rhs_matches_dense(orc, n3, a):
    p = W.small_problem(n=n3, a=a)
    u = W.random_field(n3, 13)
    nu = 0.05
    ref = (dense_coarse(n3, a, nu) @ u.ravel()).reshape(u.shape)
    got = orc.coarse_rhs(p, nu, u)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_coarse_courant_one_is_exact_shift(orc, sign, axis):
    """nu = 0, |a| h^-1 Dt = 1: one upwind Euler step moves the field by one cell
    downstream, exactly (up to rounding)."""
    n3 = (6, 7, 8)
    a = [0.0, 0.0, 0.0]
    a[axis] = sign * 1.0
    n = n3[axis]
    # Dt = T / nt_coarse must equal h / |a| = 1/n
    p = W.Problem(n=n3, a=tuple(a), nu0=0.0, nu_amp=0.0, nu_omega=0.0, T=1.0, P=1,
                  nt_fine=1, nt_coarse=n, K=0)
    u = W.random_field(n3, 14)
    got = orc.euler_step(p, 0, u)
    # storage is [z, y, x]; +a along axis d moves values to larger index
    np_axis = 2 - axis
    ref = np.roll(u, int(sign), axis=np_axis)
    assert np.max(np.abs(got - ref)) <= 1e-13


@pytest.mark.parametrize("order", [2, 4])
def test_fine_step_conserves_mean(orc, order):
    n3 = (8, 7, 6) if order == 2 else (8, 7, 6)
    p = W.small_problem(n=n3, order=order)
    u = W.random_field(n3, 15) + 3.0
    out = orc.rk4_step(p, 3, u)
    assert abs(out.sum() - u.sum()) <= 1e-12 * np.abs(u).sum()


def test_coarse_step_conserves_mean(orc):
    n3 = (8, 7, 6)
    p = W.small_problem(n=n3, a=(0.6, -0.4, 0.9))
    u = W.random_field(n3, 16) + 3.0
    out = orc.euler_step(p, 2, u)
    assert abs(out.sum() - u.sum()) <= 1e-12 * np.abs(u).sum()


@pytest.mark.parametrize("order", [2, 4])
def test_translation_equivariance_bitwise(orc, order):
    n3 = (8, 6, 7)
    p = W.small_problem(n=n3, order=order, a=(0.8, -0.3, 0.5))
    u = W.random_field(n3, 17)
    shifts = (2, -1, 3)  # along z, y, x of the array
    f1 = orc.fine_steps(p, 5, 2, np.roll(u, shifts, axis=(0, 1, 2)))
    f2 = np.roll(orc.fine_steps(p, 5, 2, u), shifts, axis=(0, 1, 2))
    assert np.array_equal(f1, f2)
    g1 = orc.coarse_steps(p, 1, 3, np.roll(u, shifts, axis=(0, 1, 2)))
    g2 = np.roll(orc.coarse_steps(p, 1, 3, u), shifts, axis=(0, 1, 2))
    assert np.array_equal(g1, g2)


def test_linearity(orc):
    n3 = (6, 6, 6)
    p = W.small_problem(n=n3)
    u, v = W.random_field(n3, 18), W.random_field(n3, 19)
    al, be = 0.75, -1.5
    lhs = orc.fine_steps(p, 0, 3, al * u + be * v)
    rhs = al * orc.fine_steps(p, 0, 3, u) + be * orc.fine_steps(p, 0, 3, v)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


@pytest.mark.parametrize("order", [2, 4])
def test_spectral_symbols_are_operator_eigenvalues(order):
    """The spectral reference's symbols equal the eigenvalues of the dense
    operators on grid exponentials (pins spectral.py's stencil algebra)."""
    n3 = (5, 6, 7)
    a = (0.9, -0.6, 0.3)
    nu = 0.043
    q = np.array([[1, 2, -3], [-2, 0, 1], [0, 0, 0], [2, -3, 3]])
    x = np.arange(n3[0]) / n3[0]
    y = np.arange(n3[1]) / n3[1]
    z = np.arange(n3[2]) / n3[2]
    Lf = dense_fine(n3, a, nu, order)
    Lc = dense_coarse(n3, a, nu)
    sDf, sAf = S.fine_symbols(q, n3, a, order)
    sDc, sAc = S.coarse_symbols(q, n3, a)
    for i, (qx, qy, qz) in enumerate(q):
        e = (np.exp(2j * np.pi * qz * z)[:, None, None] * np.exp(2j * np.pi * qy * y)[None, :, None]
             * np.exp(2j * np.pi * qx * x)[None, None, :]).ravel()
        lam_f = (Lf @ e)[0] / e[0]
        lam_c = (Lc @ e)[0] / e[0]
        assert np.allclose(Lf @ e, lam_f * e, atol=1e-10 * max(1, abs(lam_f)))
        assert abs(lam_f - (nu * sDf[i] + sAf[i])) <= 1e-11 * max(1.0, abs(lam_f))
        assert abs(lam_c - (nu * sDc[i] + sAc[i])) <= 1e-11 * max(1.0, abs(lam_c))
