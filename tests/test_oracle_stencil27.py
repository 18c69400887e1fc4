"""Pins of the 27-point path of the oracle (the trilinear finite-element
discretisation of Section 5.3, whose plane couplings E_k, F_k are 9-point
plane operators rather than diagonals)."""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle.acr import OracleACR, dense_solve
from oracle.assemble import fem_q1_operator, operator_from_coef, relres
from workloads import fem_q1_coef, helmholtz27_wavenumber, problem, rhs_normal

from test_oracle_acr import _level_matrix


@pytest.mark.parametrize("shape,k", [((4, 5, 6), 0.0), ((5, 5, 5), 3.0), ((3, 4, 7), 7.5), ((6, 6, 6), 3.0)])
def test_stencil_equals_element_assembly(shape, k):
    """The generator's tensor-product stencil equals the element-by-element
    assembly of the 8 x 8 element matrices (two independent routes)."""
    A1 = operator_from_coef(fem_q1_coef(shape, k))
    A2 = fem_q1_operator(shape, k)
    assert abs(A1 - A2).max() <= 1e-14 * abs(A2).max()
    assert A1.nnz == A2.nnz


def _dst_q1_solve(f, n, k):
    """Exact inverse of the constant-coefficient Q1 operator K - k^2 M on an
    n^3 Dirichlet grid: every 1D factor is a symmetric tridiagonal Toeplitz
    matrix diagonalised by the type-I DST, with symbols
    stiffness (2 - 2 cos t) / h and mass h (4 + 2 cos t) / 6, t = p pi h."""
    h = 1.0 / (n + 1)
    t = np.arange(1, n + 1) * np.pi * h
    ks = (2.0 - 2.0 * np.cos(t)) / h
    ms = h * (4.0 + 2.0 * np.cos(t)) / 6.0
    kz, ky, kx = ks[:, None, None], ks[None, :, None], ks[None, None, :]
    mz, my, mx = ms[:, None, None], ms[None, :, None], ms[None, None, :]
    lam = kx * my * mz + mx * ky * mz + mx * my * kz - k ** 2 * mx * my * mz
    F = sfft.dstn(f.reshape(n, n, n), type=1, norm="ortho")
    return sfft.dstn(F / lam, type=1, norm="ortho").reshape(-1)


@pytest.mark.parametrize("kind", ["fem_poisson27", "fem_helmholtz27", "nonsym27"])
@pytest.mark.parametrize("n,leaf", [(4, 4), (5, 4), (6, 9), (7, 13), (8, 16)])
def test_exact_mode_equals_dense_solve(kind, n, leaf):
    coef = problem(kind, n)
    f = rhs_normal(n ** 3)
    u = OracleACR(coef, leaf, 0.0).solve(f)
    ud = dense_solve(coef, f)
    assert np.linalg.norm(u - ud) <= 1e-11 * np.linalg.norm(ud)


@pytest.mark.parametrize("k", [0.0, None])
def test_exact_mode_equals_dst(k):
    """Poisson and the Helmholtz workload's wavenumber (n / 2) at n = 16."""
    n = 16
    k = helmholtz27_wavenumber(n) if k is None else k
    coef = fem_q1_coef((n, n, n), k)
    f = rhs_normal(n ** 3)
    u = OracleACR(coef, 32, 0.0).solve(f)
    ue = _dst_q1_solve(f, n, k)
    assert np.linalg.norm(u - ue) <= 1e-11 * np.linalg.norm(ue)


def test_dst_solver_is_the_inverse():
    """The DST reference itself against the assembled matrix (n = 5)."""
    n, k = 5, 2.5
    f = rhs_normal(n ** 3)
    A = fem_q1_operator((n, n, n), k)
    assert np.linalg.norm(A @ _dst_q1_solve(f, n, k) - f) <= 1e-12 * np.linalg.norm(f)


@pytest.mark.parametrize("nz", [6, 7, 8])
def test_levels_are_schur_complements_dense_couplings(nz):
    """eps = 0 with dense E, F: each level is the Schur complement of the
    red/black permuted previous level (Eq. schur_complement)."""
    n = 4
    coef = problem("nonsym27", n)
    coef = np.concatenate([coef] * 2, axis=1)[:, :nz]
    coef[:9, 0] = 0.0      # dz = -1 slots of the first plane
    coef[18:, -1] = 0.0    # dz = +1 slots of the last plane
    o = OracleACR(coef, 4, 0.0)
    M = o.M
    assert o.levels[0]["E"][1][0] == "dense"
    for i, lev in enumerate(o.levels):
        S = _level_matrix(o, lev)
        ev = np.concatenate([np.arange(q * M, (q + 1) * M) for q in lev["elim"]])
        od = np.concatenate([np.arange(q * M, (q + 1) * M) for q in lev["kept"]])
        schur = S[np.ix_(od, od)] - S[np.ix_(od, ev)] @ np.linalg.solve(S[np.ix_(ev, ev)], S[np.ix_(ev, od)])
        nxt = _level_matrix(o, o.levels[i + 1]) if i + 1 < len(o.levels) else o.D_last[1]
        assert np.max(np.abs(nxt - schur)) <= 1e-12 * np.max(np.abs(schur))


def test_transpose_identity_truncated_27():
    n = 8
    o = OracleACR(problem("nonsym27", n), 16, 1e-2)
    rng = np.random.default_rng(8)
    f, g = rng.standard_normal(o.N), rng.standard_normal(o.N)
    rhs = g @ o.solve(f)
    assert abs(o.solve_transpose(g) @ f - rhs) <= 1e-12 * abs(rhs)


def test_transpose_exact_mode_27():
    n = 6
    coef = problem("nonsym27", n)
    f = rhs_normal(n ** 3)
    u = OracleACR(coef, 9, 0.0).solve_transpose(f)
    ue = np.linalg.solve(operator_from_coef(coef).toarray().T, f)
    assert np.linalg.norm(u - ue) <= 1e-11 * np.linalg.norm(ue)


@pytest.mark.parametrize("kind", ["fem_poisson27", "nonsym27"])
@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_truncated_residual_bound_27(kind, eps):
    """Residual before refinement within C * eps (C = 5, as for 7 points)."""
    n = 12
    coef = problem(kind, n)
    f = rhs_normal(n ** 3)
    o = OracleACR(coef, 16, eps)
    assert float(relres(o.A, o.solve(f), f)) <= 5.0 * eps
