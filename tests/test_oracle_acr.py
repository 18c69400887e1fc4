"""Pins of the oracle's cyclic reduction against exact solvers and invariants."""
import numpy as np
import pytest
import scipy.fft as sfft
import scipy.sparse.linalg as spla

from oracle.acr import OracleACR, dense_solve
from oracle.assemble import operator_from_coef, relres
from workloads import problem, rhs_normal, diffusion_coef


@pytest.mark.parametrize("kind", ["poisson", "convdiff", "helmholtz", "laplace"])
@pytest.mark.parametrize("n,leaf", [(4, 4), (5, 4), (6, 9), (7, 13), (8, 16)])
def test_exact_mode_equals_dense_solve(kind, n, leaf):
    coef = problem(kind, n)
    f = rhs_normal(n ** 3)
    u = OracleACR(coef, leaf, 0.0).solve(f)
    ud = dense_solve(coef, f)
    assert np.linalg.norm(u - ud) <= 1e-11 * np.linalg.norm(ud)


@pytest.mark.parametrize("kind", ["poisson", "convdiff"])
def test_exact_mode_equals_sparse_lu(kind):
    n = 12
    coef = problem(kind, n)
    f = rhs_normal(n ** 3, nrhs=3)
    u = OracleACR(coef, 36, 0.0).solve(f)
    A = operator_from_coef(coef).tocsc()
    us = spla.splu(A).solve(f)
    assert np.linalg.norm(u - us) <= 1e-11 * np.linalg.norm(us)


def _dst_laplace_solve(f, n):
    """Exact inverse of the 7-point Dirichlet Laplacian by a type-I DST."""
    h = 1.0 / (n + 1)
    p = np.arange(1, n + 1)
    lam1 = (2.0 - 2.0 * np.cos(np.pi * p * h)) / h ** 2
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    F = sfft.dstn(f.reshape(n, n, n), type=1, norm="ortho")
    return sfft.dstn(F / lam, type=1, norm="ortho").reshape(-1)


def test_exact_mode_equals_dst_laplace():
    n = 16
    coef = problem("laplace", n)
    f = rhs_normal(n ** 3)
    u = OracleACR(coef, 32, 0.0).solve(f)
    ue = _dst_laplace_solve(f, n)
    assert np.linalg.norm(u - ue) <= 1e-12 * np.linalg.norm(ue)


def test_manufactured_polynomial():
    """u* = x(1-x)y(1-y)z(1-z): the 7-point stencil is exact on each quadratic factor."""
    n = 9
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    q = x * (1 - x)
    Z, Y, X = np.meshgrid(q, q, q, indexing="ij")
    ustar = (X * Y * Z).reshape(-1)
    f = (2.0 * (Y * Z + X * Z + X * Y)).reshape(-1)
    coef = diffusion_coef(np.ones((n, n, n)))
    A = operator_from_coef(coef)
    assert np.max(np.abs(A @ ustar - f)) <= 1e-11 * np.max(np.abs(f))
    u = OracleACR(coef, 9, 0.0).solve(f)
    assert np.max(np.abs(u - ustar)) <= 1e-12 * np.max(np.abs(ustar))


def _level_matrix(o, lev):
    """Dense block-tridiagonal matrix of one level from the oracle's blocks."""
    M, m = o.M, len(lev["alive"])
    S = np.zeros((m * M, m * M))
    for q in range(m):
        blk = slice(q * M, (q + 1) * M)
        S[blk, blk] = lev["D"][q][1]
        for nb, key in ((q - 1, "E"), (q + 1, "F")):
            b = lev[key][q]
            if b is None:
                continue
            assert 0 <= nb < m
            S[blk, nb * M:(nb + 1) * M] = np.diag(b[1]) if b[0] == "diag" else b[1]
    return S


@pytest.mark.parametrize("kind,nz", [("poisson", 8), ("convdiff", 7), ("helmholtz", 6)])
def test_levels_are_schur_complements(kind, nz):
    """With eps = 0 each level is A22 - A21 A11^{-1} A12 of the red/black
    permuted previous level (Eq. schur_complement), blocks and right-hand side."""
    n = 4
    coef = problem(kind, n)
    coef = np.concatenate([coef] * 2, axis=1)[:, :nz]   # stack planes to get nz planes
    coef[5, 0] = 0.0
    coef[6, -1] = 0.0
    o = OracleACR(coef, 4, 0.0)
    f = rhs_normal(o.N)
    fr = o.reduced_rhs(f)
    levels = o.levels
    M = o.M
    for i, lev in enumerate(levels):
        S = _level_matrix(o, lev)
        m = len(lev["alive"])
        ev = np.concatenate([np.arange(q * M, (q + 1) * M) for q in lev["elim"]])
        od = np.concatenate([np.arange(q * M, (q + 1) * M) for q in lev["kept"]])
        A11, A12 = S[np.ix_(ev, ev)], S[np.ix_(ev, od)]
        A21, A22 = S[np.ix_(od, ev)], S[np.ix_(od, od)]
        schur = A22 - A21 @ np.linalg.solve(A11, A12)
        fl = np.concatenate([fr[i][lev["alive"][q]] for q in range(m)])
        f_e, f_o = fl[ev], fl[od]
        fnext = f_o - A21 @ np.linalg.solve(A11, f_e)
        if i + 1 < len(levels):
            nxt = _level_matrix(o, levels[i + 1])
        else:
            nxt = o.D_last[1]
        scale = np.max(np.abs(schur))
        assert np.max(np.abs(nxt - schur)) <= 1e-12 * scale
        got = np.concatenate([fr[i + 1][p] for p in [lev["alive"][q] for q in lev["kept"]]])
        assert np.max(np.abs(got - fnext)) <= 1e-12 * np.max(np.abs(fnext))


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_truncated_residual_bound(eps):
    """Residual before refinement stays within C * eps (C = 5 measured, stated)."""
    n = 16
    coef = problem("poisson", n)
    f = rhs_normal(n ** 3)
    o = OracleACR(coef, 32, eps)
    rr = float(relres(o.A, o.solve(f), f))
    assert rr <= 5.0 * eps


def test_transpose_identity_truncated():
    """<solve_T(g), f> = <g, solve(f)> for any eps (same blocks, transposed)."""
    n = 8
    coef = problem("convdiff", n)
    o = OracleACR(coef, 16, 1e-2)
    rng = np.random.default_rng(7)
    f, g = rng.standard_normal(o.N), rng.standard_normal(o.N)
    lhs = o.solve_transpose(g) @ f
    rhs = g @ o.solve(f)
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs) * 10


def test_transpose_exact_mode():
    n = 6
    coef = problem("convdiff", n)
    f = rhs_normal(n ** 3)
    u = OracleACR(coef, 9, 0.0).solve_transpose(f)
    A = operator_from_coef(coef).toarray()
    ue = np.linalg.solve(A.T, f)
    assert np.linalg.norm(u - ue) <= 1e-11 * np.linalg.norm(ue)


def test_blocks_are_fixed_points_of_T():
    """Every stored inverse is already in HODLR form: T(G) == G."""
    from oracle.hodlr import hodlr_truncate
    n = 8
    o = OracleACR(problem("poisson", n), 16, 1e-3)
    for lev in o.levels:
        for G in lev["G"].values():
            again, _ = hodlr_truncate(G[1], o.tree, 1e-3)
            assert np.max(np.abs(again - G[1])) <= 1e-12 * np.max(np.abs(G[1]))
