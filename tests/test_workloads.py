"""Input generators: determinism, normalisation and agreement with the oracle's assembly."""
import numpy as np
import pytest

from workloads import fields, stencil, problem
from oracle.assemble import operator_from_fields, operator_from_coef


def test_deterministic_per_seed():
    a = fields.lognormal_kappa(10, seed=0)
    b = fields.lognormal_kappa(10, seed=0)
    c = fields.lognormal_kappa(10, seed=9)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(fields.rhs_normal(100), fields.rhs_normal(100))


def test_grf_normalised():
    g = fields.gaussian_random_field((12, 12, 12), seed=0)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.0) < 1e-12


def test_velocity_peclet_and_divergence():
    n = 16
    kappa = fields.lognormal_kappa(n)
    b = fields.divergence_free_velocity(kappa)
    h = fields.grid_h(n)
    assert abs(np.max(np.abs(b) * h / (2 * kappa[None])) - 1.0) < 1e-12
    # second-order central divergence is small compared with the gradients
    div = (np.gradient(b[0], h, axis=2) + np.gradient(b[1], h, axis=1) + np.gradient(b[2], h, axis=0))
    grad = np.abs(np.gradient(b[0], h, axis=2)) + np.abs(np.gradient(b[1], h, axis=1))
    assert np.max(np.abs(div[2:-2, 2:-2, 2:-2])) < 0.1 * np.max(grad)


@pytest.mark.parametrize("kind", ["poisson", "convdiff", "helmholtz", "laplace"])
def test_coef_matches_independent_assembly(kind):
    n = 7
    coef = problem(kind, n)
    A1 = operator_from_coef(coef)
    kw = {}
    if kind in ("poisson", "convdiff"):
        kw["kappa"] = fields.lognormal_kappa(n)
    if kind == "convdiff":
        kw["velocity"] = fields.divergence_free_velocity(kw["kappa"])
    if kind == "helmholtz":
        kw["speed"] = fields.helmholtz_speed(n)
        kw["omega"] = fields.helmholtz_omega(n)
    A2 = operator_from_fields((n, n, n), **kw)
    assert abs(A1 - A2).max() <= 1e-13 * abs(A2).max()


def test_upwind_exact_on_linear():
    """b . grad u with first-order upwinding is exact for u linear along b."""
    n = 6
    h = fields.grid_h(n)
    x = (np.arange(n) + 1) * h
    for bx, prof in ((2.5, x), (-1.5, 1.0 - x)):
        b = np.zeros((3, n, n, n))
        b[0] = bx
        g = np.random.default_rng(0).standard_normal((n, n))
        u = (prof[None, None, :] * g[:, :, None]).reshape(-1)
        A = operator_from_coef(stencil.add_upwind_convection(np.zeros((7, n, n, n)), b))
        want = (abs(bx) * g[:, :, None] * np.ones(n)[None, None, :]).reshape(-1)
        assert np.max(np.abs(A @ u - want)) <= 1e-10 * np.max(np.abs(want))


def test_out_of_grid_entries_zero():
    coef = problem("convdiff", 5)
    assert np.all(coef[1][:, :, 0] == 0) and np.all(coef[2][:, :, -1] == 0)
    assert np.all(coef[3][:, 0, :] == 0) and np.all(coef[4][:, -1, :] == 0)
    assert np.all(coef[5][0] == 0) and np.all(coef[6][-1] == 0)
