"""Pins of the adjoint gradient: central differences and a brute-force derivative."""
import numpy as np

from oracle.gradient import gradient, loss, gradient_formula
from oracle.assemble import operator_from_fields
from workloads import lognormal_kappa, rhs_normal, observation_cells, observation_noise


def _setup(n=6, count=20):
    kappa = lognormal_kappa(n)
    f = rhs_normal(n ** 3)
    obs = observation_cells(n ** 3, count=count)
    data = observation_noise(count) * 0.01
    return kappa, f, obs, data


def test_gradient_matches_central_differences():
    kappa, f, obs, data = _setup()
    L0, g, _, _ = gradient(kappa, f, obs, data)
    rng = np.random.default_rng(11)
    for _ in range(3):
        v = kappa * rng.standard_normal(kappa.shape)
        t = 1e-6
        fd = (loss(kappa + t * v, f, obs, data) - loss(kappa - t * v, f, obs, data)) / (2 * t)
        an = float(np.sum(g * v))
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-14


def test_gradient_formula_brute_force_derivative():
    """-lam^T (dA/dkappa_c) u with dA/dkappa_c from differencing the assembly itself."""
    n = 4
    kappa = lognormal_kappa(n)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(n ** 3)
    lam = rng.standard_normal(n ** 3)
    g = gradient_formula(kappa, u, lam)
    for c in [0, 7, 21, 63]:
        t = 1e-6 * kappa.reshape(-1)[c]
        kp, km = kappa.copy().reshape(-1), kappa.copy().reshape(-1)
        kp[c] += t
        km[c] -= t
        Ap = operator_from_fields(kappa.shape, kappa=kp.reshape(kappa.shape))
        Am = operator_from_fields(kappa.shape, kappa=km.reshape(kappa.shape))
        dA = (Ap - Am) / (2 * t)
        want = -lam @ (dA @ u)
        assert abs(g.reshape(-1)[c] - want) <= 1e-6 * abs(want)
