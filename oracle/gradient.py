"""Data-misfit loss and its gradient with respect to the nodal diffusion coefficient.

Not part of the paper: the differentiable-solver workload asks for
dL/dkappa of L = 0.5 ||P u - d||^2 with A(kappa) u = f, where A is the
variable-coefficient model operator of Section 2.2.1 (Eq. probSta).  With the
adjoint A^T lam = P^T (P u - d), dL/dkappa_c = -lam^T (dA/dkappa_c) u.

For the discretisation used here (harmonic-mean face coefficients, boundary
faces weighted by the nodal value) lam^T A u equals
h^-2 [ sum_faces k_rs (lam_r - lam_s)(u_r - u_s) + sum_r n_b(r) k_r lam_r u_r ]
and d k_rs / d k_r = 2 k_s^2 / (k_r + k_s)^2, which gives
dL/dk_c = -h^-2 [ sum_{s in nb(c)} 2 k_s^2/(k_c+k_s)^2 (lam_c-lam_s)(u_c-u_s)
                  + n_b(c) lam_c u_c ].
"""
import numpy as np
import scipy.sparse.linalg as spla

from .assemble import operator_from_fields


def loss(kappa, f, obs, data):
    A = operator_from_fields(kappa.shape, kappa=kappa)
    u = spla.spsolve(A.tocsc(), f)
    r = u[obs] - data
    return 0.5 * float(r @ r)


def gradient_formula(kappa, u, lam):
    """Per-node gradient -lam^T (dA/dkappa_c) u by the face sum above."""
    nz, ny, nx = kappa.shape
    U = u.reshape(kappa.shape)
    Lm = lam.reshape(kappa.shape)
    g = np.zeros_like(kappa)
    for axis, n in ((2, nx), (1, ny), (0, nz)):
        h2 = (1.0 / (n + 1)) ** 2
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(None, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        kr, ks = kappa[lo], kappa[hi]
        prod = (Lm[lo] - Lm[hi]) * (U[lo] - U[hi])
        g[lo] -= 2.0 * ks ** 2 / (kr + ks) ** 2 * prod / h2
        g[hi] -= 2.0 * kr ** 2 / (kr + ks) ** 2 * prod / h2
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = 0
        last[axis] = -1
        for b in (tuple(first), tuple(last)):
            g[b] -= Lm[b] * U[b] / h2
    return g


def gradient(kappa, f, obs, data):
    """Loss and dL/dkappa with exact sparse solves (forward and adjoint)."""
    A = operator_from_fields(kappa.shape, kappa=kappa).tocsc()
    u = spla.spsolve(A, f)
    r = u[obs] - data
    rhs = np.zeros_like(u)
    rhs[obs] = r
    lam = spla.spsolve(A.T.tocsc(), rhs)
    return 0.5 * float(r @ r), gradient_formula(kappa, u, lam), u, lam
