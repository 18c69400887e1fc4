"""The factorisation as a preconditioner across truncation tolerances (the
accuracy/time trade-off of Section 5: Table precond, Fig. controlAccuracy):
constant-coefficient Poisson -lap u = 1 with Dirichlet boundaries, conjugate
gradients to 1e-6 preconditioned by the truncated factorisation, eps swept as
in the paper's table.

* n = 16: the GPU's iteration counts (FP64 factors, flexible CG on the device)
  against a CPU flexible CG preconditioned by the oracle's factorisation at
  the same eps and leaf size;
* n = 32 and n = 64 (FP32 factors): every eps converges, and the counts do not
  increase as eps shrinks while the stored ranks do not decrease -- the shape
  of the paper's table (43/34/25/11/4 iterations at 0.6/0.3/0.1/1e-2/1e-3).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1701_00182_amd as acr  # noqa: E402
from oracle.acr import OracleACR  # noqa: E402
from oracle.assemble import operator_from_coef, relres  # noqa: E402
from workloads import problem  # noqa: E402

os.environ.setdefault("ACR_CHECK", "1")
DEV = torch.device("cuda:0")
EPS_SWEEP = [0.6, 0.3, 0.1, 1e-2, 1e-3]


def _fcg_cpu(A, b, precond, tol, maxit=500):
    """Flexible preconditioned CG on the host (beta from z^T (r - r_old)),
    counting preconditioner applications as the device refinement does (the
    first application gives x0 = M^{-1} b)."""
    x = precond(b)
    its = 1
    r = b - A @ x
    bn = np.linalg.norm(b)
    if np.linalg.norm(r) / bn <= tol:
        return its, np.linalg.norm(r) / bn
    z = precond(r)
    its += 1
    rz = r @ z
    p = z.copy()
    while True:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r_old = r.copy()
        r = r - alpha * q
        rel = np.linalg.norm(r) / bn
        if rel <= tol or its >= maxit:
            break
        z = precond(r)
        its += 1
        beta = (z @ r - z @ r_old) / rz
        rz = r @ z
        p = z + beta * p
    return its, np.linalg.norm(b - A @ x) / bn


def _gpu_sweep(n, leaf, precision):
    coef = problem("laplace", n)
    A = operator_from_coef(coef)
    coef_d = torch.from_numpy(coef).to(DEV)
    b = torch.ones(n ** 3, dtype=torch.float64, device=DEV)
    rows = []
    for eps in EPS_SWEEP:
        fac = acr.Factor(coef_d, eps=eps, leaf=leaf, precision=precision)
        x, info = fac.solve_refined(b, tol=1e-6, method="cg", maxit=500)
        rel = float(relres(A, x.cpu().numpy(), np.ones(n ** 3)))
        st = fac.stats()
        fac.free()
        rows.append((eps, info["iterations"], rel, st["max_rank"], info["relres0"]))
        print(f"n={n} eps={eps:g}: {info['iterations']} CG applications, relres {rel:.2e}, "
              f"unrefined {info['relres0']:.2e}, max rank {st['max_rank']}", flush=True)
    return rows


def test_precond_iterations_match_oracle_n16():
    n, leaf = 16, 32
    coef = problem("laplace", n)
    A = operator_from_coef(coef).tocsr()
    b = np.ones(n ** 3)
    gpu = _gpu_sweep(n, leaf, "fp64")
    for (eps, its, rel, _, _) in gpu:
        o = OracleACR(coef, leaf, eps)
        its_o, rel_o = _fcg_cpu(A, b, o.solve, 1e-6)
        print(f"eps={eps:g}: gpu {its} oracle {its_o} (oracle relres {rel_o:.2e})", flush=True)
        assert rel <= 1e-6
        assert abs(its - its_o) <= max(2, int(0.3 * its_o))


@pytest.mark.parametrize("n,leaf", [(32, 64), (64, 64)])
def test_precond_sweep_shape(n, leaf):
    rows = _gpu_sweep(n, leaf, "fp32")
    for eps, its, rel, _, _ in rows:
        assert rel <= 1e-6, (eps, rel)
    its = [r[1] for r in rows]
    ranks = [r[3] for r in rows]
    assert all(a >= b for a, b in zip(its, its[1:])), its
    assert all(a <= b for a, b in zip(ranks, ranks[1:])), ranks
    assert its[0] > its[-1]
