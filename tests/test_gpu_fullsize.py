"""The benchmark configurations at full size, through the C-ABI, checked by
properties that hold at any size (the oracle cannot factorise these): relative
residuals measured with an independent CPU sparse operator built from the same
seeded coefficients, and column-by-column identities of the multi-RHS solve."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1701_00182_amd as acr  # noqa: E402
from oracle.assemble import operator_from_coef, relres  # noqa: E402
from workloads import problem, rhs_normal  # noqa: E402

# host-side bounds check of every launched task at the full-size shapes
os.environ.setdefault("ACR_CHECK", "1")
DEV = torch.device("cuda:0")


def _factor(coef, **kw):
    return acr.Factor(torch.from_numpy(np.ascontiguousarray(coef)).to(DEV), **kw)


@pytest.mark.parametrize("tol", [1e-8, 1e-10])
def test_headline_convdiff_n128_fp32_gmres(tol):
    """n = 128 convection-diffusion (N = 2,097,152), eps = 1e-2, leaf 128,
    FP32 factors, two-kernel core SVD: the unrefined solve is accurate to the
    truncation level and FP64 GMRES(30) reaches the headline's 1e-8 and the
    workload's stated 1e-10, both measured again with the CPU operator.  The
    two residuals differ only by the rounding of one FP64 operator
    application (|A| |x| u / |b| ~ 1e-15), hence the 1 % margin at 1e-10."""
    n, eps = 128, 1e-2
    coef = problem("convdiff", n)
    f = rhs_normal(n ** 3)
    A = operator_from_coef(coef)
    fac = _factor(coef, eps=eps, leaf=128, precision="fp32", svd_fused_lds=-1)
    b = torch.from_numpy(f).to(DEV)
    x0 = fac.solve(b).cpu().numpy()
    assert float(relres(A, x0, f)) <= 5 * eps
    x, info = fac.solve_refined(b, tol=tol, method="gmres", maxit=300)
    rel = float(relres(A, x.cpu().numpy(), f))
    print(f"n=128 GMRES to {tol:g}: {info['iterations']} applications, relres gpu {info['relres']:.3e} "
          f"cpu {rel:.3e}", flush=True)
    assert info["converged"] and info["relres"] <= tol
    assert rel <= 1.01 * tol
    fac.free()


def test_poisson_n64_fp32_ir_to_1e8():
    """n = 64 Poisson, eps = 1e-4, leaf 64: FP32 factors with FP64 iterative
    refinement reach 1e-8, the plain FP64 form stays at the truncation level."""
    n, eps = 64, 1e-4
    coef = problem("poisson", n)
    f = rhs_normal(n ** 3)
    A = operator_from_coef(coef)
    b = torch.from_numpy(f).to(DEV)
    f32 = _factor(coef, eps=eps, leaf=64, precision="fp32")
    x, info = f32.solve_refined(b, tol=1e-8, method="ir")
    assert info["converged"] and float(relres(A, x.cpu().numpy(), f)) <= 2e-8
    f32.free()
    f64 = _factor(coef, eps=eps, leaf=64, precision="fp64")
    assert float(relres(A, f64.solve(b).cpu().numpy(), f)) <= 5 * eps
    f64.free()


@pytest.mark.parametrize("kind,tol", [("convdiff", 1e-5), ("helmholtz", 5e-3)])
def test_n64_256_rhs_columns_equal_single_solves(kind, tol):
    """n = 64, eps = 1e-3, leaf 64, FP32 factors, 256 right-hand sides in one
    solve (the multi-RHS benchmark's launch configuration: segmented leaf
    products and split inner products on the matrix cores): sampled columns
    equal their single-RHS solves (fused vector kernels).  The two paths sum
    in different orders in FP32; for convection-diffusion they agree to 1e-5.
    The indefinite Helmholtz factors at this eps amplify rounding by 1e3 - 1e5
    (their unrefined residuals are 1e2 - 1e4, and the amplification moves
    with rounding-level changes in the factors: below 1e-3 with one choice of
    launch shapes of the same kernels, 1.6e-3 with another), so the bound
    there is 5e-3."""
    n, nrhs = 64, 256
    coef = problem(kind, n)
    F = rhs_normal(n ** 3, nrhs=nrhs)
    fac = _factor(coef, eps=1e-3, leaf=64, precision="fp32")
    X = fac.solve(torch.from_numpy(np.ascontiguousarray(F.T)).to(DEV)).cpu().numpy().T
    for j in (0, 77, 255):
        xj = fac.solve(torch.from_numpy(np.ascontiguousarray(F[:, j])).to(DEV)).cpu().numpy()
        d = np.linalg.norm(X[:, j] - xj) / np.linalg.norm(xj)
        print(f"{kind} column {j}: |X_j - x_j| / |x_j| = {d:.2e}", flush=True)
        assert d <= tol
    fac.free()


def test_helmholtz_n64_refinable_factors_gmres():
    """The multi-RHS Helmholtz operator (n = 64, variable wave speed,
    indefinite) with FP32 factors at eps = 1e-6 and the operation-internal
    truncations at eps / 100: FP64 GMRES(30) reaches 1e-8 in a few tens of
    applications (14-15 measured) for each of two right-hand sides."""
    n = 64
    coef = problem("helmholtz", n)
    F = rhs_normal(n ** 3, nrhs=2)
    A = operator_from_coef(coef)
    fac = _factor(coef, eps=1e-6, leaf=64, precision="fp32", inner_eps_ratio=0.01)
    for j in range(2):
        f = np.ascontiguousarray(F[:, j])
        x, info = fac.solve_refined(torch.from_numpy(f).to(DEV), tol=1e-8, method="gmres", maxit=60,
                                    raise_on_fail=False)
        r = float(relres(A, x.cpu().numpy(), f))
        print(f"helmholtz n=64 rhs {j}: {info['iterations']} GMRES applications, relres {r:.2e}", flush=True)
        assert info["converged"] and r <= 1.01e-8
    fac.free()
