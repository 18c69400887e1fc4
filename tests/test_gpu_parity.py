"""GPU path through the C-ABI against the CPU FP64 oracle (same seeded inputs)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1701_00182_amd as acr  # noqa: E402
from oracle.acr import OracleACR  # noqa: E402
from oracle.assemble import operator_from_coef, relres  # noqa: E402
from workloads import problem, rhs_normal  # noqa: E402

# host-side bounds check of every launched task (raises instead of faulting)
os.environ.setdefault("ACR_CHECK", "1")
DEV = torch.device("cuda:0")


def _gpu(coef, **kw):
    return acr.Factor(torch.from_numpy(np.ascontiguousarray(coef)).to(DEV), **kw)


def _solve(fac, f, transpose=False):
    b = torch.from_numpy(np.ascontiguousarray(f.T if f.ndim == 2 else f)).to(DEV)
    x = fac.solve_transpose(b) if transpose else fac.solve(b)
    x = x.cpu().numpy()
    return x.T if f.ndim == 2 else x


@pytest.mark.parametrize("kind", ["poisson", "convdiff", "helmholtz"])
@pytest.mark.parametrize("n,leaf", [(4, 4), (5, 4), (6, 9), (8, 16), (8, 64), (7, 5)])
def test_exact_mode_matches_oracle(kind, n, leaf):
    print(f"case exact kind={kind} n={n} leaf={leaf}", flush=True)
    coef = problem(kind, n)
    f = rhs_normal(n ** 3, nrhs=2)
    fac = _gpu(coef, eps=0.0, leaf=leaf, precision="fp64")
    o = OracleACR(coef, leaf, 0.0)
    x = _solve(fac, f)
    ref = o.solve(f)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    xt = _solve(fac, f, transpose=True)
    reft = o.solve_transpose(f)
    assert np.linalg.norm(xt - reft) <= 1e-10 * np.linalg.norm(reft)
    fac.free()


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_truncated_fp64_config1_against_oracle(eps):
    """Poisson n = 16, leaf 32: both are eps-approximations of A^{-1} f; the
    residual stays within 5 eps and the two solutions differ by <= 20 eps."""
    n, leaf = 16, 32
    print(f"case truncated n={n} eps={eps}", flush=True)
    coef = problem("poisson", n)
    f = rhs_normal(n ** 3)
    fac = _gpu(coef, eps=eps, leaf=leaf, precision="fp64")
    x = _solve(fac, f)
    o = OracleACR(coef, leaf, eps)
    ref = o.solve(f)
    A = operator_from_coef(coef)
    assert float(relres(A, x, f)) <= 5 * eps
    assert np.linalg.norm(x - ref) <= 20 * eps * np.linalg.norm(ref)
    st = fac.stats()
    assert st["max_rank"] <= 2 * max(o.max_rank(), 1)
    fac.free()


def test_transpose_is_exact_adjoint_truncated():
    n, leaf = 12, 36
    coef = problem("convdiff", n)
    fac = _gpu(coef, eps=1e-3, leaf=leaf, precision="fp64")
    rng = np.random.default_rng(9)
    f, g = rng.standard_normal(n ** 3), rng.standard_normal(n ** 3)
    lhs = _solve(fac, g, transpose=True) @ f
    rhs = g @ _solve(fac, f)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    fac.free()


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("n,leaf,nrhs", [(8, 16, 5), (48, 64, 10)])
def test_multi_rhs_equals_single_solves(n, leaf, nrhs, transpose):
    """Several right-hand sides take the matrix-core path (segmented leaf
    products, split inner products); each column must equal its single-RHS
    solve (fused vector kernels), also for the transposed solve."""
    coef = problem("helmholtz" if n == 8 else "convdiff", n)
    f = rhs_normal(n ** 3, nrhs=nrhs)
    fac = _gpu(coef, eps=1e-3, leaf=leaf, precision="fp32")
    X = _solve(fac, f, transpose)
    for j in range(nrhs):
        xj = _solve(fac, np.ascontiguousarray(f[:, j]), transpose)
        assert np.linalg.norm(X[:, j] - xj) <= 1e-5 * np.linalg.norm(xj)
    fac.free()


@pytest.mark.parametrize("method", ["ir", "gmres", "cg"])
def test_fp32_refined_to_1e8(method):
    n, leaf = 16, 32
    coef = problem("poisson", n)
    f = rhs_normal(n ** 3)
    fac = _gpu(coef, eps=1e-4, leaf=leaf, precision="fp32")
    x, info = fac.solve_refined(torch.from_numpy(f).to(DEV), tol=1e-8, method=method)
    A = operator_from_coef(coef)
    assert info["converged"] and float(relres(A, x.cpu().numpy(), f)) <= 1e-8
    fac.free()


def test_gmres_convdiff_fp32_eps1e2_to_1e10():
    n, leaf = 16, 32
    coef = problem("convdiff", n)
    f = rhs_normal(n ** 3)
    fac = _gpu(coef, eps=1e-2, leaf=leaf, precision="fp32")
    x, info = fac.solve_refined(torch.from_numpy(f).to(DEV), tol=1e-10, method="gmres")
    A = operator_from_coef(coef)
    assert info["converged"] and float(relres(A, x.cpu().numpy(), f)) <= 1e-10
    fac.free()


@pytest.mark.parametrize("n", [32, 22])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gram_compression_matches_householder(prec, n, monkeypatch):
    """Blocks take the Gram compression path at this eps; it must agree with
    the Householder path (forced with ACR_GRAM=0) to the truncation level.
    n = 32 gives block sizes that are multiples of 32 (whole row groups and
    16-byte aligned columns); n = 22 gives odd block sizes (ragged row tails
    and columns read one element at a time)."""
    leaf, eps = 32, 1e-3
    coef = problem("convdiff", n)
    f = rhs_normal(n ** 3)
    A = operator_from_coef(coef)
    monkeypatch.setenv("ACR_GRAM", "1")
    fg = _gpu(coef, eps=eps, leaf=leaf, precision=prec)
    xg = _solve(fg, f)
    monkeypatch.setenv("ACR_GRAM", "0")
    fh = _gpu(coef, eps=eps, leaf=leaf, precision=prec)
    xh = _solve(fh, f)
    assert float(relres(A, xg, f)) <= 5 * eps
    assert float(relres(A, xh, f)) <= 5 * eps
    assert np.linalg.norm(xg - xh) <= 20 * eps * np.linalg.norm(xh)
    fg.free()
    fh.free()


@pytest.mark.parametrize("leaf", [16, 64])
@pytest.mark.parametrize("prec", ["fp32_bf16leaf", "fp32_fp16leaf"])
def test_lowp_leaf_variant(prec, leaf):
    """Leaf x leaf products on 16-bit matrix-core inputs (power-of-two panel
    scaling, FP32 accumulation): unit roundoff 2^-9 (BF16) / 2^-12 (FP16) is
    below the truncation level, so the unrefined residual stays within the
    FP32 form's bound, and FP64 GMRES still reaches 1e-10."""
    n, eps = 16, 1e-2
    coef = problem("convdiff", n)
    f = rhs_normal(n ** 3)
    A = operator_from_coef(coef)
    fr = _gpu(coef, eps=eps, leaf=leaf, precision="fp32")
    fl = _gpu(coef, eps=eps, leaf=leaf, precision=prec)
    r32 = float(relres(A, _solve(fr, f), f))
    rlo = float(relres(A, _solve(fl, f), f))
    assert rlo <= max(2.0 * r32, 5 * eps)
    x, info = fl.solve_refined(torch.from_numpy(f).to(DEV), tol=1e-10, method="gmres")
    assert info["converged"] and float(relres(A, x.cpu().numpy(), f)) <= 1e-10
    fr.free()
    fl.free()


@pytest.fixture(scope="module")
def convdiff20_oracle():
    n, leaf, eps = 20, 32, 1e-6
    coef = problem("convdiff", n)
    f = rhs_normal(n ** 3)
    return coef, f, OracleACR(coef, leaf, eps).solve(f)


@pytest.mark.parametrize("fused", ["0", "65536", "160000", "global"])
def test_svd_paths_agree(fused, monkeypatch, convdiff20_oracle):
    """The one-workgroup core SVD, the two-kernel path in LDS (pivoted QR,
    then scalar Jacobi sweeps on W^T) and the global-memory path (every core,
    blocked Jacobi sweeps on matrix cores) compute the same truncation: all
    give solutions within the eps bound of the oracle's (n = 20, FP64; eps small
    enough that stacked cores exceed 64 columns)."""
    leaf, eps = 32, 1e-6
    coef, f, xo = convdiff20_oracle
    A = operator_from_coef(coef)
    if fused == "global":
        monkeypatch.setenv("ACR_SVD_GLOBAL", "1")
    else:
        monkeypatch.setenv("ACR_FUSED_LDS", fused)
    fac = _gpu(coef, eps=eps, leaf=leaf, precision="fp64")
    x = _solve(fac, f)
    assert float(relres(A, x, f)) <= 5 * eps
    assert np.linalg.norm(x - xo) <= 20 * eps * np.linalg.norm(xo)
    fac.free()
