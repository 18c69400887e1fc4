"""Boundary paths of the C ABI that the solver tests do not reach: the
allocator callback (and its failure), leading dimensions above N, x aliasing b,
calls on a handle from two streams, and run-to-run determinism."""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1701_00182_amd as acr  # noqa: E402
from workloads import problem, rhs_normal  # noqa: E402

os.environ.setdefault("ACR_CHECK", "1")
DEV = torch.device("cuda:0")

ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def _opts(coef, eps, leaf, precision):
    o = acr.Options()
    acr.lib().acr_options_default(ctypes.byref(o))
    _, nz, ny, nx = coef.shape
    o.nx, o.ny, o.nplanes = nx, ny, nz
    o.eps, o.leaf, o.precision = eps, leaf, acr.PREC[precision]
    return o


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_allocator_callback_used_and_balanced():
    """Every device allocation goes through the callback (torch's caching
    allocator here), is released by acr_free, and the result equals the
    default allocator's."""
    n, leaf = 12, 36
    coef = torch.from_numpy(problem("convdiff", n)).to(DEV)
    b = torch.from_numpy(rhs_normal(n ** 3)).to(DEV)
    live = {}

    @ALLOC
    def alloc(nbytes, ctx, stream):
        p = torch.cuda.caching_allocator_alloc(nbytes, device=0, stream=stream or 0)
        live[p] = nbytes
        return p

    @RELEASE
    def release(p, ctx, stream):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    L = acr.lib()
    o = _opts(coef, 1e-3, leaf, "fp32")
    o.alloc = ctypes.cast(alloc, ctypes.c_void_p)
    o.release = ctypes.cast(release, ctypes.c_void_p)
    h = ctypes.c_void_p()
    assert L.acr_factor(ctypes.byref(o), ctypes.c_void_p(coef.data_ptr()), _stream(), ctypes.byref(h)) == 0
    assert len(live) > 0
    x = torch.empty_like(b)
    assert L.acr_solve(h, 1, ctypes.c_void_p(b.data_ptr()), n ** 3, ctypes.c_void_p(x.data_ptr()), n ** 3,
                       _stream()) == 0
    L.acr_free(h)
    assert live == {}
    ref = acr.Factor(coef, eps=1e-3, leaf=leaf, precision="fp32")
    xr = ref.solve(b)
    torch.cuda.synchronize()
    assert torch.equal(x, xr)
    ref.free()


def test_allocator_callback_null_is_out_of_memory():
    n, leaf = 8, 16
    coef = torch.from_numpy(problem("poisson", n)).to(DEV)
    calls = [0]

    @ALLOC
    def alloc(nbytes, ctx, stream):
        calls[0] += 1
        return None

    @RELEASE
    def release(p, ctx, stream):
        pass

    L = acr.lib()
    o = _opts(coef, 1e-3, leaf, "fp64")
    o.alloc = ctypes.cast(alloc, ctypes.c_void_p)
    o.release = ctypes.cast(release, ctypes.c_void_p)
    h = ctypes.c_void_p(1234)
    code = L.acr_factor(ctypes.byref(o), ctypes.c_void_p(coef.data_ptr()), _stream(), ctypes.byref(h))
    assert code == 2 and not h.value and calls[0] >= 1
    assert b"NULL" in L.acr_last_error_message()


def test_allocator_callback_fails_midway():
    """A callback that fails after some successful allocations: the factorisation
    returns out-of-memory and every allocation it made is released."""
    n, leaf = 12, 16
    coef = torch.from_numpy(problem("convdiff", n)).to(DEV)
    live, count = {}, [0]

    @ALLOC
    def alloc(nbytes, ctx, stream):
        count[0] += 1
        if count[0] > 3:
            return None
        p = torch.cuda.caching_allocator_alloc(nbytes, device=0, stream=stream or 0)
        live[p] = nbytes
        return p

    @RELEASE
    def release(p, ctx, stream):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    L = acr.lib()
    o = _opts(coef, 1e-3, leaf, "fp32")
    o.alloc = ctypes.cast(alloc, ctypes.c_void_p)
    o.release = ctypes.cast(release, ctypes.c_void_p)
    h = ctypes.c_void_p()
    assert L.acr_factor(ctypes.byref(o), ctypes.c_void_p(coef.data_ptr()), _stream(), ctypes.byref(h)) == 2
    assert not h.value
    assert live == {}


@pytest.mark.parametrize("nrhs", [1, 3, 9])
@pytest.mark.parametrize("transpose", [False, True])
def test_leading_dimensions_above_n(nrhs, transpose):
    n, leaf = 10, 20
    N = n ** 3
    coef = torch.from_numpy(problem("convdiff", n)).to(DEV)
    fac = acr.Factor(coef, eps=1e-4, leaf=leaf, precision="fp32")
    B = torch.from_numpy(rhs_normal(N, nrhs=nrhs).T.copy()).to(DEV)
    ref = fac.solve_transpose(B) if transpose else fac.solve(B)
    ldb, ldx = N + 5, N + 13
    Bp = torch.full((nrhs, ldb), float("nan"), dtype=torch.float64, device=DEV)
    Bp[:, :N] = B
    Xp = torch.full((nrhs, ldx), -7.0, dtype=torch.float64, device=DEV)
    fn = acr.lib().acr_solve_transpose if transpose else acr.lib().acr_solve
    assert fn(fac._h, nrhs, ctypes.c_void_p(Bp.data_ptr()), ldb, ctypes.c_void_p(Xp.data_ptr()), ldx,
              _stream()) == 0
    torch.cuda.synchronize()
    assert torch.equal(Xp[:, :N].reshape(ref.shape), ref)
    assert torch.all(Xp[:, N:] == -7.0)   # padding untouched
    fac.free()


@pytest.mark.parametrize("nrhs", [1, 6])
def test_x_aliases_b(nrhs):
    n, leaf = 10, 20
    N = n ** 3
    coef = torch.from_numpy(problem("helmholtz", n)).to(DEV)
    fac = acr.Factor(coef, eps=1e-4, leaf=leaf, precision="fp64")
    B = torch.from_numpy(rhs_normal(N, nrhs=nrhs).T.copy()).to(DEV)
    ref = fac.solve(B)
    Y = B.clone()
    assert acr.lib().acr_solve(fac._h, nrhs, ctypes.c_void_p(Y.data_ptr()), N, ctypes.c_void_p(Y.data_ptr()), N,
                               _stream()) == 0
    torch.cuda.synchronize()
    assert torch.equal(Y, ref)
    fac.free()


def test_two_streams_on_one_handle():
    """Solves issued on two streams in turn: each call waits for the handle's
    previous one (shared solve buffers), so every result equals the reference."""
    n, leaf = 12, 36
    N = n ** 3
    coef = torch.from_numpy(problem("convdiff", n)).to(DEV)
    fac = acr.Factor(coef, eps=1e-3, leaf=leaf, precision="fp32")
    bs = [torch.from_numpy(rhs_normal(N, seed=s)).to(DEV) for s in range(6)]
    refs = [fac.solve(b) for b in bs]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for i, b in enumerate(bs):
        with torch.cuda.stream(s1 if i % 2 == 0 else s2):
            outs.append(fac.solve(b))
    torch.cuda.synchronize()
    for x, r in zip(outs, refs):
        assert torch.equal(x, r)
    fac.free()


@pytest.mark.parametrize("precision,eps", [("fp32", 1e-2), ("fp64", 1e-4)])
def test_factor_and_solve_bitwise_deterministic(precision, eps):
    n, leaf = 16, 32
    N = n ** 3
    coef = torch.from_numpy(problem("convdiff", n)).to(DEV)
    B = torch.from_numpy(rhs_normal(N, nrhs=4).T.copy()).to(DEV)
    out = []
    for _ in range(2):
        fac = acr.Factor(coef, eps=eps, leaf=leaf, precision=precision)
        out.append((fac.solve(B), fac.solve(B[0].contiguous()), fac.stats()))
        fac.free()
    torch.cuda.synchronize()
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
    for k in ("max_rank", "avg_rank", "factor_bytes", "flops_gemm", "flops_svd"):
        assert out[0][2][k] == out[1][2][k], k


def test_narrow_gemm_tiles_bitwise_equal(monkeypatch):
    """FP32 products with outputs at most 32 columns wide run in 128 x 32 tiles;
    the K loop accumulates in the same order as the 64 x 64 tiles, so the
    factorisation and its solve are bitwise equal with the narrow kernel
    switched off (ACR_GEMM_NARROW=0)."""
    n, leaf = 24, 128
    coef = torch.from_numpy(problem("convdiff", n)).to(DEV)
    b = torch.from_numpy(rhs_normal(n ** 3)).to(DEV)
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("ACR_GEMM_NARROW", flag)
        fac = acr.Factor(coef, eps=1e-2, leaf=leaf, precision="fp32")
        out.append((fac.solve(b), fac.stats()))
        fac.free()
    torch.cuda.synchronize()
    assert torch.equal(out[0][0], out[1][0])
    assert out[0][1]["max_rank"] == out[1][1]["max_rank"]


@pytest.mark.parametrize("n,leaf,eps", [(24, 128, 1e-2), (32, 64, 1e-4), (16, 32, 1e-3)])
def test_register_pchol_bitwise_equals_lds_kernel(n, leaf, eps, monkeypatch):
    """The register-tiled pivoted Cholesky (no swaps; 5 x 5 tiles on 512 or
    1024 threads by order, 8 x 8 on 512 with ACR_PCHOL_TILES=512, 5 x 5 on
    1024 for every mid order with ACR_PCHOL_TILES=1024) takes the same pivots
    and does the same arithmetic per element as the right-looking LDS kernel
    (ACR_PCHOL_LDS=1), so the factorisation and its solve are bitwise equal."""
    coef = torch.from_numpy(problem("convdiff", n)).to(DEV)
    b = torch.from_numpy(rhs_normal(n ** 3)).to(DEV)
    out = []
    for lds, tiles in (("0", ""), ("0", "512"), ("0", "1024"), ("1", "")):
        monkeypatch.setenv("ACR_PCHOL_LDS", lds)
        monkeypatch.setenv("ACR_PCHOL_TILES", tiles)
        fac = acr.Factor(coef, eps=eps, leaf=leaf, precision="fp32")
        out.append((fac.solve(b), fac.stats()))
        fac.free()
    torch.cuda.synchronize()
    for o in out[1:]:
        assert out[0][1]["max_rank"] == o[1]["max_rank"]
        assert torch.equal(out[0][0], o[0])


def test_cached_device_memory_reused_and_released():
    """Freed handles leave their device buffers in the library's cache; the
    next factorisation of the same operator takes them over and gives bitwise
    the same factors and solution; acr_release_cached_memory empties the
    cache."""
    n, leaf = 16, 32
    coef = torch.from_numpy(problem("convdiff", n)).to(DEV)
    b = torch.from_numpy(rhs_normal(n ** 3)).to(DEV)
    acr.release_cached_memory()
    out = []
    for _ in range(3):
        fac = acr.Factor(coef, eps=1e-2, leaf=leaf, precision="fp32")
        out.append((fac.solve(b), fac.stats()["factor_bytes"]))
        fac.free()
    torch.cuda.synchronize()
    for o in out[1:]:
        assert torch.equal(out[0][0], o[0]) and o[1] == out[0][1]
    assert acr.release_cached_memory() > 0
    assert acr.release_cached_memory() == 0
