"""acr_solve_noalloc (the solve whose workspace is the library's fixed device
scratch) against acr_solve, through the C ABI: equal results on consecutive
calls (the second on a smaller problem, then back to the first handle, so the
scratch's task arrays are restored), no device allocation through the
handle's allocator, and a clear rejection of a workspace above the limit."""
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
SCRATCH_BYTES = 128 << 20

ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class _Counted:
    """A handle whose device allocations go through a counting callback."""

    def __init__(self, kind, n, leaf, eps, precision):
        self.count, self.live = [0], {}

        @ALLOC
        def alloc(nbytes, ctx, stream):
            self.count[0] += 1
            p = torch.cuda.caching_allocator_alloc(nbytes, device=0, stream=stream or 0)
            self.live[p] = nbytes
            return p

        @RELEASE
        def release(p, ctx, stream):
            self.live.pop(p)
            torch.cuda.caching_allocator_delete(p)

        self._cb = (alloc, release)
        self.coef = torch.from_numpy(problem(kind, n)).to(DEV)
        self.N = n ** 3
        L = acr.lib()
        o = acr.Options()
        L.acr_options_default(ctypes.byref(o))
        o.nx = o.ny = o.nplanes = n
        o.eps, o.leaf, o.precision = eps, leaf, acr.PREC[precision]
        o.alloc = ctypes.cast(alloc, ctypes.c_void_p)
        o.release = ctypes.cast(release, ctypes.c_void_p)
        self.h = ctypes.c_void_p()
        assert L.acr_factor(ctypes.byref(o), ctypes.c_void_p(self.coef.data_ptr()), _stream(),
                            ctypes.byref(self.h)) == 0

    def call(self, fn, B, X):
        nrhs = B.shape[0]
        return fn(self.h, nrhs, ctypes.c_void_p(B.data_ptr()), self.N, ctypes.c_void_p(X.data_ptr()), self.N,
                  _stream())

    def free(self):
        acr.lib().acr_free(self.h)
        assert self.live == {}


def _rhs(N, nrhs, seed):
    return torch.from_numpy(np.ascontiguousarray(rhs_normal(N, nrhs=nrhs, seed=seed).reshape(N, nrhs).T)).to(DEV)


def _check(x, ref, precision):
    # same kernels and launch order as acr_solve: equal to rounding (bitwise in
    # practice); the bound allows for a different summation order only
    tol = (1e-13 if precision == "fp64" else 1e-6) * float(ref.abs().max())
    assert float((x - ref).abs().max()) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_solve_equals_solve(precision):
    L = acr.lib()
    big = _Counted("convdiff", 16, 32, 1e-3, precision)
    small = _Counted("helmholtz", 12, 36, 1e-4, precision)
    calls = [(big, 3, 11), (small, 1, 12), (big, 3, 13), (small, 6, 14)]
    for hd, nrhs, seed in calls:
        print(f"case noalloc {precision} N={hd.N} nrhs={nrhs}", flush=True)
        B = _rhs(hd.N, nrhs, seed)
        ref = torch.empty_like(B)
        assert hd.call(L.acr_solve, B, ref) == 0
        torch.cuda.synchronize()
        before = hd.count[0]
        X = torch.full_like(B, float("nan"))
        assert hd.call(L.acr_solve_noalloc, B, X) == 0
        torch.cuda.synchronize()
        assert hd.count[0] == before, "acr_solve_noalloc allocated device memory"
        _check(X, ref, precision)
    # x aliasing b
    B = _rhs(small.N, 2, 15)
    ref = torch.empty_like(B)
    assert small.call(L.acr_solve, B, ref) == 0
    assert small.call(L.acr_solve_noalloc, B, B) == 0
    torch.cuda.synchronize()
    _check(B, ref, precision)
    big.free()
    small.free()


def test_noalloc_rejects_workspace_above_limit():
    """Right-hand sides whose vectors alone exceed the fixed scratch: a clear
    error, nothing launched (x keeps its contents)."""
    L = acr.lib()
    hd = _Counted("poisson", 16, 32, 1e-3, "fp64")
    nrhs = SCRATCH_BYTES // (hd.N * 8 * 2) + 1     # W and Ub alone exceed it
    B = torch.zeros((nrhs, hd.N), dtype=torch.float64, device=DEV)
    X = torch.full_like(B, 5.0)
    before = hd.count[0]
    assert hd.call(L.acr_solve_noalloc, B, X) == 1
    msg = L.acr_last_error_message().decode()
    assert "no-allocation scratch" in msg and str(SCRATCH_BYTES) in msg
    torch.cuda.synchronize()
    assert bool(torch.all(X == 5.0))
    assert hd.count[0] == before
    # the handle still solves afterwards, with and without the fixed scratch
    b = _rhs(hd.N, 1, 16)
    ref, x = torch.empty_like(b), torch.empty_like(b)
    assert hd.call(L.acr_solve, b, ref) == 0
    assert hd.call(L.acr_solve_noalloc, b, x) == 0
    torch.cuda.synchronize()
    _check(x, ref, "fp64")
    hd.free()
