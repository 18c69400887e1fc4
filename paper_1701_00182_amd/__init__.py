"""Accelerated cyclic reduction (Chavez et al., Parallel Computing 2017) on MI355X.

Thin Python binding of the C library ``libacr.so`` (declared in include/acr.h).
Arguments are marshalled to the C entry points; every step of the solver runs
in the library's HIP kernels.  PyTorch provides device memory and the current
stream only.  Importing never loads the library; the first call does, and it
raises if the library has not been built (``python -m paper_1701_00182_amd.build``).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libacr.so")
_LIB = None

PREC = {"fp64": 0, "fp32": 1, "fp32_bf16leaf": 2, "fp32_fp16leaf": 3, "fp32_bf16": 4, "fp32_fp16": 5}
STATUS = {0: "success", 1: "invalid value", 2: "out of memory", 3: "HIP error",
          4: "singular", 5: "rank capacity", 6: "not converged", 7: "not supported"}


class AcrError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = STATUS.get(code, str(code))
        detail = ""
        if _LIB is not None:
            detail = _LIB.acr_last_error_message().decode(errors="replace")
        super().__init__(f"{where}: {msg}" + (f" ({detail})" if detail else ""))


class Options(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nplanes", ctypes.c_int32),
                ("eps", ctypes.c_double), ("leaf", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_eps_ratio", ctypes.c_double),
                ("alloc", ctypes.c_void_p), ("release", ctypes.c_void_p), ("alloc_ctx", ctypes.c_void_p),
                ("svd_fused_lds", ctypes.c_int32), ("stencil_points", ctypes.c_int32),
                ("gemm_tiles", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("svd_fused_lds", ctypes.c_int32), ("seconds", ctypes.c_double),
                ("tried", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("gemm_tiles", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("depth", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("avg_rank", ctypes.c_double), ("factor_bytes", ctypes.c_double),
                ("factor_seconds", ctypes.c_double), ("solve_bytes", ctypes.c_double),
                ("flops_gemm", ctypes.c_double), ("flops_qr", ctypes.c_double),
                ("flops_svd", ctypes.c_double), ("flops_inverse", ctypes.c_double),
                ("launches", ctypes.c_int64), ("level_max_rank", ctypes.c_int32 * 32),
                ("level_avg_rank", ctypes.c_double * 32)]


class Structure(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("depth", ctypes.c_int32), ("nodes", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("schedule_len", ctypes.c_int32), ("last_plane", ctypes.c_int32)]


class RefineOptions(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("tol", ctypes.c_double), ("transpose", ctypes.c_int32)]


class RefineResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("relres", ctypes.c_double), ("relres0", ctypes.c_double)]


EXPORTS = ("acr_options_default", "acr_factor", "acr_solve", "acr_solve_transpose", "acr_solve_noalloc", "acr_free",
           "acr_get_stats", "acr_solve_refined", "acr_residual", "acr_assemble_diffusion",
           "acr_kappa_gradient", "acr_status_string", "acr_plan_structure", "acr_get_structure",
           "acr_release_cached_memory")


def lib():
    """Load libacr.so (once) and declare the C signatures."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1701_00182_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.acr_options_default.argtypes = [ctypes.POINTER(Options)]
        L.acr_options_default.restype = None
        L.acr_factor.argtypes = [ctypes.POINTER(Options), vp, vp, ctypes.POINTER(vp)]
        L.acr_factor.restype = ctypes.c_int
        for fn in (L.acr_solve, L.acr_solve_transpose, L.acr_solve_noalloc):
            fn.argtypes = [vp, i32, vp, i64, vp, i64, vp]
            fn.restype = ctypes.c_int
        L.acr_free.argtypes = [vp]
        L.acr_free.restype = None
        L.acr_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.acr_get_stats.restype = ctypes.c_int
        L.acr_solve_refined.argtypes = [vp, ctypes.POINTER(RefineOptions), vp, vp, vp,
                                        ctypes.POINTER(RefineResult), ctypes.POINTER(dbl), i32]
        L.acr_solve_refined.restype = ctypes.c_int
        L.acr_residual.argtypes = [vp, vp, vp, vp, i32, vp]
        L.acr_residual.restype = ctypes.c_int
        L.acr_assemble_diffusion.argtypes = [i32, i32, i32, vp, vp, vp]
        L.acr_assemble_diffusion.restype = ctypes.c_int
        L.acr_kappa_gradient.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp]
        L.acr_kappa_gradient.restype = ctypes.c_int
        L.acr_status_string.argtypes = [ctypes.c_int]
        L.acr_status_string.restype = ctypes.c_char_p
        L.acr_autotune.argtypes = [ctypes.POINTER(Options), vp, i32, ctypes.c_char_p, vp,
                                    ctypes.POINTER(TuneResult)]
        L.acr_autotune.restype = ctypes.c_int
        p32 = ctypes.POINTER(ctypes.c_int32)
        L.acr_plan_structure.argtypes = [i32, i32, i32, i32, ctypes.POINTER(Structure)] + [p32] * 6
        L.acr_plan_structure.restype = ctypes.c_int
        L.acr_get_structure.argtypes = [vp, ctypes.POINTER(Structure)] + [p32] * 6
        L.acr_get_structure.restype = ctypes.c_int
        L.acr_last_error_message.argtypes = []
        L.acr_last_error_message.restype = ctypes.c_char_p
        L.acr_release_cached_memory.argtypes = []
        L.acr_release_cached_memory.restype = ctypes.c_size_t
        _LIB = L
    return _LIB


def _structure(call, where):
    """Two-call pattern of the structure queries: sizes, then the arrays."""
    import numpy as np
    info = Structure()
    _check(call(ctypes.byref(info), *([None] * 6)), where)
    arrs = [np.zeros(max(n, 1), dtype=np.int32) for n in
            (info.M, info.nodes, info.nodes, info.levels, info.schedule_len, info.schedule_len)]
    ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for a in arrs]
    _check(call(ctypes.byref(info), *ptrs), where)
    perm, noff, nsz, lsz, splane, selim = arrs
    sched, pos = [], 0
    for i in range(info.levels):
        m = int(lsz[i])
        sched.append({"alive": splane[pos:pos + m].tolist(), "elim": selim[pos:pos + m].tolist()})
        pos += m
    return {"M": info.M, "depth": info.depth, "perm": perm[:info.M], "node_offset": noff[:info.nodes],
            "node_size": nsz[:info.nodes], "schedule": sched, "last_plane": info.last_plane}


def release_cached_memory():
    """acr_release_cached_memory: free the device buffers the library keeps for
    reuse; returns the bytes released."""
    return int(lib().acr_release_cached_memory())


def plan_structure(nx, ny, nplanes, leaf):
    """Cluster tree, permutation and level schedule for these sizes (host only,
    acr_plan_structure): dict with M, depth, perm, node_offset / node_size (node
    (d, s) at index 2^d - 1 + s), schedule (per level the alive planes and a 0/1
    eliminated flag per plane) and last_plane."""
    L = lib()
    return _structure(lambda info, *a: L.acr_plan_structure(nx, ny, nplanes, leaf, info, *a), "acr_plan_structure")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(code, where):
    if code != 0:
        raise AcrError(code, where)


def _dev_f64(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _rhs_view(b, N):
    """(N,) or (nrhs, N) tensor -> (nrhs, pointer); column j of the C matrix is row j."""
    if b.dim() == 1:
        if b.numel() != N:
            raise ValueError("right-hand side has the wrong length")
        return 1
    if b.dim() != 2 or b.shape[1] != N:
        raise ValueError("right-hand sides must be shaped (nrhs, N)")
    return b.shape[0]


class Factor:
    """ACR factorisation of a 7-point operator given as coef[7, nz, ny, nx] or a
    27-point one given as coef[27, nz, ny, nx] (FP64, CUDA)."""

    def __init__(self, coef, eps=1e-6, leaf=64, precision="fp64", max_rank=0, inner_eps_ratio=1.0,
                 svd_fused_lds=0, gemm_tiles=0):
        L = lib()
        if coef.dim() != 4 or coef.shape[0] not in (7, 27):
            raise ValueError("coef must be shaped (7, nz, ny, nx) or (27, nz, ny, nx)")
        _dev_f64(coef, "coef")
        ns, nz, ny, nx = coef.shape
        o = Options()
        L.acr_options_default(ctypes.byref(o))
        o.nx, o.ny, o.nplanes = nx, ny, nz
        o.eps, o.leaf, o.max_rank = float(eps), int(leaf), int(max_rank)
        o.precision = PREC[precision]
        o.inner_eps_ratio = float(inner_eps_ratio)
        o.svd_fused_lds = int(svd_fused_lds)
        o.stencil_points = ns
        o.gemm_tiles = int(gemm_tiles)
        h = ctypes.c_void_p()
        _check(L.acr_factor(ctypes.byref(o), ctypes.c_void_p(coef.data_ptr()), _stream(), ctypes.byref(h)),
               "acr_factor")
        self._h = h
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.precision = precision

    def _solve(self, fn, b, out=None):
        nrhs = _rhs_view(b, self.N)
        _dev_f64(b, "b")
        x = torch.empty_like(b) if out is None else out
        _check(fn(self._h, nrhs, ctypes.c_void_p(b.data_ptr()), self.N, ctypes.c_void_p(x.data_ptr()),
                  self.N, _stream()), fn.__name__)
        return x

    def solve(self, b, out=None):
        return self._solve(lib().acr_solve, b, out)

    def solve_transpose(self, b, out=None):
        return self._solve(lib().acr_solve_transpose, b, out)

    def solve_noalloc(self, b, out):
        """acr_solve_noalloc: the solve with the library's fixed device scratch
        (allocates no device memory; `out` must be given)."""
        return self._solve(lib().acr_solve_noalloc, b, out)

    def solve_refined(self, b, tol=1e-8, method="gmres", restart=30, maxit=200, transpose=False,
                      history=64, raise_on_fail=True):
        _dev_f64(b, "b")
        if b.dim() != 1:
            raise ValueError("refined solves take one right-hand side")
        x = torch.empty_like(b)
        ro = RefineOptions({"ir": 0, "gmres": 1, "cg": 2}[method], restart, maxit, tol, 1 if transpose else 0)
        rr = RefineResult()
        hist = (ctypes.c_double * history)()
        code = lib().acr_solve_refined(self._h, ctypes.byref(ro), ctypes.c_void_p(b.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()), _stream(), ctypes.byref(rr), hist, history)
        info = {"iterations": rr.iterations, "converged": bool(rr.converged), "relres": rr.relres,
                "relres0": rr.relres0, "history": [hist[i] for i in range(min(history, rr.iterations + 1))]}
        if code != 0 and (raise_on_fail or code != 6):
            raise AcrError(code, "acr_solve_refined")
        return x, info

    def residual(self, x, b, transpose=False):
        _dev_f64(x, "x")
        _dev_f64(b, "b")
        r = torch.empty_like(b)
        _check(lib().acr_residual(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                  ctypes.c_void_p(r.data_ptr()), 1 if transpose else 0, _stream()), "acr_residual")
        return r

    def structure(self):
        """The structure this handle was factorised with (acr_get_structure; the
        permutation read back from the device); same dict as plan_structure."""
        L = lib()
        return _structure(lambda info, *a: L.acr_get_structure(self._h, info, *a), "acr_get_structure")

    def stats(self):
        st = Stats()
        _check(lib().acr_get_stats(self._h, ctypes.byref(st)), "acr_get_stats")
        out = {k: getattr(st, k) for k, _ in Stats._fields_ if not k.startswith("level_")}
        out["level_max_rank"] = list(st.level_max_rank)[: st.levels + 1]
        out["level_avg_rank"] = list(st.level_avg_rank)[: st.levels]
        return out

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().acr_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def assemble_diffusion(kappa):
    """coef[7, nz, ny, nx] of -div(kappa grad u) from nodal kappa (GPU kernel)."""
    _dev_f64(kappa, "kappa")
    nz, ny, nx = kappa.shape
    coef = torch.empty((7, nz, ny, nx), dtype=torch.float64, device=kappa.device)
    _check(lib().acr_assemble_diffusion(nx, ny, nz, ctypes.c_void_p(kappa.data_ptr()),
                                        ctypes.c_void_p(coef.data_ptr()), _stream()), "acr_assemble_diffusion")
    return coef


def kappa_gradient(kappa, u, lam):
    """-lam^T (dA/dkappa_c) u for every node c (GPU kernel)."""
    for t, n in ((kappa, "kappa"), (u, "u"), (lam, "lam")):
        _dev_f64(t, n)
    nz, ny, nx = kappa.shape
    g = torch.empty_like(kappa)
    _check(lib().acr_kappa_gradient(nx, ny, nz, ctypes.c_void_p(kappa.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                    ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(g.data_ptr()), _stream()),
           "acr_kappa_gradient")
    return g


def autotune(coef, eps=1e-6, precision="fp64", leaf=64, sample_planes=16, cache=None, max_rank=0,
             inner_eps_ratio=1.0):
    """Leaf size and core-SVD dispatch picked by timing a sample of the operator
    (acr_autotune); returns a dict with leaf, svd_fused_lds, seconds, tried,
    from_cache.  Pass leaf / svd_fused_lds on to Factor."""
    if coef.dim() != 4 or coef.shape[0] not in (7, 27):
        raise ValueError("coef must be shaped (7, nz, ny, nx) or (27, nz, ny, nx)")
    _dev_f64(coef, "coef")
    L = lib()
    ns, nz, ny, nx = coef.shape
    o = Options()
    L.acr_options_default(ctypes.byref(o))
    o.nx, o.ny, o.nplanes = nx, ny, nz
    o.stencil_points = ns
    o.eps, o.leaf, o.max_rank = float(eps), int(leaf), int(max_rank)
    o.precision = PREC[precision]
    o.inner_eps_ratio = float(inner_eps_ratio)
    r = TuneResult()
    path = None if cache is None else os.fsencode(cache)
    _check(L.acr_autotune(ctypes.byref(o), ctypes.c_void_p(coef.data_ptr()), int(sample_planes), path, _stream(),
                          ctypes.byref(r)), "acr_autotune")
    return {"leaf": r.leaf, "svd_fused_lds": r.svd_fused_lds, "seconds": r.seconds, "tried": r.tried,
            "from_cache": bool(r.from_cache), "gemm_tiles": r.gemm_tiles}


class ACRSolve(torch.autograd.Function):
    """u = A(kappa)^{-1} f with an adjoint backward pass.

    Forward: assemble the diffusion stencil, factorise, solve with FP64
    refinement.  Backward: refined transpose solve A^T lam = du (reusing the
    factors) and the per-node gradient kernel; returns (dkappa, lam).
    """

    @staticmethod
    def forward(ctx, kappa, f, eps=1e-4, leaf=64, precision="fp32", tol=1e-12):
        coef = assemble_diffusion(kappa.contiguous())
        fac = Factor(coef, eps=eps, leaf=leaf, precision=precision)
        u, info = fac.solve_refined(f.contiguous(), tol=tol)
        ctx.fac = fac
        ctx.tol = tol
        ctx.save_for_backward(kappa, u)
        ctx.info = info
        return u

    @staticmethod
    def backward(ctx, du):
        kappa, u = ctx.saved_tensors
        lam, _ = ctx.fac.solve_refined(du.contiguous(), tol=ctx.tol, transpose=True)
        gk = kappa_gradient(kappa, u, lam)
        ctx.fac.free()
        return gk, lam, None, None, None, None
