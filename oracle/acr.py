"""Dense block cyclic reduction with HODLR truncation (oracle).

Follows Section 3 of the paper: the plane blocks of the block-tridiagonal
matrix (Eq. originalMatrix) are approximated block-wise (Algorithm 1, first
step), then the red/black elimination of Eq. elim runs level by level
(Algorithm 1) with the truncation T(.) of ``hodlr.hodlr_truncate`` applied to
every block an operation produces, and the solution is recovered by
Algorithm 2 / Eq. all_backSubs.

Blocks are kept dense (M x M, in cluster order) and a block that is still a
diagonal (the level-0 E_k and F_k of a 7-point stencil) is kept as its
diagonal.  With a 27-point stencil E_k and F_k are 9-point plane operators;
Eq. elim is written for general blocks, and they are approximated like D_k at
level 0.  Missing couplings
(E of the first plane, F of the last plane of a level) are ``None``: the
terms that would use them are dropped, as Section 2.2.2 prescribes for the
last plane.

With eps = 0 every truncation is the identity and the procedure is block
Gaussian elimination of the red/black permuted system (Eq. schur_complement),
so the result is A^{-1} f.
"""
import numpy as np
import scipy.linalg as sla

from .cluster import ClusterTree, level_schedule
from .hodlr import hodlr_truncate
from .assemble import operator_from_coef, plane_blocks

# A block is None, ("diag", vector) or ("dense", matrix).


def _mul(a, b):
    if a is None or b is None:
        return None
    (ka, va), (kb, vb) = a, b
    if ka == "diag" and kb == "diag":
        return ("diag", va * vb)
    if ka == "diag":
        return ("dense", va[:, None] * vb)
    if kb == "diag":
        return ("dense", va * vb[None, :])
    return ("dense", va @ vb)


def _neg(a):
    return None if a is None else (a[0], -a[1])


def _dense(a, M):
    if a is None:
        return np.zeros((M, M))
    return np.diag(a[1]) if a[0] == "diag" else a[1]


def _apply(a, v):
    """Block times vector(s); ``None`` contributes zero."""
    if a is None:
        return 0.0
    return a[1].reshape((-1,) + (1,) * (v.ndim - 1)) * v if a[0] == "diag" else a[1] @ v


def _apply_t(a, v):
    if a is None:
        return 0.0
    return a[1].reshape((-1,) + (1,) * (v.ndim - 1)) * v if a[0] == "diag" else a[1].T @ v


class OracleACR:
    """Factorisation by ACR elimination; ``solve`` / ``solve_transpose`` reuse it.

    Parameters: coef (stencil array coef[7, nz, ny, nx] or coef[27, nz, ny, nx]),
    leaf size of the cluster tree, truncation tolerance eps (relative, per block).
    """

    def __init__(self, coef, leaf, eps):
        coef = np.asarray(coef, dtype=np.float64)
        ns, nz, ny, nx = coef.shape
        self.shape = (nz, ny, nx)
        self.M = nx * ny
        self.N = self.M * nz
        self.eps = float(eps)
        self.tree = ClusterTree(nx, ny, leaf)
        self.A = operator_from_coef(coef)
        D, E, F = plane_blocks(self.A, nx, ny, nz, diagonal=ns == 7)
        p = self.tree.perm
        self.ranks = []          # (level, name, plane, ranks-per-depth)
        T = self._T
        # Algorithm 1, first step: block-wise approximation A^(0) of A
        Dc = [T(("dense", d[np.ix_(p, p)]), 0, "D", k) for k, d in enumerate(D)]
        if ns == 7:
            Ec = [None if e is None else ("diag", e[p]) for e in E]
            Fc = [None if f is None else ("diag", f[p]) for f in F]
        else:
            Ec = [None if e is None else T(("dense", e[np.ix_(p, p)]), 0, "E", k) for k, e in enumerate(E)]
            Fc = [None if f is None else T(("dense", f[np.ix_(p, p)]), 0, "F", k) for k, f in enumerate(F)]
        self.levels = []
        sched, self.last_plane = level_schedule(nz)
        cur = {"D": Dc, "E": Ec, "F": Fc}
        for i, lev in enumerate(sched):
            alive, m = lev["alive"], len(lev["alive"])
            Dl = [cur["D"][q] for q in range(m)]
            El = [cur["E"][q] for q in range(m)]
            Fl = [cur["F"][q] for q in range(m)]
            G, X, Y = {}, {}, {}
            for q in lev["elim"]:
                G[q] = T(("dense", np.linalg.inv(Dl[q][1])), i, "G", alive[q])
                X[q] = T(_mul(G[q], El[q]), i, "X", alive[q])
                Y[q] = T(_mul(G[q], Fl[q]), i, "Y", alive[q])
            nD, nE, nF = [], [], []
            for q in lev["kept"]:
                nE.append(T(_neg(_mul(El[q], X[q - 1])), i + 1, "E", alive[q]))
                acc = _dense(Dl[q], self.M).copy()
                t1 = T(_mul(El[q], Y[q - 1]), i, "EY", alive[q])
                if t1 is not None:
                    acc -= _dense(t1, self.M)
                if q + 1 < m:
                    t2 = T(_mul(Fl[q], X[q + 1]), i, "FX", alive[q])
                    if t2 is not None:
                        acc -= _dense(t2, self.M)
                    nF.append(T(_neg(_mul(Fl[q], Y[q + 1])), i + 1, "F", alive[q]))
                else:
                    nF.append(None)
                nD.append(T(("dense", acc), i + 1, "D", alive[q]))
            self.levels.append({"alive": alive, "elim": lev["elim"], "kept": lev["kept"],
                                "G": G, "D": Dl, "E": El, "F": Fl})
            cur = {"D": nD, "E": nE, "F": nF}
        # Algorithm 2, first step: the last remaining plane
        self.G_last = T(("dense", np.linalg.inv(cur["D"][0][1])), len(sched), "G", self.last_plane)
        self.D_last = cur["D"][0]

    def _T(self, a, level, name, plane):
        """Truncation T(.) of a produced block; diagonals and None pass through."""
        if a is None or a[0] == "diag":
            return a
        out, ranks = hodlr_truncate(a[1], self.tree, self.eps)
        self.ranks.append((level, name, plane, ranks))
        return ("dense", out)

    # -- solves -----------------------------------------------------------
    def _to_planes(self, f):
        f = np.asarray(f, dtype=np.float64)
        tail = f.shape[1:]
        fp = f.reshape((self.shape[0], self.M) + tail)
        return fp[:, self.tree.perm].copy()

    def _from_planes(self, u):
        out = np.empty_like(u)
        out[:, self.tree.perm] = u
        return out.reshape((self.N,) + u.shape[2:])

    def reduced_rhs(self, f):
        """Right-hand sides f^(i) of every level (Eq. elim, last line), cluster order."""
        fw = self._to_planes(f)
        out = [fw.copy()]
        for lev in self.levels:
            al, m = lev["alive"], len(lev["alive"])
            g = {q: _apply(lev["G"][q], fw[al[q]]) for q in lev["elim"]}
            for q in lev["kept"]:
                fw[al[q]] = fw[al[q]] - _apply(lev["E"][q], g[q - 1])
                if q + 1 < m:
                    fw[al[q]] = fw[al[q]] - _apply(lev["F"][q], g[q + 1])
            out.append(fw.copy())
        return out

    def solve(self, f):
        """u = M^{-1} f by forward elimination of f (Eq. elim, last line) and
        back-substitution (Eq. all_backSubs); f is (N,) or (N, nrhs), natural order."""
        fw = self._to_planes(f)
        for lev in self.levels:
            al, m = lev["alive"], len(lev["alive"])
            g = {q: _apply(lev["G"][q], fw[al[q]]) for q in lev["elim"]}
            for q in lev["kept"]:
                fw[al[q]] = fw[al[q]] - _apply(lev["E"][q], g[q - 1])
                if q + 1 < m:
                    fw[al[q]] = fw[al[q]] - _apply(lev["F"][q], g[q + 1])
        u = np.zeros_like(fw)
        u[self.last_plane] = _apply(self.G_last, fw[self.last_plane])
        for lev in reversed(self.levels):
            al, m = lev["alive"], len(lev["alive"])
            for q in lev["elim"]:
                r = fw[al[q]].copy()
                if q - 1 >= 0:
                    r = r - _apply(lev["E"][q], u[al[q - 1]])
                if q + 1 < m:
                    r = r - _apply(lev["F"][q], u[al[q + 1]])
                u[al[q]] = _apply(lev["G"][q], r)
        return self._from_planes(u)

    def solve_transpose(self, f):
        """u = M^{-T} f with the same blocks: cyclic reduction of A^T, whose
        level blocks are (D_j^T, F_{j-1}^T, E_{j+1}^T)."""
        fw = self._to_planes(f)
        for lev in self.levels:
            al, m = lev["alive"], len(lev["alive"])
            g = {q: _apply_t(lev["G"][q], fw[al[q]]) for q in lev["elim"]}
            for q in lev["kept"]:
                fw[al[q]] = fw[al[q]] - _apply_t(lev["F"][q - 1], g[q - 1])
                if q + 1 < m:
                    fw[al[q]] = fw[al[q]] - _apply_t(lev["E"][q + 1], g[q + 1])
        u = np.zeros_like(fw)
        u[self.last_plane] = _apply_t(self.G_last, fw[self.last_plane])
        for lev in reversed(self.levels):
            al, m = lev["alive"], len(lev["alive"])
            for q in lev["elim"]:
                r = fw[al[q]].copy()
                if q - 1 >= 0:
                    r = r - _apply_t(lev["F"][q - 1], u[al[q - 1]])
                if q + 1 < m:
                    r = r - _apply_t(lev["E"][q + 1], u[al[q + 1]])
                u[al[q]] = _apply_t(lev["G"][q], r)
        return self._from_planes(u)

    def max_rank(self):
        return max((max(max(r) if r else 0 for r in rk) if rk else 0)
                   for _, _, _, rk in self.ranks) if self.ranks else 0


def dense_solve(coef, f):
    """Brute force: dense LU of the assembled matrix (tiny grids only)."""
    A = operator_from_coef(coef).toarray()
    return sla.solve(A, f)
