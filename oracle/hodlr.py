"""Block-wise truncation T(.) to the weak-admissibility format (oracle).

Weak admissibility (Section 2.1.1): the (1,2) and (2,1) blocks of every node
of the cluster tree are single low-rank blocks and the (1,1), (2,2) blocks
recurse; the leaves are dense.  Every off-diagonal block is compressed with a
singular value decomposition (Section 2.1: compression by SVD) at a relative
accuracy (Section 3.1).  Reading of the accuracy criterion, which the paper
leaves to its library: block-wise relative in the spectral norm, i.e. keep the
singular values sigma_i > eps * sigma_1 of that block; eps = 0 keeps the block
unchanged (exact mode).
"""
import numpy as np
import scipy.linalg as sla


def truncate_block(B, eps):
    """Best rank-k approximation keeping sigma_i > eps * sigma_1; returns (B_k, k)."""
    if B.size == 0:
        return B.copy(), 0
    if eps == 0.0:
        return B.copy(), int(min(B.shape))
    U, s, Vt = sla.svd(B, full_matrices=False, lapack_driver="gesvd")
    if s[0] == 0.0:
        return np.zeros_like(B), 0
    k = int(np.count_nonzero(s > eps * s[0]))
    return (U[:, :k] * s[:k]) @ Vt[:k], k


def hodlr_truncate(A, tree, eps):
    """T(A): truncate every off-diagonal block of the HODLR partition of A.

    ``A`` is dense M x M in cluster order.  Returns (T(A), ranks) where
    ranks[d] lists, for depth d, the ranks of the (1,2) and (2,1) blocks of
    each node in order (2 ** (d + 1) entries).
    """
    out = np.array(A, dtype=np.float64, copy=True)
    ranks = []
    for d in range(tree.L):
        rd = []
        for b in range(2 ** d):
            s1 = tree.seg_slice(d + 1, 2 * b)
            s2 = tree.seg_slice(d + 1, 2 * b + 1)
            out[s1, s2], k12 = truncate_block(A[s1, s2], eps)
            out[s2, s1], k21 = truncate_block(A[s2, s1], eps)
            rd.extend([k12, k21])
        ranks.append(rd)
    return out, ranks


def hodlr_words(tree, ranks):
    """Words stored by the HODLR form: dense leaves plus U and V of every block."""
    words = sum(size * size for _, size in tree.segs[tree.L])
    for d in range(tree.L):
        for s, k in enumerate(ranks[d]):
            _, rows = tree.segs[d + 1][s]
            _, cols = tree.segs[d + 1][s ^ 1]
            words += k * (rows + cols)
    return words
