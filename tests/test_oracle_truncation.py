"""Pins of the block truncation T(.): Eckart-Young and exact HODLR reconstruction."""
import numpy as np
import pytest

from oracle.cluster import ClusterTree
from oracle.hodlr import truncate_block, hodlr_truncate, hodlr_words


def _with_spectrum(m, n, sigma, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, len(sigma))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(sigma))))
    return (U * sigma) @ V.T


@pytest.mark.parametrize("eps", [1e-1, 1e-3, 1e-6])
def test_eckart_young(eps):
    sigma = np.logspace(0, -9, 20) * 7.0   # no value sits on a threshold
    B = _with_spectrum(40, 33, sigma, 1)
    Bk, k = truncate_block(B, eps)
    assert k == int(np.count_nonzero(sigma > eps * sigma[0]))
    err = np.linalg.norm(B - Bk, 2)
    assert abs(err - sigma[k]) <= 1e-12 * sigma[0]
    assert err <= eps * sigma[0]
    assert np.linalg.matrix_rank(Bk, tol=1e-13 * sigma[0]) == k


def test_zero_block_and_exact_mode():
    Z = np.zeros((5, 4))
    assert truncate_block(Z, 1e-3)[1] == 0
    B = np.arange(12.0).reshape(3, 4)
    out, k = truncate_block(B, 0.0)
    assert k == 3 and np.array_equal(out, B)


def test_hodlr_exact_ranks_roundtrip():
    """A matrix built with known block ranks is reproduced and its ranks reported."""
    t = ClusterTree(8, 8, 4)
    rng = np.random.default_rng(2)
    A = np.zeros((t.M, t.M))
    want = []
    for d in range(t.L):
        rd = []
        for b in range(2 ** d):
            s1, s2 = t.seg_slice(d + 1, 2 * b), t.seg_slice(d + 1, 2 * b + 1)
            for r, c in ((s1, s2), (s2, s1)):
                k = int(rng.integers(1, min(4, r.stop - r.start) + 1))
                A[r, c] = rng.standard_normal((r.stop - r.start, k)) @ rng.standard_normal((k, c.stop - c.start))
                rd.append(k)
        want.append(rd)
    for off, size in t.segs[t.L]:
        A[off:off + size, off:off + size] = rng.standard_normal((size, size))
    out, ranks = hodlr_truncate(A, t, 1e-10)
    assert ranks == want
    assert np.max(np.abs(out - A)) <= 1e-12 * np.max(np.abs(A))
    # words: leaves plus U and V of each block
    words = hodlr_words(t, ranks)
    assert words == sum(s * s for _, s in t.segs[t.L]) + sum(
        k * (t.segs[d + 1][s][1] + t.segs[d + 1][s ^ 1][1])
        for d in range(t.L) for s, k in enumerate(ranks[d]))


def test_hodlr_truncate_blockwise_error():
    """Each off-diagonal block of T(A) is that block's Eckart-Young truncation."""
    t = ClusterTree(8, 4, 4)
    rng = np.random.default_rng(3)
    x = np.linspace(0, 1, t.M)
    A = 1.0 / (1.0 + 40.0 * np.abs(x[:, None] - x[None, :])) + 0.01 * rng.standard_normal((t.M, t.M))
    eps = 1e-2
    out, ranks = hodlr_truncate(A, t, eps)
    for d in range(t.L):
        for b in range(2 ** d):
            s1, s2 = t.seg_slice(d + 1, 2 * b), t.seg_slice(d + 1, 2 * b + 1)
            for r, c in ((s1, s2), (s2, s1)):
                sv = np.linalg.svd(A[r, c], compute_uv=False)
                k = int(np.count_nonzero(sv > eps * sv[0]))
                err = np.linalg.norm(A[r, c] - out[r, c], 2)
                assert abs(err - (sv[k] if k < len(sv) else 0.0)) <= 1e-12 * sv[0]
    for off, size in t.segs[t.L]:
        assert np.array_equal(out[off:off + size, off:off + size], A[off:off + size, off:off + size])
