"""Pins of the oracle's integer structure: level schedule and cluster tree."""
import json
import os

import numpy as np
import pytest

from oracle.cluster import ClusterTree, level_schedule, red_black_order
from oracle.assemble import operator_from_coef, plane_blocks
from workloads import problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_red_black_worked_example():
    g = _golden("red_black_n8.json")
    assert red_black_order(g["nplanes"]) == g["first_level_order"]
    levels, last = level_schedule(g["nplanes"])
    assert len(levels) == g["levels"]
    first = levels[0]
    assert [first["alive"][p] for p in first["elim"]] == g["first_level_eliminated"]
    assert [first["alive"][p] for p in first["kept"]] == g["first_level_kept"]
    # kept planes renumbered sequentially: level 1 works on planes 1,3,5,7 as 0..3
    assert levels[1]["alive"] == g["first_level_kept"]
    assert last == 7


def test_concurrency_16_planes():
    g = _golden("concurrency_n16.json")
    levels, _ = level_schedule(g["nplanes"])
    assert [len(lv["elim"]) for lv in levels] == g["eliminated_per_level"]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 9, 12, 33])
def test_schedule_any_n(n):
    levels, last = level_schedule(n)
    assert len(levels) == (int(np.floor(np.log2(n))) if n > 1 else 0)
    seen = []
    for lv in levels:
        seen += [lv["alive"][p] for p in lv["elim"]]
        m = len(lv["alive"])
        assert lv["elim"] == list(range(0, m, 2)) and lv["kept"] == list(range(1, m, 2))
    assert sorted(seen + [last]) == list(range(n))


@pytest.mark.parametrize("nx,ny,leaf", [(16, 16, 32), (64, 64, 64), (128, 128, 64),
                                        (5, 7, 4), (12, 12, 36), (10, 6, 4)])
def test_cluster_tree_bijection_and_contiguity(nx, ny, leaf):
    t = ClusterTree(nx, ny, leaf)
    assert sorted(t.perm.tolist()) == list(range(nx * ny))
    for d in range(t.L + 1):
        segs = t.segs[d]
        assert len(segs) == 2 ** d
        assert segs[0][0] == 0 and sum(s for _, s in segs) == nx * ny
        for (o1, s1), (o2, _) in zip(segs, segs[1:]):
            assert o1 + s1 == o2
        if d < t.L:
            for b in range(2 ** d):
                assert segs[b][1] == t.segs[d + 1][2 * b][1] + t.segs[d + 1][2 * b + 1][1]
    assert max(s for _, s in t.segs[t.L]) <= leaf
    assert t.L == 0 or max(s for _, s in t.segs[t.L - 1]) > leaf
    # every leaf is a rectangle of the grid, numbered row-major
    for (x0, x1, y0, y1), (off, size) in zip(t.boxes[t.L], t.segs[t.L]):
        pts = t.perm[off:off + size]
        exp = [j * nx + i for j in range(y0, y1) for i in range(x0, x1)]
        assert pts.tolist() == exp


def test_config_leaf_boxes():
    # n = 16, leaf 32 -> 4 x 8 leaves at depth 3; n = 64 / 128, leaf 64 -> 8 x 8
    t = ClusterTree(16, 16, 32)
    assert t.L == 3 and all((b[1] - b[0], b[3] - b[2]) == (4, 8) for b in t.boxes[3])
    t = ClusterTree(64, 64, 64)
    assert t.L == 6 and all((b[1] - b[0], b[3] - b[2]) == (8, 8) for b in t.boxes[6])
    t = ClusterTree(128, 128, 64)
    assert t.L == 8


def test_level0_cut_ranks():
    """Off-diagonal blocks of the exact plane operator have rank = cut length."""
    n = 16
    coef = problem("poisson", n)
    A = operator_from_coef(coef)
    D, _, _ = plane_blocks(A, n, n, n)
    t = ClusterTree(n, n, 32)
    Dc = D[3][np.ix_(t.perm, t.perm)]
    expected = {0: 16, 1: 8, 2: 8}
    for d in range(t.L):
        for b in range(2 ** d):
            s1, s2 = t.seg_slice(d + 1, 2 * b), t.seg_slice(d + 1, 2 * b + 1)
            assert np.linalg.matrix_rank(Dc[s1, s2]) == expected[d]
            assert np.linalg.matrix_rank(Dc[s2, s1]) == expected[d]


def test_single_point_split_rejected():
    with pytest.raises(ValueError):
        ClusterTree(3, 1, 1)
