"""Integer set-up of the path (planar bisection cluster tree, cluster
permutation, red/black level schedule; Section 2.1.1 and Section 2.2.2,
Eq. permuted_system / Eq. next_step): the library's host-side structure
(acr_plan_structure, no device work) equals the oracle's bit for bit."""
import numpy as np
import pytest

import paper_1701_00182_amd as acr
from oracle.cluster import ClusterTree, level_schedule

# (nx, ny, nplanes, leaf): the benchmark shapes and ragged ones
SHAPES = [(16, 16, 16, 32), (64, 64, 64, 64), (128, 128, 128, 128), (128, 128, 128, 64),
          (5, 7, 5, 4), (10, 6, 9, 4), (12, 12, 12, 36), (7, 3, 1, 4), (1, 9, 2, 2), (33, 17, 31, 5)]


def expected(nx, ny, nplanes, leaf):
    t = ClusterTree(nx, ny, leaf)
    off = np.array([o for d in range(t.L + 1) for (o, _) in t.segs[d]], dtype=np.int32)
    size = np.array([s for d in range(t.L + 1) for (_, s) in t.segs[d]], dtype=np.int32)
    levels, last = level_schedule(nplanes)
    sched = []
    for lev in levels:
        m = len(lev["alive"])
        elim = [1 if q in lev["elim"] else 0 for q in range(m)]
        assert [q for q in range(m) if not elim[q]] == lev["kept"]
        sched.append({"alive": lev["alive"], "elim": elim})
    return t, off, size, sched, last


def check_equal(got, nx, ny, nplanes, leaf):
    t, off, size, sched, last = expected(nx, ny, nplanes, leaf)
    assert got["M"] == nx * ny and got["depth"] == t.L
    np.testing.assert_array_equal(got["perm"], t.perm.astype(np.int32))
    np.testing.assert_array_equal(got["node_offset"], off)
    np.testing.assert_array_equal(got["node_size"], size)
    assert got["schedule"] == sched
    assert got["last_plane"] == last


@pytest.mark.parametrize("nx,ny,nplanes,leaf", SHAPES)
def test_plan_structure_equals_oracle(nx, ny, nplanes, leaf):
    check_equal(acr.plan_structure(nx, ny, nplanes, leaf), nx, ny, nplanes, leaf)


def test_paper_worked_example_schedule():
    """n = 8 planes: level 0 eliminates 0, 2, 4, 6 and keeps 1, 3, 5, 7; three
    levels leave plane 7 (the red/black example of Section 2.2.2)."""
    s = acr.plan_structure(4, 4, 8, 4)
    assert s["schedule"][0] == {"alive": list(range(8)), "elim": [1, 0] * 4}
    assert [lv["alive"] for lv in s["schedule"]] == [list(range(8)), [1, 3, 5, 7], [3, 7]]
    assert s["last_plane"] == 7


def test_single_point_split_rejected():
    with pytest.raises(acr.AcrError):
        acr.plan_structure(3, 3, 2, 0)
