"""Cluster tree of a plane and the cyclic-reduction level schedule (oracle).

Cluster tree (Sections 2.1.1 and 3.1: binary space partitioning of the
two-dimensional plane by planar bisection).  The paper fixes neither the split
rule nor the ordering, so the reading used here is:

* a box is split across its longer side (x on ties); the first half keeps
  ceil(side / 2) grid lines;
* the tree is complete: every box is split as long as some box of the same
  depth holds more than ``leaf`` points, so all leaves sit at one depth L;
* points are numbered leaf by leaf, first half before second half, and
  row-major (x fastest) inside a leaf.

Level schedule (Section 2.2.2, Eq. permuted_system and next_step): the planes
alive at a level are numbered 0..m-1; those at even positions are eliminated,
the odd ones are kept and renumbered 0..floor(m/2)-1; this repeats until one
plane is left.
"""
import numpy as np


def _split(box):
    x0, x1, y0, y1 = box
    w, h = x1 - x0, y1 - y0
    if w >= h:
        xm = x0 + (w + 1) // 2
        return (x0, xm, y0, y1), (xm, x1, y0, y1)
    ym = y0 + (h + 1) // 2
    return (x0, x1, y0, ym), (x0, x1, ym, y1)


def _size(box):
    return (box[1] - box[0]) * (box[3] - box[2])


class ClusterTree:
    """Complete bisection tree of an nx-by-ny plane.

    Attributes: ``L`` (leaf depth), ``boxes[d]`` (2**d boxes at depth d),
    ``segs[d]`` (list of (offset, size) of the boxes in cluster order) and
    ``perm`` (cluster position -> natural in-plane index j*nx + i).
    """

    def __init__(self, nx, ny, leaf):
        if nx < 1 or ny < 1 or leaf < 1:
            raise ValueError("nx, ny and leaf must be positive")
        self.nx, self.ny, self.leaf = nx, ny, leaf
        boxes = [[(0, nx, 0, ny)]]
        while max(_size(b) for b in boxes[-1]) > leaf:
            nxt = []
            for b in boxes[-1]:
                if _size(b) < 2:
                    raise ValueError("cluster tree would have to split a single point")
                nxt.extend(_split(b))
            boxes.append(nxt)
        self.boxes = boxes
        self.L = len(boxes) - 1
        self.M = nx * ny
        self.segs = []
        for level in boxes:
            off, segs = 0, []
            for b in level:
                segs.append((off, _size(b)))
                off += _size(b)
            self.segs.append(segs)
        perm = []
        for (x0, x1, y0, y1) in boxes[-1]:
            for j in range(y0, y1):
                for i in range(x0, x1):
                    perm.append(j * nx + i)
        self.perm = np.array(perm, dtype=np.int64)

    def seg_slice(self, d, s):
        off, size = self.segs[d][s]
        return slice(off, off + size)


def level_schedule(nplanes):
    """Per level: the alive planes (original indices) and elim/kept positions."""
    alive = list(range(nplanes))
    levels = []
    while len(alive) > 1:
        m = len(alive)
        levels.append({"alive": list(alive),
                       "elim": list(range(0, m, 2)),
                       "kept": list(range(1, m, 2))})
        alive = [alive[p] for p in range(1, m, 2)]
    return levels, alive[0]


def red_black_order(nplanes):
    """Plane order of the permuted system at the first level (even, then odd)."""
    return list(range(0, nplanes, 2)) + list(range(1, nplanes, 2))
