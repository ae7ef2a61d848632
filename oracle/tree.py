"""ORACLE -- test infrastructure only.

Plain reference for the integer work of the complex-coordinate FMM: the
adaptive tree on the real parts of the points and the interaction Lists 1-4
(Sec. 6.1 tree generation, Sec. 6.2 list generation).  Written for clarity,
not speed: every list is derived from its definition by a descent from the
root, without relying on the level restriction.

Conventions (the readings of the paper this reference fixes):

* Root cube: centre at the midpoint of the real bounding box, side
  D = max extent * (1 + 2^-20) (D = 1 if all real parts coincide);
  lo = mid - D/2.
* Integer coordinates q_d = min(max(floor((Re x_d - lo_d) * 2^B / D), 0), 2^B - 1),
  B = 31 bits per coordinate in 2D and 21 in 3D.  A point on a box face
  goes to the upper box.
* Morton key: bit b of q_d is key bit b*dim + d.  Points are sorted by key,
  ties by original index (stable sort).
* A box holding more than N_s points splits (Sec. 6.1) unless it is at level B;
  only non-empty children are created.
* Near zone (the separation reading, Sec. 6.2): boxes a, b are near iff
  ||x_a - x_b||_inf <= (k/2)(w_a + w_b) for the real centres x and widths w.
  Colleagues are same-level near boxes.
* Level restriction (Sec. 6.1): two leaves whose levels differ by two or more
  are never near; the coarser one is split until none is (the coarsest such
  refinement, which is unique).
* List 1 (leaf b):  leaves near b, b included.
  List 2 (any b):   same-level boxes not near b whose parent is near b's parent.
  List 3 (leaf b):  finer boxes not near b whose parent is near b.
  List 4:           the transpose of List 3.
* Boxes are numbered in (level, key) order; each list row is sorted.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def key_bits(dim: int) -> int:
    return 31 if dim == 2 else 21


def root_cube(re: np.ndarray):
    """lo[d], D, scale = 2^B / D from the real parts re[n, dim]."""
    dim = re.shape[1]
    B = key_bits(dim)
    mn = re.min(axis=0)
    mx = re.max(axis=0)
    mid = (mn + mx) * 0.5
    ext = float(np.max(mx - mn))
    D = ext * (1.0 + 2.0 ** -20) if ext > 0.0 else 1.0
    lo = mid - 0.5 * D
    scale = float(2.0 ** B) / D
    return lo, D, scale


def morton_keys(re: np.ndarray, lo, scale) -> np.ndarray:
    dim = re.shape[1]
    B = key_bits(dim)
    top = (1 << B) - 1
    q = np.floor((re - lo[None, :]) * scale)
    q = np.clip(q, 0, top).astype(np.uint64)
    key = np.zeros(re.shape[0], dtype=np.uint64)
    for b in range(B):
        for d in range(dim):
            bit = (q[:, d] >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(b * dim + d)
    return key


def deinterleave(prefix: int, level: int, dim: int):
    c = [0] * dim
    for b in range(level):
        for d in range(dim):
            c[d] |= ((prefix >> (b * dim + d)) & 1) << b
    return tuple(c)


@dataclass
class Tree:
    dim: int
    nbits: int
    lo: np.ndarray
    D: float
    perm: np.ndarray       # int64[n]: sorted position -> original index
    keys: np.ndarray       # uint64[n] sorted keys
    level: np.ndarray      # int32[nbox]
    prefix: np.ndarray     # uint64[nbox] key prefix at the box's level
    parent: np.ndarray     # int32[nbox] (-1 for the root)
    child0: np.ndarray     # int32[nbox] first child (-1 for a leaf)
    nchild: np.ndarray     # int32[nbox]
    pbeg: np.ndarray       # int32[nbox] first point (sorted order)
    pend: np.ndarray       # int32[nbox] one past the last point
    lists: dict            # name -> (offsets int32[nbox+1], idx int32[...])

    @property
    def nbox(self) -> int:
        return int(self.level.shape[0])

    def is_leaf(self, b) -> bool:
        return self.nchild[b] == 0

    def coords(self, b):
        return deinterleave(int(self.prefix[b]), int(self.level[b]), self.dim)

    def center_units(self, b):
        """Real centre in integer units of D / 2^(B+1)."""
        s = 1 << (self.nbits - int(self.level[b]))
        return tuple((2 * c + 1) * s for c in self.coords(b))

    def width_units(self, b) -> int:
        return 1 << (self.nbits + 1 - int(self.level[b]))

    def real_center(self, b) -> np.ndarray:
        l = int(self.level[b])
        h = self.D * 2.0 ** (-(l + 1))
        c = np.array(self.coords(b), dtype=np.float64)
        return self.lo + (2.0 * c + 1.0) * h


def _near_units(ca, wa, cb, wb, k) -> bool:
    return all(2 * abs(x - y) <= k * (wa + wb) for x, y in zip(ca, cb))


def build_tree(points: np.ndarray, leaf_size: int, sep: int = 1, top_level: int = 0) -> Tree:
    """Adaptive level-restricted tree of complex points (uses Re only)."""
    pts = np.asarray(points)
    dim = pts.shape[1]
    re = np.ascontiguousarray(pts.real, dtype=np.float64)
    B = key_bits(dim)
    lo, D, scale = root_cube(re)
    keys = morton_keys(re, lo, scale)
    perm = np.argsort(keys, kind="stable").astype(np.int64)
    skeys = keys[perm]
    n = skeys.shape[0]

    # box dictionary: (level, prefix) -> [pbeg, pend]; children created lazily
    boxes = {(0, 0): [0, n]}
    children = {}

    def split(bk):
        lvl, pre = bk
        b0, b1 = boxes[bk]
        sh = np.uint64(dim * (B - lvl - 1))
        sub = (skeys[b0:b1] >> sh).astype(np.uint64)
        kids = []
        start = b0
        for i in range(b0 + 1, b1 + 1):
            if i == b1 or sub[i - b0] != sub[i - 1 - b0]:
                ck = (lvl + 1, int(sub[start - b0]))
                boxes[ck] = [start, i]
                kids.append(ck)
                start = i
        children[bk] = kids
        return kids

    # refinement by occupancy
    frontier = [(0, 0)]
    while frontier:
        nxt = []
        for bk in frontier:
            b0, b1 = boxes[bk]
            if b1 - b0 > leaf_size and bk[0] < B:
                nxt.extend(split(bk))
        frontier = nxt

    def geom(bk):
        lvl, pre = bk
        s = 1 << (B - lvl)
        c = tuple((2 * x + 1) * s for x in deinterleave(pre, lvl, dim))
        return c, 1 << (B + 1 - lvl)

    def near(a, b):
        ca, wa = geom(a)
        cb, wb = geom(b)
        return _near_units(ca, wa, cb, wb, sep)

    def near_leaves(b):
        out = []
        stack = [(0, 0)]
        while stack:
            a = stack.pop()
            if not near(a, b):
                continue
            if a in children:
                stack.extend(children[a])
            else:
                out.append(a)
        return out

    # level restriction: split coarse leaves near much finer leaves
    while True:
        leaves = [bk for bk in boxes if bk not in children]
        to_split = set()
        for b in leaves:
            for a in near_leaves(b):
                if a[0] <= b[0] - 2:
                    to_split.add(a)
        if not to_split:
            break
        for a in to_split:
            split(a)

    order = sorted(boxes.keys())
    index = {bk: i for i, bk in enumerate(order)}
    nb = len(order)
    level = np.array([bk[0] for bk in order], dtype=np.int32)
    prefix = np.array([bk[1] for bk in order], dtype=np.uint64)
    parent = np.full(nb, -1, dtype=np.int32)
    child0 = np.full(nb, -1, dtype=np.int32)
    nchild = np.zeros(nb, dtype=np.int32)
    pbeg = np.array([boxes[bk][0] for bk in order], dtype=np.int32)
    pend = np.array([boxes[bk][1] for bk in order], dtype=np.int32)
    for bk, kids in children.items():
        i = index[bk]
        ks = sorted(index[c] for c in kids)
        child0[i] = ks[0]
        nchild[i] = len(ks)
        assert ks == list(range(ks[0], ks[0] + len(ks)))
        for c in ks:
            parent[c] = i

    t = Tree(dim, B, lo, D, perm, skeys, level, prefix, parent, child0, nchild,
             pbeg, pend, {})
    t.lists = build_lists(t, sep, top_level)
    return t


def build_lists(t: Tree, sep: int, top_level: int = 0) -> dict:
    """Lists 1-4.  Boxes coarser than `top_level` carry no expansions: for the
    lists, any pair involving such a box counts as near, so far interactions
    start at `top_level` (List 2 there holds every non-near box of the level)."""
    nb = t.nbox
    cen = [t.center_units(b) for b in range(nb)]
    wid = [t.width_units(b) for b in range(nb)]

    def near(a, b):
        if t.level[a] < top_level or t.level[b] < top_level:
            return True
        return _near_units(cen[a], wid[a], cen[b], wid[b], sep)

    def kids(a):
        return range(t.child0[a], t.child0[a] + t.nchild[a]) if t.nchild[a] else range(0)

    def near_boxes(b):
        out = []
        stack = [0]
        while stack:
            a = stack.pop()
            if not near(a, b):
                continue
            out.append(a)
            stack.extend(kids(a))
        return out

    L1 = [[] for _ in range(nb)]
    L2 = [[] for _ in range(nb)]
    L3 = [[] for _ in range(nb)]
    L4 = [[] for _ in range(nb)]
    for b in range(nb):
        nbs = near_boxes(b)
        leaf = t.nchild[b] == 0
        if leaf:
            L1[b] = sorted(a for a in nbs if t.nchild[a] == 0)
            L3[b] = sorted(c for a in nbs if t.level[a] >= t.level[b]
                           for c in kids(a) if not near(c, b))
        p = t.parent[b]
        if p >= 0:
            pc = [a for a in near_boxes(p) if t.level[a] == t.level[p]]
            L2[b] = sorted(c for a in pc for c in kids(a) if not near(c, b))
    for b in range(nb):
        for c in L3[b]:
            L4[c].append(b)
    for b in range(nb):
        L4[b].sort()

    def csr(rows):
        off = np.zeros(nb + 1, dtype=np.int32)
        for i, r in enumerate(rows):
            off[i + 1] = off[i] + len(r)
        idx = np.array([x for r in rows for x in r], dtype=np.int32)
        return off, idx

    return {"L1": csr(L1), "L2": csr(L2), "L3": csr(L3), "L4": csr(L4)}


def complex_centers(t: Tree, points: np.ndarray) -> np.ndarray:
    """Complexified box centres x_b + i * mean of Im over the box's points (Sec. 6.1)."""
    pts = np.asarray(points)[t.perm]
    out = np.empty((t.nbox, t.dim), dtype=np.complex128)
    for b in range(t.nbox):
        im = pts[t.pbeg[b]:t.pend[b]].imag.mean(axis=0)
        out[b] = t.real_center(b) + 1j * im
    return out
