"""Pins of the oracle tree and lists (Sec. 6.1, Sec. 6.2) against geometry and
brute force: containment of every point in its leaf, occupancy, the level
restriction over all leaf pairs, and that every (target, source) pair is
accounted for exactly once by List 1, List 2 at one ancestor pair, List 3 or
List 4."""
import numpy as np
import pytest

import synth
from oracle import tree as T


def _clustered2d(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 0.01, (n // 2, 2)) + 0.3
    b = rng.uniform(-1, 1, (n - n // 2, 2))
    re = np.concatenate([a, b])
    return re + 0.2j * np.abs(re)


def _clustered3d(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 0.02, (n // 2, 3)) - 0.4
    b = rng.uniform(-1, 1, (n - n // 2, 3))
    re = np.concatenate([a, b])
    return re + 0.1j * np.abs(re)


CASES = [
    ("curve2d", lambda: synth.curve2d(1500, 7), 16, 1),
    ("curve2d_k2", lambda: synth.curve2d(1500, 8), 16, 2),
    ("cluster2d", lambda: _clustered2d(1200, 9), 8, 1),
    ("cluster2d_k2", lambda: _clustered2d(1200, 10), 8, 2),
    ("plane3d", lambda: synth.plane3d_bumps(30, 11), 16, 1),
    ("cluster3d", lambda: _clustered3d(1000, 12), 8, 1),
]


def _leaf_geom(t, b):
    w = t.D * 2.0 ** (-int(t.level[b]))
    return t.real_center(b), w


def _near_real(t, a, b, k):
    ca, wa = _leaf_geom(t, a)
    cb, wb = _leaf_geom(t, b)
    return np.all(np.abs(ca - cb) <= 0.5 * k * (wa + wb) * (1 + 1e-12))


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def built(request):
    name, make, ns, k = request.param
    pts = make()
    return pts, T.build_tree(pts, ns, k), ns, k


# The library starts the far field at a level >= 2 (boxes coarser than that
# carry no expansions and count as near everything), so the lists are also
# pinned at the top levels it uses.
TOPS = [2, 3, 4]


@pytest.fixture(scope="module", params=[(c, top) for c in CASES for top in TOPS],
                ids=[f"{c[0]}-top{top}" for c in CASES for top in TOPS])
def built_top(request):
    (name, make, ns, k), top = request.param
    pts = make()
    return pts, T.build_tree(pts, ns, k, top_level=top), ns, k, top


def test_points_lie_in_their_leaf_and_occupancy(built):
    pts, t, ns, k = built
    assert sorted(t.perm.tolist()) == list(range(pts.shape[0]))
    assert np.all(np.diff(t.keys.astype(np.float64)) >= 0)
    seen = np.zeros(pts.shape[0], dtype=int)
    for b in range(t.nbox):
        if t.nchild[b]:
            # children partition the parent's point range
            kids = range(t.child0[b], t.child0[b] + t.nchild[b])
            assert t.pbeg[t.child0[b]] == t.pbeg[b]
            assert t.pend[t.child0[b] + t.nchild[b] - 1] == t.pend[b]
            for c in kids:
                assert t.parent[c] == b and t.level[c] == t.level[b] + 1
            continue
        assert t.pend[b] - t.pbeg[b] >= 1
        if t.level[b] < t.nbits:
            assert t.pend[b] - t.pbeg[b] <= ns
        c, w = _leaf_geom(t, b)
        re = pts[t.perm[t.pbeg[b]:t.pend[b]]].real
        tol = 1e-12 * t.D
        assert np.all(re >= c - 0.5 * w - tol) and np.all(re <= c + 0.5 * w + tol)
        seen[t.perm[t.pbeg[b]:t.pend[b]]] += 1
    assert np.all(seen == 1)


def test_level_restriction_all_leaf_pairs(built):
    pts, t, ns, k = built
    leaves = np.flatnonzero(t.nchild == 0)
    for a in leaves:
        for b in leaves:
            if t.level[a] <= t.level[b] - 2:
                assert not _near_real(t, a, b, k)


def _ancestors(t, b):
    out = []
    while b >= 0:
        out.append(b)
        b = t.parent[b]
    return out


def _coverage(t):
    rows = {name: [set(idx[off[b]:off[b + 1]].tolist()) for b in range(t.nbox)]
            for name, (off, idx) in t.lists.items()}
    leaves = np.flatnonzero(t.nchild == 0)
    anc = {b: _ancestors(t, b) for b in leaves}
    for b in leaves:           # target leaf
        for a in leaves:       # source leaf
            n = int(a in rows["L1"][b])
            n += sum(1 for B in anc[b] for A in anc[a] if A in rows["L2"][B])
            n += sum(1 for A in anc[a] if A in rows["L3"][b])
            n += sum(1 for B in anc[b] if a in rows["L4"][B])
            assert n == 1, (b, a, n)


def test_every_pair_covered_exactly_once(built):
    pts, t, ns, k = built
    _coverage(t)


def test_every_pair_covered_exactly_once_above_top(built_top):
    pts, t, ns, k, top = built_top
    _coverage(t)


def _structure(t, k, top):
    """Row order and symmetry, plus each list's geometric definition, where a
    box coarser than `top` is near every box (it carries no expansion)."""
    def near(a, b):
        if t.level[a] < top or t.level[b] < top:
            return True
        return _near_real(t, a, b, k)

    rows = {name: [idx[off[b]:off[b + 1]].tolist() for b in range(t.nbox)]
            for name, (off, idx) in t.lists.items()}
    for b in range(t.nbox):
        for name in rows:
            assert rows[name][b] == sorted(set(rows[name][b]))
        for a in rows["L1"][b]:
            assert b in rows["L1"][a] and near(a, b)
        for a in rows["L2"][b]:
            assert b in rows["L2"][a] and t.level[a] == t.level[b]
            assert t.level[a] >= top
            assert not near(a, b)
            assert near(t.parent[a], t.parent[b])
        for a in rows["L3"][b]:
            assert b in rows["L4"][a] and t.level[a] > t.level[b]
            assert t.level[a] >= top
            assert not near(a, b) and near(t.parent[a], b)
        if t.nchild[b]:
            assert not rows["L1"][b] and not rows["L3"][b]
        if t.level[b] < top:
            # no expansion at b: every interaction of b is direct
            assert not rows["L2"][b] and not rows["L3"][b] and not rows["L4"][b]
    # List 2 is complete: every same-level pair at or below top that is not
    # near but whose parents are near is in it
    for l in range(max(top, 1), int(t.level.max()) + 1):
        bl = np.flatnonzero(t.level == l)
        for b in bl:
            want = sorted(int(a) for a in bl if not near(a, b) and near(t.parent[a], t.parent[b]))
            assert rows["L2"][b] == want, (b, l)


def test_list_structure(built):
    pts, t, ns, k = built
    _structure(t, k, 0)


def test_list_structure_above_top(built_top):
    pts, t, ns, k, top = built_top
    _structure(t, k, top)


def _cube_members(t, re, b):
    """Indices of the points whose real part lies in box b's half-open cube
    [lo + c w, lo + (c + 1) w) per coordinate, from the box geometry alone."""
    w = t.D * 2.0 ** (-int(t.level[b]))
    c = np.array(t.coords(b), dtype=np.float64)
    lo = t.lo + c * w
    hi = lo + w
    inside = np.all((re >= lo) & (re < hi), axis=1)
    return np.flatnonzero(inside)


@pytest.mark.parametrize("case", CASES[:1] + CASES[2:3] + CASES[4:5], ids=lambda c: c[0])
def test_complex_centers_definition(case):
    """The complexified centre of every box (Sec. 6.1): its real part is the
    cube's geometric centre and its imaginary part the mean imaginary part of
    the points whose real parts lie in the cube, descendants included; the
    membership here comes from the cube bounds, not from the sorted ranges."""
    name, make, ns, k = case
    pts = make()
    t = T.build_tree(pts, ns, k)
    cen = T.complex_centers(t, pts)
    re = pts.real
    for b in range(t.nbox):
        members = _cube_members(t, re, b)
        assert members.size == t.pend[b] - t.pbeg[b] and members.size > 0
        w = t.D * 2.0 ** (-int(t.level[b]))
        mid = t.lo + (np.array(t.coords(b), dtype=np.float64) + 0.5) * w
        assert np.array_equal(cen[b].real, mid)
        want = pts[members].imag.mean(axis=0)
        assert np.allclose(cen[b].imag, want, rtol=1e-13, atol=1e-15 * np.abs(pts.imag).max())


def test_complex_centers_planted_box():
    """Hand-made case: four points in two quadrants of the unit square; the
    level-1 boxes' centres are known in closed form."""
    pts = np.array([[0.1 + 0.2j, 0.1 + 0.0j], [0.2 + 0.4j, 0.3 - 0.2j],
                    [0.9 + 1.0j, 0.8 + 0.5j], [0.0 + 0.0j, 1.0 + 0.0j]])
    t = T.build_tree(pts, 2, 1)
    cen = T.complex_centers(t, pts)
    lo, D = t.lo, t.D
    assert np.allclose(cen[0], (lo + 0.5 * D) + 1j * pts.imag.mean(axis=0), rtol=0, atol=1e-15)
    for b in range(t.nbox):
        if t.level[b] != 1:
            continue
        members = _cube_members(t, pts.real, b)
        expect_im = pts[members].imag.mean(axis=0)
        assert np.allclose(cen[b].imag, expect_im, rtol=0, atol=1e-15)
    # the lower-left quadrant holds points 0 and 1: Im mean (0.3, -0.1)
    ll = [b for b in range(t.nbox) if t.level[b] == 1 and t.coords(b) == (0, 0)]
    assert len(ll) == 1
    assert np.allclose(cen[ll[0]].imag, [0.3, -0.1], rtol=0, atol=1e-15)
