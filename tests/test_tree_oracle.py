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


def test_every_pair_covered_exactly_once(built):
    pts, t, ns, k = built
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


def test_list_structure(built):
    pts, t, ns, k = built
    rows = {name: [idx[off[b]:off[b + 1]].tolist() for b in range(t.nbox)]
            for name, (off, idx) in t.lists.items()}
    for b in range(t.nbox):
        for name in rows:
            assert rows[name][b] == sorted(set(rows[name][b]))
        for a in rows["L1"][b]:
            assert b in rows["L1"][a] and _near_real(t, a, b, k)
        for a in rows["L2"][b]:
            assert b in rows["L2"][a] and t.level[a] == t.level[b]
            assert not _near_real(t, a, b, k)
            assert _near_real(t, t.parent[a], t.parent[b], k)
        for a in rows["L3"][b]:
            assert b in rows["L4"][a] and t.level[a] > t.level[b]
            assert not _near_real(t, a, b, k) and _near_real(t, t.parent[a], b, k)
        if t.nchild[b]:
            assert not rows["L1"][b] and not rows["L3"][b]
