"""Hand-built cases for remeshing, reconnection and small-loop removal
(exact integer outcomes) plus invariants of the rules."""

import numpy as np
import pytest

import workloads as wl
from oracle import topology, coupled, vfm
from oracle.lbm import Lattice


def _loop(points):
    pos = np.asarray(points, dtype=np.float64)
    n = pos.shape[0]
    nxt = (np.arange(n) + 1) % n
    return pos, nxt, coupled.prev_from_next(nxt)


def _loops_of(nxt):
    seen = np.zeros(nxt.shape[0], dtype=bool)
    loops = []
    for k in range(nxt.shape[0]):
        if seen[k]:
            continue
        lp = [k]
        seen[k] = True
        p = nxt[k]
        while p != k:
            lp.append(p)
            seen[p] = True
            p = nxt[p]
        loops.append(lp)
    return loops


LAT = Lattice(32, 32, 32)


def test_uniform_ring_untouched():
    pos, nxt = wl.ring((16.0, 16.0, 16.0), 8.0, (0, 0, 1), 64)
    prv = coupled.prev_from_next(nxt)
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
    assert nd == 0 and ni == 0
    np.testing.assert_array_equal(p2, pos)
    np.testing.assert_array_equal(n2, nxt)


def test_one_long_segment_one_insertion():
    # square-ish loop of 8 points spaced 0.9 except one gap of 1.6
    pts = [(10 + 0.9 * i, 10.0, 10.0) for i in range(5)]  # x 10 .. 13.6
    pts += [(13.6, 10.9, 10.0), (12.0, 10.9, 10.0), (11.1, 10.9, 10.0), (10.2, 10.9, 10.0)]
    pos, nxt, prv = _loop(pts)
    # segment 5 -> 6 has length 1.6 (> 0.95); every other is in [0.7, 0.95]
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
    assert nd == 0 and ni == 1
    assert p2.shape[0] == 10
    np.testing.assert_allclose(p2[9], [12.8, 10.9, 10.0], atol=1e-15)  # midpoint, appended
    assert n2[5] == 9 and n2[9] == 6 and q2[9] == 5 and q2[6] == 9


def test_short_segment_deletes_later_point():
    pts = [(10 + 0.8 * i, 10.0, 10.0) for i in range(4)]  # 10, 10.8, 11.6, 12.4
    pts.insert(2, (11.0, 10.0, 10.0))  # 10.8 -> 11.0 is 0.2 long
    pts += [(12.4, 10.8, 10.0), (11.6, 10.8, 10.0), (10.8, 10.8, 10.0), (10.0, 10.8, 10.0)]
    pos, nxt, prv = _loop(pts)
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
    # point 2 (the later point of the short segment 1->2) goes
    assert nd == 1
    assert p2.shape[0] == len(pts) - 1 + ni
    assert not np.any(np.all(np.isclose(p2, [11.0, 10.0, 10.0]), axis=1))
    # the joined segment 1 -> old 3 is 0.8 long: no insertion
    assert ni == 0
    assert n2[1] == 2 and np.allclose(p2[2], [11.6, 10.0, 10.0])


def test_no_two_neighbours_deleted():
    pts = [(10.0, 10.0, 10.0), (10.3, 10.0, 10.0), (10.6, 10.0, 10.0), (10.9, 10.0, 10.0),
           (11.7, 10.0, 10.0), (11.7, 10.9, 10.0), (10.9, 10.9, 10.0), (10.0, 10.9, 10.0)]
    pos, nxt, prv = _loop(pts)
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
    # incoming segments of 1, 2, 3 are 0.3 long; 3 is no candidate because
    # dropping it would leave the chord 10.6 -> 11.7 = 1.1 > dxi_max; of the
    # run (1, 2) every other one goes: only 1, never two neighbours
    assert nd == 1
    np.testing.assert_allclose(p2[1], [10.6, 10.0, 10.0])


def test_deletion_never_forces_insertion():
    # a split segment: halves 0.5 < dxi_min, but the merged chord 1.0 >
    # dxi_max, so nothing is deleted and the split is stable
    pts = [(10.0, 10.0, 10.0), (10.9, 10.0, 10.0), (11.4, 10.0, 10.0), (11.9, 10.0, 10.0),
           (11.9, 10.9, 10.0), (11.0, 10.9, 10.0), (10.1, 10.9, 10.0)]
    pos, nxt, prv = _loop(pts)
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
    assert nd == 0 and ni == 0
    np.testing.assert_array_equal(p2, pos)


def test_all_candidate_loop_thinned():
    # a loop of 7 points 0.3 apart: all candidates; positions 0, 2, 4 from
    # the lowest index go, the last (6) stays because 7 is odd
    th = 2 * np.pi * np.arange(7) / 7
    R = 0.3 / (2 * np.sin(np.pi / 7))
    pts = np.stack([10 + R * np.cos(th), 10 + R * np.sin(th), np.full(7, 10.0)], axis=1)
    pos, nxt, prv = _loop(pts)
    cand = np.ones(7, dtype=bool)
    dele = topology._deletion_flags(cand, nxt, prv)
    assert dele.tolist() == [True, False, True, False, True, False, False]


def test_remesh_keeps_links_consistent():
    # dense rings (spacing <= 0.5: deletions) with noise (long segments: insertions)
    pos, nxt = wl.random_rings(9, 20, 3.0, 6.0, (32, 32, 32), (False,) * 3, 0.5)
    rng = np.random.default_rng(9)
    pos = pos + 0.2 * rng.standard_normal(pos.shape)
    pos = vfm.wrap_positions(pos, LAT)
    prv = coupled.prev_from_next(nxt)
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
    assert nd > 0 and ni > 0
    np.testing.assert_array_equal(q2[n2], np.arange(p2.shape[0]))
    assert len(_loops_of(n2)) == 20


def _two_lines(d, antiparallel=True, n=16, L=16):
    """Two straight lines along z through the periodic box, separated by d in x."""
    lat = Lattice(L, L, L)
    z = (np.arange(n) + 0.5) * L / n
    a = np.stack([np.full(n, 7.0), np.full(n, 8.0), z], axis=1)
    b = np.stack([np.full(n, 7.0 + d), np.full(n, 8.0), z], axis=1)
    na = (np.arange(n) + 1) % n
    if antiparallel:
        nb = n + (np.arange(n) - 1) % n
    else:
        nb = n + (np.arange(n) + 1) % n
    pos = np.concatenate([a, b])
    nxt = np.concatenate([na, nb])
    return lat, pos, nxt, coupled.prev_from_next(nxt)


def test_antiparallel_lines_annihilate_pairwise():
    """Antiparallel lines 0.3 apart, spacing 0.8: the same-height pairs would
    lengthen the line and are refused; every diagonal pair (k, next on the
    other line) shortens it, is disjoint from the others, and is taken."""
    lat, pos, nxt, prv = _two_lines(0.3, n=20)
    n2, q2, nr = topology.reconnect(pos, nxt, prv, lat, 0.95)
    assert nr == 20
    np.testing.assert_array_equal(q2[n2], np.arange(pos.shape[0]))
    loops = _loops_of(n2)
    assert sorted(len(lp) for lp in loops) == [2] * 20
    assert not topology.small_loops(n2, 5).any()


def test_parallel_lines_do_not_reconnect():
    lat, pos, nxt, prv = _two_lines(0.3, antiparallel=False, n=20)
    n2, q2, nr = topology.reconnect(pos, nxt, prv, lat, 0.95)
    assert nr == 0
    np.testing.assert_array_equal(n2, nxt)


def test_reconnection_exact_small_case():
    """Two antiparallel strands 0.3 apart, x spacing 0.9 (hand-derived).
    Same-x pairs (d = 0.3) would lengthen the line: refused.  Diagonal pairs
    (0,6), (1,5), (2,4) (d^2 = 0.9) shorten it from 1.8 to 0.6: taken; the
    other diagonal (1,7), (2,6), (3,5) lengthen it: refused."""
    lat = Lattice(32, 32, 32)
    A = [(10.0, 10.0, 10.0), (10.9, 10.0, 10.0), (11.8, 10.0, 10.0), (12.7, 10.0, 10.0)]
    B = [(12.7, 10.3, 10.0), (11.8, 10.3, 10.0), (10.9, 10.3, 10.0), (10.0, 10.3, 10.0)]
    pos = np.array(A + B)
    nxt = np.array([1, 2, 3, 0, 5, 6, 7, 4])
    prv = coupled.prev_from_next(nxt)
    n2, q2, nr = topology.reconnect(pos, nxt, prv, lat, 0.95)
    assert nr == 3
    expect = nxt.copy()
    expect[[0, 6, 1, 5, 2, 4]] = [7, 1, 6, 2, 5, 3]
    np.testing.assert_array_equal(n2, expect)
    assert sorted(sorted(lp) for lp in _loops_of(n2)) == [[0, 3, 4, 7], [1, 6], [2, 5]]


def test_reconnection_greedy_order():
    """Point 0 is close to both 4 and 8; the closer partner wins and the
    other exchange is dropped because 0 is used."""
    lat = Lattice(32, 32, 32)
    A = [(10.0, 10.0, 10.0), (10.9, 10.0, 10.0), (11.8, 10.0, 10.0), (12.7, 10.0, 10.0)]
    # strand B: 4 at (10.9, 10.2) heading -x so nxt[4] sits above point 0
    B = [(10.9, 10.2, 10.0), (10.0, 10.2, 10.0), (9.1, 10.2, 10.0), (8.2, 10.2, 10.0)]
    # strand C: 8 at (10.9, 9.7) heading -x
    Cs = [(10.9, 9.7, 10.0), (10.0, 9.7, 10.0), (9.1, 9.7, 10.0), (8.2, 9.7, 10.0)]
    pos = np.array(A + B + Cs)
    nxt = np.array([1, 2, 3, 0, 5, 6, 7, 4, 9, 10, 11, 8])
    prv = coupled.prev_from_next(nxt)
    n2, q2, nr = topology.reconnect(pos, nxt, prv, lat, 0.95)
    # (0,4): d^2 = 0.81 + 0.04; (0,8): d^2 = 0.81 + 0.09 -> (0,4) first
    assert n2[0] == 5 and n2[4] == 1
    assert n2[8] == 9  # C untouched: 0 already used
    np.testing.assert_array_equal(q2[n2], np.arange(12))


def test_small_loop_removed():
    big = wl.ring((8.0, 8.0, 8.0), 3.0, (0, 0, 1), 24)
    small = wl.ring((20.0, 20.0, 20.0), 0.5, (0, 1, 0), 4)
    pos, nxt = wl.concat_loops([big, small])
    alive = topology.small_loops(nxt, 5)
    assert alive[:24].all() and not alive[24:].any()
    five = wl.ring((20.0, 20.0, 20.0), 0.7, (0, 1, 0), 5)
    pos, nxt = wl.concat_loops([big, five])
    assert topology.small_loops(nxt, 5).all()


def test_compaction_renumbers_links():
    pos, nxt = wl.concat_loops([wl.ring((8.0, 8.0, 8.0), 2.0, (0, 0, 1), 6),
                               wl.ring((20.0, 8.0, 8.0), 2.0, (0, 0, 1), 7)])
    prv = coupled.prev_from_next(nxt)
    alive = np.ones(13, dtype=bool)
    alive[:6] = False
    p2, n2, q2 = topology.compact(pos, nxt, prv, alive)
    np.testing.assert_array_equal(p2, pos[6:])
    np.testing.assert_array_equal(n2, (np.arange(7) + 1) % 7)
    np.testing.assert_array_equal(q2, (np.arange(7) - 1) % 7)


# ---- long runs of deletion candidates (reading R10: every run is thinned,
# however long).  Hand counts: a loop of L points that are all candidates
# loses floor(L / 2), the points at even distance from its lowest index
# (the last one kept when L is odd); an open run of m candidates loses the
# 1st, 3rd, ... of them, ceil(m / 2).

def _fine_ring(L, spacing=0.45, centre=(16.0, 16.0, 16.0)):
    """Regular L-gon of side ``spacing`` in the plane z = centre_z."""
    R = spacing / (2.0 * np.sin(np.pi / L))
    th = 2.0 * np.pi * (np.arange(L) + 0.5) / L
    pts = np.stack([centre[0] + R * np.cos(th), centre[1] + R * np.sin(th),
                    np.full(L, centre[2])], 1)
    return _loop(pts)


@pytest.mark.parametrize("L", [30, 33, 34, 40, 64])
def test_all_candidate_ring_is_thinned(L):
    pos, nxt, prv = _fine_ring(L)
    # every point is a candidate: incoming side 0.45 < 0.70, chord over two
    # sides 2 * 0.45 cos(pi / L) < 0.95
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
    assert nd == L // 2 and ni == 0
    keep = [k for k in range(L) if not (k % 2 == 0 and not (k == L - 1 and L % 2 == 1))]
    np.testing.assert_array_equal(p2, pos[keep])
    assert len(_loops_of(n2)) == 1
    # every new side is the chord over two old sides (or one old side where
    # the odd loop kept its last point)
    seg = np.linalg.norm(vfm.min_image(p2[n2] - p2, LAT), axis=1)
    assert seg.max() <= 0.95


def test_open_run_of_forty_candidates():
    """Arc of a circle of radius 10: 41 sides of 0.45 (points 0 .. 41), then
    equal sides of about 0.807 closing the loop.  The candidates are points
    1 .. 40 (incoming side 0.45 and chord over both sides <= 0.95; point 41's
    chord includes a long side, point 0's incoming side is long): one run of
    40, of which points 1, 3, ..., 39 go."""
    R = 10.0
    t1 = 2.0 * np.arcsin(0.45 / (2.0 * R))
    rest = 2.0 * np.pi - 41 * t1
    m = 55
    th = np.concatenate([np.arange(42) * t1, 41 * t1 + np.arange(1, m) * rest / m])
    pts = np.stack([16.0 + R * np.cos(th), 16.0 + R * np.sin(th), np.full(th.size, 16.0)], 1)
    pos, nxt, prv = _loop(pts)
    long_side = np.linalg.norm(pts[42] - pts[41])
    assert 0.70 < long_side < 0.95
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
    assert nd == 20 and ni == 0
    gone = set(range(1, 40, 2))
    keep = [k for k in range(pts.shape[0]) if k not in gone]
    np.testing.assert_array_equal(p2, pos[keep])


def test_shrinking_ring_keeps_the_lower_bound():
    """Repeated passes on an over-resolved ring: each pass halves it until
    every side is at least dxi_min (the resolution bound of Sec. II.A)."""
    pos, nxt, prv = _fine_ring(96, spacing=0.2)
    sizes = []
    for _ in range(4):
        pos, nxt, prv, nd, ni = topology.remesh(pos, nxt, prv, LAT, 0.7, 0.95)
        sizes.append(pos.shape[0])
    assert sizes[:2] == [48, 24]
    seg = np.linalg.norm(vfm.min_image(pos[nxt] - pos, LAT), axis=1)
    assert seg.min() >= 0.7 and seg.max() <= 0.95
