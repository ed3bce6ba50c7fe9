"""Discrete filament operations, plain loops (paper Sec. II.A and III.B).

The paper fixes only the resolution bounds (segment lengths kept between
dxi_min and dxi_max, Sec. II.A and III) and that the legs of two vortices
are exchanged when they come within the resolution (Sec. II.A; "within
dxi_max", Sec. III.B).  The concrete rules below are readings R10 and R11.
They are written so that every decision is a comparison of squared FP64
distances summed as dx*dx + dy*dy + dz*dz, left to right, with no fused
multiply-add; any implementation that sums in that order reaches the same
integer result.

Index conventions (so that integer outputs can be compared exactly):
  * deleted points are removed and the survivors keep their relative order;
  * points inserted by remeshing are appended after all old points, in
    ascending order of the segment they split.
"""

import numpy as np

from .lbm import Lattice
from .vfm import min_image, wrap_positions


def _sq(d):
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2]


def compact(pos, nxt, prv, alive):
    """Drop dead points; survivors keep their order; links are renumbered."""
    alive = np.asarray(alive, dtype=bool)
    new_index = np.cumsum(alive) - 1
    keep = np.nonzero(alive)[0]
    pos2 = pos[keep].copy()
    nxt2 = new_index[nxt[keep]].astype(np.int64)
    prv2 = new_index[prv[keep]].astype(np.int64)
    return pos2, nxt2, prv2


def _deletion_flags(cand, nxt, prv):
    """Which deletion candidates go in one pass (reading R10).  Along a run
    of consecutive candidates the 1st, 3rd, 5th, ... go: candidate k is
    deleted when the number c of candidates directly before it (walking
    back along prv to the first point of the run, however long the run) is
    even.  A loop made only of candidates is counted from its lowest index,
    and its last point is kept when the loop length is odd.  No two
    neighbours are ever deleted in the same pass, and a run of m candidates
    loses ceil(m / 2) of them (a loop of L candidates floor(L / 2)), so that
    every run is thinned in one pass however long it is (the segment-length
    bounds of Sec. II.A hold for any resolution of the input)."""
    N = cand.shape[0]
    dele = np.zeros(N, dtype=bool)
    for k in range(N):
        if not cand[k]:
            continue
        c = 0
        p = prv[k]
        while cand[p] and p != k:
            c += 1
            p = prv[p]
        if p == k:  # the whole loop (c + 1 points) is candidates
            L = c + 1
            members = [k]
            q = nxt[k]
            while q != k:
                members.append(q)
                q = nxt[q]
            m = min(members)
            pos = 0
            q = m
            while q != k:
                pos += 1
                q = nxt[q]
            dele[k] = (pos % 2 == 0) and not (pos == L - 1 and L % 2 == 1)
        else:
            dele[k] = c % 2 == 0
    return dele


def remesh(pos, nxt, prv, lat: Lattice, dxi_min, dxi_max):
    """Keep segment lengths inside [dxi_min, dxi_max] (Sec. II.A; reading R10).

    1. Deletion.  The ends of an open line are never deleted (reading
       F1b); any other point k is a candidate when its incoming segment
       (prv[k] -> k) is shorter than dxi_min and the chord prv[k] -> nxt[k]
       that would replace its two segments is not longer than dxi_max (so a
       deletion never calls for a new insertion: with the paper's bounds,
       dxi_max < 2 dxi_min, a split segment has halves below dxi_min, and
       deleting one of them would recreate the long segment every pass).
       Along each run of consecutive
       candidates every other one is deleted (see _deletion_flags), so no
       two neighbours go in one pass; the predecessor and successor of a
       deleted point are joined.
    2. Insertion, on the joined loops.  Every segment j -> nxt[j] longer than
       dxi_max gets one new point at its midpoint (nearest image, wrapped),
       appended after the old points in ascending j.
    3. Compaction.
    Returns (pos, nxt, prv, n_deleted, n_inserted)."""
    N = pos.shape[0]
    nxt = nxt.copy()
    prv = prv.copy()
    mn2 = dxi_min * dxi_min
    mx2 = dxi_max * dxi_max
    cand = np.zeros(N, dtype=bool)
    for k in range(N):
        if nxt[k] == k or prv[k] == k:
            continue  # the ends of an open line stay on their walls (F1b)
        d = min_image((pos[k] - pos[prv[k]])[None, :], lat)[0]
        chord = min_image((pos[nxt[k]] - pos[prv[k]])[None, :], lat)[0]
        cand[k] = (_sq(d) < mn2) and (_sq(chord) <= mx2)
    dele = _deletion_flags(cand, nxt, prv)
    for k in range(N):
        if dele[k]:
            p, n = prv[k], nxt[k]
            nxt[p] = n
            prv[n] = p
    new_pos = []
    for j in range(N):
        if dele[j]:
            continue
        seg = min_image((pos[nxt[j]] - pos[j])[None, :], lat)[0]
        if _sq(seg) > mx2:
            new_pos.append((j, pos[j] + 0.5 * seg))
    M = len(new_pos)
    if M:
        pos = np.concatenate([pos, np.array([p for _, p in new_pos])], axis=0)
        pos = wrap_positions(pos, lat)
        nxt = np.concatenate([nxt, np.zeros(M, dtype=np.int64)])
        prv = np.concatenate([prv, np.zeros(M, dtype=np.int64)])
        for r, (j, _) in enumerate(new_pos):
            q = N + r
            n = nxt[j]
            nxt[j] = q
            prv[q] = j
            nxt[q] = n
            prv[n] = q
    alive = np.concatenate([~dele, np.ones(M, dtype=bool)])
    pos, nxt, prv = compact(pos, nxt, prv, alive)
    return pos, nxt, prv, int(dele.sum()), M


def reconnect(pos, nxt, prv, lat: Lattice, dist):
    """Exchange the legs of two vortices that come closer than ``dist``
    (Sec. II.A and III.B; reading R11).

    Candidates: pairs i < j with |s_j - s_i| < dist (nearest image) that are
    more than two links apart along the loop, and both of which have a
    segment (the last point of an open line has none, reading F1b; the
    exchange keeps every open line open, with its ends on the walls).  A
    candidate is kept if the
    exchange i -> nxt[j], j -> nxt[i] does not lengthen the line:
    |s_nxt[j] - s_i| + |s_nxt[i] - s_j| <= |s_nxt[i] - s_i| + |s_nxt[j] - s_j|.
    Kept candidates are taken greedily in ascending (d^2, i, j); a point
    takes part in at most one exchange per call.
    Returns (nxt, prv, n_reconnections)."""
    N = pos.shape[0]
    nxt = nxt.copy()
    prv = prv.copy()
    d2max = dist * dist
    cands = []
    for i in range(N):
        if nxt[i] == i:
            continue
        near = {nxt[i], nxt[nxt[i]], prv[i], prv[prv[i]]}
        for j in range(i + 1, N):
            if j in near or nxt[j] == j:
                continue
            d = min_image((pos[j] - pos[i])[None, :], lat)[0]
            d2 = _sq(d)
            if not d2 < d2max:
                continue
            a = min_image((pos[nxt[i]] - pos[i])[None, :], lat)[0]
            b = min_image((pos[nxt[j]] - pos[j])[None, :], lat)[0]
            c = min_image((pos[nxt[j]] - pos[i])[None, :], lat)[0]
            e = min_image((pos[nxt[i]] - pos[j])[None, :], lat)[0]
            before = np.sqrt(_sq(a)) + np.sqrt(_sq(b))
            after = np.sqrt(_sq(c)) + np.sqrt(_sq(e))
            if after <= before:
                cands.append((d2, i, j))
    cands.sort()
    used = np.zeros(N, dtype=bool)
    n_rec = 0
    for d2, i, j in cands:
        if used[i] or used[j]:
            continue
        ni, nj = nxt[i], nxt[j]
        nxt[i] = nj
        prv[nj] = i
        nxt[j] = ni
        prv[ni] = j
        used[i] = used[j] = True
        n_rec += 1
    return nxt, prv, n_rec


def small_loops(nxt, min_pts, prv=None):
    """Mark points on filaments with fewer than ``min_pts`` points (they are
    removed: such loops are below the resolution): closed loops, and open
    lines counted from their first to their last point (reading F1b; needs
    ``prv``).  Returns alive mask."""
    N = nxt.shape[0]
    alive = np.ones(N, dtype=bool)
    for k in range(N):
        # forward: back to k (a loop), or to the last point of an open line
        p = k
        fwd = 0
        closed = False
        while fwd < min_pts:
            q = nxt[p]
            if q == p:
                break
            if q == k:
                closed = True
                break
            p = q
            fwd += 1
        if closed:
            alive[k] = fwd + 1 >= min_pts
            continue
        if nxt[p] != p:
            continue  # min_pts points ahead already
        # open line: back to its first point
        b = 0
        p = k
        while b < min_pts and prv[p] != p:
            p = prv[p]
            b += 1
        if prv[p] == p and fwd + b + 1 < min_pts:
            alive[k] = False
    return alive


def check_lines(pos, nxt, lat: Lattice):
    """Validate the links of a filament state (reading F1b): every point has
    at most one predecessor besides itself, and the ends of open lines (a
    point that links to itself, or that no other point links to) lie on a
    wall plane of a closed axis; a single point that is both is not a line.
    Raises ValueError."""
    nxt = np.asarray(nxt)
    N = nxt.shape[0]
    if N == 0:
        return
    if nxt.min() < 0 or nxt.max() >= N:
        raise ValueError("next[] out of range")
    ks = np.arange(N)
    real = nxt != ks
    indeg = np.bincount(nxt[real], minlength=N)
    if indeg.max(initial=0) > 1:
        raise ValueError("a point has two predecessors")
    last = ~real
    first = indeg == 0
    if np.any(last & first):
        raise ValueError("a one-point line")
    on_wall = np.zeros(N, dtype=bool)
    for a in range(3):
        if lat.walls[a]:
            on_wall |= (pos[:, a] == -0.5) | (pos[:, a] == lat.dims[a] - 0.5)
    if np.any((last | first) & ~on_wall):
        raise ValueError("an open line ends off the wall planes")


def topology_update(pos, nxt, prv, lat: Lattice, vp):
    """Remeshing, then small-loop removal and compaction; then, if enabled,
    reconnection followed by small-loop removal and compaction again."""
    stats = dict(deleted=0, inserted=0, reconnections=0, loops_removed_pts=0)
    if vp.remesh:
        pos, nxt, prv, nd, ni = remesh(pos, nxt, prv, lat, vp.dxi_min, vp.dxi_max)
        stats["deleted"], stats["inserted"] = nd, ni
    alive = small_loops(nxt, vp.min_loop_pts, prv)
    stats["loops_removed_pts"] += int((~alive).sum())
    pos, nxt, prv = compact(pos, nxt, prv, alive)
    if vp.reconnect:
        nxt, prv, nr = reconnect(pos, nxt, prv, lat, vp.reconnect_dist)
        stats["reconnections"] = nr
        alive = small_loops(nxt, vp.min_loop_pts, prv)
        stats["loops_removed_pts"] += int((~alive).sum())
        pos, nxt, prv = compact(pos, nxt, prv, alive)
    return pos, nxt, prv, stats
