"""Cell-multipole approximation of the non-local Biot-Savart sum, plain
FP64 (an extension for large tangles: Sec. II.A computes the full
non-local integral, which grows as N^2 while the tangles of Sec. III.C
grow; reading F2).  Test infrastructure only (see the package docstring):
the reference that the library's far-field sum is checked against.

Positions are first reduced into [0, L) on every axis (the box is periodic
on all three axes).  The box is cut into a uniform grid of cells of edge
h (h divides every L_a).  Each segment k (start s_k, vector d_k at the
nearest image, circulation kappa) belongs to the cell of its midpoint m_k
(reduced into [0, L)).  About the cell centre c, with y_k = m_k - c at the
nearest image, the segment's vorticity kappa d_k is spread along
y_k + t d_k, t in [-1/2, 1/2]; the cell's moments are
    M0 = sum kappa d,  M1 = sum kappa d (x) y,
    M2 = sum kappa d (x) (y (x) y + d (x) d / 12),
and its radius rad = max_k (|y_k| + |d_k| / 2).
The field of a vortex element a at offset y seen from r, a x (r - y) /
|r - y|^3 / (4 pi), expanded about the centre to second order in y, gives
the velocity at R = r - c
    v_m = eps_mnp g_np / (4 pi),
    g_np = M0_n R_p / r^3 - M1_np / r^3 + 3 (M1 R)_n R_p / r^5
         + (15 (R M2_n R) R_p / r^7 - 3 tr(M2_n) R_p / r^5 - 6 (M2_n R)_p / r^5) / 2.

Periodic images (reading R12 decides the image of each segment by its
start, per target).  For target r, segment k of cell c sits at the image
whose start is s_k - r + n_k L (the nearest image on the 32-bit grid, as
in the direct sum); that image places the cell centre at
    C_k = (s_k - r + n_k L) + d_k / 2 - y_k = (c - r) + K_k L,
with an integer vector K_k, the segment's image class.  The segments of a
cell take one class unless the plane half a box from the target crosses
their starts.  Per target and cell:
  * one class K: the cell is far when |R|^2 theta^2 >= rad^2 with
    R = (c - r) + K L, and contributes its expansion at that image;
  * two classes differing on one axis (the plane crosses the starts on
    that axis only): when both images pass the same test the cell is
    split, each class contributing the expansion of its own segments'
    moments at its image;
  * otherwise (an image too close, or starts crossed on two or more axes)
    the cell's segments are summed directly with the exact straight-
    segment integral at their own images, the target's own two segments
    excluded, as in vfm.biot_savart_nonlocal.
theta < 1 keeps the target's own segments in direct cells (a segment that
touches r lies within rad of its cell centre).  Decisions are made in FP64
with the sums written left to right.

Levels.  With ``levels`` = l > 1 the cells of edge h 2^m (m = 0 .. l - 1)
form a hierarchy, each cell the union of 8 cells of the level below, each
with its own moments and radius about its own centre.  Per target the
cells of the coarsest level are classified as above; a coarse cell that is
neither far nor split is opened: its 8 children are classified in turn,
down to edge h, where the cells that are neither far nor split are summed
directly.
"""

import numpy as np

from .lbm import Lattice
from .vfm import bs_image_offsets, min_image, segment_velocity, wrap_positions


def cell_grid(lat: Lattice, h):
    """Cells per axis and their edge: nc_a = L_a / h (h must divide L_a)."""
    nc = []
    for n in lat.dims:
        if n % h:
            raise ValueError("the cell edge must divide every box length")
        nc.append(n // h)
    return np.array(nc, dtype=np.int64), np.array([float(h)] * 3)


def cell_moments(pos, nxt, lat: Lattice, h, kappa):
    """Segment cells and the per-cell moments (module docstring), for
    positions already in [0, L).  Returns a dict: key (N,) cell of each
    segment, order (segments sorted by cell, stable), starts / ends (per
    cell, into order), centre (C, 3), y (N, 3), d (N, 3), M0 (C, 3),
    M1 (C, 3, 3), M2 (C, 3, 3, 3), rad (C,)."""
    nc, hh = cell_grid(lat, h)
    L = np.array(lat.dims, dtype=np.float64)
    d = min_image(pos[nxt] - pos, lat)
    mid = pos + 0.5 * d
    mid = mid - L * np.floor(mid / L)
    idx = np.minimum(np.floor(mid / hh).astype(np.int64), nc - 1)
    key = (idx[:, 2] * nc[1] + idx[:, 1]) * nc[0] + idx[:, 0]
    C = int(nc.prod())
    cid = np.arange(C)
    ci = np.stack([cid % nc[0], (cid // nc[0]) % nc[1], cid // (nc[0] * nc[1])], 1)
    centre = (ci + 0.5) * hh
    y = min_image(mid - centre[key], lat)
    M0, M1, M2 = _moments(key, y, d, kappa, C)
    ny = np.sqrt(y[:, 0] * y[:, 0] + y[:, 1] * y[:, 1] + y[:, 2] * y[:, 2])
    nd = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
    rad = np.zeros(C)
    np.maximum.at(rad, key, ny + 0.5 * nd)
    order = np.argsort(key, kind="stable")
    starts = np.searchsorted(key[order], cid)
    ends = np.searchsorted(key[order], cid, side="right")
    return dict(key=key, order=order, starts=starts, ends=ends, centre=centre, y=y, d=d, M0=M0,
                M1=M1, M2=M2, rad=rad)


def _moments(key, y, d, kappa, C):
    """M0, M1, M2 of the segments (key, y, d) added into C cells."""
    a = kappa * d
    M0 = np.zeros((C, 3))
    M1 = np.zeros((C, 3, 3))
    M2 = np.zeros((C, 3, 3, 3))
    np.add.at(M0, key, a)
    np.add.at(M1, key, a[:, :, None] * y[:, None, :])
    yy = y[:, :, None] * y[:, None, :] + d[:, :, None] * d[:, None, :] / 12.0
    np.add.at(M2, key, a[:, :, None, None] * yy[:, None, :, :])
    return M0, M1, M2


def m2p(R, M0, M1, M2):
    """Velocity (without kappa / (4 pi) folded in: the moments carry kappa)
    of cells with moments M0 (C, 3), M1 (C, 3, 3), M2 (C, 3, 3, 3) at
    offsets R (C, 3) from their centres, times 4 pi; summed over C."""
    r2 = R[:, 0] * R[:, 0] + R[:, 1] * R[:, 1] + R[:, 2] * R[:, 2]
    r = np.sqrt(r2)
    r3 = 1.0 / (r2 * r)
    r5 = r3 / r2
    r7 = r5 / r2
    g = M0[:, :, None] * R[:, None, :] * r3[:, None, None]
    g = g - M1 * r3[:, None, None]
    g = g + 3.0 * np.einsum("cnq,cq->cn", M1, R)[:, :, None] * R[:, None, :] * r5[:, None, None]
    RMR = np.einsum("cnjk,cj,ck->cn", M2, R, R)
    tr = np.einsum("cnjj->cn", M2)
    MR = np.einsum("cnjk,ck->cnj", M2, R)
    g = g + 0.5 * (15.0 * RMR[:, :, None] * R[:, None, :] * r7[:, None, None]
                   - 3.0 * tr[:, :, None] * R[:, None, :] * r5[:, None, None]
                   - 6.0 * MR * r5[:, None, None])
    v = np.stack([g[:, 1, 2] - g[:, 2, 1], g[:, 2, 0] - g[:, 0, 2], g[:, 0, 1] - g[:, 1, 0]], 1)
    return v.sum(axis=0)


EMPTY, FAR, SPLIT, NEAR = 0, 1, 2, 3


def classify(r, pos, cm, lat: Lattice, theta):
    """Per-cell decisions for target r (module docstring).  Returns a dict:
    kind (C,) in EMPTY / FAR / SPLIT / NEAR, K (N, 3) image class of every
    segment, Kmin / Kmax (C, 3) the classes' extremes per axis, axis (C,)
    the crossed axis of a split cell, Rlo / Rhi (C, 3) the centre's images
    (c - r) + K L for Kmin and Kmax (source minus target)."""
    L = np.array(lat.dims, dtype=np.float64)
    key = cm["key"]
    C = cm["centre"].shape[0]
    base = cm["centre"] - r[None, :]
    R1 = bs_image_offsets(pos, r[None, :], lat)
    Cimg = R1 + 0.5 * cm["d"] - cm["y"]
    K = np.rint((Cimg - base[key]) / L).astype(np.int64)
    big = np.iinfo(np.int64).max
    Kmin = np.full((C, 3), big)
    Kmax = np.full((C, 3), -big)
    np.minimum.at(Kmin, key, K)
    np.maximum.at(Kmax, key, K)
    ne = cm["ends"] > cm["starts"]
    Kmin[~ne] = 0
    Kmax[~ne] = 0
    crossed = Kmax > Kmin
    ncross = crossed.sum(axis=1)
    Rlo = base + Kmin * L
    Rhi = base + Kmax * L
    th2 = theta * theta
    rad2 = cm["rad"] * cm["rad"]
    ok_lo = (Rlo[:, 0] * Rlo[:, 0] + Rlo[:, 1] * Rlo[:, 1] + Rlo[:, 2] * Rlo[:, 2]) * th2 >= rad2
    ok_hi = (Rhi[:, 0] * Rhi[:, 0] + Rhi[:, 1] * Rhi[:, 1] + Rhi[:, 2] * Rhi[:, 2]) * th2 >= rad2
    kind = np.full(C, NEAR, dtype=np.int64)
    kind[ne & (ncross == 0) & ok_lo] = FAR
    kind[ne & (ncross == 1) & ok_lo & ok_hi] = SPLIT
    kind[~ne] = EMPTY
    return dict(kind=kind, K=K, Kmin=Kmin, Kmax=Kmax, axis=np.argmax(crossed, axis=1), Rlo=Rlo,
                Rhi=Rhi)


def _children(nc_fine):
    """Parent index (at the level with half the cells per axis) of every
    cell of a level with nc_fine cells per axis."""
    cid = np.arange(int(np.prod(nc_fine)))
    ci = np.stack([cid % nc_fine[0], (cid // nc_fine[0]) % nc_fine[1],
                   cid // (nc_fine[0] * nc_fine[1])], 1) // 2
    pn = np.asarray(nc_fine) // 2
    return (ci[:, 2] * pn[1] + ci[:, 1]) * pn[0] + ci[:, 0]


def biot_savart_farfield(pos, nxt, prv, lat: Lattice, kappa, h, theta, targets=None, levels=1):
    """Non-local superfluid velocity at ``targets`` (default: all) by the
    cell-multipole approximation (module docstring), with ``levels`` levels
    of cells (edge h at the finest).  Returns (T, 3) and a dict of the mean
    numbers of far cells, split cells (all levels) and direct pairs per
    target."""
    if any(lat.walls):
        raise ValueError("the far-field sum is defined for periodic boxes")
    if not 0.0 < theta < 1.0:
        raise ValueError("theta must lie in (0, 1)")
    if levels < 1:
        raise ValueError("levels must be >= 1")
    pos = wrap_positions(pos, lat)
    N = pos.shape[0]
    if targets is None:
        targets = np.arange(N)
    cms = [cell_moments(pos, nxt, lat, h * 2 ** m, kappa) for m in range(levels)]
    parents = [_children(cell_grid(lat, h * 2 ** m)[0]) for m in range(levels - 1)]
    out = np.zeros((len(targets), 3))
    n_far = n_split = n_dir = 0
    for t, j in enumerate(targets):
        r = pos[j]
        v = np.zeros(3)
        consider = np.ones(cms[-1]["centre"].shape[0], dtype=bool)
        for m in range(levels - 1, -1, -1):
            cm = cms[m]
            key, d, y = cm["key"], cm["d"], cm["y"]
            C = cm["centre"].shape[0]
            cl = classify(r, pos, cm, lat, theta)
            kind = np.where(consider, cl["kind"], EMPTY)
            far = kind == FAR
            if far.any():
                v += m2p(-cl["Rlo"][far], cm["M0"][far], cm["M1"][far], cm["M2"][far]) / (4.0 * np.pi)
            split = kind == SPLIT
            if split.any():
                # lower class: the segments of split cells whose class on the
                # crossed axis is the smaller one; the others form the upper
                ks = np.nonzero(split[key])[0]
                kc = key[ks]
                ax = cl["axis"][kc]
                lower = cl["K"][ks, ax] == cl["Kmin"][kc, ax]
                lo, hi = ks[lower], ks[~lower]
                M0l, M1l, M2l = _moments(key[lo], y[lo], d[lo], kappa, C)
                M0h, M1h, M2h = _moments(key[hi], y[hi], d[hi], kappa, C)
                v += m2p(-cl["Rlo"][split], M0l[split], M1l[split], M2l[split]) / (4.0 * np.pi)
                v += m2p(-cl["Rhi"][split], M0h[split], M1h[split], M2h[split]) / (4.0 * np.pi)
            n_far += int(far.sum())
            n_split += int(split.sum())
            opened = kind == NEAR
            if m > 0:
                consider = opened[parents[m - 1]]
                continue
            near = np.nonzero(opened)[0]
            if near.size:
                ks = np.concatenate([cm["order"][cm["starts"][c]:cm["ends"][c]] for c in near])
                ks = ks[(ks != j) & (ks != prv[j])]
                R1 = bs_image_offsets(pos[ks], r[None, :], lat)
                v = v + segment_velocity(R1, R1 + d[ks], kappa).sum(axis=0)
                n_dir += ks.size
        out[t] = v
    T = max(len(targets), 1)
    return out, dict(far=n_far / T, split=n_split / T, direct=n_dir / T)
