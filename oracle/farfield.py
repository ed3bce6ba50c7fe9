"""Cell-multipole approximation of the non-local Biot-Savart sum, plain
FP64 (an extension for large tangles: Sec. II.A computes the full
non-local integral, which grows as N^2 while the tangles of Sec. III.C
grow; reading F2).  Test infrastructure only (see the package docstring):
the reference of the far-field analysis, which has no GPU counterpart in
the library (the direct sum is kept; the analysis is in the pins).

The box is cut into a uniform grid of cells of edge h_a = L_a / nc_a.  Each
segment k (start s_k, vector d_k at the nearest image, circulation kappa)
belongs to the cell of its midpoint m_k.  About the cell centre c the
segment's vorticity kappa d_k is spread along y = m_k - c + t d_k,
t in [-1/2, 1/2]; its moments are
    M0 = sum kappa d,  M1 = sum kappa d (x) y,
    M2 = sum kappa d (x) (y (x) y + d (x) d / 12).
The field of a vortex element a at offset y seen from r, a x (r - y) /
|r - y|^3 / (4 pi), expanded about the centre to second order in y, gives
the cell's velocity at R = r - c (nearest image of the centre)
    v_m = eps_mnp g_np / (4 pi),
    g_np = M0_n R_p / r^3 - M1_np / r^3 + 3 (M1 R)_n R_p / r^5
         + (15 (R M2_n R) R_p / r^7 - 3 tr(M2_n) R_p / r^5 - 6 (M2_n R)_p / r^5) / 2.
A cell is far from target r when |R| theta >= rad (rad: the largest
|y| + |d|/2 of its segments) and, on every periodic axis a,
|R_a| + ext_a < L_a / 2 (ext_a: the largest |s_k,a - c_a| of its segment
starts), so that every segment start of the cell takes the nearest image
of the centre (reading R12 decides images per segment start).  Far cells
contribute their expansion; every other cell contributes the exact
straight-segment integrals of its segments (nearest image per segment
start, the target's own two segments excluded, as in
vfm.biot_savart_nonlocal).  Decisions are made in FP64 with the sums
written left to right.
"""

import numpy as np

from .lbm import Lattice
from .vfm import bs_image_offsets, min_image, segment_velocity


def cell_grid(lat: Lattice, h):
    """Cells per axis and their edge: nc_a = L_a / h (h must divide L_a)."""
    nc = []
    for n in lat.dims:
        if n % h:
            raise ValueError("the cell edge must divide every box length")
        nc.append(n // h)
    return np.array(nc, dtype=np.int64), np.array([float(h)] * 3)


def cell_moments(pos, nxt, lat: Lattice, h, kappa):
    """Segment cells and the per-cell moments (see the module docstring).
    Returns a dict: key (N,), order (segments sorted by cell, stable),
    starts / ends (per cell), centre (C, 3), M0 (C, 3), M1 (C, 3, 3),
    M2 (C, 3, 3, 3), rad (C,), ext (C, 3)."""
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
    a = kappa * d
    M0 = np.zeros((C, 3))
    M1 = np.zeros((C, 3, 3))
    M2 = np.zeros((C, 3, 3, 3))
    np.add.at(M0, key, a)
    np.add.at(M1, key, a[:, :, None] * y[:, None, :])
    yy = y[:, :, None] * y[:, None, :] + d[:, :, None] * d[:, None, :] / 12.0
    np.add.at(M2, key, a[:, :, None, None] * yy[:, None, :, :])
    ny = np.sqrt(y[:, 0] * y[:, 0] + y[:, 1] * y[:, 1] + y[:, 2] * y[:, 2])
    nd = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
    rad = np.zeros(C)
    np.maximum.at(rad, key, ny + 0.5 * nd)
    ext = np.zeros((C, 3))
    np.maximum.at(ext, key, np.abs(min_image(pos - centre[key], lat)))
    order = np.argsort(key, kind="stable")
    starts = np.searchsorted(key[order], cid)
    ends = np.searchsorted(key[order], cid, side="right")
    return dict(key=key, order=order, starts=starts, ends=ends, centre=centre, M0=M0, M1=M1,
                M2=M2, rad=rad, ext=ext, d=d)


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


def far_mask(r, cm, lat: Lattice, theta):
    """Which cells are far from target r (module docstring): (C,) bool.
    Empty cells are never far (they add nothing either way)."""
    R = min_image(r[None, :] - cm["centre"], lat)
    d2 = R[:, 0] * R[:, 0] + R[:, 1] * R[:, 1] + R[:, 2] * R[:, 2]
    far = (d2 * (theta * theta) >= cm["rad"] * cm["rad"]) & (cm["ends"] > cm["starts"])
    for a, n in enumerate(lat.dims):
        if lat.walls[a]:
            continue
        far &= np.abs(R[:, a]) + cm["ext"][:, a] < 0.5 * float(n)
    return far, R


def biot_savart_farfield(pos, nxt, prv, lat: Lattice, kappa, h, theta, targets=None):
    """Non-local superfluid velocity at ``targets`` (default: all) by the
    cell-multipole approximation (module docstring).  Returns (T, 3) and the
    mean numbers of far cells and direct pairs per target."""
    if any(lat.walls):
        raise ValueError("the far-field sum is defined for periodic boxes")
    N = pos.shape[0]
    if targets is None:
        targets = np.arange(N)
    cm = cell_moments(pos, nxt, lat, h, kappa)
    d = cm["d"]
    out = np.zeros((len(targets), 3))
    n_far = 0
    n_dir = 0
    for t, j in enumerate(targets):
        r = pos[j]
        far, R = far_mask(r, cm, lat, theta)
        v = m2p(R[far], cm["M0"][far], cm["M1"][far], cm["M2"][far]) / (4.0 * np.pi) \
            if far.any() else np.zeros(3)
        near = np.nonzero(~far & (cm["ends"] > cm["starts"]))[0]
        if near.size:
            ks = np.concatenate([cm["order"][cm["starts"][c]:cm["ends"][c]] for c in near])
            ks = ks[(ks != j) & (ks != prv[j])]
            R1 = bs_image_offsets(pos[ks], r[None, :], lat)
            v = v + segment_velocity(R1, R1 + d[ks], kappa).sum(axis=0)
            n_dir += ks.size
        n_far += int(far.sum())
        out[t] = v
    return out, n_far / max(len(targets), 1), n_dir / max(len(targets), 1)
