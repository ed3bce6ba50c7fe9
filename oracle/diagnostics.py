"""Diagnostics of the coupled state, plain FP64 (paper Sec. III.A, III.C, IV).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper judges its runs by the vortex line length and line density
(Sec. III.C, Fig. VLD (a); Sec. IV, Fig. Wall_density: total length and the
density along the channel), by the fluctuations of the normal-fluid velocity
about its mean, component by component (Sec. III.C, Eq. for v_n = V_n +
delta v_n, Fig. VLD (b)-(c)), and by the vorticity omega = curl v of the
normal fluid (Sec. III.A).  The readings taken where the paper gives no
discrete definition:

  D1  The filament is the chain of straight segments s_j -> s_next(j) at the
      nearest periodic image (as in the Biot-Savart sum).  The line length
      inside the slab of node z is measured along the z axis, the slab being
      [z - 1/2, z + 1/2) (periodic z wraps); a segment is split in
      proportion to its z extent, and a segment with no z extent belongs to
      the slab of its start point.
  D2  The velocity statistics use the bare velocity u_b = sum c f / sum f of
      the current populations (velocity planes applied), the field the
      filaments see.  Per z slice: the mean of each component and the root
      mean square of its deviation from that mean; over the whole lattice:
      the same with the lattice mean.
  D3  The vorticity is the curl of u_b by central differences; periodic
      axes wrap, and a node beyond a wall carries u = 0 (the convention of
      the interpolation, R14).
  D5  Cylindrical components about an axis (point, direction): see
      vorticity_cylindrical.
"""

import numpy as np

from .lbm import Lattice
from .vfm import min_image


def segment_vectors(pos, nxt, lat: Lattice):
    """s_next(j) - s_j at the nearest periodic image (D1)."""
    pos = np.asarray(pos, dtype=np.float64)
    return min_image(pos[np.asarray(nxt)] - pos, lat)


def line_length(pos, nxt, lat: Lattice):
    """Total vortex line length: the sum of the segment lengths (D1)."""
    d = segment_vectors(pos, nxt, lat)
    return float(np.sqrt((d * d).sum(axis=1)).sum())


def _slab_of(z, lat: Lattice):
    """Index of the slab [k - 1/2, k + 1/2) that contains coordinate z."""
    k = int(np.floor(z + 0.5))
    if lat.walls[2]:
        return min(max(k, 0), lat.nz - 1)
    return k % lat.nz


def line_length_slabs(pos, nxt, lat: Lattice):
    """Line length inside each z slab (D1): every segment's length is split
    over the slabs its z extent crosses, in proportion to the overlap."""
    pos = np.asarray(pos, dtype=np.float64)
    d = segment_vectors(pos, nxt, lat)
    ell = np.sqrt((d * d).sum(axis=1))
    nz = lat.nz
    out = np.zeros(nz)
    slab_lo = np.arange(nz) - 0.5
    images = (0,) if lat.walls[2] else (-1, 0, 1)
    for j in range(pos.shape[0]):
        a = pos[j, 2]
        b = a + d[j, 2]
        lo, hi = min(a, b), max(a, b)
        if hi == lo:
            out[_slab_of(a, lat)] += ell[j]
            continue
        for k in images:
            s_lo = slab_lo + k * nz
            s_hi = s_lo + 1.0
            ov = np.maximum(0.0, np.minimum(hi, s_hi) - np.maximum(lo, s_lo))
            out += ell[j] * ov / (hi - lo)
    return out


def flow_stats(u, lat: Lattice):
    """Velocity statistics of a vector field u of shape (3, nz, ny, nx) (D2).
    Returns (slice_mean, slice_rms, mean, rms) with shapes (nz, 3), (nz, 3),
    (3,), (3,)."""
    u = np.asarray(u, dtype=np.float64)
    sm = u.mean(axis=(2, 3))                     # (3, nz)
    srms = np.sqrt(((u - sm[:, :, None, None]) ** 2).mean(axis=(2, 3)))
    m = u.mean(axis=(1, 2, 3))
    rms = np.sqrt(((u - m[:, None, None, None]) ** 2).mean(axis=(1, 2, 3)))
    return sm.T.copy(), srms.T.copy(), m, rms


def _shifted(f, lat: Lattice, a, s):
    """Scalar field f (nz, ny, nx) at x + s e_a (s = +-1): periodic axes
    wrap, beyond a wall the value is 0 (D3)."""
    ax = 2 - a
    g = np.roll(f, -s, axis=ax)
    if lat.walls[a]:
        idx = [slice(None)] * 3
        idx[ax] = -1 if s > 0 else 0
        g[tuple(idx)] = 0.0
    return g


def _ddx(f, lat: Lattice, a):
    return 0.5 * (_shifted(f, lat, a, 1) - _shifted(f, lat, a, -1))


def vorticity(u, lat: Lattice):
    """omega = curl u by central differences (D3); u and omega have shape
    (3, nz, ny, nx)."""
    u = np.asarray(u, dtype=np.float64)
    ux, uy, uz = u
    wx = _ddx(uz, lat, 1) - _ddx(uy, lat, 2)
    wy = _ddx(ux, lat, 2) - _ddx(uz, lat, 0)
    wz = _ddx(uy, lat, 0) - _ddx(ux, lat, 1)
    return np.stack([wx, wy, wz])


def vorticity_cylindrical(w, lat: Lattice, point, direction):
    """Cylindrical components (omega_rho, omega_phi, omega_axis) of a vector
    field w (3, nz, ny, nx) about the axis through ``point`` along
    ``direction`` (Sec. III.A: the vorticity of a ring in the cylindrical
    frame of its axis).  Reading D5: a node's offset from the point is taken
    at the nearest periodic image; rho_hat is the unit offset perpendicular
    to the axis and phi_hat = axis x rho_hat; on the axis itself (no
    perpendicular offset) omega_rho = omega_phi = 0."""
    w = np.asarray(w, dtype=np.float64)
    a = np.asarray(direction, dtype=np.float64)
    a = a / np.sqrt((a * a).sum())
    z, y, x = np.meshgrid(np.arange(lat.nz), np.arange(lat.ny), np.arange(lat.nx), indexing="ij")
    r = np.stack([x - point[0], y - point[1], z - point[2]], axis=-1).astype(np.float64)
    r = min_image(r, lat)
    ra = (r * a).sum(axis=-1)
    rp = r - ra[..., None] * a
    n = np.sqrt((rp * rp).sum(axis=-1))
    with np.errstate(invalid="ignore", divide="ignore"):
        rho_hat = np.where(n[..., None] > 0, rp / n[..., None], 0.0)
    phi_hat = np.cross(a, rho_hat)
    wv = np.moveaxis(w, 0, -1)
    out = np.stack([(wv * rho_hat).sum(-1), (wv * phi_hat).sum(-1), (wv * a).sum(-1)])
    return out
