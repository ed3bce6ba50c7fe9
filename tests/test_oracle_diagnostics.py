"""Pins of the diagnostics oracle (CPU): closed forms, invariants and
hand-derived cases that a dropped term, a wrong sign or a wrong slab rule
would break."""

import numpy as np
import pytest

import workloads as wl
from oracle import diagnostics as dg
from oracle.lbm import Lattice


def _ring(n, R, centre, normal_axis=2, phase=0.0):
    t = 2 * np.pi * (np.arange(n) + phase) / n
    p = np.zeros((n, 3))
    a, b = [k for k in range(3) if k != normal_axis]
    p[:, a] = centre[a] + R * np.cos(t)
    p[:, b] = centre[b] + R * np.sin(t)
    p[:, normal_axis] = centre[normal_axis]
    return p, (np.arange(n) + 1) % n


@pytest.mark.parametrize("n", [8, 37, 64])
def test_polygon_ring_length(n):
    """A regular n-gon of circumradius R has perimeter 2 n R sin(pi / n)."""
    lat = Lattice(40, 40, 40)
    pos, nxt = _ring(n, 7.5, (20.0, 20.0, 20.0))
    assert abs(dg.line_length(pos, nxt, lat) - 2 * n * 7.5 * np.sin(np.pi / n)) < 1e-12


def test_ring_across_periodic_boundary():
    """The same ring shifted across a periodic boundary keeps its length
    (nearest-image segments)."""
    lat = Lattice(16, 16, 16)
    pos, nxt = _ring(24, 5.0, (1.0, 2.0, 8.0))
    pos = np.mod(pos, 16.0)
    assert abs(dg.line_length(pos, nxt, lat) - 2 * 24 * 5.0 * np.sin(np.pi / 24)) < 1e-12


def test_straight_line_fills_every_slab_equally():
    """A straight periodic line along z with points at z = k * L / n + 0.3:
    the length inside every slab is exactly 1."""
    nz = 12
    lat = Lattice(8, 8, nz)
    n = 30
    pos = np.zeros((n, 3))
    pos[:, 0], pos[:, 1] = 3.0, 4.0
    pos[:, 2] = np.mod(np.arange(n) * nz / n + 0.3, nz)
    nxt = (np.arange(n) + 1) % n
    s = dg.line_length_slabs(pos, nxt, lat)
    np.testing.assert_allclose(s, np.ones(nz), rtol=0, atol=1e-12)
    assert abs(dg.line_length(pos, nxt, lat) - nz) < 1e-12


def test_flat_ring_in_one_slab():
    """A ring in a plane of constant z has no z extent: all of its length is
    in the slab of that plane (z = 5.3 lies in [4.5, 5.5))."""
    lat = Lattice(24, 24, 10, walls=(True, True, True))
    pos, nxt = _ring(20, 4.0, (12.0, 12.0, 5.3))
    s = dg.line_length_slabs(pos, nxt, lat)
    total = dg.line_length(pos, nxt, lat)
    assert abs(s[5] - total) < 1e-12 and np.abs(np.delete(s, 5)).max() == 0.0


def test_hand_segment_split():
    """A two-point loop from (2, 1, 1.2) to (2, 4, 2.7) and back: each of its
    two segments (length sqrt(9 + 2.25)) lies 0.3 / 1.5 in slab 1, 1.0 / 1.5
    in slab 2 and 0.2 / 1.5 in slab 3."""
    lat = Lattice(8, 8, 8)
    pos = np.array([[2.0, 1.0, 1.2], [2.0, 4.0, 2.7]])
    nxt = np.array([1, 0])
    s = dg.line_length_slabs(pos, nxt, lat)
    ell = np.sqrt(9.0 + 2.25)
    want = np.zeros(8)
    want[1], want[2], want[3] = 2 * ell * 0.2, 2 * ell * 1.0 / 1.5, 2 * ell * 0.2 / 1.5
    np.testing.assert_allclose(s, want, rtol=0, atol=1e-12)


def test_segment_across_periodic_z_boundary():
    """A segment from z = nz - 0.2 to z = 0.4 (nearest image: +0.6) lies
    entirely in slab 0 = [-1/2, 1/2) wrapped."""
    lat = Lattice(8, 8, 10)
    pos = np.array([[1.0, 1.0, 9.8], [1.0, 1.0, 0.4]])
    s = dg.line_length_slabs(pos, np.array([1, 0]), lat)
    want = np.zeros(10)
    want[0] = 1.2
    np.testing.assert_allclose(s, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("walls", [(False, False, False), (True, True, False), (True, True, True)])
def test_slabs_add_up_to_total(walls):
    dims = (20, 18, 24)
    lat = Lattice(*dims, walls=walls)
    pos, nxt = wl.random_rings(5, 6, 2.0, 5.0, dims, walls, 0.95)
    s = dg.line_length_slabs(pos, nxt, lat)
    assert abs(s.sum() - dg.line_length(pos, nxt, lat)) < 1e-10
    assert s.min() >= 0.0


def test_flow_stats_checkerboard():
    """u_z = c + a (-1)^(x + y) with even nx, ny: every slice has mean c and
    rms |a|; u_x = const has rms 0."""
    nz, ny, nx = 5, 6, 8
    lat = Lattice(nx, ny, nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((3, nz, ny, nx))
    u[0] = 0.01
    u[2] = 0.02 + 3e-4 * (-1.0) ** (x + y)
    sm, srms, m, rms = dg.flow_stats(u, lat)
    np.testing.assert_allclose(sm[:, 2], 0.02, rtol=0, atol=1e-15)
    np.testing.assert_allclose(srms[:, 2], 3e-4, rtol=1e-12)
    np.testing.assert_allclose(srms[:, 0], 0.0, atol=1e-15)
    np.testing.assert_allclose(rms, [0.0, 0.0, 3e-4], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, [0.01, 0.0, 0.02], atol=1e-15)


def test_flow_stats_linear_in_z():
    """u_x = z: each slice is uniform (rms 0, mean z); over the lattice the
    mean is (nz - 1) / 2 and the rms sqrt((nz^2 - 1) / 12)."""
    nz, ny, nx = 9, 4, 4
    lat = Lattice(nx, ny, nz)
    u = np.zeros((3, nz, ny, nx))
    u[0] = np.arange(nz, dtype=float)[:, None, None]
    sm, srms, m, rms = dg.flow_stats(u, lat)
    np.testing.assert_allclose(sm[:, 0], np.arange(nz), atol=1e-14)
    np.testing.assert_allclose(srms[:, 0], 0.0, atol=1e-14)
    assert abs(m[0] - (nz - 1) / 2) < 1e-14
    assert abs(rms[0] - np.sqrt((nz * nz - 1) / 12.0)) < 1e-13


def test_vorticity_sinusoid_closed_form():
    """u_x = sin(2 pi y / ny), u_y = sin(2 pi z / nz) on a periodic lattice:
    the central difference of sin(k y) is cos(k y) sin(k), so
    omega_z = -cos(2 pi y / ny) sin(2 pi / ny) and
    omega_x = -cos(2 pi z / nz) sin(2 pi / nz), omega_y = 0."""
    nz, ny, nx = 10, 12, 6
    lat = Lattice(nx, ny, nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ky, kz = 2 * np.pi / ny, 2 * np.pi / nz
    u = np.zeros((3, nz, ny, nx))
    u[0] = np.sin(ky * y)
    u[1] = np.sin(kz * z)
    w = dg.vorticity(u, lat)
    np.testing.assert_allclose(w[2], -np.cos(ky * y) * np.sin(ky), atol=1e-14)
    np.testing.assert_allclose(w[0], -np.cos(kz * z) * np.sin(kz), atol=1e-14)
    np.testing.assert_allclose(w[1], 0.0, atol=1e-14)


def test_vorticity_at_walls():
    """u_z = 1 with walls on x: beyond the walls u = 0, so
    omega_y = -d u_z / dx is -1/2 at x = 0, +1/2 at x = nx - 1, 0 inside."""
    nz, ny, nx = 4, 5, 6
    lat = Lattice(nx, ny, nz, walls=(True, False, False))
    u = np.zeros((3, nz, ny, nx))
    u[2] = 1.0
    w = dg.vorticity(u, lat)
    want = np.zeros(nx)
    want[0], want[-1] = -0.5, 0.5
    np.testing.assert_allclose(w[1], np.broadcast_to(want, (nz, ny, nx)), atol=1e-15)
    np.testing.assert_allclose(w[0], 0.0, atol=1e-15)
    np.testing.assert_allclose(w[2], 0.0, atol=1e-15)


def test_cylindrical_rigid_rotation():
    """u = Omega x r (rigid rotation about an axis through c) has the
    discrete curl 2 Omega away from the periodic seams; about that axis its
    cylindrical components are (0, 0, 2 |Omega|)."""
    n = 24
    lat = Lattice(n, n, n)
    c = np.array([11.3, 12.1, 12.7])
    om = np.array([0.3, -0.2, 0.5])
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.stack([x - c[0], y - c[1], z - c[2]])
    u = np.stack([om[1] * r[2] - om[2] * r[1], om[2] * r[0] - om[0] * r[2], om[0] * r[1] - om[1] * r[0]])
    w = dg.vorticity(u, lat)
    inner = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    np.testing.assert_allclose(w[inner], np.broadcast_to(2 * om[:, None, None, None], w[inner].shape),
                               atol=1e-12)
    cyl = dg.vorticity_cylindrical(w, lat, c, om)
    np.testing.assert_allclose(cyl[0][inner[1:]], 0.0, atol=1e-12)
    np.testing.assert_allclose(cyl[1][inner[1:]], 0.0, atol=1e-12)
    np.testing.assert_allclose(cyl[2][inner[1:]], 2 * np.linalg.norm(om), atol=1e-12)


def test_cylindrical_hand_case_and_norm():
    """omega = x_hat at the node one unit along +y from an axis along z:
    rho_hat = y_hat, phi_hat = z_hat x y_hat = -x_hat, so (0, -1, 0); on the
    axis the radial and azimuthal parts are 0; the three components keep
    |omega| everywhere off the axis."""
    lat = Lattice(8, 8, 8)
    w = np.zeros((3, 8, 8, 8))
    w[0] = 1.0
    cyl = dg.vorticity_cylindrical(w, lat, (4.0, 3.0, 0.0), (0.0, 0.0, 1.0))
    np.testing.assert_allclose(cyl[:, 5, 4, 4], [0.0, -1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(cyl[:, 2, 3, 4], [0.0, 0.0, 0.0], atol=1e-15)
    rng = np.random.default_rng(3)
    w = rng.standard_normal((3, 8, 8, 8))
    cyl = dg.vorticity_cylindrical(w, lat, (3.7, 4.2, 1.1), (1.0, 2.0, -0.5))
    np.testing.assert_allclose((cyl ** 2).sum(0), (w ** 2).sum(0), rtol=1e-12)
