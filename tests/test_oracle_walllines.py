"""Pins of open vortex lines bound to the walls (reading F1b of the
closed-channel initial condition of Sec. IV: lines bound to the solid
walls; the line continues into its mirror image in the wall, whose flow is
the image term v_s,b of Sec. II.A, Eq. Biot-Savart).

Each pin compares with something the open-line rules do not compute
themselves: a straight line at rest, the closed form of a finite straight
line (the partner line and its two wall images are one straight line),
the closed full ring evaluated by the closed-loop path (a half ring on a
wall is half of that ring, plus the far wall's image placed by hand),
hand-counted remeshing and small-line removal, and link validation."""

import numpy as np
import pytest

import workloads as wl
from oracle import coupled, diagnostics, topology, vfm
from oracle.lbm import Lattice
from oracle.vfm import VortexParams

KAPPA = 0.1


def _params(**kw):
    base = dict(kappa=KAPPA, alpha=0.0, alpha_p=0.0, wall_images=True)
    base.update(kw)
    return VortexParams(**base)


def _still(lat):
    return np.zeros((3,) + lat.shape)


def test_prev_from_next_and_link_validation():
    lat = Lattice(8, 8, 6, walls=(False, False, True))
    pos, nxt = wl.wall_line((3.0, 4.0), 2, 6, 8)
    prv = coupled.prev_from_next(nxt)
    assert prv[0] == 0 and nxt[-1] == 7
    assert np.array_equal(prv[1:], np.arange(7))
    topology.check_lines(pos, nxt, lat)
    # an end off the wall plane
    bad = pos.copy()
    bad[-1, 2] = 5.4
    with pytest.raises(ValueError):
        topology.check_lines(bad, nxt, lat)
    # an open line on an axis without walls
    with pytest.raises(ValueError):
        topology.check_lines(pos, nxt, Lattice(8, 8, 6))
    # two predecessors
    n2 = nxt.copy()
    n2[3] = 5
    with pytest.raises(ValueError):
        topology.check_lines(pos, n2, lat)
    # a one-point line
    with pytest.raises(ValueError):
        topology.check_lines(pos[:1], np.array([0]), lat)


def test_straight_line_between_walls_is_at_rest():
    """A straight line from wall to wall continues into its images as one
    straight line: every term of its velocity vanishes (no NaN from the
    image segments that meet its ends)."""
    lat = Lattice(16, 16, 12, walls=(False, False, True))
    pos, nxt = wl.wall_line((7.3, 8.1), 2, 12, 15)
    prv = coupled.prev_from_next(nxt)
    out = vfm.line_velocity(pos, nxt, prv, _still(lat), None, lat, _params(), want_force=True)
    assert np.all(np.isfinite(out["sdot"]))
    assert np.abs(out["sdot"]).max() == 0.0
    geo = out["geo"]
    np.testing.assert_array_equal(geo["sp"][[0, -1]], [[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])


@pytest.mark.parametrize("nz", [12, 21])
def test_antiparallel_lines_between_walls(nz):
    """Two straight lines from wall to wall, antiparallel at distance D: with
    the wall images each is a straight line of length 3 nz (z from -nz-1/2
    to 2 nz - 1/2), so each point moves with the finite-line closed form
    k/(4 pi D) (b/sqrt(b^2+D^2) - a/sqrt(a^2+D^2)), perpendicular to the
    pair's plane, both lines the same way."""
    lat = Lattice(24, 24, nz, walls=(False, False, True))
    D = 2.5
    n_pts = nz + 2
    pa, na = wl.wall_line((9.0, 7.0), 2, nz, n_pts)
    pb, nb = wl.wall_line((9.0, 7.0 + D), 2, nz, n_pts, reverse=True)
    pos, nxt = wl.concat_loops([(pa, na), (pb, nb)])
    prv = coupled.prev_from_next(nxt)
    out = vfm.line_velocity(pos, nxt, prv, _still(lat), None, lat, _params())
    lo, hi = -nz - 0.5, 2 * nz - 0.5
    z = pos[:, 2]
    a, b = lo - z, hi - z
    speed = KAPPA / (4 * np.pi * D) * (b / np.sqrt(b * b + D * D) - a / np.sqrt(a * a + D * D))
    want = np.zeros_like(pos)
    want[:, 0] = -speed
    np.testing.assert_allclose(out["sdot"], want, rtol=0, atol=1e-14)
    # without the images the ends feel only the real partner segment
    out0 = vfm.line_velocity(pos, nxt, prv, _still(lat), None, lat, _params(wall_images=False))
    a0, b0 = -0.5 - z, nz - 0.5 - z
    s0 = KAPPA / (4 * np.pi * D) * (b0 / np.sqrt(b0 * b0 + D * D) - a0 / np.sqrt(a0 * a0 + D * D))
    np.testing.assert_allclose(out0["sdot"][:, 0], -s0, rtol=0, atol=1e-14)


def _free_loop_velocity(pts, kappa, vp):
    """v_s of a closed loop alone in space (nearest images never cross):
    the closed-loop path of the oracle on a box far larger than the loop."""
    big = Lattice(4096, 4096, 4096)
    shift = np.array([2048.0, 2048.0, 2048.0]) - pts.mean(axis=0)
    p = pts + shift
    n = p.shape[0]
    nxt = (np.arange(n) + 1) % n
    prv = coupled.prev_from_next(nxt)
    geo = vfm.geometry(p, nxt, prv, big)
    return vfm.biot_savart_nonlocal(p, nxt, prv, big, kappa) + vfm.lia_velocity(geo, vp)


def test_half_ring_on_a_wall_is_half_of_the_full_ring():
    """A half ring standing on the wall z = -1/2 is half of the closed ring
    that its image completes: its v_s equals the full ring's at the same
    points, plus the image in the far wall (sign -1, placed by hand)."""
    nz = 40
    lat = Lattice(32, 32, nz, walls=(False, False, True))
    R, m = 5.0, 18
    th = np.pi * np.arange(m + 1) / m
    half = np.stack([15.0 + R * np.cos(th), np.full(m + 1, 16.0), -0.5 + R * np.sin(th)], 1)
    half[0, 2] = half[-1, 2] = -0.5
    nxt = np.arange(1, m + 2)
    nxt[-1] = m
    prv = coupled.prev_from_next(nxt)
    vp = _params()
    out = vfm.line_velocity(half, nxt, prv, _still(lat), None, lat, vp)
    # the full ring: the half ring, then its mirror image below the wall
    # (points m-1 .. 1 mirrored), closed
    lower = half[m - 1:0:-1].copy()
    lower[:, 2] = -1.0 - lower[:, 2]
    full = np.concatenate([half, lower], axis=0)
    want = _free_loop_velocity(full, KAPPA, vp)[: m + 1]
    # the far wall's image of the half ring, by hand
    far = half.copy()
    far[:, 2] = 2.0 * (nz - 0.5) - far[:, 2]
    seg = half[nxt] - half
    fseg = seg * np.array([1.0, 1.0, -1.0])
    for j in range(m + 1):
        R1 = far - half[j]
        want[j] -= vfm.segment_velocity(R1, R1 + fseg, KAPPA).sum(axis=0)
    np.testing.assert_allclose(out["vs"], want, rtol=0, atol=2e-13)
    # the ends slide on the wall: no velocity normal to it
    assert out["sdot"][0, 2] == 0.0 and out["sdot"][-1, 2] == 0.0
    np.testing.assert_array_equal(out["sdot"][1:-1], out["vs"][1:-1])


def test_end_points_slide_and_carry_half_their_segment():
    """Without images (v_s,b = 0) and with a normal-fluid flow through the
    wall, the ends still keep no normal velocity, an RK4 step leaves them
    on the wall plane exactly, and the force at an end carries half of its
    one real segment (the line length of Sec. II.B is the real length)."""
    nz = 10
    lat = Lattice(16, 16, nz, walls=(False, False, True))
    pos, nxt = wl.wall_line((7.0, 8.0), 2, nz, 13, amp=0.6, turns=1.0, phase=0.1)
    prv = coupled.prev_from_next(nxt)
    ub = np.zeros((3,) + lat.shape)
    ub[0] = 0.004
    ub[2] = 0.01
    vp = VortexParams(kappa=KAPPA, wall_images=False)
    out = vfm.line_velocity(pos, nxt, prv, ub, None, lat, vp, want_force=True)
    assert out["sdot"][0, 2] == 0.0 and out["sdot"][-1, 2] == 0.0
    assert np.abs(out["sdot"][1:-1, 2]).min() > 0.0
    s1, _ = coupled.filament_advance(pos, nxt, prv, ub, None, lat, vp)
    assert s1[0, 2] == -0.5 and s1[-1, 2] == nz - 0.5
    geo = out["geo"]
    l_first = np.linalg.norm(pos[1] - pos[0])
    l_last = np.linalg.norm(pos[-1] - pos[-2])
    sp, sd, vs = geo["sp"], out["sdot"], out["vs"]
    for j, ell in ((0, l_first), (len(pos) - 1, l_last)):
        g = vp.rho_s_over_rho_n * KAPPA * np.cross(sp[j], sd[j] - vs[j]) * (0.5 * ell)
        np.testing.assert_allclose(out["force"][j], g, rtol=1e-15, atol=0)
    # the lengths the points carry add up to the line length (D1)
    total = 0.5 * (geo["lp_real"] + geo["lm_real"]).sum()
    assert total == pytest.approx(diagnostics.line_length(pos, nxt, lat), rel=1e-14)


def test_remesh_keeps_the_ends_and_thins_the_inside():
    """Hand count on one open line (dxi 0.70 / 0.95): the short first
    segment's inner point goes, the short last segment stays (ends are never
    deleted), the long segment is split."""
    nz = 8
    lat = Lattice(12, 12, nz, walls=(False, False, True))
    # the last segment (6.9 -> 7.5) is short too, but only its end could go
    z = np.array([-0.5, -0.3, 0.3, 1.2, 2.1, 3.0, 4.2, 5.1, 6.0, 6.9, 7.5])
    pos = np.stack([np.full(z.size, 5.0), np.full(z.size, 6.0), z], 1)
    nxt = np.arange(1, z.size + 1)
    nxt[-1] = z.size - 1
    prv = coupled.prev_from_next(nxt)
    p2, n2, q2, nd, ni = topology.remesh(pos, nxt, prv, lat, 0.70, 0.95)
    assert (nd, ni) == (1, 1)
    # walk the line from its first point
    order = [0]
    while n2[order[-1]] != order[-1]:
        order.append(n2[order[-1]])
    zz = p2[order, 2]
    want = [-0.5, 0.3, 1.2, 2.1, 3.0, 3.6, 4.2, 5.1, 6.0, 6.9, 7.5]
    np.testing.assert_allclose(zz, want, rtol=0, atol=1e-15)
    assert zz[0] == -0.5 and zz[-1] == 7.5
    topology.check_lines(p2, n2, lat)
    assert np.array_equal(q2, coupled.prev_from_next(n2))


def test_small_lines_and_loops_are_removed():
    """Open lines and closed loops below 5 points go; 5 points stay."""
    lat = Lattice(12, 12, 3, walls=(False, False, True))
    l4 = wl.wall_line((2.0, 2.0), 2, 3, 4)
    l5 = wl.wall_line((6.0, 2.0), 2, 3, 5)
    r4 = wl.ring((3.0, 8.0, 1.0), 0.5, (0.0, 0.0, 1.0), 4)
    r5 = wl.ring((8.0, 8.0, 1.0), 0.6, (0.0, 0.0, 1.0), 5)
    pos, nxt = wl.concat_loops([l4, l5, r4, r5])
    prv = coupled.prev_from_next(nxt)
    alive = topology.small_loops(nxt, 5, prv)
    want = np.array([False] * 4 + [True] * 5 + [False] * 4 + [True] * 5)
    np.testing.assert_array_equal(alive, want)


def test_reconnection_skips_the_last_point_of_a_line():
    """The only close pair involves the last point of a line (it has no
    segment to exchange): no reconnection.  Moved one point inwards, the
    pair of interior points reconnects and the lines stay open with their
    ends on the walls."""
    nz = 6
    lat = Lattice(12, 12, nz, walls=(False, False, True))
    a = wl.wall_line((5.0, 5.0), 2, nz, 8)
    b = wl.wall_line((5.6, 5.0), 2, nz, 8, reverse=True)
    # b's first point sits on the upper wall next to a's last point; move
    # every other point of b away
    pb = b[0].copy()
    pb[1:, 0] += 3.0
    pos, nxt = wl.concat_loops([a, (pb, b[1])])
    prv = coupled.prev_from_next(nxt)
    n2, q2, nr = topology.reconnect(pos, nxt, prv, lat, 0.95)
    # a's last point (7) and b's first (8) are 0.6 apart: 7 has no segment
    assert nr == 0
    # now two antiparallel interior stretches 0.5 apart with short segments
    z = np.array([-0.5, 0.5, 1.1, 1.7, 2.3, 5.5])
    la = np.stack([np.full(6, 4.0), np.full(6, 4.0), z], 1)
    lb = np.stack([np.full(6, 4.5), np.full(6, 4.0), z[::-1]], 1)
    lb[[0, -1], 0] = 8.0  # b's ends far away on the walls
    lb[[0, -1], 2] = [nz - 0.5, -0.5]
    la[-1, 0] = 1.0
    na = np.arange(1, 7)
    na[-1] = 5
    pos = np.concatenate([la, lb])
    nxt = np.concatenate([na, na + 6])
    prv = coupled.prev_from_next(nxt)
    n2, q2, nr = topology.reconnect(pos, nxt, prv, lat, 0.95)
    assert nr >= 1
    topology.check_lines(pos, n2, lat)
    assert np.array_equal(q2, coupled.prev_from_next(n2))
    ks = np.arange(12)
    assert (n2 == ks).sum() == 2 and (q2 == ks).sum() == 2


def test_coupled_steps_keep_the_lines_on_the_walls():
    """A few coupled steps of a small closed channel (lines bound to the end
    walls, two rings, reconnection on): the links stay valid, every open
    line keeps its two ends on the wall planes, nothing is non-finite."""
    cfg = wl.config_closed_channel(nxy=16, nz=24)
    lv = cfg["lattice"]
    lat = Lattice(lv["nx"], lv["ny"], lv["nz"], tau=lv["tau"], walls=lv["walls"],
                  plane_lo=lv["plane_lo"], plane_hi=lv["plane_hi"], plane_u=lv["plane_u"])
    vp = VortexParams(**{k: cfg["vortex"][k] for k in VortexParams.__dataclass_fields__
                         if k in cfg["vortex"]})
    st = coupled.make_state(cfg["rho"], cfg["u"], cfg["pos"], cfg["nxt"], lat)
    topology.check_lines(st.pos, st.nxt, lat)
    for _ in range(3):
        st = coupled.coupled_step(st, lat, vp)
        assert np.all(np.isfinite(st.pos))
        topology.check_lines(st.pos, st.nxt, lat)
        ks = np.arange(st.nxt.shape[0])
        assert (st.nxt == ks).sum() == 4 and (st.prv == ks).sum() == 4
        assert np.array_equal(st.prv, coupled.prev_from_next(st.nxt))
