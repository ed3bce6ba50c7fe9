"""Pins of the boundary superflow from image vortices (reading F1 of the
superfluid wall term v_s,b in Sec. II.A, Eq. Biot-Savart): closed forms of
straight lines parallel to one and two walled axes, written out here with
the images placed by hand, and the sense of the image flow on a ring that
approaches a wall head-on."""

import numpy as np
import pytest

import workloads as wl
from oracle import coupled, vfm
from oracle.lbm import Lattice
from oracle.vfm import VortexParams

KAPPA = 0.1


def _line(x0, y0, nz):
    """Straight line along +z through (x0, y0): nz points at z = k + 1/2."""
    pos = np.stack([np.full(nz, x0), np.full(nz, y0), np.arange(nz) + 0.5], 1)
    nxt = (np.arange(nz) + 1) % nz
    return pos, nxt


def _finite_line(D, a, b):
    """Speed times 4 pi D / circulation of a straight line from a to b
    (along its direction, measured from the foot of the perpendicular) at
    distance D: b / sqrt(b^2 + D^2) - a / sqrt(a^2 + D^2)."""
    return b / np.sqrt(b * b + D * D) - a / np.sqrt(a * a + D * D)


def _line_images_by_hand(images, x0, y0, nz):
    """Velocity at a point of the line (x0, y0) from image lines along z:
    ``images`` = [(x, y, circulation sign)].  Each image segment is taken at
    the nearest periodic image of its start (odd nz: starts at -(nz-1)/2 ..
    (nz-1)/2 from the target, so the image line covers a = -(nz-1)/2 to
    b = (nz+1)/2)."""
    a, b = -(nz - 1) / 2.0, (nz + 1) / 2.0
    v = np.zeros(3)
    for xi, yi, sgn in images:
        r = np.array([x0 - xi, y0 - yi, 0.0])
        D = np.linalg.norm(r)
        speed = sgn * KAPPA / (4 * np.pi * D) * _finite_line(D, a, b)
        v += speed * np.cross([0.0, 0.0, 1.0], r / D)
    return v


def test_line_parallel_to_one_pair_of_walls():
    """Walls on x only: the images of a line at distance d_lo / d_hi from
    the walls lie at -1 - x0 and 2 n - 1 - x0 with circulation -kappa; the
    line moves parallel to the walls at about kappa/(4 pi)(1/d_hi - 1/d_lo)
    (exactly the finite-line form of the periodic segment sum)."""
    nx, ny, nz = 16, 8, 15
    lat = Lattice(nx, ny, nz, walls=(True, False, False))
    x0, y0 = 3.3, 4.1
    pos, nxt = _line(x0, y0, nz)
    prv = coupled.prev_from_next(nxt)
    got = vfm.biot_savart_images(pos, nxt, coupled.prev_from_next(nxt), lat, KAPPA)
    want = _line_images_by_hand([(-1.0 - x0, y0, -1.0), (2 * nx - 1.0 - x0, y0, -1.0)],
                                x0, y0, nz)
    np.testing.assert_allclose(got, np.tile(want, (nz, 1)), rtol=0, atol=1e-15)
    # direction and size: along -y, near the infinite-line value
    d_lo, d_hi = x0 + 0.5, nx - 0.5 - x0
    assert want[1] < 0 and abs(want[0]) < 1e-18 and want[2] == 0.0
    inf = KAPPA / (4 * np.pi) * (1 / d_hi - 1 / d_lo)
    assert want[1] == pytest.approx(inf, rel=0.25)
    # the whole line velocity: a straight line has no self-induced part
    vp = VortexParams(kappa=KAPPA, wall_images=True)
    out = vfm.line_velocity(pos, nxt, prv, np.zeros((3,) + lat.shape), None, lat, vp)
    np.testing.assert_allclose(out["vs"], np.tile(want, (nz, 1)), rtol=0, atol=1e-15)
    vp0 = VortexParams(kappa=KAPPA)
    out0 = vfm.line_velocity(pos, nxt, prv, np.zeros((3,) + lat.shape), None, lat, vp0)
    np.testing.assert_allclose(out0["vs"], 0.0, atol=1e-17)


def test_line_in_a_channel_corner():
    """Walls on x and y: 4 face images (-kappa) and 4 edge images (+kappa,
    mirrored twice)."""
    nx, ny, nz = 12, 10, 9
    lat = Lattice(nx, ny, nz, walls=(True, True, False))
    x0, y0 = 1.2, 7.9
    pos, nxt = _line(x0, y0, nz)
    xs = {0: x0, 1: -1.0 - x0, 2: 2 * nx - 1.0 - x0}
    ys = {0: y0, 1: -1.0 - y0, 2: 2 * ny - 1.0 - y0}
    images = [(xs[i], ys[k], (-1.0) ** ((i > 0) + (k > 0)))
              for i in range(3) for k in range(3) if (i, k) != (0, 0)]
    want = _line_images_by_hand(images, x0, y0, nz)
    got = vfm.biot_savart_images(pos, nxt, coupled.prev_from_next(nxt), lat, KAPPA)
    np.testing.assert_allclose(got, np.tile(want, (nz, 1)), rtol=0, atol=1e-15)
    assert len(vfm.image_copies(lat)) == 8


def test_ring_approaching_a_wall_is_slowed_and_stretched():
    """A ring moving head-on toward the wall x = -1/2: its image (opposite
    circulation) pushes every point away from the wall and outward, with no
    swirl about the axis."""
    lat = Lattice(32, 32, 32, walls=(True, False, False))
    pos, nxt = wl.ring((4.0, 16.0, 16.0), 3.0, (-1.0, 0.0, 0.0), 40)
    prv = coupled.prev_from_next(nxt)
    vs = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, KAPPA)
    geo = vfm.geometry(pos, nxt, prv, lat)
    v_self = vs + vfm.lia_velocity(geo, VortexParams(kappa=KAPPA))
    assert (v_self[:, 0] < 0).all()        # the ring moves toward the wall
    vb = vfm.biot_savart_images(pos, nxt, coupled.prev_from_next(nxt), lat, KAPPA)
    rad = pos[:, 1:] - 16.0
    rad /= np.linalg.norm(rad, axis=1)[:, None]
    radial = (vb[:, 1:] * rad).sum(axis=1)
    phi = np.stack([-rad[:, 1], rad[:, 0]], 1)
    swirl = (vb[:, 1:] * phi).sum(axis=1)
    assert (vb[:, 0] > 0).all() and (radial > 0).all()
    assert np.abs(swirl).max() < 1e-9 * np.abs(vb).max()


def test_images_equal_mirrored_loops_run_backwards():
    """Circulation -kappa on the mirrored loop equals +kappa on the mirrored
    loop traversed backwards: the image sum equals the plain non-local sum
    over real + mirrored-and-reversed loops, minus the real loops' own sum
    (a tilted ring, whose segments cross the wall normal, next to both walls
    of a closed x axis)."""
    nx = 20
    lat = Lattice(nx, 24, 24, walls=(True, False, False))
    pos, nxt = wl.ring((3.1, 12.0, 12.0), 2.6, (0.6, 1.0, 0.3), 23)
    n = pos.shape[0]
    prv = coupled.prev_from_next(nxt)
    mirrored = [(-1.0 - pos[:, 0]), (2 * nx - 1.0 - pos[:, 0])]
    all_pos, all_nxt = [pos], [nxt]
    for c, mx in enumerate(mirrored):
        mp = pos.copy()
        mp[:, 0] = mx
        all_pos.append(mp)
        all_nxt.append(prv + (c + 1) * n)   # backwards
    P = np.concatenate(all_pos)
    Nx = np.concatenate(all_nxt)
    Pv = coupled.prev_from_next(Nx)
    combined = vfm.biot_savart_nonlocal(P, Nx, Pv, lat, KAPPA, targets=np.arange(n))
    real = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, KAPPA)
    got = vfm.biot_savart_images(pos, nxt, coupled.prev_from_next(nxt), lat, KAPPA)
    np.testing.assert_allclose(got, combined - real, rtol=1e-12, atol=1e-16)
