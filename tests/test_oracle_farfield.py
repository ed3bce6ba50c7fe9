"""Pins of the cell-multipole far-field sum (reading F2) against the direct
sum and the order of its expansion: with every cell near it is the direct
sum; one segment's expansion error falls as the cube of the distance (the
square without the quadrupole term, so a wrong quadrupole shows); on a
random tangle its error stays inside the stated bound; cells whose segment
starts straddle the plane half a box from the target are never far."""

import numpy as np
import pytest

import workloads as wl
from oracle import coupled, farfield, vfm
from oracle.lbm import Lattice

KAPPA = 0.1


def _tangle(n, n_rings, seed, r_lo=2.0, r_hi=5.0):
    lat = Lattice(n, n, n)
    pos, nxt = wl.random_rings(seed, n_rings, r_lo, r_hi, (n, n, n), (False, False, False), 0.95,
                               min_sep=1.0)
    pos = vfm.wrap_positions(pos, lat)
    return lat, pos, nxt, coupled.prev_from_next(nxt)


def test_all_cells_near_is_the_direct_sum():
    lat, pos, nxt, prv = _tangle(32, 12, 3)
    for h in (8, 16):
        got, n_far, _ = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, h, 1e-9)
        assert n_far == 0
        ref = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, KAPPA)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def _one_segment_error(D, quad=True):
    """Expansion of one segment about a centre 0.3 away from its midpoint,
    seen from distance D: |approx - exact| / |exact|."""
    c = np.zeros(3)
    y0 = np.array([0.2, -0.1, 0.2])
    d = np.array([0.5, 0.7, -0.3])
    s = c + y0 - 0.5 * d
    r = np.array([0.6, 0.8, 0.0]) * D + np.array([0.0, 0.0, 0.37])
    exact = vfm.segment_velocity((s - r)[None, :], (s + d - r)[None, :], KAPPA)[0]
    a = KAPPA * d
    M0 = a[None, :]
    M1 = (a[:, None] * y0[None, :])[None]
    M2 = (a[:, None, None] * (np.outer(y0, y0) + np.outer(d, d) / 12.0)[None, :, :])[None]
    if not quad:
        M2 = np.zeros_like(M2)
    approx = farfield.m2p((r - c)[None, :], M0, M1, M2) / (4.0 * np.pi)
    return np.linalg.norm(approx - exact) / np.linalg.norm(exact)


def test_expansion_error_falls_as_the_cube_of_the_distance():
    e = [_one_segment_error(D) for D in (8.0, 16.0, 32.0)]
    assert 6.5 < e[0] / e[1] < 9.5 and 6.5 < e[1] / e[2] < 9.5
    assert e[2] < 1e-4
    # without the quadrupole term the error falls as the square only
    e2 = [_one_segment_error(D, quad=False) for D in (8.0, 16.0, 32.0)]
    assert 3.2 < e2[0] / e2[1] < 4.8 and 3.2 < e2[1] / e2[2] < 4.8


def test_error_bound_on_a_random_tangle():
    """64^3 periodic box, 60 rings: relative L2 error of the non-local
    velocity at 150 sampled targets <= 1e-3 at h = 16, theta = 0.25, and it
    grows with theta."""
    lat, pos, nxt, prv = _tangle(64, 60, 5, 2.0, 6.0)
    t = np.random.default_rng(7).choice(pos.shape[0], 150, replace=False)
    ref = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, KAPPA, targets=t)
    errs = {}
    for theta in (0.25, 0.5):
        got, n_far, n_dir = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, 16, theta,
                                                          targets=t)
        errs[theta] = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert n_far > 0
    assert errs[0.25] <= 1e-3
    assert errs[0.5] > errs[0.25]


def test_cells_straddling_the_half_box_are_never_far():
    """A cell whose segment starts lie on both sides of the plane half a box
    from the target is evaluated directly even when the opening angle would
    accept it."""
    lat = Lattice(64, 64, 64)
    # a short line along x through x = 32.0 (half a box from a target at x = 0)
    xs = np.arange(28.0, 36.5, 0.8)
    pos = np.stack([xs, np.full(xs.size, 40.0), np.full(xs.size, 40.0)], 1)
    nxt = np.concatenate([np.arange(1, xs.size), [xs.size - 1]])  # open: last links to itself
    cm = farfield.cell_moments(pos, nxt, lat, 16, KAPPA)
    target = np.array([0.0, 40.0, 40.0])
    far, R = farfield.far_mask(target, cm, lat, 1.0)
    # the cell around x = 32 holds starts on both sides of the plane x = 32
    c = int(cm["key"][np.searchsorted(xs, 32.0)])
    assert cm["rad"][c] < np.linalg.norm(R[c])  # the opening angle alone would accept it
    assert not far[c]
