"""Pins of the cell-multipole far-field sum (reading F2) against the direct
sum and the order of its expansion: with every cell near it is the direct
sum; one segment's expansion error falls as the cube of the distance (the
square without the quadrupole term, so a wrong quadrupole shows); a cell
whose segment starts the half-box plane crosses on one axis is split into
its two image classes, which matches the direct sum where one image would
be wrong by the cell's whole contribution; a cell crossed on two axes is
summed directly; on random tangles with many split cells the error stays
inside the stated bound."""

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


@pytest.mark.parametrize("levels", [1, 2])
def test_all_cells_near_is_the_direct_sum(levels):
    lat, pos, nxt, prv = _tangle(32, 12, 3)
    for h in (4, 8):
        got, st = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, h, 1e-9,
                                                levels=levels)
        assert st["far"] == 0 and st["split"] == 0
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


def _chain_and_ring(target, chain_from, chain_to, n_chain):
    """An open chain of n_chain points from chain_from to chain_to (its last
    point links to itself) and a ring of radius 1 through the target point
    (index n_chain: the evaluation point), positions wrapped into the 64^3
    box."""
    t = np.linspace(0.0, 1.0, n_chain)[:, None]
    chain = np.asarray(chain_from) + t * (np.asarray(chain_to) - np.asarray(chain_from))
    phi = np.arange(12) * (2.0 * np.pi / 12)
    ring = np.asarray(target) + np.stack([np.cos(phi) - 1.0, np.sin(phi), 0.0 * phi], 1)
    pos = np.concatenate([chain, ring])
    pos = vfm.wrap_positions(pos, Lattice(64, 64, 64))
    nxt = np.concatenate([np.arange(1, n_chain), [n_chain - 1],
                          n_chain + (np.arange(1, 13) % 12)])
    return pos, nxt


def test_a_cell_crossed_on_one_axis_is_split_by_image():
    """64^3, h = 8: the target sits at x = 3.8, so the plane x = 35.8 half a
    box away cuts the cell [32, 40) x [40, 48) x [40, 48), whose diagonal
    chain segments start on both sides of it.  The cell is split; each
    class lies at its own image (starts below the plane at +32 on x, the
    others at -32), and the far field then matches the direct sum to the
    expansion error, while the cell's whole moments at one image miss by a
    large part of the cell's own contribution."""
    lat = Lattice(64, 64, 64)
    r = np.array([3.8, 20.2, 20.7])
    pos, nxt = _chain_and_ring(r, [32.4, 40.6, 44.6], [39.2, 47.4, 44.6], 13)
    prv = coupled.prev_from_next(nxt)
    j = 13
    cm = farfield.cell_moments(pos, nxt, lat, 8, KAPPA)
    cl = farfield.classify(r, pos, cm, lat, 0.25)
    c = int(cm["key"][3])
    assert cl["kind"][c] == farfield.SPLIT and cl["axis"][c] == 0
    ks = np.nonzero(cm["key"] == c)[0]
    R1 = vfm.bs_image_offsets(pos[ks], r[None, :], lat)
    lower = cl["K"][ks, 0] == cl["Kmin"][c, 0]
    # the lower class takes the image at -L on x, the upper the one at +L/2
    assert lower.any() and (~lower).any()
    assert np.all(R1[lower, 0] < 0.0) and np.all(R1[~lower, 0] > 0.0)
    assert np.all(pos[ks[lower], 0] >= 35.8) and np.all(pos[ks[~lower], 0] < 35.8)
    got, st = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, 8, 0.25, targets=[j])
    assert st["split"] >= 1
    ref = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, KAPPA, targets=[j])
    cell = vfm.segment_velocity(R1, R1 + cm["d"][ks], KAPPA).sum(axis=0)
    assert np.linalg.norm(got[0] - ref[0]) < 1e-2 * np.linalg.norm(cell)
    # one image for the whole cell is wrong by most of the cell's contribution
    one = farfield.m2p(-cl["Rlo"][c][None], cm["M0"][c][None], cm["M1"][c][None],
                       cm["M2"][c][None]) / (4.0 * np.pi)
    assert np.linalg.norm(one - cell) > 0.5 * np.linalg.norm(cell)


def test_a_cell_crossed_on_two_axes_is_summed_directly():
    """The plane crossings x = 33.3 and y = 33.7 both cut the starts of the
    cell [32, 40) x [32, 40) x [40, 48): it is summed directly."""
    lat = Lattice(64, 64, 64)
    r = np.array([1.3, 1.7, 20.7])
    pos, nxt = _chain_and_ring(r, [32.2, 32.6, 44.6], [38.2, 38.6, 44.6], 9)
    prv = coupled.prev_from_next(nxt)
    cm = farfield.cell_moments(pos, nxt, lat, 8, KAPPA)
    cl = farfield.classify(r, pos, cm, lat, 0.25)
    c = int(cm["key"][2])
    assert (cl["Kmax"][c] > cl["Kmin"][c]).sum() == 2
    assert cl["kind"][c] == farfield.NEAR
    got, _ = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, 8, 0.25, targets=[9])
    ref = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, KAPPA, targets=[9])
    # every chain cell is near or split at this distance; the ring is direct
    np.testing.assert_allclose(got, ref, rtol=1e-3)


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("n,h,n_rings,seed", [(64, 16, 60, 5), (128, 8, 260, 9)])
def test_error_bound_on_a_random_tangle(n, h, n_rings, seed, levels):
    """Random rings: relative L2 error of the non-local velocity at 150
    sampled targets <= 1e-3 at theta = 0.25, larger at theta = 0.5; the
    128^3 box with 8^3 cells has many far and split cells per target, and
    with a second level of 16^3 cells fewer of them."""
    lat, pos, nxt, prv = _tangle(n, n_rings, seed, 2.0, 6.0)
    t = np.random.default_rng(7).choice(pos.shape[0], 150, replace=False)
    ref = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, KAPPA, targets=t)
    errs = {}
    for theta in (0.25, 0.5):
        got, st = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, h, theta, targets=t,
                                                levels=levels)
        errs[theta] = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert st["far"] > 0
        if n == 128:
            assert st["split"] > 20
            if levels == 2:
                # coarse cells stand for groups of fine ones
                _, st1 = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, h, theta,
                                                       targets=t)
                assert st["far"] + st["split"] < st1["far"] + st1["split"]
    assert errs[0.25] <= 1e-3
    assert errs[0.5] > errs[0.25]


def test_line_velocity_switch():
    """VortexParams.ff_cell routes the non-local term of the line velocity
    through the far field: with nothing far (theta tiny) it is the direct
    line velocity, at theta 0.3 it differs by the approximation's size."""
    import dataclasses

    lat, pos, nxt, prv = _tangle(32, 12, 3)
    vp = vfm.VortexParams(kappa=KAPPA)
    ub = np.zeros((3, lat.nz, lat.ny, lat.nx))
    ref = vfm.line_velocity(pos, nxt, prv, ub, None, lat, vp)
    tiny = vfm.line_velocity(pos, nxt, prv, ub, None, lat,
                             dataclasses.replace(vp, ff_cell=8, ff_levels=2, ff_theta=1e-9))
    np.testing.assert_allclose(tiny["vs"], ref["vs"], rtol=0, atol=1e-13 * np.abs(ref["vs"]).max())
    ff = vfm.line_velocity(pos, nxt, prv, ub, None, lat,
                           dataclasses.replace(vp, ff_cell=4, ff_theta=0.3))
    e = np.linalg.norm(ff["vs"] - ref["vs"]) / np.linalg.norm(ref["vs"])
    assert 1e-8 < e < 1e-2
