"""GPU parity of the far-field approximation of the non-local Biot-Savart
sum (vlb_biot_savart_farfield, reading F2) against the oracle of the same
approximation (oracle/farfield.py) through the C ABI: every target of
small periodic tangles (uniform and non-uniform grids, several cell edges
and opening parameters), sampled targets of a 128^3 tangle with many split
cells and of the 256^3 tangle at full size, open lines, determinism, and
the approximation's error against the GPU's direct FP32 sum."""

import numpy as np
import pytest

import workloads as wl
from oracle import coupled, farfield, vfm
from oracle.lbm import Lattice
from tests._cases import rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_04435_amd as vlb  # noqa: E402

KAPPA = 0.1
# FP32 arithmetic against the FP64 oracle of the same approximation
TOL = 1e-5


def _tangle(dims, n_rings, seed, r_lo=2.0, r_hi=6.0):
    lat = Lattice(*dims)
    pos, nxt = wl.random_rings(seed, n_rings, r_lo, r_hi, dims, (False, False, False), 0.95,
                               min_sep=1.0)
    pos = vfm.wrap_positions(pos, lat)
    return lat, pos, nxt, coupled.prev_from_next(nxt)


def _check(got, ref, tag):
    e = rel_l2(got, ref)
    emax = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"{tag}: rel L2 {e:.2e}, max {emax:.2e}")
    assert e <= TOL
    assert emax <= 5 * TOL


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("dims,cell,theta", [
    ((64, 64, 64), 16, 0.5), ((64, 64, 64), 8, 0.25), ((64, 64, 64), 8, 0.6),
    ((64, 64, 128), 8, 0.4), ((48, 48, 48), 6, 0.5)])
def test_farfield_every_target(dims, cell, theta, levels):
    """Small tangles, every target: 64^3 is a uniform grid (direct pairs in
    grid units), 64x64x128 and 48^3 are not (lattice units); one level of
    cells and two."""
    lat, pos, nxt, prv = _tangle(dims, 60, 5)
    say(f"farfield every target {dims} cell {cell} theta {theta} levels {levels}: "
        f"{pos.shape[0]} points")
    got = vlb.biot_savart_farfield(pos, nxt, dims, cell, theta, KAPPA, levels=levels)
    ref, st = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, cell, theta,
                                            levels=levels)
    say(f"  oracle far {st['far']:.1f}, split {st['split']:.1f}, direct {st['direct']:.0f}")
    assert st["far"] > 0
    _check(got, ref, "every target")


@pytest.mark.parametrize("levels", [1, 2])
def test_farfield_many_split_cells(levels):
    """128^3, 8^3 cells (and 16^3 above them), theta 0.25: about 60 split
    cells per target."""
    dims = (128, 128, 128)
    lat, pos, nxt, prv = _tangle(dims, 260, 9)
    say(f"farfield 128^3 split cells, levels {levels}: {pos.shape[0]} points")
    got = vlb.biot_savart_farfield(pos, nxt, dims, 8, 0.25, KAPPA, levels=levels)
    t = np.random.default_rng(3).choice(pos.shape[0], 300, replace=False)
    ref, st = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, 8, 0.25, targets=t,
                                            levels=levels)
    assert st["split"] > 20
    _check(got[t], ref, "128^3 sampled")


def test_farfield_open_lines_and_split_pin():
    """An open chain crossing the half-box plane of a ring's point (the
    oracle's split pin) plus a few rings: every target."""
    dims = (64, 64, 64)
    lat = Lattice(*dims)
    t = np.linspace(0.0, 1.0, 13)[:, None]
    chain = np.array([32.4, 40.6, 44.6]) + t * np.array([6.8, 6.8, 0.0])
    pos_r, nxt_r = wl.random_rings(4, 6, 2.0, 4.0, dims, (False, False, False), 0.95, min_sep=1.0)
    phi = np.arange(12) * (2.0 * np.pi / 12)
    ring = np.array([3.8, 20.2, 20.7]) + np.stack([np.cos(phi) - 1.0, np.sin(phi), 0 * phi], 1)
    pos = vfm.wrap_positions(np.concatenate([chain, ring, pos_r]), lat)
    nxt = np.concatenate([np.arange(1, 13), [12], 13 + (np.arange(1, 13) % 12), 25 + nxt_r])
    prv = coupled.prev_from_next(nxt)
    say(f"farfield open chain: {pos.shape[0]} points")
    for levels in (1, 2):
        got = vlb.biot_savart_farfield(pos, nxt, dims, 8, 0.25, KAPPA, levels=levels)
        ref, st = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, 8, 0.25,
                                                levels=levels)
        assert st["split"] > 0
        _check(got, ref, f"open chain, levels {levels}")


def test_farfield_deterministic_and_degenerate():
    """Two calls give the same bits; one point and no points are handled;
    a cell as large as the box (one cell: nothing is far) is the direct
    sum."""
    dims = (32, 32, 32)
    lat, pos, nxt, prv = _tangle(dims, 12, 3, 2.0, 5.0)
    say(f"farfield determinism: {pos.shape[0]} points")
    for levels in (1, 2):
        a = vlb.biot_savart_farfield(pos, nxt, dims, 8, 0.5, KAPPA, levels=levels)
        b = vlb.biot_savart_farfield(pos, nxt, dims, 8, 0.5, KAPPA, levels=levels)
        assert np.array_equal(a, b)
    one = vlb.biot_savart_farfield(np.array([[1.0, 2.0, 3.0]]), np.array([0]), dims, 8, 0.5, KAPPA)
    assert np.array_equal(one, np.zeros((1, 3)))
    assert vlb.biot_savart_farfield(np.zeros((0, 3)), np.zeros(0, np.int32), dims, 8, 0.5,
                                    KAPPA).shape == (0, 3)
    whole = vlb.biot_savart_farfield(pos, nxt, dims, 32, 0.5, KAPPA)
    direct = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, KAPPA)
    _check(whole, direct, "one cell")


@pytest.mark.parametrize("levels", [1, 2])
def test_farfield_tangle_256_full_size(levels):
    """The 256^3 tangle (2000 rings, about 1e5 points), 16^3 cells (and
    32^3 above them), theta 0.25: 64 sampled targets against the oracle of
    the approximation, and every target against the GPU's direct FP32 sum
    within the approximation's error (relative L2 <= 1e-3)."""
    cfg = wl.config_tangle()
    dims = (256, 256, 256)
    lat = Lattice(*dims)
    pos = vfm.wrap_positions(cfg["pos"], lat)
    nxt = cfg["nxt"]
    prv = coupled.prev_from_next(nxt)
    say(f"farfield 256^3 tangle, levels {levels}: {pos.shape[0]} points")
    got = vlb.biot_savart_farfield(pos, nxt, dims, 16, 0.25, KAPPA, levels=levels)
    t = np.random.default_rng(11).choice(pos.shape[0], 64, replace=False)
    ref, st = farfield.biot_savart_farfield(pos, nxt, prv, lat, KAPPA, 16, 0.25, targets=t,
                                            levels=levels)
    say(f"  oracle far {st['far']:.0f}, split {st['split']:.0f}, direct {st['direct']:.0f}")
    _check(got[t], ref, "256^3 sampled")
    direct = vlb.biot_savart(pos, nxt, dims, kappa=KAPPA, precision="f32")
    e = rel_l2(got, direct)
    say(f"  approximation error against the direct sum: {e:.2e}")
    assert e <= 1e-3


# ---- the far-field sum inside coupled runs (vortex descriptor ff_cell)

RUN_TOL = {"f32": 1e-5, "f16": 1e-3}


def _ff_run_case(precision, levels, n_rings=20):
    """64^3 periodic tangle of 20 rings with mass balance; the non-local sum
    of every stage by the far field (cells of 8, theta 0.3)."""
    cfg = wl.config_tangle(precision=precision, n=64, n_rings=n_rings, seed=5)
    cfg["vortex"] = dict(cfg["vortex"], ff_cell=8, ff_levels=levels, ff_theta=0.3)
    return cfg


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_run_eval_with_farfield(precision, levels):
    """First-stage line velocity, force and spread force of a run whose
    non-local sum is the far field, against the oracle's line velocity with
    the same approximation; it differs from the direct sum's by about the
    approximation's error (so the approximation is the one in use)."""
    import dataclasses

    from oracle import lbm
    from tests._cases import oracle_state

    cfg = _ff_run_case(precision, levels)
    say(f"run eval with far field {precision} levels {levels}: {cfg['pos'].shape[0]} points")
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    F_g = run.read_force()
    lat, vp, st = oracle_state(cfg)
    assert vp.ff_cell == 8 and vp.ff_levels == levels
    _, ub = lbm.bare_velocity(st.f, lat)
    Vs = lbm.mass_balance_superflow(st.f, lat, vp.rho_s_over_rho_n) if vp.mass_balance else None
    ref = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, Vs, lat, vp, want_force=True)
    for k in ("vs", "vn", "sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(f"  {k}: {err:.2e}")
        assert err <= RUN_TOL[precision], (k, err)
    F_o = vfm.spread(ref["force"], st.pos, lat)
    assert rel_l2(F_g, F_o) <= RUN_TOL[precision]
    direct = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, Vs, lat,
                               dataclasses.replace(vp, ff_cell=0))
    e = rel_l2(got["vs"], direct["vs"])
    say(f"  against the direct sum: {e:.2e}")
    assert 1e-7 < e < 1e-2
    run.close()


def test_run_steps_with_farfield():
    """FP32 coupled steps with the two-level far field against the oracle's
    steps with the same approximation: links equal after every step,
    positions within 1e-4, velocity field within 1e-5."""
    from oracle import lbm
    from tests._cases import oracle_state

    cfg = _ff_run_case("f32", 2)
    say(f"run steps with far field: {cfg['pos'].shape[0]} points")
    run = vlb.run_from_config(cfg)
    lat, vp, st = oracle_state(cfg)
    for k in range(3):
        run.step(1)
        run.sync()
        st = coupled.coupled_step(st, lat, vp)
        pos_g, nxt_g = run.read_filaments()
        assert nxt_g.shape == st.nxt.shape and (nxt_g == st.nxt).all(), k
        d = np.abs(vfm.min_image(pos_g - st.pos, lat)).max()
        say(f"  step {k + 1}: max position difference {d:.2e}")
        assert d < 1e-4
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) <= 1e-5
    run.close()


def test_run_farfield_graph_replay_matches_direct_steps():
    """Steps with the far field replayed from a captured HIP graph are
    bitwise equal to steps enqueued one by one (several replays)."""
    cfg = _ff_run_case("f16", 2)
    say("run far field graph replay")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        direct = vlb.run_from_config(cfg)
    with torch.cuda.stream(s2):
        graphed = vlb.run_from_config(cfg)
        for _ in range(3):
            direct.step(4)
            graphed.step_graph(4)
            direct.sync()
            graphed.sync()
            pa, na = direct.read_filaments()
            pb, nb = graphed.read_filaments()
            np.testing.assert_array_equal(na, nb)
            np.testing.assert_array_equal(pa, pb)
            np.testing.assert_array_equal(direct.read_populations(), graphed.read_populations())
    direct.close()
    graphed.close()
