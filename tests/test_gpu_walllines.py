"""GPU parity of open vortex lines bound to the walls (the closed-channel
initial condition of Sec. IV; reading F1b) against the oracle, through the
C ABI: first-stage line velocity, force and spread force with and without
the wall images, coupled steps with exact topology and the ends kept on
their wall planes, the seeding checks, and the stand-alone Biot-Savart sum
of open lines."""

import numpy as np
import pytest

import workloads as wl
from oracle import coupled, lbm, topology, vfm
from tests._cases import oracle_state, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_04435_amd as vlb  # noqa: E402

TOL = {"f64": 1e-10, "f32": 1e-5, "f16": 1e-3}


def _case(precision, images=True, nxy=16, nz=24, seed=6):
    cfg = wl.config_closed_channel(precision=precision, nxy=nxy, nz=nz, seed=seed)
    if not images:
        cfg["vortex"] = dict(cfg["vortex"], wall_images=False)
    return cfg


def _ends(nxt, prv):
    ks = np.arange(nxt.shape[0])
    return np.nonzero((nxt == ks) | (prv == ks))[0]


@pytest.mark.parametrize("images", [True, False])
@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_wall_lines_eval(precision, images):
    cfg = _case(precision, images)
    say("wall lines eval", precision, images, cfg["pos"].shape[0])
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    F_g = run.read_force()
    lat, vp, st = oracle_state(cfg)
    _, ub = lbm.bare_velocity(st.f, lat)
    Vs = lbm.mass_balance_superflow(st.f, lat, vp.rho_s_over_rho_n) if vp.mass_balance else None
    ref = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, Vs, lat, vp, want_force=True)
    F_o = vfm.spread(ref["force"], st.pos, lat)
    for k in ("vs", "vn", "sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err <= TOL[precision], (k, err)
    assert rel_l2(F_g, F_o) <= TOL[precision]
    ends = _ends(st.nxt, st.prv)
    assert ends.size == 8
    # the ends slide on the z walls
    assert np.all(got["sdot"][ends, 2] == 0.0)
    run.close()


def test_wall_lines_coupled_f64():
    """Coupled FP64 steps (remeshing, reconnection, images): links exact,
    positions and the lattice within 1e-10, ends on the wall planes."""
    cfg = _case("f64")
    say("wall lines coupled f64")
    run = vlb.run_from_config(cfg)
    lat, vp, st = oracle_state(cfg)
    for s in range(8):
        run.step(1)
        st = coupled.coupled_step(st, lat, vp)
        run.sync()
        pos_g, nxt_g = run.read_filaments()
        np.testing.assert_array_equal(nxt_g, st.nxt)
        assert np.abs(vfm.min_image(pos_g - st.pos, lat)).max() < 1e-10, s
    ends = _ends(st.nxt, st.prv)
    assert ends.size == 8
    assert np.all(np.isin(pos_g[ends, 2], (-0.5, lat.nz - 0.5)))
    topology.check_lines(pos_g, nxt_g, lat)
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) < 1e-10
    run.close()


def test_wall_lines_steps_reduced_precision():
    """FP32 and FP16 storage: the ends stay exactly on their planes and the
    lines stay valid over coupled steps."""
    for precision in ("f32", "f16"):
        cfg = _case(precision)
        say("wall lines steps", precision)
        run = vlb.run_from_config(cfg)
        lat, _, _ = oracle_state(cfg)
        run.step(10)
        run.sync()
        pos_g, nxt_g = run.read_filaments()
        assert np.all(np.isfinite(pos_g))
        topology.check_lines(pos_g, nxt_g, lat)
        prv = coupled.prev_from_next(nxt_g)
        ends = _ends(nxt_g, prv)
        assert ends.size == 8
        assert np.all(np.isin(pos_g[ends, 2], (-0.5, lat.nz - 0.5)))
        run.close()


def test_seed_checks_open_lines():
    cfg = _case("f64")
    run = vlb.Run(cfg["lattice"], cfg["vortex"], n_cap=2 * cfg["pos"].shape[0])
    pos, nxt = cfg["pos"], cfg["nxt"]
    bad = []
    p = pos.copy(); p[0, 2] = -0.4; bad.append((p, nxt))          # an end off its plane
    q = nxt.copy(); q[5] = 5; bad.append((pos, q))                # a new end off the walls
    q = nxt.copy(); q[3] = q[2]; bad.append((pos, q))             # two predecessors
    q = nxt.copy(); q[0] = 0; bad.append((pos, q))                # a one-point line
    for p, q in bad:
        with pytest.raises(vlb.VlbError) as ei:
            run.seed(p, q)
        assert ei.value.code == vlb.VLB_EINVAL
    # an open line along a periodic axis
    cfgp = dict(cfg, lattice=dict(cfg["lattice"], walls=(False, False, False)))
    runp = vlb.Run(cfgp["lattice"], cfgp["vortex"], n_cap=2 * pos.shape[0])
    with pytest.raises(vlb.VlbError):
        runp.seed(pos, nxt)
    runp.close()
    run.seed(pos, nxt)
    got, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, nxt)
    run.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_standalone_biot_savart_open_lines(precision):
    """The stand-alone sum (no images) of open lines and loops: the last
    point's zero segment adds nothing, the first point has no incoming
    segment to exclude."""
    cfg = _case("f64")
    lat, vp, st = oracle_state(cfg)
    v = vlb.biot_savart(st.pos, st.nxt, lat.dims, lat.walls, kappa=vp.kappa,
                        precision=precision)
    ref = vfm.biot_savart_nonlocal(st.pos, st.nxt, st.prv, lat, vp.kappa)
    err = rel_l2(v, ref)
    say("standalone", precision, err)
    assert err <= TOL[precision]


def _ring_meets_line():
    """A ring 0.62 beside a wall-bound line, oriented so that the two
    reconnect in the first step (the ring becomes part of the line)."""
    lat = wl.lattice_preset(16, 16, 24, tau=0.8, walls=(False, False, True), precision="f64")
    vor = wl.vortex_preset(reconnect=True, wall_images=True)
    rho, u = wl.velocity_field(9, (16, 16, 24), (0.0, 0.0, 0.0), 1e-4)
    line = wl.wall_line((8.0, 8.0), 2, 24, int(np.ceil(24 / 0.85)) + 1)
    ring = wl.ring((10.62, 8.0, 11.8), 2.0, (0.0, -1.0, 0.0), 14)
    pos, nxt = wl.concat_loops([line, ring])
    return dict(name="ring_meets_line", lattice=lat, vortex=vor, rho=rho, u=u, pos=pos, nxt=nxt)


def test_ring_reconnects_with_a_wall_line_f64():
    cfg = _ring_meets_line()
    say("ring meets line")
    run = vlb.run_from_config(cfg)
    lat, vp, st = oracle_state(cfg)
    n_rec = 0
    for s in range(6):
        run.step(1)
        st = coupled.coupled_step(st, lat, vp)
        n_rec += st.stats["reconnections"]
        run.sync()
        pos_g, nxt_g = run.read_filaments()
        np.testing.assert_array_equal(nxt_g, st.nxt)
        assert np.abs(vfm.min_image(pos_g - st.pos, lat)).max() < 1e-10, s
    assert n_rec >= 1
    ks = np.arange(nxt_g.shape[0])
    assert (nxt_g == ks).sum() == 1
    topology.check_lines(pos_g, nxt_g, lat)
    run.close()


def _state(run):
    buf, step = run.read_state()
    pos, nxt = run.read_filaments()
    return buf.cpu().numpy(), pos, nxt, step


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_wall_lines_checkpoint_resume_bitwise(precision):
    """Checkpoint at an odd step (swapped AA layout) of a closed channel and
    resume in a new run: bitwise equal to the uninterrupted run."""
    cfg = _case(precision)
    say("wall lines checkpoint", precision)
    a = vlb.run_from_config(cfg)
    a.step(5)
    a.sync()
    buf, step = a.read_state()
    pos, nxt = a.read_filaments()
    b = vlb.Run(cfg["lattice"], cfg["vortex"], a.n_cap)
    b.write_state(buf, step)
    b.seed(pos, nxt)
    a.step(6)
    b.step(6)
    a.sync()
    b.sync()
    sa, sb = _state(a), _state(b)
    for x, y in zip(sa[:3], sb[:3]):
        np.testing.assert_array_equal(x, y)
    assert sa[3] == sb[3]
    a.close()
    b.close()


def test_wall_lines_graph_replay_matches_direct_steps():
    """Steps of a closed channel replayed from a captured HIP graph are
    bitwise equal to steps enqueued one by one (several replays)."""
    cfg = _case("f32")
    say("wall lines graph replay")
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


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_wall_lines_coupled_reduced_precision(precision):
    """Step by step against the FP64 oracle: the links equal the oracle's
    after every step, positions agree to the precision form's tolerance."""
    cfg = _case(precision)
    say("wall lines coupled", precision)
    run = vlb.run_from_config(cfg)
    lat, vp, st = oracle_state(cfg)
    for k in range(8):
        run.step(1)
        run.sync()
        st = coupled.coupled_step(st, lat, vp)
        pos_g, nxt_g = run.read_filaments()
        assert nxt_g.shape == st.nxt.shape and (nxt_g == st.nxt).all(), k
        d = np.abs(vfm.min_image(pos_g - st.pos, lat)).max()
        assert d < (1e-4 if precision == "f32" else 1e-2), (k, d)
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) <= TOL[precision]
    run.close()


def test_wall_lines_step_many_equals_single_runs():
    """Closed channels of three seeds advanced by one vlb_step_many call are
    bitwise equal to the same runs stepped one by one."""
    cfgs = [_case("f32", seed=s) for s in (6, 7, 8)]
    together = [vlb.run_from_config(c) for c in cfgs]
    alone = [vlb.run_from_config(c) for c in cfgs]
    vlb.step_many(together, 5)
    for r in alone:
        r.step(5)
    for a, b in zip(together, alone):
        a.sync()
        b.sync()
        pa, na = a.read_filaments()
        pb, nb = b.read_filaments()
        np.testing.assert_array_equal(na, nb)
        np.testing.assert_array_equal(pa, pb)
        np.testing.assert_array_equal(a.read_populations(), b.read_populations())
    for r in together + alone:
        r.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_wall_lines_eval_full_size(precision):
    """The closed-channel workload at its full size (48 x 48 x 128, 692
    points, the bench's configuration): first-stage line velocity, force and
    spread force against the oracle."""
    cfg = wl.config_closed_channel(precision=precision)
    say("wall lines full size", precision, cfg["pos"].shape[0])
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    F_g = run.read_force()
    lat, vp, st = oracle_state(cfg)
    _, ub = lbm.bare_velocity(st.f, lat)
    ref = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, None, lat, vp, want_force=True)
    F_o = vfm.spread(ref["force"], st.pos, lat)
    for k in ("vs", "vn", "sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err <= TOL[precision], (k, err)
    assert rel_l2(F_g, F_o) <= TOL[precision]
    run.close()
