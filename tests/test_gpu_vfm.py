"""GPU parity of the filament side and of the coupled step against the
oracle, through the C ABI: line velocity (Biot-Savart + LIA + superflow +
interpolation + Schwarz), mutual-friction force and its spreading, full
coupled steps, topology (exact integers)."""

import numpy as np
import pytest

import workloads as wl
from oracle import coupled, lbm, topology, vfm
from tests._cases import oracle_state, rel_l2, say, small_channel, small_periodic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_04435_amd as vlb  # noqa: E402

# velocity tolerance (relative L2 over all points / nodes)
TOL = {"f64": 1e-10, "f32": 1e-5, "f16": 1e-3}

CASES = {
    "ring32": lambda p: wl.config_ring32(precision=p),
    "channel": lambda p: small_channel(precision=p),
    "periodic": lambda p: small_periodic(precision=p),
    "heater": lambda p: small_channel(precision=p, planes=True, seed=23),
    # more than 512 LBM blocks: the update beside the filament kernels
    # strides its narrow grid over them
    "wide": lambda p: small_channel(precision=p, seed=28, n_rings=8, nxy=64, nz=40),
}


def _oracle_eval(cfg):
    lat, vp, st = oracle_state(cfg)
    _, ub = lbm.bare_velocity(st.f, lat)
    Vs = lbm.mass_balance_superflow(st.f, lat, vp.rho_s_over_rho_n) if vp.mass_balance else None
    out = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, Vs, lat, vp, want_force=True)
    F = vfm.spread(out["force"], st.pos, lat)
    return out, F, st


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_line_velocity_and_force(case, precision):
    cfg = CASES[case](precision)
    say("eval", case, precision, cfg["pos"].shape[0], "points")
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    F_g = run.read_force()
    ref, F_o, st = _oracle_eval(cfg)
    pos_g, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, st.nxt)
    np.testing.assert_array_equal(pos_g, st.pos)
    tol = TOL[precision]
    for k in ("vs", "vn", "sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err <= tol, (k, err)
    errF = rel_l2(F_g, F_o)
    say("spread force", errF)
    assert errF <= tol


@pytest.mark.parametrize("n_cap", [13312, 40000])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_line_velocity_large_capacity(n_cap, precision):
    # The Biot-Savart launch is sized by the capacity: with a few hundred
    # points in it most source chunks hold a handful of sources (some
    # waves get none) and the last chunks are empty; the sum must not care.
    cfg = CASES["channel"](precision)
    say("eval large capacity", precision, cfg["pos"].shape[0], "points, n_cap", n_cap)
    run = vlb.run_from_config(cfg, n_cap=n_cap)
    got = run.eval_line_velocity()
    ref, _, _ = _oracle_eval(cfg)
    tol = TOL[precision]
    for k in ("vs", "sdot"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err <= tol, (k, err)
    run.close()


@pytest.mark.parametrize("case", ["ring32", "channel", "heater", "wide"])
def test_coupled_steps_f64(case):
    cfg = CASES[case]("f64")
    steps = 12
    say("coupled", case, steps)
    run = vlb.run_from_config(cfg)
    run.step(steps)
    run.sync()
    lat, vp, st = oracle_state(cfg)
    for _ in range(steps):
        st = coupled.coupled_step(st, lat, vp)
    pos_g, nxt_g = run.read_filaments()
    # no topology event may differ: compare integer links exactly
    np.testing.assert_array_equal(nxt_g, st.nxt)
    d = vfm.min_image(pos_g - st.pos, lat)
    assert np.abs(d).max() < 1e-10
    rho_g, u_g = run.read_fields()
    rho_o, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) < 1e-10
    np.testing.assert_allclose(rho_g, rho_o, rtol=0, atol=1e-12)


@pytest.mark.parametrize("case", ["channel", "wide"])
@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_coupled_steps_reduced_precision(precision, case):
    """Step by step against the FP64 oracle: the topology (links) must be
    the oracle's after every step, and then positions and velocity agree to
    the precision form's tolerance."""
    cfg = CASES[case](precision)
    steps = 10
    say("coupled reduced", case, precision)
    run = vlb.run_from_config(cfg)
    lat, vp, st = oracle_state(cfg)
    for k in range(steps):
        run.step(1)
        run.sync()
        st = coupled.coupled_step(st, lat, vp)
        pos_g, nxt_g = run.read_filaments()
        assert nxt_g.shape == st.nxt.shape and (nxt_g == st.nxt).all(), \
            f"{precision} topology differs from the oracle's after step {k + 1}"
        d = vfm.min_image(pos_g - st.pos, lat)
        assert np.abs(d).max() < (1e-4 if precision == "f32" else 1e-2), (k, np.abs(d).max())
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    err = rel_l2(u_g, u_o)
    say("velocity", err)
    assert err <= TOL[precision]


def test_ring32_hundred_steps_f64():
    """The plain small case in full: 32^3 periodic lattice, one ring of 64
    points, 100 coupled FP64 steps against the oracle: links exact,
    positions within 1e-10, velocity field and line velocity within 1e-10
    (relative L2)."""
    cfg = wl.config_ring32(precision="f64")
    say("ring32 100 steps")
    run = vlb.run_from_config(cfg)
    lat, vp, st = oracle_state(cfg)
    for _ in range(10):
        run.step(10)
        for _ in range(10):
            st = coupled.coupled_step(st, lat, vp)
        run.sync()
        pos_g, nxt_g = run.read_filaments()
        np.testing.assert_array_equal(nxt_g, st.nxt)
        assert np.abs(vfm.min_image(pos_g - st.pos, lat)).max() < 1e-10
    assert run.get_step() == 100
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) < 1e-10
    got = run.eval_line_velocity()
    _, ub = lbm.bare_velocity(st.f, lat)
    ref = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, None, lat, vp, want_force=True)
    for k in ("vs", "vn", "sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err < 1e-10, (k, err)
    run.close()


def test_ring_relations_in_fluid_at_rest_f64():
    """Sec. II.A, Eq. (E of M) for a circular ring in a normal fluid at rest
    (v_n = 0): the line moves with (1 - alpha') V along its axis and shrinks
    at alpha V, V the self-induced speed, which the GPU's own v_s gives."""
    n = 32
    lat = wl.lattice_preset(n, n, n, tau=0.8, precision="f64")
    vor = wl.vortex_preset(alpha=0.2, alpha_p=0.05, coupling=False)
    pos, nxt = wl.ring((16.0, 16.0, 16.0), 8.0, (0.0, 0.0, 1.0), 64, phase=0.5)
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    cfg = dict(name="ring_at_rest", lattice=lat, vortex=vor, rho=rho, u=u, pos=pos, nxt=nxt,
               steps=1)
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    pos_g, _ = run.read_filaments()
    radial = pos_g[:, :2] - 16.0
    radial /= np.linalg.norm(radial, axis=1)[:, None]
    V = got["vs"][:, 2]
    assert np.abs(got["vn"]).max() < 1e-15
    np.testing.assert_allclose(got["sdot"][:, 2], (1.0 - 0.05) * V, rtol=1e-12, atol=0)
    dr = (got["sdot"][:, :2] * radial).sum(axis=1)
    np.testing.assert_allclose(dr, -0.2 * V, rtol=1e-12, atol=0)
    run.close()


def test_interpolation_exact_on_a_linear_field_f64():
    """The two-point delta interpolation (Sec. II.B, Eq. delta_2pt) is
    trilinear, so it reproduces a linear normal-fluid velocity u = A x + b
    at every point whose stencil lies away from the periodic seams."""
    n = 32
    lat = wl.lattice_preset(n, n, n, tau=0.8, precision="f64")
    A = np.array([[1e-4, -2e-4, 3e-4], [2e-4, 1e-4, -1e-4], [-3e-4, 2e-4, 2e-4]])
    b = np.array([0.002, -0.001, 0.004])
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X = np.stack([x, y, z]).astype(np.float64)
    u = np.einsum("ab,b...->a...", A, X) + b[:, None, None, None]
    rho = np.ones((n, n, n))
    pos, nxt = wl.ring((15.3, 16.1, 15.7), 6.0, (0.3, -0.4, 0.866), 48, phase=0.5)
    cfg = dict(name="linear_field", lattice=lat, vortex=wl.vortex_preset(coupling=False),
               rho=rho, u=u, pos=pos, nxt=nxt, steps=1)
    run = vlb.run_from_config(cfg)
    vn = run.eval_line_velocity()["vn"]
    p, _ = run.read_filaments()
    want = p @ A.T + b
    np.testing.assert_allclose(vn, want, rtol=0, atol=1e-15)
    run.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_thin_ring_speed_closed_form(precision):
    """Biot-Savart sum plus LIA term (Sec. II.A, reading R3, C = 1/2) of a
    thin ring, R = 8, a = 1e-3, 64 segments, in a 64^3 box: the self-induced
    speed is the closed form kappa / (4 pi R) (ln(8 R / a) - 1/2) to within
    1% (the discrete ring is faster by a chord-versus-arc offset of about
    +0.65%), the same at every point, along the axis."""
    n = 64
    lat = wl.lattice_preset(n, n, n, tau=0.8, precision=precision)
    kappa, R, a = 0.1, 8.0, 1e-3
    vor = wl.vortex_preset(kappa=kappa, core_a=a, coupling=False)
    pos, nxt = wl.ring((32.0, 32.0, 32.0), R, (0.0, 0.0, 1.0), 64, phase=0.5)
    cfg = dict(name="thin_ring", lattice=lat, vortex=vor, rho=np.ones((n, n, n)),
               u=np.zeros((3, n, n, n)), pos=pos, nxt=nxt, steps=1)
    run = vlb.run_from_config(cfg)
    vs = run.eval_line_velocity()["vs"]
    closed = kappa / (4.0 * np.pi * R) * (np.log(8.0 * R / a) - 0.5)
    V = vs[:, 2]
    say("ring speed / closed form", V.mean() / closed)
    assert abs(V.mean() / closed - 1.0) < 0.01
    assert 0.0 < V.mean() / closed - 1.0
    assert np.abs(V - V.mean()).max() < (1e-12 if precision == "f64" else 1e-6) * V.mean()
    assert np.abs(vs[:, :2]).max() < (1e-12 if precision == "f64" else 1e-6) * V.mean()
    run.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_spread_force_sums_to_the_point_forces(precision):
    """Spreading with delta_2pt weights that sum to one (Sec. II.B) keeps
    the total: away from walls the lattice force field adds up to the sum
    of the point forces."""
    cfg = small_periodic(precision=precision)
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    F = run.read_force()
    tot_pts = got["force"].sum(axis=0)
    tot_lat = F.reshape(3, -1).sum(axis=1)
    scale = np.abs(got["force"]).sum(axis=0)
    tol = 1e-13 if precision == "f64" else 1e-6
    assert (np.abs(tot_lat - tot_pts) <= tol * scale).all(), (tot_lat, tot_pts)
    run.close()


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_ring32_hundred_steps_reduced_precision(precision):
    """The precision forms over the plain small case: 100 coupled steps with
    FP32 or FP16 population storage against the FP64 oracle; the ring stays
    inside the remeshing bounds (no topology event), so the links stay the
    oracle's; velocity field and line velocity within the form's tolerance
    (FP32 1e-5, FP16 1e-3, relative L2)."""
    cfg = wl.config_ring32(precision=precision)
    say("ring32 100 steps", precision)
    run = vlb.run_from_config(cfg)
    lat, vp, st = oracle_state(cfg)
    for _ in range(10):
        run.step(10)
        for _ in range(10):
            st = coupled.coupled_step(st, lat, vp)
        run.sync()
        pos_g, nxt_g = run.read_filaments()
        np.testing.assert_array_equal(nxt_g, st.nxt)
        d = np.abs(vfm.min_image(pos_g - st.pos, lat)).max()
        assert d < (1e-4 if precision == "f32" else 1e-2), d
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    err = rel_l2(u_g, u_o)
    say("velocity field", err, "positions", d)
    assert err <= TOL[precision]
    got = run.eval_line_velocity()
    ref = vfm.line_velocity(st.pos, st.nxt, st.prv, u_o, None, lat, vp, want_force=True)
    for k in ("vs", "vn", "sdot"):
        e = rel_l2(got[k], ref[k])
        say(k, e)
        assert e <= TOL[precision], (k, e)
    run.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["channel", "periodic"])
def test_applied_superflow_eval(case, precision):
    """A nonzero applied superflow v_s,a (Eq. Biot-Savart) in the line
    velocity, the force and the spread force field."""
    cfg = CASES[case](precision)
    cfg["vortex"] = dict(cfg["vortex"], vs_applied=(0.004, -0.003, 0.006))
    say("applied superflow", case, precision)
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    F_g = run.read_force()
    ref, F_o, _ = _oracle_eval(cfg)
    for k in ("vs", "vn", "sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err <= TOL[precision], (k, err)
    assert rel_l2(F_g, F_o) <= TOL[precision]
    # the applied term is really in: without it v_s differs by about its size
    cfg0 = dict(cfg, vortex=dict(cfg["vortex"], vs_applied=(0.0, 0.0, 0.0)))
    ref0, _, _ = _oracle_eval(cfg0)
    assert rel_l2(got["vs"], ref0["vs"]) > 100 * TOL[precision]
    run.close()


def _perturbed_rings(seed, n_rings, dims, walls, amp):
    pos, nxt = wl.random_rings(seed, n_rings, 2.5, 5.0, dims, walls, 0.95)
    rng = np.random.default_rng(seed + 100)
    pos = pos + amp * rng.standard_normal(pos.shape)
    return pos, nxt


@pytest.mark.parametrize("walls", [(False, False, False), (True, True, False)])
def test_remesh_exact(walls):
    dims = (24, 24, 32)
    lat = wl.lattice_preset(*dims, walls=walls, precision="f64")
    vor = wl.vortex_preset()
    pos, nxt = _perturbed_rings(41, 12, dims, walls, 0.3)
    say("remesh", walls, pos.shape[0])
    run = vlb.Run(lat, vor, n_cap=2 * pos.shape[0])
    run.seed(pos, nxt)
    stats = run.apply_topology()
    pos_g, nxt_g = run.read_filaments()
    from tests._cases import oracle_lattice, oracle_vortex
    olat = oracle_lattice(lat)
    p0 = vfm.wrap_positions(pos, olat)
    p1, n1, q1, st = topology.topology_update(p0, nxt, coupled.prev_from_next(nxt), olat,
                                              oracle_vortex(vor))
    say("stats gpu", stats, "oracle", st)
    assert stats["deleted"] == st["deleted"] and stats["inserted"] == st["inserted"]
    assert st["deleted"] > 0 and st["inserted"] > 0
    np.testing.assert_array_equal(nxt_g, n1)
    np.testing.assert_array_equal(pos_g, p1)


def _long_candidate_runs():
    """Loops whose points are all deletion candidates (regular 30/33/34/40/64
    and 150-gons of side 0.45, centred in separate places) plus one loop
    with an open run of 40 candidates (an arc of 41 sides of 0.45 closed by
    sides of about 0.81): the oracle thins every run, however long."""
    loops = []
    for i, L in enumerate((30, 33, 34, 40, 64, 150)):
        R = 0.45 / (2.0 * np.sin(np.pi / L))
        th = 2.0 * np.pi * (np.arange(L) + 0.5) / L
        c = (24.0 + 0.0 * i, 24.0, 4.0 + 7.5 * i)
        pts = np.stack([c[0] + R * np.cos(th), c[1] + R * np.sin(th), np.full(L, c[2])], 1)
        loops.append((pts, (np.arange(L) + 1) % L))
    R = 10.0
    t1 = 2.0 * np.arcsin(0.45 / (2.0 * R))
    rest = 2.0 * np.pi - 41 * t1
    th = np.concatenate([np.arange(42) * t1, 41 * t1 + np.arange(1, 55) * rest / 55])
    pts = np.stack([12.0 + R * np.cos(th), 12.0 + R * np.sin(th), np.full(th.size, 47.0)], 1)
    loops.append((pts, (np.arange(th.size) + 1) % th.size))
    return wl.concat_loops(loops)


def test_remesh_long_runs_exact():
    dims = (48, 48, 56)
    lat = wl.lattice_preset(*dims, precision="f64")
    vor = wl.vortex_preset()
    pos, nxt = _long_candidate_runs()
    say("remesh long runs", pos.shape[0])
    run = vlb.Run(lat, vor, n_cap=2 * pos.shape[0])
    run.seed(pos, nxt)
    from tests._cases import oracle_lattice, oracle_vortex
    olat = oracle_lattice(lat)
    p0, n0 = vfm.wrap_positions(pos, olat), nxt
    for rnd in range(3):
        stats = run.apply_topology()
        pos_g, nxt_g = run.read_filaments()
        p0, n0, _, st = topology.topology_update(p0, n0, coupled.prev_from_next(n0), olat,
                                                 oracle_vortex(vor))
        say("round", rnd, "gpu", stats, "oracle", st)
        assert stats["deleted"] == st["deleted"] and stats["inserted"] == st["inserted"]
        np.testing.assert_array_equal(nxt_g, n0)
        np.testing.assert_array_equal(pos_g, p0)
        if rnd == 0:
            # floor(L / 2) of each all-candidate loop, half the open run
            assert st["deleted"] == 15 + 16 + 17 + 20 + 32 + 75 + 20
    run.close()


def test_reconnection_exact():
    dims = (16, 16, 16)
    lat = wl.lattice_preset(*dims, precision="f64")
    vor = wl.vortex_preset(reconnect=True, remesh=False)
    # antiparallel lines 0.3 apart (pairwise annihilation) plus a tangle of
    # perturbed rings with many close approaches
    n = 20
    z = (np.arange(n) + 0.5) * 16 / n
    a = np.stack([np.full(n, 7.0), np.full(n, 8.0), z], 1)
    b = np.stack([np.full(n, 7.3), np.full(n, 8.0), z], 1)
    rp, rn = _perturbed_rings(43, 25, dims, (False,) * 3, 0.2)
    pos = np.concatenate([a, b, rp])
    nxt = np.concatenate([(np.arange(n) + 1) % n, n + (np.arange(n) - 1) % n, rn + 2 * n])
    say("reconnect", pos.shape[0])
    run = vlb.Run(lat, vor, n_cap=2 * pos.shape[0], recon_cap=1 << 14)
    run.seed(pos, nxt)
    stats = run.apply_topology()
    pos_g, nxt_g = run.read_filaments()
    from tests._cases import oracle_lattice, oracle_vortex
    olat = oracle_lattice(lat)
    p0 = vfm.wrap_positions(pos, olat)
    p1, n1, q1, st = topology.topology_update(p0, nxt, coupled.prev_from_next(nxt), olat,
                                              oracle_vortex(vor))
    say("stats gpu", stats, "oracle", st)
    assert st["reconnections"] >= 20
    assert stats["reconnections"] == st["reconnections"]
    np.testing.assert_array_equal(nxt_g, n1)
    np.testing.assert_array_equal(pos_g, p1)


def test_no_vortices_is_pure_lbm():
    cfg = small_channel(precision="f64")
    say("no vortices")
    run = vlb.Run(cfg["lattice"], cfg["vortex"], n_cap=16)
    run.write_fields(cfg["rho"], cfg["u"])
    run.step(4)
    run.sync()
    lat, vp, st = oracle_state(cfg)
    f = st.f
    for _ in range(4):
        f = lbm.lbm_step(f, np.zeros((3,) + lat.shape), lat)
    np.testing.assert_allclose(run.read_populations(), f, rtol=0, atol=1e-14)
    assert run.n_points() == 0


def test_capacity_overflow_reported():
    dims = (24, 24, 24)
    lat = wl.lattice_preset(*dims, precision="f64")
    vor = wl.vortex_preset()
    # a ring with spacing 1.9: every segment gets a midpoint -> 2x points
    pos, nxt = wl.ring((12.0, 12.0, 12.0), 6.0, (0, 0, 1), 20)
    run = vlb.Run(lat, vor, n_cap=25)
    run.seed(pos, nxt)
    say("capacity")
    with pytest.raises(vlb.VlbError) as ei:
        run.apply_topology()
    assert ei.value.code == vlb.VLB_ECAPACITY
    assert run.n_points() == 20  # insertion skipped, state intact


def _final_state(run):
    pos, nxt = run.read_filaments()
    return pos, nxt, run.read_populations()


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_bitwise_deterministic(precision):
    """No atomics on floating-point sums: two runs give identical bits."""
    cfg = small_channel(precision=precision, reconnect=True, seed=24)
    say("determinism", precision)
    outs = []
    for _ in range(2):
        run = vlb.run_from_config(cfg)
        run.step(8)
        run.sync()
        outs.append(_final_state(run))
        run.close()
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)


def test_graph_replay_matches_direct_steps():
    """Steps replayed from a captured HIP graph are bitwise equal to steps
    enqueued one by one (several replays, with eager work in between)."""
    cfg = small_channel(precision="f32", reconnect=True, seed=25)
    say("graph replay")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        direct = vlb.run_from_config(cfg)
    with torch.cuda.stream(s2):
        graphed = vlb.run_from_config(cfg)
    with torch.cuda.stream(s2):
        for _ in range(3):
            direct.step(4)
            graphed.step_graph(4)
            direct.sync()
            graphed.sync()
            a = _final_state(direct)
            b = _final_state(graphed)
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)
        assert graphed.get_step() == 12
        direct.close()
        graphed.close()


def test_one_call_equals_single_steps():
    """n steps in one call (the next step's moments computed at the end of
    the previous step on the side stream) are bitwise equal to n calls of
    one step (each forking and joining the side stream)."""
    cfg = small_channel(precision="f32", reconnect=True, seed=26)
    say("one call vs single steps")
    a = vlb.run_from_config(cfg)
    b = vlb.run_from_config(cfg)
    a.step(6)
    for _ in range(6):
        b.step(1)
    a.sync()
    b.sync()
    for x, y in zip(_final_state(a), _final_state(b)):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_uncoupled_run(precision):
    """Coupling off: the filaments move in the normal fluid, which evolves
    as if they were absent (no spreading, no force in the LBM update)."""
    cfg = small_channel(precision=precision)
    cfg["vortex"] = dict(cfg["vortex"], coupling=False)
    steps = 6
    say("uncoupled", precision)
    run = vlb.run_from_config(cfg)
    run.step(steps)
    run.sync()
    lat, vp, st = oracle_state(cfg)
    assert not vp.coupling
    for _ in range(steps):
        st = coupled.coupled_step(st, lat, vp)
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) <= TOL[precision]
    pos_g, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, st.nxt)
    d = vfm.min_image(pos_g - st.pos, lat)
    assert np.abs(d).max() < (1e-10 if precision == "f64" else 1e-4)
    assert np.abs(run.read_force()).max() == 0.0


def test_all_loops_vanish():
    """A loop shorter than the minimum is removed by the first topology
    pass; the run continues with no points as a pure LBM run."""
    cfg = small_channel(precision="f64")
    pos, nxt = wl.ring((8.0, 8.0, 16.0), 0.6, (0, 0, 1), 4)
    cfg = dict(cfg, pos=pos, nxt=nxt)
    say("all loops vanish")
    run = vlb.run_from_config(cfg)
    run.step(3)
    run.sync()
    assert run.n_points() == 0
    lat, vp, st = oracle_state(cfg)
    for _ in range(3):
        st = coupled.coupled_step(st, lat, vp)
    assert st.pos.shape[0] == 0
    np.testing.assert_allclose(run.read_populations(), st.f, rtol=0, atol=1e-12)


def _bundle(n_b, r=0.4, nz=20, L=16.0):
    """Line A along +z through (8, 8) and n_b lines along -z at distance r
    around it: every point of A has one exchange candidate on each B line."""
    z = (np.arange(nz) + 0.5) * L / nz
    pos = [np.stack([np.full(nz, 8.0), np.full(nz, 8.0), z], 1)]
    nxt = [(np.arange(nz) + 1) % nz]
    for m in range(n_b):
        ang = 2 * np.pi * m / n_b
        pos.append(np.stack([np.full(nz, 8.0 + r * np.cos(ang)), np.full(nz, 8.0 + r * np.sin(ang)), z], 1))
        nxt.append((m + 1) * nz + (np.arange(nz) - 1) % nz)
    return np.concatenate(pos), np.concatenate(nxt)


def test_reconnection_slot_overflow_skips():
    """More candidates at one point than its slots: the step reports
    VLB_ECAPACITY and leaves the links unchanged (reconnection skipped)."""
    lat = wl.lattice_preset(16, 16, 16, precision="f64")
    vor = wl.vortex_preset(reconnect=True, remesh=False)
    pos, nxt = _bundle(9)
    say("slot overflow", pos.shape[0])
    run = vlb.Run(lat, vor, n_cap=2 * pos.shape[0], recon_cap=1 << 14)
    run.seed(pos, nxt)
    with pytest.raises(vlb.VlbError) as ei:
        run.apply_topology()
    assert ei.value.code == vlb.VLB_ECAPACITY
    _, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, nxt)
    # with slots to spare (4 lines) the same kind of bundle reconnects
    pos4, nxt4 = _bundle(4)
    run4 = vlb.Run(lat, vor, n_cap=2 * pos4.shape[0], recon_cap=1 << 14)
    run4.seed(pos4, nxt4)
    stats = run4.apply_topology()
    assert stats["reconnections"] > 0


def test_reconnection_list_capacity_skips():
    """More candidates in the step than recon_cap: VLB_ECAPACITY, links
    unchanged."""
    lat = wl.lattice_preset(16, 16, 16, precision="f64")
    vor = wl.vortex_preset(reconnect=True, remesh=False)
    pos, nxt = _bundle(2)
    say("list capacity", pos.shape[0])
    run = vlb.Run(lat, vor, n_cap=2 * pos.shape[0], recon_cap=4)
    run.seed(pos, nxt)
    with pytest.raises(vlb.VlbError) as ei:
        run.apply_topology()
    assert ei.value.code == vlb.VLB_ECAPACITY
    _, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, nxt)


def test_nonfinite_velocity_is_flagged():
    """A non-finite normal-fluid field makes the line velocity non-finite:
    the step latches VLB_ENUMERIC, reported by the next sync; positions
    that blew up still index inside the lattice (no fault)."""
    cfg = small_channel(precision="f64")
    u = cfg["u"].copy()
    u[:] = np.nan
    cfg = dict(cfg, u=u)
    say("non-finite")
    run = vlb.run_from_config(cfg)
    run.step(2)
    with pytest.raises(vlb.VlbError) as ei:
        run.sync()
    assert ei.value.code == vlb.VLB_ENUMERIC
    run.close()


def test_graph_rejects_odd_parity():
    """A graph captured at one AA / point-array parity refuses to launch
    after an odd number of direct steps, and launches again after the next
    one; the replay then matches direct stepping."""
    cfg = small_channel(precision="f32", seed=27)
    say("graph parity")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = vlb.run_from_config(cfg)
        d = vlb.run_from_config(cfg)
        h = g.graph(2)
        g.step(1)
        d.step(1)
        # the C ABI refuses the graph captured at the other parity
        assert g.lib.vlb_graph_launch(h) == vlb.VLB_ESTATE
        g.step(1)
        d.step(1)
        assert g.lib.vlb_graph_launch(h) == vlb.VLB_OK
        d.step(2)
        # the binding captures a second graph at the odd parity
        g.step(1)
        d.step(1)
        g.step_graph(2)
        d.step(2)
        g.sync()
        d.sync()
        assert g.get_step() == d.get_step() == 7
        for x, y in zip(_final_state(g), _final_state(d)):
            np.testing.assert_array_equal(x, y)
        g.close()
        d.close()


def test_seed_rejects_invalid_positions():
    """Seeding checks on the host: a coordinate more than one length outside
    the box, a non-finite one, or a next[] that is not a permutation gives
    VLB_EINVAL and leaves the run usable; one period out is wrapped."""
    lat = wl.lattice_preset(16, 16, 16, walls=(True, False, False), precision="f64")
    vor = wl.vortex_preset()
    pos, nxt = wl.random_rings(31, 1, 3.0, 4.0, (16, 16, 16), (True, False, False), 0.95)
    say("seed checks", pos.shape[0])
    run = vlb.Run(lat, vor, n_cap=2 * pos.shape[0])
    bad_cases = []
    p = pos.copy(); p[0, 1] = -17.0; bad_cases.append((p, nxt))  # periodic y, two periods
    p = pos.copy(); p[0, 0] = 40.0; bad_cases.append((p, nxt))   # wall x, beyond one mirror
    p = pos.copy(); p[0, 2] = np.inf; bad_cases.append((p, nxt))
    q = nxt.copy(); q[1] = q[0]; bad_cases.append((pos, q))
    for p, q in bad_cases:
        with pytest.raises(vlb.VlbError) as ei:
            run.seed(p, q)
        assert ei.value.code == vlb.VLB_EINVAL
    p = pos.copy(); p[:, 2] -= 16.0  # one period below on z
    run.seed(p, nxt)
    got, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, nxt)
    np.testing.assert_allclose(got, pos, rtol=0, atol=1e-12)
    run.close()


def test_graph_rejects_seeding_after_lattice_only_capture():
    """A graph captured before any filament was seeded replays the lattice
    alone: after seeding it refuses to launch (VLB_ESTATE)."""
    lat = wl.lattice_preset(16, 16, 16, precision="f32")
    vor = wl.vortex_preset()
    pos, nxt = wl.random_rings(32, 1, 3.0, 4.0, (16, 16, 16), (False, False, False), 0.95)
    say("graph seeding")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        run = vlb.Run(lat, vor, n_cap=2 * pos.shape[0])
        run.graph(2)
        run.step_graph(2)
        run.seed(pos, nxt)
        with pytest.raises(vlb.VlbError) as ei:
            run.step_graph(2)
        assert ei.value.code == vlb.VLB_ESTATE
        run.step(2)
        run.sync()
        run.close()


def _with_friction_profile(cfg):
    nz = cfg["lattice"]["nz"]
    z = np.arange(nz)
    vor = dict(cfg["vortex"])
    vor["alpha_z"] = tuple(0.2 + 0.08 * np.sin(2 * np.pi * z / nz))
    vor["alpha_p_z"] = tuple(0.01 + 0.006 * np.cos(2 * np.pi * z / nz))
    return dict(cfg, vortex=vor)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_friction_profile_line_velocity(precision):
    """alpha(z), alpha'(z) profiles: the line velocity and force of the
    first stage against the oracle."""
    cfg = _with_friction_profile(CASES["channel"](precision))
    say("friction profile eval", precision)
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    ref, F_o, _ = _oracle_eval(cfg)
    for k in ("vs", "sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err <= TOL[precision], (k, err)
    run.close()


@pytest.mark.parametrize("case", ["channel", "periodic"])
def test_friction_profile_coupled_f64(case):
    cfg = _with_friction_profile(CASES[case]("f64"))
    steps = 8
    say("friction profile coupled", case)
    run = vlb.run_from_config(cfg)
    run.step(steps)
    run.sync()
    lat, vp, st = oracle_state(cfg)
    assert vp.alpha_z is not None
    for _ in range(steps):
        st = coupled.coupled_step(st, lat, vp)
    pos_g, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, st.nxt)
    assert np.abs(vfm.min_image(pos_g - st.pos, lat)).max() < 1e-10
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) < 1e-10
    run.close()


def test_friction_profile_reset_and_graph():
    """Restoring the constants gives bitwise the run that never had a
    profile; a graph captured before the profile was set follows it."""
    cfg = small_channel(precision="f32", seed=30)
    prof = _with_friction_profile(cfg)["vortex"]
    say("friction profile reset / graph")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = vlb.run_from_config(cfg)
        b = vlb.run_from_config(cfg)
        b.set_friction_profile(prof["alpha_z"], prof["alpha_p_z"])
        b.set_friction_profile(None, None)
        a.step(4)
        b.step(4)
        for x, y in zip(_final_state(a), _final_state(b)):
            np.testing.assert_array_equal(x, y)
        g = vlb.run_from_config(cfg)
        d = vlb.run_from_config(cfg)
        g.graph(2)
        g.set_friction_profile(prof["alpha_z"], prof["alpha_p_z"])
        d.set_friction_profile(prof["alpha_z"], prof["alpha_p_z"])
        g.step_graph(2)
        d.step(2)
        g.sync()
        d.sync()
        for x, y in zip(_final_state(g), _final_state(d)):
            np.testing.assert_array_equal(x, y)
        # and the profile changes the result
        a2 = vlb.run_from_config(cfg)
        a2.step(2)
        a2.sync()
        assert not np.array_equal(_final_state(a2)[0], _final_state(d)[0])
        with pytest.raises(ValueError):
            a.set_friction_profile(prof["alpha_z"][:-1], prof["alpha_p_z"][:-1])
        one = np.zeros(1)
        assert a.lib.vlb_set_friction_profile(a.h, None, one.ctypes.data) == vlb.VLB_EINVAL
        bad = np.array(prof["alpha_z"])
        bad[3] = np.nan
        with pytest.raises(vlb.VlbError):
            a.set_friction_profile(bad, prof["alpha_p_z"])
        for r in (a, b, g, d, a2):
            r.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_literal_force_model_eval(precision):
    """force_model 1 (the printed Eq. (f), for ablation): the per-point force
    and its spreading against the oracle."""
    cfg = CASES["channel"](precision)
    cfg = dict(cfg, vortex=dict(cfg["vortex"], force_model=1))
    say("literal force eval", precision)
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    F_g = run.read_force()
    ref, F_o, _ = _oracle_eval(cfg)
    for k in ("sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err <= TOL[precision], (k, err)
    assert rel_l2(F_g, F_o) <= TOL[precision]
    run.close()


def test_literal_force_model_coupled_f64():
    cfg = CASES["channel"]("f64")
    cfg = dict(cfg, vortex=dict(cfg["vortex"], force_model=1))
    steps = 8
    say("literal force coupled")
    run = vlb.run_from_config(cfg)
    run.step(steps)
    run.sync()
    lat, vp, st = oracle_state(cfg)
    assert vp.force_model == 1
    for _ in range(steps):
        st = coupled.coupled_step(st, lat, vp)
    pos_g, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, st.nxt)
    assert np.abs(vfm.min_image(pos_g - st.pos, lat)).max() < 1e-10
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) < 1e-10
    run.close()


def _walled_case(walls, precision, seed=61, n_rings=5, dims=(20, 18, 24)):
    lat = wl.lattice_preset(*dims, walls=walls, precision=precision,
                            body_force=(0.0, 0.0, 0.0 if walls[2] else 1e-5))
    vor = wl.vortex_preset(wall_images=True, mass_balance=not walls[2])
    rho, u = wl.velocity_field(seed, dims, (0.0, 0.0, 0.01), 2e-3)
    # rings close to the walls (margin 0.3): the image terms are large there
    pos, nxt = wl.random_rings(seed, n_rings, 2.0, 4.0, dims, walls, 0.95, margin=0.3)
    return dict(name=f"walled{walls}", lattice=lat, vortex=vor, rho=rho, u=u, pos=pos,
                nxt=nxt, steps=6)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("walls", [(True, False, False), (True, True, False), (True, True, True)])
def test_wall_images_eval(walls, precision):
    """Superfluid wall term from image filaments (3^w - 1 mirrored copies):
    line velocity, force and spread force against the oracle; without the
    images the velocity differs by far more than the tolerance."""
    cfg = _walled_case(walls, precision, n_rings=16)
    say("wall images", walls, precision, cfg["pos"].shape[0])
    run = vlb.run_from_config(cfg)
    got = run.eval_line_velocity()
    F_g = run.read_force()
    ref, F_o, _ = _oracle_eval(cfg)
    for k in ("vs", "vn", "sdot", "force"):
        err = rel_l2(got[k], ref[k])
        say(k, err)
        assert err <= TOL[precision], (k, err)
    assert rel_l2(F_g, F_o) <= TOL[precision]
    cfg0 = dict(cfg, vortex=dict(cfg["vortex"], wall_images=False))
    ref0, _, _ = _oracle_eval(cfg0)
    assert rel_l2(ref0["vs"], ref["vs"]) > 100 * TOL[precision]
    run.close()


def test_wall_images_coupled_f64():
    cfg = _walled_case((True, True, False), "f64", seed=62)
    say("wall images coupled")
    run = vlb.run_from_config(cfg)
    lat, vp, st = oracle_state(cfg)
    assert vp.wall_images
    for _ in range(6):
        run.step(1)
        st = coupled.coupled_step(st, lat, vp)
    run.sync()
    pos_g, nxt_g = run.read_filaments()
    np.testing.assert_array_equal(nxt_g, st.nxt)
    assert np.abs(vfm.min_image(pos_g - st.pos, lat)).max() < 1e-10
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, lat)
    assert rel_l2(u_g, u_o) < 1e-10
    run.close()
