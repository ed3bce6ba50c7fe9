"""GPU parity of the normal-fluid update (collide + stream, walls, planes,
body force) against the oracle, through the C ABI."""

import numpy as np
import pytest

import workloads as wl
from oracle import lbm
from oracle.lbm import Lattice
from tests._cases import oracle_lattice, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_04435_amd as vlb  # noqa: E402

LBM_CASES = {
    "periodic": dict(n=(12, 10, 9), walls=(False, False, False), planes=False, body=(1e-5, -2e-5, 3e-5)),
    "walls_xy": dict(n=(11, 13, 10), walls=(True, True, False), planes=False, body=(0.0, 0.0, 4e-5)),
    "walls_xyz": dict(n=(9, 8, 10), walls=(True, True, True), planes=False, body=(2e-5, 0.0, 1e-5)),
    "planes": dict(n=(10, 12, 14), walls=(True, True, False), planes=True, body=(0.0, 0.0, 0.0)),
    # rows longer than one block (256 nodes) with a ragged second block
    "wide_x": dict(n=(261, 5, 4), walls=(True, False, False), planes=False, body=(1e-5, 0.0, 2e-5)),
    # rows of exactly 256 nodes periodic in x and y: with FP16 storage four
    # nodes per lane (x-shifted directions across lanes, x wrapping at lane
    # 63), also next to z walls (per-node path for those slices' odd passes)
    # and on velocity planes
    "rows256": dict(n=(256, 6, 5), walls=(False, False, False), planes=False, body=(1e-5, -2e-5, 3e-5)),
    "rows256_zwalls": dict(n=(256, 5, 6), walls=(False, False, True), planes=False, body=(2e-5, 1e-5, 0.0)),
    "rows256_planes": dict(n=(256, 4, 8), walls=(False, False, False), planes=True, body=(0.0, 0.0, 0.0)),
}

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}


def _run_case(name, precision, steps):
    c = LBM_CASES[name]
    lat = wl.lattice_preset(*c["n"], tau=0.8, walls=c["walls"], plane_lo=c["planes"],
                            plane_hi=c["planes"], plane_u=(0.0, 0.0, 0.02),
                            body_force=c["body"], precision=precision)
    vor = wl.vortex_preset()
    rho, u = wl.velocity_field(31, c["n"], (0.01, -0.005, 0.02), 3e-3)
    rho = rho + 0.01 * np.random.default_rng(32).standard_normal(rho.shape)
    say("lbm", name, precision, steps)
    run = vlb.Run(lat, vor, n_cap=1)
    run.write_fields(rho, u)
    run.step(steps)
    run.sync()
    olat = oracle_lattice(lat)
    f = lbm.init_equilibrium(rho, u)
    zero = np.zeros((3,) + olat.shape)
    for _ in range(steps):
        f = lbm.lbm_step(f, zero, olat)
    return run, f, olat, rho


@pytest.mark.parametrize("name", list(LBM_CASES))
@pytest.mark.parametrize("steps", [1, 2, 5])
def test_lbm_f64_populations(name, steps):
    run, f, olat, _ = _run_case(name, "f64", steps)
    fg = run.read_populations()
    np.testing.assert_allclose(fg, f, rtol=0, atol=1e-14)
    rho_g, u_g = run.read_fields()
    rho_o, u_o = lbm.bare_velocity(f, olat)
    np.testing.assert_allclose(rho_g, rho_o, rtol=0, atol=1e-13)
    np.testing.assert_allclose(u_g, u_o, rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", list(LBM_CASES))
@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_lbm_reduced_precision(name, precision):
    steps = 20
    run, f, olat, _ = _run_case(name, precision, steps)
    rho_g, u_g = run.read_fields()
    rho_o, u_o = lbm.bare_velocity(f, olat)
    err = rel_l2(u_g, u_o)
    say("velocity L2 rel", precision, name, err)
    assert err <= TOL[precision]
    assert np.abs(rho_g - rho_o).max() < (1e-6 if precision == "f32" else 2e-4)


def test_lbm_mass_conserved_f64():
    """Walls + periodic, no planes: total mass exact over 50 steps."""
    run, f, olat, rho0 = _run_case("walls_xy", "f64", 50)
    rho_g, _ = run.read_fields()
    assert abs(rho_g.sum() - rho0.sum()) / rho0.sum() < 1e-13


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_lbm_mass_drift_ten_thousand_steps(precision):
    """Exact mass conservation of the scheme (Sec. II.B: collision and the
    forcing term conserve mass; halfway bounce-back and periodic streaming
    move every population to one slot): a channel 16 nodes across (walls on
    x and y, periodic z), body force along z, 1e4 steps.  The FP64 total
    drifts by round-off only (below 1e-12 relative); the storage forms'
    drift is reported and stays inside their tolerances."""
    n = (16, 16, 8)
    lat = wl.lattice_preset(*n, tau=0.8, walls=(True, True, False), body_force=(0.0, 0.0, 1e-5),
                            precision=precision)
    rho, u = wl.velocity_field(33, n, (0.0, 0.0, 0.01), 1e-3)
    run = vlb.Run(lat, wl.vortex_preset(), n_cap=1)
    run.write_fields(rho, u)
    m0 = run.read_fields()[0].sum()
    run.step(10000)
    run.sync()
    m1 = run.read_fields()[0].sum()
    drift = abs(m1 - m0) / m0
    say("mass drift over 1e4 steps", precision, drift)
    assert drift < {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}[precision]
    run.close()


def test_uniform_equilibrium_is_a_fixed_point_f64():
    """A uniform flow at equilibrium with no force on a periodic lattice
    stays where it is (Sec. II.B: f^eq collides to itself, streaming moves
    equal values): populations after 100 steps equal the initial ones to
    round-off."""
    n = (12, 10, 9)
    lat = wl.lattice_preset(*n, tau=0.8, precision="f64")
    rho = np.full((n[2], n[1], n[0]), 1.0)
    u = np.zeros((3, n[2], n[1], n[0]))
    u[0], u[1], u[2] = 0.01, -0.02, 0.015
    run = vlb.Run(lat, wl.vortex_preset(), n_cap=1)
    run.write_fields(rho, u)
    f0 = run.read_populations()
    run.step(100)
    run.sync()
    f1 = run.read_populations()
    assert np.abs(f1 - f0).max() <= 1e-15
    run.close()


def test_body_force_momentum_bookkeeping_f64():
    """Guo forcing adds exactly the body force to the momentum of a periodic
    lattice per step (Sec. II.B, Eq. F_i: collision gives g / (2 tau), the
    forcing term (1 - 1 / (2 tau)) g): after N steps sum(rho u) has grown by
    N cells g, u being the force-shifted velocity."""
    n = (10, 8, 12)
    g = np.array([2e-5, -1e-5, 3e-5])
    lat = wl.lattice_preset(*n, tau=0.9, body_force=tuple(g), precision="f64")
    rho, u = wl.velocity_field(34, n, (0.005, 0.0, -0.01), 2e-3)
    run = vlb.Run(lat, wl.vortex_preset(), n_cap=1)
    run.write_fields(rho, u)
    r0, u0 = run.read_fields()
    steps = 40
    run.step(steps)
    run.sync()
    r1, u1 = run.read_fields()
    cells = n[0] * n[1] * n[2]
    for a in range(3):
        gain = (r1 * u1[a]).sum() - (r0 * u0[a]).sum()
        assert abs(gain - steps * cells * g[a]) < 1e-12, (a, gain, steps * cells * g[a])
    run.close()


def test_poiseuille_gpu_f64():
    """Exact discrete Poiseuille profile reached by the GPU (plane channel,
    walls on y, body force along x)."""
    H, tau, g = 8, 1.0, 1e-6
    lat = wl.lattice_preset(4, H, 4, tau=tau, walls=(False, True, False), body_force=(g, 0, 0),
                            precision="f64")
    run = vlb.Run(lat, wl.vortex_preset(), n_cap=1)
    rho = np.ones((4, H, 4))
    u = np.zeros((3, 4, H, 4))
    say("poiseuille gpu")
    run.write_fields(rho, u)
    run.step(3000)
    _, ub = run.read_fields()
    nu = (tau - 0.5) / 3
    y = np.arange(H) - (H - 1) / 2
    exact = (g / (2 * nu)) * ((H / 2) ** 2 - y ** 2 + (16 * (tau - 0.5) ** 2 - 3) / 12)
    ux = ub[0, 1, :, 2] + 0.5 * g  # force-shifted velocity (rho = 1)
    assert np.abs(ux / exact - 1).max() < 1e-9


@pytest.mark.parametrize("precision,dims", [("f64", (320, 320, 280)), ("f32", (400, 400, 360))])
def test_lbm_large_array_crop(precision, dims):
    """A population array above 4 GiB (the odd pass then addresses the
    neighbours' slots with 64-bit offsets): two updates (both AA parities)
    from f = f^eq(rho, u), checked on an interior window against the oracle
    stepping the window with a two-node halo from the same initial state."""
    nx, ny, nz = dims
    b = 8 if precision == "f64" else 4
    assert 19 * nx * ny * nz * b >= 1 << 32
    lat = wl.lattice_preset(nx, ny, nz, tau=0.8, body_force=(1e-6, 0.0, 2e-6), precision=precision)
    rho, u = wl.velocity_field(51, dims, (0.01, -0.005, 0.02), 3e-3)
    say("large array", precision, dims)
    run = vlb.Run(lat, wl.vortex_preset(), n_cap=1)
    run.write_fields(rho, u)
    run.step(2)
    run.sync()
    _, u_g = run.read_fields()
    run.close()
    w, h = 16, 2
    c = (nz // 2, ny // 2, nx // 2)
    win = tuple(slice(ci - w // 2 - h, ci + w // 2 + h) for ci in c)
    clat = Lattice(w + 2 * h, w + 2 * h, w + 2 * h, tau=0.8, body_force=(1e-6, 0.0, 2e-6))
    f = lbm.init_equilibrium(rho[win], u[(slice(None),) + win])
    zero = np.zeros((3,) + clat.shape)
    for _ in range(2):
        f = lbm.lbm_step(f, zero, clat)
    _, u_o = lbm.bare_velocity(f, clat)
    inner = (slice(None),) + (slice(h, -h),) * 3
    got = u_g[(slice(None),) + win][inner]
    err = rel_l2(got, u_o[inner])
    say("large array crop velocity", precision, err)
    assert err <= (1e-12 if precision == "f64" else 1e-5)


def _rows256_coupled(precision="f16", seed=41):
    """256 x 8 x 8 periodic lattice (rows of 256 nodes) with a ring of 16
    points around the x axis, so that the update reads a spread force."""
    lat = wl.lattice_preset(256, 8, 8, tau=0.8, precision=precision)
    vor = wl.vortex_preset()
    rho, u = wl.velocity_field(seed, (256, 8, 8), (0.01, 0.0, 0.005), 1e-3)
    pos, nxt = wl.ring((128.3, 4.1, 3.9), 2.2, (1.0, 0.0, 0.0), 16, phase=0.5)
    return dict(name="rows256_ring", lattice=lat, vortex=vor, rho=rho, u=u, pos=pos, nxt=nxt)


def test_rows256_coupled_f16_against_oracle():
    """Coupled FP16-storage steps on rows of 256 nodes (four nodes per lane,
    spread force read as four-node groups) against the FP64 oracle: links
    equal, positions within 1e-2, velocity field within 1e-3."""
    from oracle import coupled, vfm
    from tests._cases import oracle_state

    cfg = _rows256_coupled()
    say("rows256 coupled f16")
    run = vlb.run_from_config(cfg)
    olat, vp, st = oracle_state(cfg)
    for k in range(6):
        run.step(1)
        run.sync()
        st = coupled.coupled_step(st, olat, vp)
        pos_g, nxt_g = run.read_filaments()
        assert (nxt_g == st.nxt).all(), k
        assert np.abs(vfm.min_image(pos_g - st.pos, olat)).max() < 1e-2, k
    _, u_g = run.read_fields()
    _, u_o = lbm.bare_velocity(st.f, olat)
    err = rel_l2(u_g, u_o)
    say("velocity L2 rel", err)
    assert err <= TOL["f16"]
    run.close()


def test_rows256_checkpoint_resume_bitwise():
    """FP16 rows of 256 nodes: a run resumed from the state read after an
    odd number of steps (swapped AA layout) continues bit for bit."""
    cfg = _rows256_coupled(seed=42)
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
    np.testing.assert_array_equal(a.read_state()[0].cpu().numpy(), b.read_state()[0].cpu().numpy())
    np.testing.assert_array_equal(a.read_filaments()[0], b.read_filaments()[0])
    a.close()
    b.close()
