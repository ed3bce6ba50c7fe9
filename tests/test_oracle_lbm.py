"""Pins of the oracle's lattice-Boltzmann part against closed forms, exact
invariants and brute force (none of them re-types the oracle's formulas)."""

import itertools
import os

import numpy as np
import pytest

from oracle import lbm
from oracle.d3q19 import C, W, OPP, Q
from oracle.lbm import Lattice


def _table1(golden_dir):
    shells = []
    with open(os.path.join(golden_dir, "d3q19_table1.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            num, den, vel = line.split(None, 2)
            vs = [tuple(int(c) for c in v.split(",")) for v in vel.split(";")]
            shells.append((int(num) / int(den), vs))
    return shells


def test_d3q19_matches_table1(golden_dir):
    """Velocities and weights are exactly Table I (order inside shells free)."""
    shells = _table1(golden_dir)
    table = {}
    for w, vs in shells:
        for v in vs:
            table[v] = w
    assert len(table) == 19
    mine = {tuple(int(x) for x in C[i]): W[i] for i in range(Q)}
    assert set(mine) == set(table)
    for v in table:
        assert mine[v] == pytest.approx(table[v], abs=0, rel=1e-15)
    # the paper's index 1 is the rest velocity
    assert tuple(C[0]) == (0, 0, 0)
    for i in range(Q):
        assert (C[OPP[i]] == -C[i]).all()


def test_lattice_isotropy():
    """Moment identities of the D3Q19 weights (c_s^2 = 1/3)."""
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    for a in range(3):
        assert abs((W * C[:, a]).sum()) < 1e-16
        for b in range(3):
            m2 = (W * C[:, a] * C[:, b]).sum()
            assert m2 == pytest.approx((1.0 / 3.0) if a == b else 0.0, abs=1e-15)
    for a, b, c_, d in itertools.product(range(3), repeat=4):
        m4 = (W * C[:, a] * C[:, b] * C[:, c_] * C[:, d]).sum()
        delta = lambda i, j: 1.0 if i == j else 0.0  # noqa: E731
        exp = (delta(a, b) * delta(c_, d) + delta(a, c_) * delta(b, d) + delta(a, d) * delta(b, c_)) / 9.0
        assert m4 == pytest.approx(exp, abs=1e-15)


def test_equilibrium_moments():
    """sum f^eq = rho, sum c f^eq = rho u, sum c c f^eq = rho (u u + I/3)."""
    rng = np.random.default_rng(0)
    rho = 1.0 + 0.1 * rng.random((2, 3, 4))
    u = 0.05 * rng.standard_normal((3, 2, 3, 4))
    feq = lbm.equilibrium(rho, u)
    np.testing.assert_allclose(feq.sum(0), rho, rtol=0, atol=1e-15)
    for a in range(3):
        ja = sum(C[i, a] * feq[i] for i in range(Q))
        np.testing.assert_allclose(ja, rho * u[a], rtol=0, atol=1e-15)
        for b in range(3):
            pab = sum(C[i, a] * C[i, b] * feq[i] for i in range(Q))
            np.testing.assert_allclose(pab, rho * (u[a] * u[b] + (a == b) / 3.0), atol=1e-15)


def test_forcing_moments():
    """Guo term: sum F_i = 0 and sum c_i F_i = (1 - 1/(2 tau)) g."""
    rng = np.random.default_rng(1)
    u = 0.05 * rng.standard_normal((3, 5))
    g = 1e-3 * rng.standard_normal((3, 5))
    tau = 0.8
    F = lbm.forcing(u, g, tau)
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-18)
    for a in range(3):
        ja = sum(C[i, a] * F[i] for i in range(Q))
        np.testing.assert_allclose(ja, (1 - 0.5 / tau) * g[a], rtol=1e-13, atol=1e-19)


def _poiseuille(H, tau, steps):
    g = 1e-6
    lat = Lattice(1, H, 1, tau=tau, walls=(False, True, False), body_force=(g, 0.0, 0.0))
    nu = (tau - 0.5) / 3.0
    lam = (tau - 0.5) ** 2
    y = np.arange(H) - (H - 1) / 2.0
    exact = (g / (2.0 * nu)) * ((H / 2.0) ** 2 - y ** 2 + (16.0 * lam - 3.0) / 12.0)
    rho = np.ones(lat.shape)
    u = np.zeros((3,) + lat.shape)
    f = lbm.init_equilibrium(rho, u)
    F0 = np.zeros((3,) + lat.shape)
    for _ in range(steps):
        f = lbm.lbm_step(f, F0, lat)
    r = lbm.density(f)[0, :, 0]
    ux = (lbm.momentum(f)[0, 0, :, 0] + 0.5 * g) / r
    return ux, exact


@pytest.mark.parametrize("tau", [1.0, 0.5 + np.sqrt(3.0 / 16.0)])
def test_poiseuille_exact_discrete(tau):
    """Force-driven plane Poiseuille flow between halfway bounce-back walls:
    BGK's steady state is exactly u(y) = g/(2 nu) [(H/2)^2 - y^2 + (16 L - 3)/12],
    nu = (tau - 1/2)/3, L = (tau - 1/2)^2, with u the force-shifted velocity
    (sum c f + g/2)/rho; at L = 3/16 the wall slip vanishes."""
    ux, exact = _poiseuille(8, tau, 3000)
    assert np.abs(ux / exact - 1).max() < 1e-10
    if abs((tau - 0.5) ** 2 - 3.0 / 16.0) < 1e-12:
        # the same solution is the continuum parabola
        H = 8
        y = np.arange(H) - (H - 1) / 2.0
        par = (1e-6 / (2 * (tau - 0.5) / 3)) * ((H / 2.0) ** 2 - y ** 2)
        assert np.abs(ux / par - 1).max() < 1e-10


def test_poiseuille_dropped_wall_term_detected():
    """The continuum parabola is NOT the discrete answer at tau = 1: the
    (16 L - 3)/12 slip term is needed (guards against a wrong wall rule)."""
    ux, exact = _poiseuille(8, 1.0, 3000)
    H = 8
    y = np.arange(H) - (H - 1) / 2.0
    par = (1e-6 / (2 * 0.5 / 3)) * ((H / 2.0) ** 2 - y ** 2)
    assert np.abs(ux / par - 1).max() > 1e-3


def _random_f(shape, seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.01 * rng.standard_normal(shape)
    u = 0.02 * rng.standard_normal((3,) + shape)
    return lbm.equilibrium(rho, u) * (1 + 0.01 * rng.standard_normal((Q,) + shape))


@pytest.mark.parametrize("walls", [(False, False, False), (True, True, False), (True, True, True)])
def test_mass_conservation(walls):
    """Periodic faces and bounce-back walls conserve total mass exactly."""
    lat = Lattice(5, 4, 6, tau=0.7, walls=walls, body_force=(1e-4, -2e-4, 3e-4))
    f = _random_f(lat.shape, 3)
    m0 = f.sum()
    rng = np.random.default_rng(4)
    g = 1e-4 * rng.standard_normal((3,) + lat.shape)
    for _ in range(50):
        f = lbm.lbm_step(f, g, lat)
    assert abs(f.sum() - m0) / m0 < 1e-13


def test_momentum_bookkeeping():
    """Fully periodic: every step adds exactly sum g to the total momentum
    (collision gives g/(2 tau), the forcing term (1 - 1/(2 tau)) g)."""
    lat = Lattice(4, 5, 3, tau=0.9)
    f = _random_f(lat.shape, 5)
    rng = np.random.default_rng(6)
    g = 1e-3 * rng.standard_normal((3,) + lat.shape)
    for _ in range(5):
        j0 = lbm.momentum(f).sum(axis=(1, 2, 3))
        f = lbm.lbm_step(f, g, lat)
        j1 = lbm.momentum(f).sum(axis=(1, 2, 3))
        np.testing.assert_allclose(j1 - j0, g.sum(axis=(1, 2, 3)), rtol=1e-10, atol=1e-15)


def test_uniform_equilibrium_is_fixed_point():
    """A uniform equilibrium without force is stationary (periodic)."""
    lat = Lattice(3, 4, 5, tau=0.8)
    rho = np.full(lat.shape, 1.02)
    u = np.zeros((3,) + lat.shape)
    u[0], u[1], u[2] = 0.01, -0.02, 0.015
    f = lbm.init_equilibrium(rho, u)
    f1 = lbm.lbm_step(f, np.zeros((3,) + lat.shape), lat)
    np.testing.assert_allclose(f1, f, rtol=0, atol=1e-16)


def _push_stream(fp, lat):
    """Independent push formulation with explicit node loops: each
    population leaves x towards x + c_i; if that lies beyond a wall it turns
    round and is stored at x in the opposite direction."""
    nz, ny, nx = fp.shape[1:]
    dims = (nx, ny, nz)
    out = np.full_like(fp, np.nan)
    for i in range(Q):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    d = [x + C[i, 0], y + C[i, 1], z + C[i, 2]]
                    hit = False
                    for a in range(3):
                        if lat.walls[a]:
                            if d[a] < 0 or d[a] >= dims[a]:
                                hit = True
                        else:
                            d[a] %= dims[a]
                    if hit:
                        out[OPP[i], z, y, x] = fp[i, z, y, x]
                    else:
                        out[i, d[2], d[1], d[0]] = fp[i, z, y, x]
    return out


@pytest.mark.parametrize("walls", [(False, False, False), (True, False, False), (True, True, False),
                                   (False, True, True)])
def test_stream_matches_push_brute_force(walls):
    lat = Lattice(4, 3, 5, walls=walls)
    rng = np.random.default_rng(7)
    fp = rng.random((Q,) + lat.shape)
    out = lbm.stream(fp, lat)
    ref = _push_stream(fp, lat)
    assert not np.isnan(ref).any()
    np.testing.assert_array_equal(out, ref)


def test_velocity_planes():
    """Plane nodes carry rho = 1 and bare velocity U_plane; others untouched."""
    lat = Lattice(4, 4, 6, plane_lo=True, plane_hi=True, plane_u=(0.0, 0.0, 0.03),
                  walls=(True, True, False))
    f = _random_f(lat.shape, 8)
    rho, ub = lbm.bare_velocity(f, lat)
    for z in (0, lat.nz - 1):
        np.testing.assert_allclose(rho[z], 1.0, atol=1e-15)
        np.testing.assert_allclose(ub[2, z], 0.03, atol=1e-15)
        np.testing.assert_allclose(ub[0, z], 0.0, atol=1e-16)
    np.testing.assert_array_equal(rho[1:-1], lbm.density(f)[1:-1])


def test_mass_balance_uniform_flow():
    """Uniform u -> V_s = -(rho_n/rho_s) u_z (Sec. III.C, Eq. mass cons)."""
    lat = Lattice(4, 3, 5)
    rho = np.ones(lat.shape)
    u = np.zeros((3,) + lat.shape)
    u[2] = 0.02
    f = lbm.init_equilibrium(rho, u)
    Vs = lbm.mass_balance_superflow(f, lat, 1.35)
    np.testing.assert_allclose(Vs, -0.02 / 1.35, rtol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mass_balance_along_each_axis(axis):
    """The superflow follows the flow axis a (Sec. III.C, Eq. mass cons: the
    mean over each cross-section normal to a of u_a): with u_a = g(x_a)
    plus a part of zero mean over every cross-section, V_s = -(rho_n/rho_s)
    g exactly; the other components, made large here, do not enter."""
    lat = Lattice(6, 4, 5)
    n = lat.dims[axis]
    rho = np.ones(lat.shape)
    z, y, x = np.meshgrid(np.arange(5), np.arange(4), np.arange(6), indexing="ij")
    coord = (x, y, z)
    g = 0.01 + 0.004 * np.arange(n) / n
    u = np.zeros((3,) + lat.shape)
    for c in range(3):
        u[c] = 0.05 * (c + 1)
    o1, o2 = [b for b in range(3) if b != axis]
    u[axis] = (g[coord[axis]] + 0.003 * np.cos(2 * np.pi * coord[o1] / lat.dims[o1])
               + 0.002 * np.sin(2 * np.pi * coord[o2] / lat.dims[o2]))
    f = lbm.init_equilibrium(rho, u)
    Vs = lbm.mass_balance_superflow(f, lat, 1.35, axis)
    assert Vs.shape == (n,)
    np.testing.assert_allclose(Vs, -g / 1.35, rtol=0, atol=1e-15)
