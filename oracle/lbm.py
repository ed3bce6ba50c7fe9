"""Lattice-Boltzmann normal fluid, plain FP64 (paper Sec. II.B).

Field layout: populations ``f`` have shape (19, nz, ny, nx); scalar fields
(nz, ny, nx); vector fields (3, nz, ny, nx) with components (x, y, z).
Lattice units: dx = dt = 1, c_s^2 = 1/3 (Sec. II.B, Step 1).

Boundary conditions (readings of the paper):
  * an axis is either periodic or closed by two halfway bounce-back walls
    that sit half a cell outside the first and last node (R15);
  * optional velocity planes at z = 0 (heater) and z = nz-1 (cooler): the
    populations on those nodes are replaced by f^eq(rho=1, U_plane) before
    each collision, which is the same as overwriting them right after the
    previous streaming (R16, Sec. III.C and IV: velocities set by hand at the
    lattice sites next to the end walls).
"""

from dataclasses import dataclass, field

import numpy as np

from .d3q19 import C, W, OPP, Q


@dataclass
class Lattice:
    nx: int
    ny: int
    nz: int
    tau: float = 0.8
    walls: tuple = (False, False, False)  # per axis (x, y, z): bounce-back walls
    plane_lo: bool = False  # velocity plane on z = 0
    plane_hi: bool = False  # velocity plane on z = nz-1
    plane_u: tuple = (0.0, 0.0, 0.0)
    body_force: tuple = (0.0, 0.0, 0.0)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def dims(self):
        return (self.nx, self.ny, self.nz)


def equilibrium(rho, u):
    """f_i^eq = w_i rho (1 + u.c_i/c_s^2 + (u.c_i)^2/(2 c_s^4) - u.u/(2 c_s^2))
    (Sec. II.B, Step 1), with c_s^2 = 1/3."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    feq = np.empty((Q,) + rho.shape, dtype=np.float64)
    for i in range(Q):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        feq[i] = W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
    return feq


def density(f):
    """rho = sum_i f_i (Sec. II.B)."""
    return f.sum(axis=0)


def momentum(f):
    """j = sum_i c_i f_i (Sec. II.B); the paper's u is j / rho."""
    j = np.zeros((3,) + f.shape[1:], dtype=np.float64)
    for i in range(Q):
        for a in range(3):
            if C[i, a] != 0:
                j[a] += C[i, a] * f[i]
    return j


def forcing(u, g, tau):
    """Cheng-Li / Guo force term (Sec. II.B, Eq. for F_i):
    F_i = (1 - 1/(2 tau)) w_i ((c_i - u)/c_s^2 + (c_i.u) c_i / c_s^4) . g.
    The paper prints e_i in the first bracket; it is c_i (reading R22)."""
    F = np.empty((Q,) + u.shape[1:], dtype=np.float64)
    pref = 1.0 - 1.0 / (2.0 * tau)
    for i in range(Q):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        s = np.zeros(u.shape[1:], dtype=np.float64)
        for a in range(3):
            s = s + (3.0 * (C[i, a] - u[a]) + 9.0 * cu * C[i, a]) * g[a]
        F[i] = pref * W[i] * s
    return F


def apply_planes(f, lat: Lattice):
    """Velocity planes (reading R16): the nodes of z = 0 / z = nz-1 carry
    f^eq(1, U_plane).  Returns the effective populations; ``f`` is not
    modified."""
    if not (lat.plane_lo or lat.plane_hi):
        return f
    fe = f.copy()
    U = np.array(lat.plane_u, dtype=np.float64)
    one = np.ones((lat.ny, lat.nx))
    uu = np.broadcast_to(U[:, None, None], (3, lat.ny, lat.nx))
    feq = equilibrium(one, uu)
    if lat.plane_lo:
        fe[:, 0] = feq
    if lat.plane_hi:
        fe[:, lat.nz - 1] = feq
    return fe


def bare_velocity(f, lat: Lattice):
    """Bare velocity u_b = (sum_i c_i f_i) / (sum_i f_i) of the effective
    populations (planes applied), and the density.  This is the normal-fluid
    velocity that is interpolated onto the filaments (reading R17)."""
    fe = apply_planes(f, lat)
    rho = density(fe)
    return rho, momentum(fe) / rho


def collide(f, g, tau):
    """Forced BGK collision, the paper's four equations LBM 1-3 (Sec. II.B):
        f'   = f + F/2
        f''  = f' - (f - f^eq)/tau
        f''' = f'' + F/2
    with f^eq and F built from rho and the force-shifted velocity
    u = (sum_i c_i f_i + g/2) / rho (reading R2).  ``g`` has shape
    (3, nz, ny, nx)."""
    rho = density(f)
    u = (momentum(f) + 0.5 * g) / rho
    feq = equilibrium(rho, u)
    F = forcing(u, g, tau)
    f1 = f + 0.5 * F
    f2 = f1 - (f - feq) / tau
    f3 = f2 + 0.5 * F
    return f3


def stream(fp, lat: Lattice):
    """Streaming f_i(x + c_i, t + 1) = f'''_i(x, t) (Sec. II.B, Step 3 and
    Eq. LBM 4), written as a pull: the value arriving at node x in direction
    i comes from node x - c_i.  On a periodic axis the source wraps; if the
    source lies beyond a bounce-back wall the population is the one that left
    x towards that wall, reflected: f_i(x, t+1) = f'''_opp(i)(x, t)
    (halfway bounce-back, reading R15)."""
    nz, ny, nx = fp.shape[1:]
    dims = (nx, ny, nz)
    out = np.empty_like(fp)
    # node coordinate grids, (z, y, x) indexing
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = (xx, yy, zz)
    for i in range(Q):
        src = []
        outside = np.zeros(fp.shape[1:], dtype=bool)
        for a in range(3):
            s = coords[a] - C[i, a]
            if lat.walls[a]:
                outside |= (s < 0) | (s >= dims[a])
                s = np.clip(s, 0, dims[a] - 1)
            else:
                s = np.mod(s, dims[a])
            src.append(s)
        pulled = fp[i][src[2], src[1], src[0]]
        out[i] = np.where(outside, fp[OPP[i]], pulled)
    return out


def lbm_step(f, g_field, lat: Lattice):
    """One normal-fluid update f^n -> f^{n+1}: velocity planes, forced
    collision with g = body force + spread mutual-friction force, streaming."""
    fe = apply_planes(f, lat)
    g = np.array(g_field, dtype=np.float64, copy=True)
    for a in range(3):
        g[a] = g[a] + lat.body_force[a]
    return stream(collide(fe, g, lat.tau), lat)


def init_equilibrium(rho, u):
    """Initial populations f = f^eq(rho, u) (used by write_fields)."""
    return equilibrium(rho, u)


def mass_balance_superflow(f, lat: Lattice, rho_s_over_rho_n, axis=2):
    """Superflow from mass conservation (Sec. III.C, Eq. mass cons) along the
    flow axis a (the paper's is x; the channel workloads here use z):
    V_s(x_a) = -(rho_n/rho_s) (1/A) sum over the cross-section normal to
    axis a of u_n,a, with u_n the bare velocity of the effective
    populations and A the node count of a cross-section.  Returns one value
    per node along axis a."""
    _, ub = bare_velocity(f, lat)
    # ub[c] is indexed [z, y, x]: lattice axis a is array axis 2 - a
    others = tuple(k for k in range(3) if k != 2 - axis)
    area = (lat.nx * lat.ny * lat.nz) // lat.dims[axis]
    return -(1.0 / rho_s_over_rho_n) * ub[axis].sum(axis=others) / area
