"""One coupled VFM-LBM time step, plain FP64 (paper Sec. II).

Order inside a step (the paper does not state one; reading R17):
  1. From the normal-fluid state f^n: bare velocity field u_b and, if
     enabled, the mass-balance superflow V_s(z) (Sec. III.C).
  2. Filaments: classical RK4 with dt = 1 lattice step (reading R6) on the
     equation of motion (Sec. II.A, Eq. E of M), with u_b and V_s frozen at
     time n.  The mutual-friction force is taken from the first stage (the
     positions s^n).
  3. Normal fluid: the force is spread onto the lattice (Sec. II.B) and one
     forced LBM update f^n -> f^{n+1} is made.
  4. Topology: remeshing, reconnection, small-loop removal (Sec. II.A, III.B).
"""

from dataclasses import dataclass, field

import numpy as np

from . import lbm, vfm, topology
from .lbm import Lattice
from .vfm import VortexParams


@dataclass
class State:
    f: np.ndarray
    pos: np.ndarray
    nxt: np.ndarray
    prv: np.ndarray
    step: int = 0
    force: np.ndarray = None  # last spread force field (3, nz, ny, nx)
    stats: dict = field(default_factory=dict)


def prev_from_next(nxt):
    """Predecessors: prv[nxt[k]] = k for every real link; the first point
    of an open line (no predecessor) is its own (reading F1b)."""
    nxt = np.asarray(nxt)
    ks = np.arange(nxt.shape[0])
    prv = ks.copy()
    real = nxt != ks
    prv[nxt[real]] = ks[real]
    return prv


def make_state(rho, u, pos, nxt, lat: Lattice):
    """Initial state: f = f^eq(rho, u), filaments as given (wrapped)."""
    f = lbm.init_equilibrium(rho, u)
    pos = vfm.wrap_positions(np.asarray(pos, dtype=np.float64), lat)
    nxt = np.asarray(nxt, dtype=np.int64)
    return State(f=f, pos=pos, nxt=nxt, prv=prev_from_next(nxt),
                 force=np.zeros((3,) + lat.shape))


def filament_rk4(pos, nxt, prv, ub, Vs, lat: Lattice, vp: VortexParams):
    """Classical RK4 of ds/dt on the filaments; returns the new positions,
    the stage-1 quantities (velocities and force per point)."""
    s0 = pos
    st1 = vfm.line_velocity(s0, nxt, prv, ub, Vs, lat, vp, want_force=vp.coupling)
    k1 = st1["sdot"]
    y = vfm.wrap_positions(s0 + 0.5 * k1, lat)
    k2 = vfm.line_velocity(y, nxt, prv, ub, Vs, lat, vp)["sdot"]
    y = vfm.wrap_positions(s0 + 0.5 * k2, lat)
    k3 = vfm.line_velocity(y, nxt, prv, ub, Vs, lat, vp)["sdot"]
    y = vfm.wrap_positions(s0 + k3, lat)
    k4 = vfm.line_velocity(y, nxt, prv, ub, Vs, lat, vp)["sdot"]
    s1 = vfm.wrap_positions(s0 + (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0, lat)
    return s1, st1


def coupled_step(st: State, lat: Lattice, vp: VortexParams):
    """Advance the state by one step (see module docstring)."""
    _, ub = lbm.bare_velocity(st.f, lat)
    Vs = lbm.mass_balance_superflow(st.f, lat, vp.rho_s_over_rho_n) if vp.mass_balance else None
    if st.pos.shape[0] > 0:
        s1, st1 = filament_rk4(st.pos, st.nxt, st.prv, ub, Vs, lat, vp)
        if vp.coupling:
            F = vfm.spread(st1["force"], st.pos, lat)
        else:
            F = np.zeros((3,) + lat.shape)
    else:
        s1 = st.pos
        F = np.zeros((3,) + lat.shape)
    f1 = lbm.lbm_step(st.f, F, lat)
    pos, nxt, prv = s1, st.nxt, st.prv
    stats = {}
    if pos.shape[0] > 0:
        pos, nxt, prv, stats = topology.topology_update(pos, nxt, prv, lat, vp)
    return State(f=f1, pos=pos, nxt=nxt, prv=prv, step=st.step + 1, force=F, stats=stats)
