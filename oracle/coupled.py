"""One coupled VFM-LBM time step, plain FP64 (paper Sec. II).

Order inside a step (the paper does not state one; reading R17):
  1. From the normal-fluid state f^n: bare velocity field u_b and, if
     enabled, the mass-balance superflow V_s along the flow axis (Sec.
     III.C).
  2. Filaments: the equation of motion (Sec. II.A, Eq. E of M) integrated
     over dt = 1 lattice step (reading R6) by an explicit Runge-Kutta
     method (by default the classical RK4 in one step; optionally 1 or 2
     stages and several substeps of 1/m), with u_b and V_s frozen at time
     n.  The mutual-friction force is taken from the first stage of the
     first substep (the positions s^n).
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


def rk_step(s0, velocity, wrap, h, stages, k1=None):
    """One step of length h of ds/dt = velocity(s) by an explicit
    Runge-Kutta method: stages = 1 forward Euler, 2 the midpoint rule, 4 the
    classical fourth-order method.  ``wrap`` maps positions back into the
    box after every update; ``k1`` is velocity(s0) when already known."""
    if k1 is None:
        k1 = velocity(s0)
    if stages == 1:
        return wrap(s0 + h * k1)
    hh = 0.5 * h
    k2 = velocity(wrap(s0 + hh * k1))
    if stages == 2:
        return wrap(s0 + h * k2)
    if stages != 4:
        raise ValueError("rk_stages must be 1, 2 or 4")
    k3 = velocity(wrap(s0 + hh * k2))
    k4 = velocity(wrap(s0 + h * k3))
    return wrap(s0 + h * ((k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0))


def filament_advance(pos, nxt, prv, ub, Vs, lat: Lattice, vp: VortexParams):
    """Positions after one lattice step: vp.vfm_substeps steps of length
    1/vfm_substeps of the vp.rk_stages-stage method, with u_b and V_s
    frozen.  Returns the new positions and the quantities of the first
    stage of the first substep (velocities and force per point)."""
    m = int(vp.vfm_substeps)
    if m < 1:
        raise ValueError("vfm_substeps must be >= 1")
    h = 1.0 / m
    st1 = vfm.line_velocity(pos, nxt, prv, ub, Vs, lat, vp, want_force=vp.coupling)

    def velocity(y):
        return vfm.line_velocity(y, nxt, prv, ub, Vs, lat, vp)["sdot"]

    def wrap(y):
        return vfm.wrap_positions(y, lat)

    s = pos
    for i in range(m):
        s = rk_step(s, velocity, wrap, h, vp.rk_stages, k1=st1["sdot"] if i == 0 else None)
    return s, st1


def coupled_step(st: State, lat: Lattice, vp: VortexParams):
    """Advance the state by one step (see module docstring)."""
    _, ub = lbm.bare_velocity(st.f, lat)
    Vs = (lbm.mass_balance_superflow(st.f, lat, vp.rho_s_over_rho_n, vp.mass_balance_axis)
          if vp.mass_balance else None)
    if st.pos.shape[0] > 0:
        s1, st1 = filament_advance(st.pos, st.nxt, st.prv, ub, Vs, lat, vp)
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
