"""Shared helpers of the GPU parity tests: building oracle objects from the
plain-data workload presets and comparison metrics.  (Test code only.)"""

import sys

import numpy as np

import workloads as wl
from oracle import coupled
from oracle.lbm import Lattice
from oracle.vfm import VortexParams


def oracle_lattice(lat: dict) -> Lattice:
    return Lattice(lat["nx"], lat["ny"], lat["nz"], tau=lat["tau"], walls=tuple(lat["walls"]),
                   plane_lo=lat["plane_lo"], plane_hi=lat["plane_hi"],
                   plane_u=tuple(lat["plane_u"]), body_force=tuple(lat["body_force"]))


def oracle_vortex(vor: dict) -> VortexParams:
    keys = VortexParams.__dataclass_fields__.keys()
    return VortexParams(**{k: vor[k] for k in keys if k in vor})


def oracle_state(cfg):
    lat = oracle_lattice(cfg["lattice"])
    st = coupled.make_state(cfg["rho"], cfg["u"], cfg["pos"], cfg["nxt"], lat)
    return lat, oracle_vortex(cfg["vortex"]), st


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt((b * b).sum())
    return float(np.sqrt(((a - b) ** 2).sum()) / (den if den > 0 else 1.0))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def small_channel(precision="f64", seed=21, n_rings=6, nxy=16, nz=32, mass_balance=True,
                  planes=False, reconnect=False, body=2e-5):
    """Small walled channel (walls on x and y, periodic z) with a few rings:
    several tiles and ragged tails for every kernel, sizes the oracle does in
    seconds."""
    lat = wl.lattice_preset(nxy, nxy, nz, tau=0.8, walls=(True, True, False), plane_lo=planes,
                            plane_hi=planes, plane_u=(0.0, 0.0, 0.02 if planes else 0.0),
                            body_force=(0.0, 0.0, 0.0 if planes else body), precision=precision)
    vor = wl.vortex_preset(mass_balance=mass_balance, reconnect=reconnect)
    rho, u = wl.velocity_field(seed, (nxy, nxy, nz), (0.0, 0.0, 0.015), 2e-3)
    pos, nxt = wl.random_rings(seed, n_rings, 2.0, 4.5, (nxy, nxy, nz), (True, True, False), 0.95)
    return dict(name=f"channel{nxy}x{nxy}x{nz}", lattice=lat, vortex=vor, rho=rho, u=u, pos=pos,
                nxt=nxt, steps=10)


def small_periodic(precision="f64", seed=22, n_rings=5, n=(20, 16, 24)):
    lat = wl.lattice_preset(*n, tau=0.9, precision=precision)
    vor = wl.vortex_preset(mass_balance=True)
    rho, u = wl.velocity_field(seed, n, (0.004, -0.003, 0.01), 2e-3)
    pos, nxt = wl.random_rings(seed, n_rings, 2.0, 5.0, n, (False, False, False), 0.95)
    return dict(name=f"periodic{n}", lattice=lat, vortex=vor, rho=rho, u=u, pos=pos, nxt=nxt,
                steps=10)


def duct(axis, precision="f64", seed=31, n_rings=6, n_flow=32, n_side=16, body=2e-5):
    """Walled duct along `axis` (bounce-back walls on the other two axes,
    periodic along it) with a body force and the mass-balance superflow
    along it, and a few rings; the flow axis is longer than the others so
    that an axis mix-up changes shapes."""
    dims = [n_side] * 3
    dims[axis] = n_flow
    walls = [True] * 3
    walls[axis] = False
    bf = [0.0] * 3
    bf[axis] = body
    u0 = [0.0] * 3
    u0[axis] = 0.015
    lat = wl.lattice_preset(*dims, tau=0.8, walls=tuple(walls), body_force=tuple(bf),
                            precision=precision)
    vor = wl.vortex_preset(mass_balance=True, mass_balance_axis=axis)
    rho, u = wl.velocity_field(seed, tuple(dims), tuple(u0), 2e-3)
    pos, nxt = wl.random_rings(seed, n_rings, 2.0, 4.5, tuple(dims), tuple(walls), 0.95)
    return dict(name=f"duct{'xyz'[axis]}{tuple(dims)}", lattice=lat, vortex=vor, rho=rho, u=u,
                pos=pos, nxt=nxt, steps=8)
