"""Parity at the full workload sizes, in the launch configuration bench.py
times (capacity, chunking), on outputs the oracle can compute one by one:
the line velocity of sampled filament points (Biot-Savart over ALL
segments, LIA, superflow, interpolation, Schwarz) and one LBM update of a
crop of the lattice, both from the GPU's own current state."""

import numpy as np
import pytest

import workloads as wl
from oracle import lbm, vfm
from oracle.lbm import Lattice
from tests._cases import oracle_lattice, oracle_vortex, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_04435_amd as vlb  # noqa: E402

TOL = {"f32": 1e-5, "f16": 1e-3}


def _bench_run(cfg):
    n0 = cfg["pos"].shape[0]
    return vlb.run_from_config(cfg, n_cap=int(n0 * 1.4) + 256, recon_cap=1 << 18)


def _oracle_line_velocity_sample(run, cfg, sample, ub, Vs):
    lat = oracle_lattice(cfg["lattice"])
    vp = oracle_vortex(cfg["vortex"])
    pos, nxt = run.read_filaments()
    prv = np.empty_like(nxt)
    prv[nxt] = np.arange(nxt.shape[0])
    geo = vfm.geometry(pos, nxt, prv, lat)
    vs = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, vp.kappa, targets=sample)
    sub = {k: v[sample] for k, v in geo.items()}
    vs = vs + vfm.lia_velocity(sub, vp) + np.array(vp.vs_applied)[None, :]
    if Vs is not None:
        vs[:, 2] += vfm.superflow_at(Vs, pos[sample, 2], lat.nz)
    vn = vfm.interpolate(ub, pos[sample], lat)
    sdot = vfm.schwarz_velocity(vs, vn, sub["sp"], vp.alpha, vp.alpha_p)
    return dict(vs=vs, vn=vn, sdot=sdot)


def _mass_balance_from_u(u, rs_rn):
    return -(1.0 / rs_rn) * u[2].mean(axis=(1, 2))


CONFIGS = {
    "counterflow": lambda: wl.config_counterflow(precision="f32"),
    "heater": lambda: wl.config_heater(precision="f32"),
    "tangle": lambda: wl.config_tangle(precision="f16"),
}


@pytest.mark.parametrize("name", list(CONFIGS))
def test_line_velocity_sampled_fullsize(name):
    cfg = CONFIGS[name]()
    prec = cfg["lattice"]["precision"]
    say("full size", name, cfg["pos"].shape[0], "points")
    run = _bench_run(cfg)
    run.step(3)
    run.sync()
    got = run.eval_line_velocity()
    _, u = run.read_fields()
    Vs = _mass_balance_from_u(u, cfg["vortex"]["rho_s_over_rho_n"]) if cfg["vortex"]["mass_balance"] else None
    n = got["vs"].shape[0]
    rng = np.random.default_rng(5)
    # a ragged sample: the first and last targets plus random ones
    sample = np.unique(np.concatenate([[0, 1, n - 2, n - 1], rng.choice(n, 60, replace=False)]))
    ref = _oracle_line_velocity_sample(run, cfg, sample, u, Vs)
    for k in ("vs", "vn", "sdot"):
        err = rel_l2(got[k][sample], ref[k])
        say(name, k, err)
        assert err <= TOL[prec], (k, err)
    run.close()


@pytest.mark.parametrize("name,crop", [("heater", (64, 64, 64)), ("tangle", (32, 32, 32))])
def test_lbm_crop_step_fullsize(name, crop):
    """One normal-fluid update on a crop (interior nodes of a window with a
    1-node halo) recomputed by the oracle from the GPU's populations and
    force field, compared with the GPU's next populations."""
    cfg = CONFIGS[name]()
    prec = cfg["lattice"]["precision"]
    L = cfg["lattice"]
    say("crop", name, crop)
    run = _bench_run(cfg)
    run.step(2)
    run.sync()
    f0 = run.read_populations()
    run.step(1)
    run.sync()
    f1 = run.read_populations()
    F = run.read_force()
    cz, cy, cx = L["nz"] // 2, L["ny"] // 2, L["nx"] // 2
    wx, wy, wz = crop
    sl = (slice(cz - wz // 2 - 1, cz + wz // 2 + 1), slice(cy - wy // 2 - 1, cy + wy // 2 + 1),
          slice(cx - wx // 2 - 1, cx + wx // 2 + 1))
    fc = f0[(slice(None),) + sl]
    Fc = F[(slice(None),) + sl]
    clat = Lattice(wx + 2, wy + 2, wz + 2, tau=L["tau"], body_force=tuple(L["body_force"]))
    out = lbm.lbm_step(fc, Fc, clat)
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    got = f1[(slice(None),) + sl][inner]
    ref = out[inner]
    _, ug = lbm.bare_velocity(got, Lattice(wx, wy, wz))
    _, uo = lbm.bare_velocity(ref, Lattice(wx, wy, wz))
    err = rel_l2(ug, uo)
    say(name, "crop velocity", err, "max |df|", np.abs(got - ref).max())
    assert err <= TOL[prec]
    assert np.abs(got - ref).max() < (1e-6 if prec == "f32" else 2e-5)
    run.close()
