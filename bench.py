"""Benchmark of the coupled VFM-LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision P] [--rows P,P] [--graph G]

Default workload (the precision form, the largest single-GPU case): a 256^3
periodic lattice, f^eq(1, 0.02 z + N(0, 1e-4^2)) initial populations, a
seeded random tangle of 2000 rings (R ~ U[4, 12], about 1.04e5 points at
remeshing spacing 0.95), mass balance on z, populations stored as FP16
deviations with FP32 arithmetic, FP32 Biot-Savart, FP64 positions.  The
same workload with FP32-deviation storage and on the plain FP64 path is
measured beside it (``rows``).  Inputs are synthetic and already resident
in HBM when the timed region starts.  One step = one pass of the whole
coupled step (mass-balance superflow, 4 RK stages of Biot-Savart + LIA +
interpolation + Schwarz, force spreading, LBM collide+stream, remeshing).

Stepping: ``--graph 0`` (default for the 256^3 and 128x128x512 cases)
enqueues steps one by one with HIP events around every step on the run's
stream, so p50/p99 are per step; ``--graph G`` (G even, default for the
small cases) advances in launches of a G-step HIP graph and steps any
remainder of --steps / --warmup directly.

Prints ONE JSON line.  ``value`` is coupled steps per second on the one GPU
for the headline precision; ``roofline`` is the dominant kernel (the FP32
Biot-Savart pair sum), priced at 35 flops per (target, segment) pair against
the FP32 vector peak, its launch duration measured with HIP events around
each of its launches inside the timed steps on the run's stream;
``lbm_roofline`` is the LBM update against the HBM peak.  ``cpu_baseline``
times the FP64 oracle on a bounded sample of the same workload on the
host's cores; the same sample gives each precision's error against the
oracle after one coupled step from the seeded state.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 work of one (target, segment) pair of the straight-segment
# Biot-Savart closed form (Sec. II.A, Eq. Biot-Savart), counting a fused
# multiply-add as 2 flops and a reciprocal / square root as 1.  Per source
# point, amortised over the two segments that share it: separation R = s - r
# (3), |R|^2 (5), its root (1) -> 9.  Per segment: R1 x R2 (9), R1.R2 (5),
# the products and sums of the norms (4), a reciprocal (1), the scale (1),
# the 3-component accumulation (6) -> 26.  Total 35.
FLOPS_PER_PAIR = 35
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_FP64_VECTOR_TFLOPS = 78.6    # MI355X published FP64 vector peak
PEAK_HBM_GBS = 8000.0             # MI355X published HBM3E bandwidth
LLC_BYTES = 256 << 20             # MI355X last-level (Infinity) cache

WORKLOADS = ("tangle", "counterflow", "ring32", "heater", "closed_channel", "serve")
DEFAULT_PRECISION = {"tangle": "f16", "counterflow": "f32", "ring32": "f64", "heater": "f32",
                     "closed_channel": "f64"}
DEFAULT_GRAPH = {"tangle": 0, "heater": 0, "counterflow": 10, "ring32": 10, "closed_channel": 10}
STORE_BYTES = {"f64": 8, "f32": 4, "f16": 2}


def make_workload(name, precision=None):
    import workloads as wl

    p = precision or DEFAULT_PRECISION.get(name)
    if name == "counterflow":
        return wl.config_counterflow(precision=p)
    if name == "ring32":
        return wl.config_ring32(precision=p)
    if name == "heater":
        return wl.config_heater(precision=p)
    if name == "tangle":
        return wl.config_tangle(precision=p)
    if name == "closed_channel":
        return wl.config_closed_channel(precision=p)
    raise SystemExit(f"unknown workload {name}")


def with_precision(cfg, precision):
    out = dict(cfg)
    out["lattice"] = dict(cfg["lattice"], precision=precision)
    return out


def step_plan(n, chunk):
    """Split n steps into graph launches of ``chunk`` steps and a direct
    remainder: a list of ("graph" | "direct", steps).  chunk = 0: every step
    direct, one entry per step (so that each step gets its own events)."""
    if n < 0:
        raise ValueError("step count must be >= 0")
    if chunk == 0:
        return [("direct", 1)] * n
    if chunk < 2 or chunk % 2:
        raise ValueError("--graph needs an even chunk >= 2 (or 0 for direct stepping)")
    plan = [("graph", chunk)] * (n // chunk)
    if n % chunk:
        plan.append(("direct", n % chunk))
    return plan


def traffic_record(kernel_src, workload):
    """HBM bytes per launch of the Biot-Savart kernel from committed
    rocprofv3 counter runs, if they were taken on the current source and on
    this workload."""
    path = os.path.join(ROOT, "profiles", "k_bs_f32_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha") != h or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def valu_record(kernel_src, workload):
    """Measured shader clock and VALU issue rate of the Biot-Savart kernel
    from committed rocprofv3 counter runs (SQ_INSTS_VALU, GRBM_GUI_ACTIVE),
    if taken on the current source and on this workload."""
    path = os.path.join(ROOT, "profiles", "k_bs_f32_valu.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha") != h or rec.get("workload") != workload:
        return None
    return {"clock_ghz": rec["clock_ghz"],
            "valu_wave_instr_per_cu_cycle": rec["valu_wave_instr_per_cu_cycle"],
            "note": "one wave64 VALU instruction per CU per cycle is the issue limit without "
                    "packed FP32; transcendentals issue beside the others"}


# ----------------------------------------------------------------- oracle leg
# Everything under oracle/ is called from this leg only: the oracle is timed
# on a bounded sample of the workload, and its values on that sample are
# what each precision's GPU result is compared with.

_POOL_ARGS = None


def _pool_bs(targets):
    from oracle import vfm

    pos, nxt, prv, lat, kappa, images = _POOL_ARGS
    t0 = time.perf_counter()
    v = vfm.biot_savart_nonlocal(pos, nxt, prv, lat, kappa, targets=targets, chunk=16)
    if images:
        v = v + vfm.biot_savart_images(pos, nxt, prv, lat, kappa, targets=targets, chunk=16)
    return v, time.perf_counter() - t0


def sample_window(cfg, width=32):
    """Origin and width of the lattice crop the accuracy sample uses: a
    cube of ``width`` nodes centred in the lattice (interior: no wall, plane
    or periodic seam inside it)."""
    L = cfg["lattice"]
    dims = (L["nx"], L["ny"], L["nz"])
    w = min(width, min(dims) // 2)
    o = tuple((d - w) // 2 for d in dims)
    return o, w


def cpu_baseline(cfg, workers=None, per_worker=128, single=48, width=None):
    """The FP64 oracle on a bounded sample of the workload, on the host's
    cores, from the seeded state:
      * Biot-Savart sums (every segment) at sampled targets: the points of a
        slab of the lattice around a centred crop (all points whose force
        reaches the crop, plus a random draw from the slab), split over a
        fork pool of ``workers`` processes; ``single`` of them again in this
        process for the single-thread rate;
      * the rest of the first RK stage at those targets (LIA, applied and
        mass-balance superflow from the slab's slices, interpolated v_n,
        Schwarz line velocity, mutual-friction force);
      * one forced LBM update of the crop (with the force the sampled points
        spread into it).
    The rates are scaled to one coupled step of the whole workload (4
    Biot-Savart evaluations of n (n - 2) pairs, one update of every node).
    Returns (baseline dict, reference values for the accuracy check)."""
    import multiprocessing as mp

    from oracle import coupled, lbm, vfm
    from oracle.lbm import Lattice
    from oracle.vfm import VortexParams

    global _POOL_ARGS
    L = cfg["lattice"]
    dims = (L["nx"], L["ny"], L["nz"])
    walls = tuple(L["walls"])
    lat = Lattice(*dims, tau=L["tau"], walls=walls, plane_lo=L["plane_lo"],
                  plane_hi=L["plane_hi"], plane_u=tuple(L["plane_u"]),
                  body_force=tuple(L["body_force"]))
    vp = VortexParams(**{k: cfg["vortex"][k] for k in VortexParams.__dataclass_fields__
                         if k in cfg["vortex"]})
    pos = vfm.wrap_positions(np.asarray(cfg["pos"], dtype=np.float64), lat)
    nxt = np.asarray(cfg["nxt"], dtype=np.int64)
    prv = coupled.prev_from_next(nxt)
    n = pos.shape[0]
    o, w = sample_window(cfg, width if width is not None else cfg.get("crop_width", 32))
    o_arr = np.array(o, dtype=np.float64)

    # targets: every point whose stencil reaches the crop, plus a random draw
    # from the slab o_z - 1 < z < o_z + w (v_n and V_s known there)
    box = np.all((pos > o_arr - 1.0) & (pos < o_arr + w), axis=1)
    slab = (pos[:, 2] > o[2] - 1.0) & (pos[:, 2] < o[2] + w)
    nw = workers or max(1, min(16, os.cpu_count() or 1))
    want = nw * per_worker
    rng = np.random.Generator(np.random.PCG64(12345))
    box_idx = np.nonzero(box)[0]
    rest = np.setdiff1d(np.nonzero(slab)[0], box_idx)
    extra = rng.choice(rest, size=max(0, min(rest.size, want - box_idx.size)), replace=False)
    targets = np.sort(np.concatenate([box_idx, extra])).astype(np.int64)

    # Biot-Savart at the targets: fork pool (no GPU has been touched yet)
    _POOL_ARGS = (pos, nxt, prv, lat, vp.kappa, vp.wall_images)
    copies = len(vfm.image_copies(lat)) + 1 if vp.wall_images else 1
    parts = np.array_split(targets, nw)
    t0 = time.perf_counter()
    if nw > 1:
        with mp.get_context("fork").Pool(nw) as pool:
            res = pool.map(_pool_bs, parts)
    else:
        res = [_pool_bs(parts[0])]
    t_pool = time.perf_counter() - t0
    bs = np.concatenate([r[0] for r in res], axis=0)
    pairs_pool = targets.size * ((n - 2) + (copies - 1) * n)
    t_single = time.perf_counter()
    _pool_bs(targets[:single])
    t_single = time.perf_counter() - t_single
    pairs_single = min(single, targets.size) * ((n - 2) + (copies - 1) * n)

    # the rest of stage 1 at the targets, from the slab z in [o_z-2, o_z+w+2)
    t1 = time.perf_counter()
    z0, nzs = o[2] - 2, w + 4
    zs = np.arange(z0, z0 + nzs) % dims[2]
    slat = Lattice(dims[0], dims[1], nzs, tau=L["tau"], walls=(walls[0], walls[1], True))
    f_slab = lbm.init_equilibrium(cfg["rho"][zs], cfg["u"][:, zs])
    _, ub_slab = lbm.bare_velocity(f_slab, slat)
    Vs = (lbm.mass_balance_superflow(f_slab, slat, vp.rho_s_over_rho_n)
          if vp.mass_balance else None)
    del f_slab
    geo = vfm.geometry(pos, nxt, prv, lat)
    pt = pos[targets]
    pt_slab = pt - np.array([0.0, 0.0, float(z0)])
    vs = bs + vfm.lia_velocity(geo, vp)[targets] + np.array(vp.vs_applied)[None, :]
    if Vs is not None:
        vs[:, 2] += vfm.superflow_at(Vs, pt_slab[:, 2], nzs)
    vn = vfm.interpolate(ub_slab, pt_slab, slat)
    alpha, alpha_p = vfm.friction_at(vp, pt[:, 2], lat)
    sp = geo["sp"][targets]
    sdot = vfm.schwarz_velocity(vs, vn, sp, alpha, alpha_p)
    dxi = 0.5 * (geo["lp"] + geo["lm"])[targets]
    force = vfm.mutual_friction_force(sdot, vs, sp, dxi, vp)
    t_stage = time.perf_counter() - t1

    # one forced LBM update of the crop [o, o+w)^3 (interior [o+1, o+w-1)^3
    # is exact: its pulls stay inside the crop)
    inbox = box[targets]
    clat = Lattice(w, w, w, tau=L["tau"], walls=(True, True, True))
    F = (vfm.spread(force[inbox], pt[inbox] - o_arr, clat) if vp.coupling
         else np.zeros((3, w, w, w)))
    sl = (slice(o[2], o[2] + w), slice(o[1], o[1] + w), slice(o[0], o[0] + w))
    f_crop = lbm.init_equilibrium(cfg["rho"][sl], cfg["u"][(slice(None),) + sl])
    plat = Lattice(w, w, w, tau=L["tau"], body_force=tuple(L["body_force"]))
    t2 = time.perf_counter()
    f1 = lbm.lbm_step(f_crop, F, plat)
    t_lbm = time.perf_counter() - t2
    _, u1 = lbm.bare_velocity(f1, plat)
    u_crop = u1[:, 1:-1, 1:-1, 1:-1]

    cells = dims[0] * dims[1] * dims[2]
    rate_pool = pairs_pool / t_pool
    rate_single = pairs_single / t_single
    rate_lbm = w ** 3 / t_lbm
    pairs_step = 4.0 * n * ((n - 2) + (copies - 1) * n)
    t_step = pairs_step / rate_pool + cells / rate_lbm
    t_step_1 = pairs_step / rate_single + cells / rate_lbm
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    base = dict(
        value=1.0 / t_step, unit="steps/s", cores=nw, kind="oracle",
        single_thread_value=1.0 / t_step_1,
        bs_gpairs_s=rate_pool / 1e9, bs_gpairs_s_single=rate_single / 1e9,
        lbm_mlups_single=rate_lbm / 1e6,
        host_cpu=cpu, host_nproc=os.cpu_count(),
        sample=(f"FP64 numpy oracle: Biot-Savart sums at {targets.size} targets x {n - 2} "
                f"segments on a fork pool of {nw} processes ({t_pool:.1f} s; {single} targets "
                f"again in one process, {t_single:.1f} s), one LBM update of a {w}^3 crop "
                f"({t_lbm:.2f} s, one thread), the rest of RK stage 1 at the targets "
                f"({t_stage:.1f} s); scaled to one coupled step of the whole workload "
                f"(4 x {n} targets x {(n - 2) + (copies - 1) * n} segments + {cells} node updates; "
                f"the O(N) filament work "
                f"and the topology are not counted)"),
    )
    ref = dict(targets=targets, vs=vs, vn=vn, sdot=sdot, force=force, origin=o, width=w,
               u_crop=u_crop)
    return base, ref


# ------------------------------------------------------------------ GPU legs

def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float(np.sqrt((b * b).sum()))
    return float(np.sqrt(((a - b) ** 2).sum()) / (den if den > 0 else 1.0))


def accuracy(run, ref):
    """Errors of the run's first coupled step from the seeded state against
    the oracle's values on the sample: the first-stage velocities at the
    sampled targets (evaluated, not advanced), then, after one step, the
    bare normal-fluid velocity on the crop's interior.  Leaves the run one
    step on."""
    torch = run.torch
    out = run.eval_line_velocity()
    t = ref["targets"]
    err = {k: rel_l2(out[k][t], ref[k]) for k in ("vs", "vn", "sdot", "force")}
    run.step(1)
    run.sync()
    u = torch.empty((3,) + run.shape, dtype=torch.float64, device=run.device)
    run._check(run.lib.vlb_read_fields(run.h, None, run._ptr(u)))
    o, w = ref["origin"], ref["width"]
    crop = u[:, o[2] + 1:o[2] + w - 1, o[1] + 1:o[1] + w - 1, o[0] + 1:o[0] + w - 1]
    err["u_crop"] = rel_l2(crop.cpu().numpy(), ref["u_crop"])
    del u
    return {"line_velocity_rel_l2": {k: float(f"{v:.3e}") for k, v in err.items() if k != "u_crop"},
            "lattice_velocity_rel_l2": float(f"{err['u_crop']:.3e}"),
            "sample": f"{t.size} targets; crop interior {w - 2}^3 nodes at {tuple(x + 1 for x in o)}"}


def measure(cfg, args, ref, graph):
    """One precision row: accuracy from the seeded state (if the oracle leg
    ran), warm-up, the timed steps, and the kernel timings inside them."""
    import torch

    import paper_2108_04435_amd as vlb

    lat = cfg["lattice"]
    prec = lat["precision"]
    n0 = cfg["pos"].shape[0]
    stream = torch.cuda.Stream()   # default priority; graphs need a non-null stream
    torch.cuda.set_stream(stream)
    run = vlb.run_from_config(cfg, n_cap=point_capacity(n0, args.capacity_factor),
                              recon_cap=1 << 18)
    cells = lat["nx"] * lat["ny"] * lat["nz"]
    acc = accuracy(run, ref) if ref is not None else None

    def advance(plan, events=None):
        for kind, k in plan:
            if events is not None:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
            if kind == "graph":
                run.step_graph(k)
            else:
                run.step(k)
            if events is not None:
                b.record(stream)
                events.append((a, b, k))

    advance(step_plan(args.warmup, graph))
    run.sync()
    direct = graph == 0
    # two events per timed launch: every stage's sum and the LBM update
    launches = int(cfg["vortex"].get("rk_stages", 4)) * int(cfg["vortex"].get("vfm_substeps", 1)) + 1
    run.set_timing(direct, reserve=2 * launches * args.steps + 64)  # also zeroes the work counters
    ev = []
    plan = step_plan(args.steps, graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(plan, ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    run.sync()
    step_ms = np.concatenate([np.full(k, a.elapsed_time(b) / k) for a, b, k in ev]) \
        if ev else np.zeros(1)
    nodes, pairs = run.work()
    n_end = run.n_points()
    if direct:
        bs_ms, bs_n = run.timing(0)
        lbm_ms, lbm_n = run.timing(1)
        bs_basis = f"HIP events around each of the {bs_n} launches inside the timed steps"
    else:   # graphs carry no per-launch events: the kernels alone at the final state
        bs_ms, bs_n = run.time_kernel(0, reps=20) * 20, 20
        pairs = 20 * n_end * (n_end - 2)
        lbm_ms, lbm_n = run.time_kernel(1, reps=20) * 20, 20
        bs_basis = "20 launches back to back at the final state (HIP events)"
    bs_us = bs_ms * 1e3 / max(bs_n, 1)
    pairs_launch = pairs / max(bs_n, 1)
    lbm_us = lbm_ms * 1e3 / max(lbm_n, 1)
    # populations read and written, plus the spread force field (three
    # components in the arithmetic type) that a coupled update reads
    force_node = 3 * (8 if prec == "f64" else 4) if cfg["vortex"].get("coupling", True) else 0
    lbm_node = 2 * 19 * STORE_BYTES[prec] + force_node
    lbm_bytes = lbm_node * cells
    row = {
        "precision": prec,
        "value": round(args.steps / wall, 4),
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "step_ms_p50": round(float(np.percentile(step_ms, 50)), 4),
        "step_ms_p99": round(float(np.percentile(step_ms, 99)), 4),
        "step_time_basis": ("per step (HIP events around each step)" if direct else
                            f"per graph launch of {graph} steps / {graph} (direct remainder "
                            "per call)"),
        "mlups": round(cells * args.steps / wall / 1e6, 1),
        "bs_gpairs_s": round(pairs / max(bs_n, 1) * bs_n / wall / 1e9, 2) if direct else None,
        "points_start": int(n0),
        "points_end": int(n_end),
        "bs_kernel": {"name": "k_bs_f64" if prec == "f64" else "k_bs_f32",
                      "avg_launch_us": round(bs_us, 2), "launches": int(bs_n),
                      "pairs_per_launch": int(pairs_launch),
                      "tpairs_s": round(pairs_launch / (bs_us * 1e-6) / 1e12, 4),
                      "basis": bs_basis},
        "lbm_kernel": {"avg_launch_us": round(lbm_us, 2), "launches": int(lbm_n),
                       "glups": round(cells / (lbm_us * 1e-6) / 1e9, 3),
                       "bytes_per_node": lbm_node,
                       "force_bytes_per_node": force_node,
                       "algorithmic_GBs": round(lbm_bytes / (lbm_us * 1e-6) / 1e9, 1),
                       "population_bytes": 19 * STORE_BYTES[prec] * cells,
                       "cache_resident": 19 * STORE_BYTES[prec] * cells <= LLC_BYTES},
        "accuracy_vs_oracle": acc,
    }
    extra = {"run": run, "cells": cells, "pairs_launch": pairs_launch, "bs_us": bs_us,
             "lbm_us": lbm_us, "lbm_bytes": lbm_bytes, "n_end": n_end}
    return row, extra


def point_capacity(n0, factor=1.4):
    """Point capacity of a run from n0 points: room for the remeshing's
    growth (the tangle grows by 28% over 100 steps, counterflow by 26% over
    220); the capacity also sizes the Biot-Savart launch."""
    return int(n0 * factor) + 256


def lbm_kernel_name(lat):
    """The update kernel the library launches for a lattice: FP16 storage on
    rows of 256 nodes periodic in x and y takes four nodes per lane."""
    if lat["precision"] == "f16" and lat["nx"] == 256 and not lat["walls"][0] \
            and not lat["walls"][1]:
        return "k_collide_rows4"
    return "k_collide_stream"


def lbm_only(n, precision, steps=20, lattice=None):
    """The normal-fluid update alone on an n^3 periodic lattice (working set
    far above the 256 MB last-level cache), or on ``lattice`` (a lattice
    dict: its walls and planes), full grid: kernel time from HIP events
    around each launch, per AA parity."""
    import paper_2108_04435_amd as vlb
    import workloads as wl

    lat = dict(lattice, precision=precision) if lattice is not None else \
        wl.lattice_preset(n, n, n, tau=0.8, precision=precision)
    dims = (lat["nx"], lat["ny"], lat["nz"])
    run = vlb.Run(lat, wl.vortex_preset(), n_cap=1)
    rho, u = wl.velocity_field(4, dims, (0.0, 0.0, 0.02), 1e-4)
    run.write_fields(rho, u)
    del rho, u
    run.step(4)
    run.sync()
    run.set_timing(True, reserve=4 * steps)
    run.step(steps)
    run.sync()
    ms, k = run.timing(1)
    bytes_node = 2 * 19 * STORE_BYTES[precision]
    cells = dims[0] * dims[1] * dims[2]
    gbs = bytes_node * cells * k / (ms * 1e-3) / 1e9
    run.close()
    return dict(lattice="x".join(str(d) for d in dims), precision=precision,
                kernel_us=round(ms * 1e3 / k, 1),
                glups=round(cells * k / (ms * 1e-3) / 1e9, 2), bytes_per_node=bytes_node,
                achieved_GBs=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4))


def time_diagnostics(run, cells, precision, n_points, reps=10):
    """Host-visible time of one call of each diagnostic at the final state
    (median of reps calls; each call launches its kernels and synchronises
    with its copy to the host), with the algorithmic bytes of the lattice
    ones: the velocity statistics read the populations twice; the vorticity
    reads them once, writes the velocity, reads it back and writes the curl."""
    import torch

    b = STORE_BYTES[precision]

    def med(fn):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    u = torch.empty((3,) + run.shape, dtype=torch.float64, device=run.device)
    w = torch.empty_like(u)
    pu, pw = run._ptr(u), run._ptr(w)

    def vort():
        run._check(run.lib.vlb_read_vorticity(run.h, pu, pw))

    t_len = med(run.line_length)
    t_st = med(run.flow_stats)
    t_w = med(vort)
    st_bytes = 2 * 19 * b * cells
    w_bytes = (19 * b + 24 + 24 + 24) * cells
    return {
        "line_length": {"call_us": round(t_len * 1e6, 1), "points": int(n_points)},
        "flow_stats": {"call_us": round(t_st * 1e6, 1), "bytes": st_bytes,
                       "GBs": round(st_bytes / t_st / 1e9, 1)},
        "vorticity": {"call_us": round(t_w * 1e6, 1), "bytes": w_bytes,
                      "GBs": round(w_bytes / t_w / 1e9, 1),
                      "note": "device outputs (u and omega stay in HBM)"},
    }


def hbm_copy(torch, nbytes=1 << 30, reps=10):
    """A plain device-to-device copy far above the last-level cache: the
    practical HBM rate (read + write bytes over time) beside the peak."""
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        y.copy_(x)
    b.record(s)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    torch.cuda.empty_cache()
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    return dict(bytes=2 * nbytes, ms=round(ms, 4), GBs=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4))


def farfield_bench(torch, vlb, cfg, cell, theta, levels, reps=10):
    """The far-field approximation of the non-local Biot-Savart sum
    (vlb_biot_savart_farfield, reading F2) beside the direct FP32 sum
    (vlb_biot_savart) on the workload's filaments, both through the C ABI
    with device-resident inputs: time per call (HIP events around ``reps``
    calls on torch's stream, every kernel of each call inside) and the
    approximation's relative L2 error against the direct sum.  Periodic
    boxes only (None otherwise)."""
    lat = cfg["lattice"]
    dims = (lat["nx"], lat["ny"], lat["nz"])
    if any(lat["walls"]) or any(d % cell for d in dims):
        return None
    L = np.array(dims, dtype=np.float64)
    pos = np.mod(cfg["pos"], L)
    nxt = np.ascontiguousarray(cfg["nxt"], dtype=np.int32)
    n = pos.shape[0]
    kappa = cfg["vortex"]["kappa"]
    p = torch.as_tensor(np.ascontiguousarray(pos)).cuda()
    q = torch.as_tensor(nxt).cuda()
    v = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    lib = vlb.load_library()
    d = vlb.bs_desc(dims, (False, False, False), kappa, "f32")
    nb = vlb.ctypes.c_uint64(0)
    vlb._raise(lib, lib.vlb_biot_savart_workspace(vlb.ctypes.byref(d), n, vlb.ctypes.byref(nb)))
    ws = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    s = torch.cuda.current_stream()
    vp = vlb.ctypes.c_void_p

    def direct():
        vlb._raise(lib, lib.vlb_biot_savart(vlb.ctypes.byref(d), n, vp(p.data_ptr()),
                                            vp(q.data_ptr()), vp(v.data_ptr()), vp(wp),
                                            vlb.ctypes.c_uint64(int(nb.value)), vp(s.cuda_stream)))

    ff = vlb.FarField(dims, n, cell, theta, kappa, levels=levels)

    def far():
        ff.run(p, q, v)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(reps):
            fn()
        b.record(s)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_dir = timed(direct)
    v_dir = v.cpu().numpy()
    t_far = timed(far)
    v_far = v.cpu().numpy()
    err = float(np.linalg.norm(v_far - v_dir) / np.linalg.norm(v_dir))
    del ws, ff, p, q, v
    torch.cuda.empty_cache()
    return dict(points=n, cell=cell, levels=levels, theta=theta,
                cells=int(np.prod([x // cell for x in dims])),
                direct_f32_ms=round(t_dir, 4), farfield_ms=round(t_far, 4),
                speedup=round(t_dir / t_far, 3), rel_l2_vs_direct=float(f"{err:.3e}"),
                basis="HIP events around %d calls each, inputs resident on the GPU" % reps)


def farfield_steps(torch, vlb, cfg, args, cell, theta, levels):
    """Coupled steps of the workload with the far-field approximation as the
    non-local sum of every stage (vortex descriptor ff_cell), timed as the
    headline is (same warm-up, steps and graph chunks).  Periodic boxes
    with FP32 arithmetic only (None otherwise)."""
    lat = cfg["lattice"]
    dims = (lat["nx"], lat["ny"], lat["nz"])
    if any(lat["walls"]) or lat["precision"] == "f64" or any(d % (cell * levels) for d in dims):
        return None
    cfg = dict(cfg, vortex=dict(cfg["vortex"], ff_cell=cell, ff_levels=levels, ff_theta=theta))
    n0 = cfg["pos"].shape[0]
    stream = torch.cuda.Stream()   # default priority; graphs need a non-null stream
    torch.cuda.set_stream(stream)
    run = vlb.run_from_config(cfg, n_cap=point_capacity(n0, args.capacity_factor),
                              recon_cap=1 << 18)
    graph = args.graph

    def advance(plan, events=None):
        for kind, k in plan:
            if events is not None:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
            if kind == "graph":
                run.step_graph(k)
            else:
                run.step(k)
            if events is not None:
                b.record(stream)
                events.append((a, b, k))

    advance(step_plan(args.warmup, graph))
    run.sync()
    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(step_plan(args.steps, graph), ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    run.sync()
    step_ms = np.concatenate([np.full(k, a.elapsed_time(b) / k) for a, b, k in ev])
    n_end = run.n_points()
    run.close()
    torch.cuda.empty_cache()
    cells = dims[0] * dims[1] * dims[2]
    return dict(value=round(args.steps / wall, 4), unit="steps/s",
                ms_per_step=round(1e3 * wall / args.steps, 4),
                step_ms_p50=round(float(np.percentile(step_ms, 50)), 4),
                step_ms_p99=round(float(np.percentile(step_ms, 99)), 4),
                mlups=round(cells * args.steps / wall / 1e6, 1), precision=lat["precision"],
                points_start=int(n0), points_end=int(n_end), graph_steps=graph)


def serve_run(n_requests, budget_gb, slots, per_run_graphs):
    """The served form on a request stream of ``n_requests`` counterflow
    runs (seed 5, Poisson arrivals at 2/s, lattices {32^3, 64^3, 64x64x256,
    128x128x256}, 1k-20k points, alpha U[0.1,0.3], alpha' U[0,0.02], v_n
    U[0.01,0.04], 500-2000 steps), admitted by HBM budget and slots and
    stepped in chunks: run latency (arrival to completion) p50 / p99 and
    aggregate MLUPS."""
    import workloads as wl
    from paper_2108_04435_amd import serve

    reqs = wl.serving_requests(seed=5, n_requests=n_requests)
    srv = serve.Server(budget_bytes=int(budget_gb * (1 << 30)), max_slots=slots, chunk=10,
                       group=not per_run_graphs)
    res, makespan = srv.serve(reqs)
    s = serve.summarize(res, makespan)
    pairs = sum(r.steps * 4 * r.points_start * (r.points_start - 2) for r in res)
    return {
        "config": {"workload": f"serving_{n_requests}_requests_poisson_2_per_s",
                   "budget_gb": budget_gb, "slots": slots, "chunk": 10,
                   "grouped_step_many": not per_run_graphs},
        **s,
        "approx_bs_gpairs_s": round(pairs / makespan / 1e9, 1),
        "arrival_span_s": round(max(r["arrival"] for r in reqs), 2),
    }


def serve_bench(args):
    """Served form: 64 counterflow requests arriving as a Poisson stream at
    2/s (serve_run)."""
    r = serve_run(args.serve_requests, args.serve_budget_gb, args.serve_slots,
                  args.serve_per_run_graphs)
    out = {
        "metric": "served coupled runs: p50/p99 run latency, aggregate MLUPS",
        "value": r["aggregate_mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        **r,
    }
    print(json.dumps(out), flush=True)


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tangle", choices=WORKLOADS)
    ap.add_argument("--precision", default=None, choices=("f64", "f32", "f16"))
    ap.add_argument("--rows", default=None,
                    help="comma-separated precisions measured beside the headline "
                         "(default for the 256^3 tangle: f32,f64; 'none' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--wall-images", action="store_true",
                    help="superfluid wall term from image filaments (walled workloads)")
    ap.add_argument("--graph", type=int, default=None,
                    help="advance in HIP-graph launches of this many steps (even); 0: direct")
    ap.add_argument("--no-diagnostics", action="store_true")
    ap.add_argument("--lbm-probe", action="store_true",
                    help="also time the LBM update alone on 256^3 (FP16, FP32, FP64 storage)")
    ap.add_argument("--baseline-workers", type=int, default=None)
    ap.add_argument("--ff-cell", type=int, default=16,
                    help="cell edge of the far-field approximation measured beside the direct "
                         "sum (periodic workloads; 0: not measured)")
    ap.add_argument("--ff-theta", type=float, default=0.25)
    ap.add_argument("--ff-levels", type=int, default=2, choices=(1, 2))
    ap.add_argument("--rk-stages", type=int, default=None, choices=(1, 2, 4),
                    help="Runge-Kutta stages of the filament integration (default: the workload's, 4)")
    ap.add_argument("--vfm-substeps", type=int, default=None,
                    help="filament substeps per lattice step (default: the workload's, 1)")
    ap.add_argument("--capacity-factor", type=float, default=1.4,
                    help="point capacity of the runs as a multiple of the seeded points "
                         "(raise it for long runs)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--served-requests", type=int, default=16,
                    help="requests of the short served mix in the tangle line (0: none)")
    ap.add_argument("--serve-budget-gb", type=float, default=6.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-per-run-graphs", action="store_true",
                    help="served form: each run launches its own chunk graph instead of the idle "
                         "runs advancing together (one vlb_step_many call per chunk)")
    args = ap.parse_args(argv)
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be >= 1 and --warmup >= 0")
    if args.workload != "serve":
        if args.graph is None:
            args.graph = DEFAULT_GRAPH[args.workload]
        step_plan(args.steps, args.graph)   # validates the chunk
        head = args.precision or DEFAULT_PRECISION[args.workload]
        if args.rows is None:
            rows = ["f32", "f64"] if args.workload == "tangle" else []
        elif args.rows in ("", "none"):
            rows = []
        else:
            rows = [p.strip() for p in args.rows.split(",") if p.strip()]
        for p in rows:
            if p not in STORE_BYTES:
                ap.error(f"unknown precision {p} in --rows")
        args.head_precision = head
        args.row_precisions = [p for p in rows if p != head]
    return args


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this program runs on one GPU only (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        import torch

        torch.cuda.set_device(0)
        serve_bench(args)
        return

    t_setup = time.perf_counter()
    cfg = make_workload(args.workload, args.head_precision)
    if args.wall_images:
        cfg["vortex"] = dict(cfg["vortex"], wall_images=True)
    # time integration of the filaments (classical RK4 in one step unless set)
    if args.rk_stages is not None or args.vfm_substeps is not None:
        cfg["vortex"] = dict(cfg["vortex"],
                             rk_stages=args.rk_stages or cfg["vortex"].get("rk_stages", 4),
                             vfm_substeps=args.vfm_substeps or cfg["vortex"].get("vfm_substeps", 1))
    print(f"[bench] workload {cfg['name']}: {cfg['pos'].shape[0]} points, "
          f"{time.perf_counter() - t_setup:.1f} s", file=sys.stderr, flush=True)
    base, ref = None, None
    if not args.no_cpu_baseline:
        # before any GPU work: the oracle leg forks its worker pool
        base, ref = cpu_baseline(cfg, workers=args.baseline_workers)
        print(f"[bench] oracle leg done: {base['sample']}", file=sys.stderr, flush=True)

    import torch

    import paper_2108_04435_amd as vlb

    vlb.load_library()   # raises if the HIP library is not built
    torch.cuda.set_device(0)

    lat = cfg["lattice"]
    prec = args.head_precision
    head, hx = measure(cfg, args, ref, args.graph)
    print(f"[bench] {prec}: {head['value']} steps/s", file=sys.stderr, flush=True)
    diagnostics = None if args.no_diagnostics else time_diagnostics(
        hx["run"], hx["cells"], prec, hx["n_end"])
    hx["run"].close()
    del hx["run"]
    torch.cuda.empty_cache()

    rows = []
    for p in args.row_precisions:
        r, rx = measure(with_precision(cfg, p), args, ref, args.graph)
        rx["run"].close()
        del rx["run"]
        torch.cuda.empty_cache()
        print(f"[bench] {p}: {r['value']} steps/s", file=sys.stderr, flush=True)
        rows.append(r)
    plain = [r for r in [head] + rows if r["precision"] == "f64"]
    if plain:
        for r in [head] + rows:
            r["speedup_vs_f64"] = round(r["value"] / plain[0]["value"], 3)

    f64 = prec == "f64"
    peak = PEAK_FP64_VECTOR_TFLOPS if f64 else PEAK_FP32_VECTOR_TFLOPS
    achieved = FLOPS_PER_PAIR * hx["pairs_launch"] / (hx["bs_us"] * 1e-6) / 1e12
    src = os.path.join(ROOT, "paper_2108_04435_amd", "csrc", "bs.hip")
    roofline = {
        "bound": "alu",
        "kernel": head["bs_kernel"]["name"],
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": None if f64 else traffic_record(src, cfg["name"]),
        "avg_launch_us": head["bs_kernel"]["avg_launch_us"],
        "pairs_per_launch": head["bs_kernel"]["pairs_per_launch"],
        "flops_per_pair": FLOPS_PER_PAIR,
        "basis": head["bs_kernel"]["basis"],
        "issue": None if f64 else valu_record(src, cfg["name"]),
    }
    lbm_gbs = hx["lbm_bytes"] / (hx["lbm_us"] * 1e-6) / 1e9
    # the update alone on the workload's lattice (uncoupled: populations
    # only), full grid, beside the in-step launches, which run on a narrow
    # grid next to a Biot-Savart launch that holds every CU
    alone = lbm_only(0, prec, lattice=lat)
    torch.cuda.empty_cache()
    lbm_roofline = {
        "bound": "hbm", "kernel": lbm_kernel_name(lat),
        "achieved": alone["achieved_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": alone["frac"],
        "bytes_per_launch": alone["bytes_per_node"] * lat["nx"] * lat["ny"] * lat["nz"],
        "avg_launch_us": alone["kernel_us"],
        "basis": "the update alone on the workload's lattice, full grid, HIP events around "
                 "each of 20 launches (populations read and written once each)",
        "in_step": {
            "achieved": round(lbm_gbs, 1), "frac": round(lbm_gbs / PEAK_HBM_GBS, 4),
            "bytes_per_launch": hx["lbm_bytes"],
            "avg_launch_us": head["lbm_kernel"]["avg_launch_us"],
            "basis": "in the coupled steps: populations and the spread force, on a narrow "
                     "grid beside the Biot-Savart launches",
        },
        "cache_resident": head["lbm_kernel"]["cache_resident"],
    }
    out = {
        "metric": "coupled steps/s (LBM MLUPS + Biot-Savart Gpairs/s), FP32/FP16 vs FP64; p99",
        "value": head["value"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f16-storage/f32"}[prec],
        "data": "synthetic",
        "config": {
            "workload": cfg["name"],
            "lattice": [lat["nx"], lat["ny"], lat["nz"]],
            "precision": prec,
            "points_start": head["points_start"],
            "points_end": head["points_end"],
            "walls": list(lat["walls"]),
            "mass_balance": bool(cfg["vortex"]["mass_balance"]),
            "reconnect": bool(cfg["vortex"]["reconnect"]),
            "wall_images": bool(cfg["vortex"].get("wall_images", False)),
            "rk_stages": int(cfg["vortex"].get("rk_stages", 4)),
            "vfm_substeps": int(cfg["vortex"].get("vfm_substeps", 1)),
            "graph_steps": args.graph,
        },
        "step_ms_p50": head["step_ms_p50"],
        "step_ms_p99": head["step_ms_p99"],
        "step_time_basis": head["step_time_basis"],
        "mlups": head["mlups"],
        "bs_gpairs_s": head["bs_gpairs_s"],
        "roofline": roofline,
        "lbm_roofline": lbm_roofline,
        "headline": head,
        "rows": rows,
        "diagnostics": diagnostics,
    }
    if args.lbm_probe:
        out["lbm_256cubed"] = [lbm_only(256, p) for p in ("f16", "f32", "f64")]
        torch.cuda.empty_cache()
    if args.ff_cell > 0:
        out["farfield"] = farfield_bench(torch, vlb, cfg, args.ff_cell, args.ff_theta,
                                         args.ff_levels)
        if out["farfield"] is not None:
            st = farfield_steps(torch, vlb, cfg, args, args.ff_cell, args.ff_theta,
                                args.ff_levels)
            if st is not None:
                st["speedup_vs_direct_steps"] = round(st["value"] / head["value"], 3)
                print(f"[bench] {prec} with the far field: {st['value']} steps/s",
                      file=sys.stderr, flush=True)
            out["farfield"]["coupled_steps"] = st
    out["hbm_copy"] = hbm_copy(torch)
    if args.served_requests > 0 and args.workload == "tangle":
        # a short served mix beside the headline (the served form's latency
        # and throughput; --workload serve runs the full 64 requests)
        torch.cuda.empty_cache()
        out["served"] = serve_run(args.served_requests, args.serve_budget_gb, args.serve_slots,
                                  args.serve_per_run_graphs)
        print(f"[bench] served {args.served_requests} requests: latency p50 "
              f"{out['served']['latency_p50_s']} s, p99 {out['served']['latency_p99_s']} s, "
              f"{out['served']['aggregate_mlups']} MLUPS", file=sys.stderr, flush=True)
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
