"""Benchmark of the coupled VFM-LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload: the counterflow channel, 64x64x256 lattice with bounce-back
walls on x and y, periodic z, Guo body force for a mean normal-fluid velocity
of about 0.02, 200 seeded rings (R ~ U[4,12], ~1.0e4 points), remeshing
spacing 1.0, mass balance on z, FP32 deviation storage and FP32
Biot-Savart.  Inputs are synthetic and already resident in HBM when the
timed region starts.  One step = one pass of the whole coupled step
(mass-balance superflow, 4 RK stages of Biot-Savart + LIA + interpolation +
Schwarz, force spreading, LBM collide+stream, remeshing).

The run advances in launches of a HIP graph holding 10 captured steps
(``--graph 0``: steps enqueued one by one).

Prints ONE JSON line.  ``value`` is coupled steps per second on the one GPU;
``roofline`` is for the dominant kernel (the Biot-Savart pair sum), its
launch duration measured with HIP events on the run's stream (50 launches
back to back at the final state, after the timed steps); ``cpu_baseline``
times the FP64 oracle on the host on a bounded sample of the same workload.
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
# Biot-Savart closed form as evaluated (R1 = s_k - r, d = segment vector,
# R1 x R2 = R1 x d, |R2|^2 = |R1|^2 + 2 R1.d + |d|^2), counting a fused
# multiply-add as 2 flops and a reciprocal / reciprocal square root as 1:
# separation 3, R1.d 5, |R1|^2 5, |R2|^2 3, R1.R2 1, two inverse norms 2,
# cross product 9, product of inverse norms 1, denominator 2, reciprocal 1,
# numerator and scale 3, accumulation 6.
FLOPS_PER_PAIR = 41
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_FP64_VECTOR_TFLOPS = 78.6    # MI355X published FP64 vector peak
PEAK_HBM_GBS = 8000.0             # MI355X published HBM3E bandwidth
# Issue ceiling of the FP32 pair loop: packed FP32 is not used, so a SIMD
# issues one VALU instruction per lane per cycle: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz.  The unrolled loop body of the built kernel holds 117
# VALU instructions per 4 pairs (its 12 transcendental ones issue beside
# them), i.e. 29.25 per pair.
VALU_LANE_ISSUE_PER_S = 256 * 4 * 16 * 2.4e9
VALU_PER_PAIR_F32 = 29.25

WORKLOADS = ("counterflow", "ring32", "heater", "tangle", "serve")


def make_workload(name, precision=None):
    import workloads as wl

    if name == "counterflow":
        cfg = wl.config_counterflow(precision=precision or "f32")
    elif name == "ring32":
        cfg = wl.config_ring32(precision=precision or "f64")
    elif name == "heater":
        cfg = wl.config_heater(precision=precision or "f32")
    elif name == "tangle":
        cfg = wl.config_tangle(precision=precision or "f16")
    else:
        raise SystemExit(f"unknown workload {name}")
    return cfg


def traffic_record(kernel_src, workload):
    """HBM bytes per launch of the Biot-Savart kernel from committed
    rocprofv3 counter runs, if they were taken on the current source and on
    this workload (FP32 storage)."""
    path = os.path.join(ROOT, "profiles", "bs_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha") != h or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(cfg, n_evals=2):
    """Oracle (plain FP64 numpy) on the host: one full LBM update of the
    lattice plus n_evals full Biot-Savart sums (every target against every
    segment), scaled to one coupled step (4 Biot-Savart evaluations)."""
    from oracle import coupled, lbm, vfm
    from oracle.lbm import Lattice
    from oracle.vfm import VortexParams

    L = cfg["lattice"]
    lat = Lattice(L["nx"], L["ny"], L["nz"], tau=L["tau"], walls=tuple(L["walls"]),
                  plane_lo=L["plane_lo"], plane_hi=L["plane_hi"], plane_u=tuple(L["plane_u"]),
                  body_force=tuple(L["body_force"]))
    vp = VortexParams(**{k: cfg["vortex"][k] for k in VortexParams.__dataclass_fields__
                         if k in cfg["vortex"]})
    st = coupled.make_state(cfg["rho"], cfg["u"], cfg["pos"], cfg["nxt"], lat)
    n = st.pos.shape[0]
    t0 = time.perf_counter()
    _, ub = lbm.bare_velocity(st.f, lat)
    if vp.mass_balance:
        lbm.mass_balance_superflow(st.f, lat, vp.rho_s_over_rho_n)
    lbm.lbm_step(st.f, np.zeros((3,) + lat.shape), lat)
    t1 = time.perf_counter()
    for _ in range(n_evals):
        vfm.biot_savart_nonlocal(st.pos, st.nxt, st.prv, lat, vp.kappa)
    t2 = time.perf_counter()
    t_step = (t1 - t0) + 4.0 * (t2 - t1) / n_evals
    return dict(value=1.0 / t_step, unit="steps/s", cores=1, kind="oracle",
                sample=f"one FP64 LBM update of all {lat.nx}x{lat.ny}x{lat.nz} nodes plus "
                       f"{n_evals} full Biot-Savart sums ({n} targets x all segments), scaled to "
                       f"one coupled step (4 evaluations); numpy, single thread; "
                       f"measured {t2 - t0:.1f} s")


def lbm_only(torch, vlb, wl, n, precision, steps=20):
    """Normal-fluid update alone on an n^3 periodic lattice (working set far
    above the 256 MB last-level cache): kernel GB/s from HIP events."""
    lat = wl.lattice_preset(n, n, n, tau=0.8, precision=precision)
    run = vlb.Run(lat, wl.vortex_preset(), n_cap=1)
    rho, u = wl.velocity_field(4, (n, n, n), (0.0, 0.0, 0.02), 1e-4)
    run.write_fields(rho, u)
    del rho, u
    run.step(4)
    run.sync()
    run.set_timing(True, reserve=4 * steps)
    run.step(steps)
    run.sync()
    ms, k = run.timing(1)
    b = {"f64": 8, "f32": 4, "f16": 2}[precision]
    bytes_node = 2 * 19 * b
    cells = n ** 3
    gbs = bytes_node * cells * k / (ms * 1e-3) / 1e9
    run.close()
    return dict(lattice=f"{n}^3", precision=precision, kernel_ms=ms / k,
                glups=cells * k / (ms * 1e-3) / 1e9, bytes_per_node=bytes_node,
                achieved_GBs=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4))


def hbm_copy(torch, nbytes=1 << 30, reps=10):
    """A plain device-to-device copy far above the last-level cache: the
    practical HBM rate (read + write bytes over time) beside the peak."""
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    torch.cuda.empty_cache()
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    return dict(bytes=2 * nbytes, ms=round(ms, 4), GBs=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4))


def serve_bench(args):
    """Served form: 64 counterflow requests arriving as a Poisson stream at
    2/s, lattices {32^3, 64^3, 64x64x256, 128x128x256}, 1k-20k points,
    alpha U[0.1,0.3], alpha' U[0,0.02], v_n U[0.01,0.04], 500-2000 steps,
    admitted by HBM budget and slots, stepped in graph-captured chunks."""
    import workloads as wl
    from paper_2108_04435_amd import serve

    reqs = wl.serving_requests(seed=5, n_requests=args.serve_requests)
    srv = serve.Server(budget_bytes=int(args.serve_budget_gb * (1 << 30)),
                       max_slots=args.serve_slots, chunk=10)
    res, makespan = srv.serve(reqs)
    s = serve.summarize(res, makespan)
    pairs = sum(r.steps * 4 * r.points_start * (r.points_start - 2) for r in res)
    out = {
        "metric": "served coupled runs: p50/p99 run latency, aggregate MLUPS",
        "value": s["aggregate_mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving_64_requests_poisson_2_per_s",
                   "budget_gb": args.serve_budget_gb, "slots": args.serve_slots, "chunk": 10},
        **s,
        "approx_bs_gpairs_s": round(pairs / makespan / 1e9, 1),
        "arrival_span_s": round(max(r["arrival"] for r in reqs), 2),
    }
    print(json.dumps(out), flush=True)


def time_diagnostics(run, cells, precision, n_points, reps=10):
    """Host-visible time of one call of each diagnostic at the final state
    (median of reps calls; each call launches its kernels and synchronises
    with its copy to the host), with the algorithmic bytes of the lattice
    ones: the velocity statistics read the populations twice; the vorticity
    reads them once, writes the velocity, reads it back and writes the curl."""
    b = {"f64": 8, "f32": 4, "f16": 2}[precision]

    def med(fn):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    import ctypes
    import torch

    u = torch.empty((3,) + run.shape, dtype=torch.float64, device=run.device)
    w = torch.empty_like(u)
    pu, pw = ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(w.data_ptr())

    def vort():
        if run.lib.vlb_read_vorticity(run.h, pu, pw) != 0:
            raise RuntimeError("vlb_read_vorticity failed")

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="counterflow", choices=WORKLOADS)
    ap.add_argument("--precision", default=None, choices=("f64", "f32", "f16"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", type=int, default=10,
                    help="advance in HIP-graph launches of this many steps (even); 0: direct")
    ap.add_argument("--no-lbm-probe", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-budget-gb", type=float, default=6.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this program runs on one GPU only (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2108_04435_amd as vlb
    import workloads as wl

    if not os.path.exists(vlb.LIB_PATH):
        from paper_2108_04435_amd import build as b
        b.build()

    torch.cuda.set_device(0)
    if args.workload == "serve":
        serve_bench(args)
        return
    cfg = make_workload(args.workload, args.precision)
    lat = cfg["lattice"]
    n0 = cfg["pos"].shape[0]
    run = vlb.run_from_config(cfg, n_cap=int(n0 * 1.4) + 256,
                              recon_cap=1 << 18)
    cells = lat["nx"] * lat["ny"] * lat["nz"]

    G = args.graph
    if G:
        if G % 2 or args.steps % G or args.warmup % G:
            raise SystemExit("--graph needs an even chunk dividing --steps and --warmup")
        stream = torch.cuda.Stream()
        torch.cuda.set_stream(stream)
        run.close()
        run = vlb.run_from_config(cfg, n_cap=int(n0 * 1.4) + 256, recon_cap=1 << 18)
        run.graph(G)
        adv, unit = (lambda: run.step_graph(G)), G
    else:
        adv, unit = (lambda: run.step(1)), 1
    for _ in range(args.warmup // unit):
        adv()
    run.sync()
    K = args.steps
    nev = K // unit
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(nev)]
    # per-launch kernel events inside the steps only when stepping directly
    run.set_timing(not G, reserve=2 * 6 * K + 64)  # also zeroes the work counters
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nev):
        ev[k][0].record(stream)
        adv()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run.sync()
    wall = t1 - t0
    step_ms = np.array([a.elapsed_time(b) for a, b in ev]) / unit
    nodes, pairs = run.work()
    in_step = None
    if not G:
        bs_ms, bs_n = run.timing(0)
        in_step = {"bs_avg_launch_us": round(bs_ms * 1e3 / max(bs_n, 1), 2),
                   "bs_pairs_per_launch": int(pairs / max(bs_n, 1)),
                   "note": "HIP events around every launch inside the steps (adds event overhead)"}
    n_end = run.n_points()
    # the dominant kernel alone, launched back to back on the final state
    bs_iso_ms = run.time_kernel(0, reps=50)
    pairs_iso = n_end * (n_end - 2)
    # the LBM update alone (advances the fluid; after the timed region)
    lbm_iso_ms = run.time_kernel(1, reps=20)
    diagnostics = time_diagnostics(run, cells, lat["precision"], n_end)

    value = K / wall
    achieved = FLOPS_PER_PAIR * pairs_iso / (bs_iso_ms * 1e-3) / 1e12
    src = os.path.join(ROOT, "paper_2108_04435_amd", "csrc", "bs.hip")
    f64 = lat["precision"] == "f64"
    peak = PEAK_FP64_VECTOR_TFLOPS if f64 else PEAK_FP32_VECTOR_TFLOPS
    roofline = {
        "bound": "alu",
        "kernel": "k_bs_f64" if f64 else "k_bs_f32",
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": traffic_record(src, cfg["name"]) if lat["precision"] == "f32" else None,
        "avg_launch_us": round(bs_iso_ms * 1e3, 2),
        "pairs_per_launch": int(pairs_iso),
        "flops_per_pair": FLOPS_PER_PAIR,
        "in_step": in_step,
    }
    if not f64:
        ceiling = VALU_LANE_ISSUE_PER_S / VALU_PER_PAIR_F32
        rate = pairs_iso / (bs_iso_ms * 1e-3)
        roofline["issue_ceiling"] = {"valu_per_pair": VALU_PER_PAIR_F32,
                                     "pairs_per_s": round(ceiling / 1e12, 4) * 1e12,
                                     "frac": round(rate / ceiling, 4)}
    b = {"f64": 8, "f32": 4, "f16": 2}[lat["precision"]]
    lbm_bytes = 2 * 19 * b * cells
    out = {
        "metric": "coupled steps/s (LBM MLUPS + Biot-Savart Gpairs/s), FP32/FP16 vs FP64; p99",
        "value": round(value, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f16-storage/f32"}[lat["precision"]],
        "data": "synthetic",
        "config": {
            "workload": cfg["name"],
            "lattice": [lat["nx"], lat["ny"], lat["nz"]],
            "precision": lat["precision"],
            "points_start": int(n0),
            "points_end": int(n_end),
            "walls": list(lat["walls"]),
            "mass_balance": bool(cfg["vortex"]["mass_balance"]),
            "reconnect": bool(cfg["vortex"]["reconnect"]),
        },
        "graph_steps": G,
        "step_ms_p50": round(float(np.percentile(step_ms, 50)), 4),
        "step_ms_p99": round(float(np.percentile(step_ms, 99)), 4),
        "step_time_basis": (f"per graph launch of {G} steps / {G}" if G else "per step"),
        "mlups": round(cells * K / wall / 1e6, 1),
        "bs_gpairs_s": round(pairs / wall / 1e9, 2),
        "bs_kernel_gpairs_s": round(pairs_iso / (bs_iso_ms * 1e-3) / 1e9, 2),
        "lbm_kernel": {"avg_launch_us": round(lbm_iso_ms * 1e3, 2),
                       "glups": round(cells / (lbm_iso_ms * 1e-3) / 1e9, 2),
                       "algorithmic_GBs": round(lbm_bytes / (lbm_iso_ms * 1e-3) / 1e9, 1),
                       "note": "20 launches back to back; this lattice fits the 256 MB last-level cache"},
        "roofline": roofline,
        "diagnostics": diagnostics,
    }
    run.close()
    del run
    torch.cuda.empty_cache()

    if args.copy_probe:
        x = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * x.numel()
        del x, y

    if not args.no_lbm_probe:
        out["lbm_256cubed"] = [lbm_only(torch, vlb, wl, 256, p) for p in ("f32", "f16", "f64")]
        torch.cuda.empty_cache()
        out["hbm_copy"] = hbm_copy(torch)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
