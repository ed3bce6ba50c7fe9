"""Served form of the coupled step: a persistent request loop with
continuous batching on one GPU.

Requests (counterflow runs of different lattice sizes, vortex counts,
mutual-friction coefficients and heat fluxes) arrive over time.  The loop
  * admits an arrived request when a slot is free and its device footprint
    (``vlb_query_footprint``) fits in what is left of the HBM budget;
  * keeps every admitted run resident in its own workspace, on one stream of
    a fixed pool (one stream per slot, default priority);
  * advances every resident run by chunks of steps: each chunk is one
    launch of a HIP graph captured once per run, or (group=True) all the
    idle runs that have a whole chunk left advance together, enqueued by
    one library call (vlb_step_many, step by step across the runs); a
    remainder is stepped directly at the end; runs on different streams
    overlap on the GPU;
  * retires a run when its last chunk has completed: reads its final state,
    frees its workspace, and records arrival -> completion latency.
A run's kernels touch only its own workspace and no result depends on a
reduction across runs, so every result is the same alone and in the mix.
"""

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import Run, load_library, lattice_desc, step_many, vortex_desc, VlbError  # noqa: F401


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    cells: int
    points_start: int
    points_end: int
    footprint: int
    pos: np.ndarray = None
    nxt: np.ndarray = None
    u: np.ndarray = None
    error: str = ""

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class _Active:
    req: dict
    run: Run
    slot: int
    remaining: int
    admitted: float
    footprint: int
    event: object = None
    points_start: int = 0


def footprint(cfg, n_cap, recon_cap):
    import ctypes

    lib = load_library()
    ld = lattice_desc(cfg["lattice"])
    vd = vortex_desc(cfg["vortex"], n_cap, recon_cap)
    nb = ctypes.c_uint64(0)
    code = lib.vlb_query_footprint(ctypes.byref(ld), ctypes.byref(vd), ctypes.byref(nb))
    if code != 0:
        raise VlbError(code, lib.vlb_last_error(None).decode())
    return int(nb.value) + 256


class Server:
    def __init__(self, budget_bytes, max_slots=16, chunk=10, device=0, keep_fields=False,
                 cap_factor=6.0, recon_cap=1 << 16, group=False):
        import torch

        if chunk < 2 or chunk % 2:
            raise ValueError("chunk must be even and >= 2")
        self.torch = torch
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.device = torch.device("cuda", device)
        self.keep_fields = keep_fields
        self.cap_factor = cap_factor
        self.recon_cap = recon_cap
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.max_slots)]
        # group=True: the idle runs with a whole chunk left advance together,
        # enqueued by one vlb_step_many call; else each run launches its own
        # chunk graph
        self.group = bool(group)

    def _n_cap(self, cfg):
        return max(4096, int(cfg["pos"].shape[0] * self.cap_factor) + 256)

    def _admit(self, req, slot, now):
        torch = self.torch
        cfg = req["cfg"]
        n_cap = self._n_cap(cfg)
        with torch.cuda.stream(self.streams[slot]):
            run = Run(cfg["lattice"], cfg["vortex"], n_cap, device=self.device.index,
                      recon_cap=self.recon_cap, stream=self.streams[slot])
            try:
                run.write_fields(cfg["rho"], cfg["u"])
                run.seed(cfg["pos"], cfg["nxt"])
                if cfg["vortex"].get("alpha_z") is not None:
                    run.set_friction_profile(cfg["vortex"]["alpha_z"],
                                             cfg["vortex"]["alpha_p_z"])
            except Exception:
                run.close()
                run.ws = None
                raise
        return _Active(req=req, run=run, slot=slot, remaining=int(req["steps"]), admitted=now,
                       footprint=footprint(cfg, n_cap, self.recon_cap),
                       points_start=int(cfg["pos"].shape[0]))

    def _advance_group(self, group):
        """One vlb_step_many call advancing every run of ``group`` (idle, a
        whole chunk left) by one chunk, each on its own stream."""
        torch = self.torch
        step_many([a.run for a in group], self.chunk)
        for a in group:
            a.remaining -= self.chunk
            ev = torch.cuda.Event()
            ev.record(self.streams[a.slot])
            a.event = ev

    def _advance(self, a):
        torch = self.torch
        with torch.cuda.stream(self.streams[a.slot]):
            k = min(self.chunk, a.remaining)
            if k == self.chunk:
                a.run.step_graph(k)
            else:
                a.run.step(k)
            a.remaining -= k
            ev = torch.cuda.Event()
            ev.record(self.streams[a.slot])
            a.event = ev

    def _retire(self, a, now):
        torch = self.torch
        cfg = a.req["cfg"]
        lat = cfg["lattice"]
        res = Result(rid=a.req["rid"], arrival=a.req["arrival"], admitted=a.admitted, finished=0.0,
                     steps=int(a.req["steps"]), cells=lat["nx"] * lat["ny"] * lat["nz"],
                     points_start=a.points_start, points_end=0, footprint=a.footprint)
        with torch.cuda.stream(self.streams[a.slot]):
            try:
                a.run.sync()
                pos, nxt = a.run.read_filaments()
                res.points_end = pos.shape[0]
                res.pos, res.nxt = pos, nxt
                if self.keep_fields:
                    res.u = a.run.read_fields()[1]
            except VlbError as e:
                res.error = str(e)
            a.run.close()
            a.run.ws = None
        res.finished = time.perf_counter() - self.t0
        return res

    def _failed(self, req, msg, admitted=0.0):
        lat = req["cfg"]["lattice"]
        return Result(rid=req["rid"], arrival=req["arrival"], admitted=admitted,
                      finished=time.perf_counter() - self.t0, steps=int(req["steps"]),
                      cells=lat["nx"] * lat["ny"] * lat["nz"],
                      points_start=int(req["cfg"]["pos"].shape[0]), points_end=0, footprint=0,
                      error=msg or "failed")

    def serve(self, requests, time_scale=1.0):
        """Run the request loop until every request is served.  ``requests``
        are dicts with rid, arrival (s from the start), steps, cfg.
        ``time_scale`` stretches (> 1) or compresses arrival times."""
        pending = deque(sorted(requests, key=lambda r: r["arrival"]))
        active = []
        free_slots = list(range(self.max_slots))
        used = 0
        results = []
        self.t0 = time.perf_counter()
        fps = {}
        for r in list(pending):
            # a request that cannot be served (invalid descriptors, or more
            # memory than the whole budget) is answered with an error and
            # does not stop the others
            try:
                fps[r["rid"]] = footprint(r["cfg"], self._n_cap(r["cfg"]), self.recon_cap)
                if fps[r["rid"]] > self.budget:
                    raise ValueError(f"needs {fps[r['rid']]} bytes, over the budget")
            except (VlbError, ValueError) as e:
                pending.remove(r)
                results.append(self._failed(r, str(e)))
        while pending or active:
            now = time.perf_counter() - self.t0
            progressed = False
            # retire runs whose last chunk completed
            for a in list(active):
                if a.remaining == 0 and a.event is not None and a.event.query():
                    results.append(self._retire(a, now))
                    used -= a.footprint
                    free_slots.append(a.slot)
                    free_slots.sort()
                    active.remove(a)
                    progressed = True
            # admit arrived requests while a slot and memory are free
            while (pending and pending[0]["arrival"] * time_scale <= now and free_slots
                   and used + fps[pending[0]["rid"]] <= self.budget):
                req = pending.popleft()
                slot = free_slots.pop(0)
                progressed = True
                try:
                    a = self._admit(req, slot, now)
                except (VlbError, ValueError, RuntimeError) as e:
                    # e.g. seed points the library rejects: the slot is free again
                    results.append(self._failed(req, str(e), admitted=now))
                    free_slots.append(slot)
                    free_slots.sort()
                    continue
                used += a.footprint
                active.append(a)
            # keep every resident run busy
            idle = [a for a in active if a.remaining > 0 and (a.event is None or a.event.query())]
            if self.group:
                full = [a for a in idle if a.remaining >= self.chunk]
                if len(full) > 1:
                    self._advance_group(full)
                    progressed = True
                    idle = [a for a in idle if a not in full]
            for a in idle:
                self._advance(a)
                progressed = True
            if not progressed:
                time.sleep(2e-4)
        makespan = time.perf_counter() - self.t0
        results.sort(key=lambda r: r.rid)
        return results, makespan


def summarize(results, makespan):
    done = [r for r in results if not r.error]
    lat = np.array([r.latency for r in done] or [0.0])
    cells_steps = sum(r.cells * r.steps for r in done)
    return dict(
        requests=len(results),
        errors=sum(1 for r in results if r.error),
        error_list=[(r.rid, r.error) for r in results if r.error][:8],
        makespan_s=round(makespan, 3),
        latency_p50_s=round(float(np.percentile(lat, 50)), 4),
        latency_p99_s=round(float(np.percentile(lat, 99)), 4),
        aggregate_mlups=round(cells_steps / makespan / 1e6, 1),
        steps_total=int(sum(r.steps for r in done)),
    )
