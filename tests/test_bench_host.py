"""Host-side part of bench.py that needs no GPU: the oracle baseline leg
on a tiny workload, with and without optional workload keys."""

import bench
import workloads as wl


def test_cpu_baseline_leg_runs_on_a_tiny_workload():
    cfg = wl.config_ring32()
    out = bench.cpu_baseline(cfg, n_evals=1)
    assert out["kind"] == "oracle" and out["value"] > 0 and out["cores"] >= 1


def test_cpu_baseline_with_friction_profile_keys():
    """Workload dicts may carry the optional friction profiles."""
    cfg = wl.config_ring32()
    nz = cfg["lattice"]["nz"]
    cfg["vortex"] = dict(cfg["vortex"], alpha_z=(0.2,) * nz, alpha_p_z=(0.01,) * nz)
    out = bench.cpu_baseline(cfg, n_evals=1)
    assert out["value"] > 0
