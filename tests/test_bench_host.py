"""Host-side parts of bench.py that need no GPU: the argument handling and
step plan for the driver's argument set, and the oracle leg on a small
workload, with and without optional workload keys."""

import numpy as np
import pytest

import bench
import workloads as wl


def test_step_plan_covers_any_count():
    # graph chunks plus a direct remainder, for every split of 20 / 5 steps
    assert bench.step_plan(20, 10) == [("graph", 10), ("graph", 10)]
    assert bench.step_plan(5, 10) == [("direct", 5)]
    assert bench.step_plan(25, 10) == [("graph", 10), ("graph", 10), ("direct", 5)]
    assert bench.step_plan(0, 10) == []
    assert bench.step_plan(3, 0) == [("direct", 1)] * 3
    for n in range(0, 40):
        for g in (0, 2, 4, 10):
            assert sum(k for _, k in bench.step_plan(n, g)) == n
    with pytest.raises(ValueError):
        bench.step_plan(10, 3)


@pytest.mark.parametrize("argv", [
    ["--gpus", "1", "--steps", "20", "--warmup", "5"],
    ["--gpus", "1", "--steps", "20", "--warmup", "5", "--workload", "counterflow"],
    ["--gpus", "1", "--steps", "7", "--warmup", "3", "--workload", "ring32", "--graph", "4"],
])
def test_driver_arguments_parse(argv):
    a = bench.parse_args(argv)
    assert a.steps == int(argv[3]) and a.warmup == int(argv[5])
    plan = bench.step_plan(a.warmup, a.graph) + bench.step_plan(a.steps, a.graph)
    assert sum(k for _, k in plan) == a.steps + a.warmup


def test_default_workload_is_the_precision_form():
    a = bench.parse_args([])
    assert a.workload == "tangle" and a.head_precision == "f16"
    assert a.row_precisions == ["f32", "f64"] and a.graph == 0


def test_cpu_baseline_leg_runs_on_a_small_workload():
    cfg = wl.config_ring32()
    base, ref = bench.cpu_baseline(cfg, workers=2, per_worker=16, single=8)
    assert base["kind"] == "oracle" and base["value"] > 0 and base["cores"] == 2
    assert base["single_thread_value"] > 0
    # every point whose force reaches the crop is a target
    o, w = ref["origin"], ref["width"]
    pos = cfg["pos"]
    box = np.all((pos > np.array(o) - 1.0) & (pos < np.array(o) + w), axis=1)
    assert set(np.nonzero(box)[0]) <= set(ref["targets"].tolist())
    assert ref["u_crop"].shape == (3, w - 2, w - 2, w - 2)


def test_cpu_baseline_sample_matches_full_oracle():
    """The sampled first-stage values and the crop update equal the oracle's
    full-state computation at those targets / nodes."""
    from oracle import coupled, lbm, vfm
    import tests._cases as cases

    cfg = wl.config_ring32()
    base, ref = bench.cpu_baseline(cfg, workers=1, per_worker=64, single=4)
    lat, vp, st = cases.oracle_state(cfg)
    _, ub = lbm.bare_velocity(st.f, lat)
    Vs = lbm.mass_balance_superflow(st.f, lat, vp.rho_s_over_rho_n) if vp.mass_balance else None
    full = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, Vs, lat, vp, want_force=True)
    t = ref["targets"]
    for k in ("vs", "vn", "sdot", "force"):
        np.testing.assert_allclose(ref[k], full[k][t], rtol=0, atol=1e-14)
    F = vfm.spread(full["force"], st.pos, lat)
    f1 = lbm.lbm_step(st.f, F, lat)
    _, u1 = lbm.bare_velocity(f1, lat)
    o, w = ref["origin"], ref["width"]
    crop = u1[:, o[2] + 1:o[2] + w - 1, o[1] + 1:o[1] + w - 1, o[0] + 1:o[0] + w - 1]
    np.testing.assert_allclose(ref["u_crop"], crop, rtol=0, atol=1e-15)


def test_cpu_baseline_with_friction_profile_keys():
    """Workload dicts may carry the optional friction profiles."""
    cfg = wl.config_ring32()
    nz = cfg["lattice"]["nz"]
    cfg["vortex"] = dict(cfg["vortex"], alpha_z=(0.2,) * nz, alpha_p_z=(0.01,) * nz)
    base, _ = bench.cpu_baseline(cfg, workers=1, per_worker=8, single=4)
    assert base["value"] > 0


def test_cpu_baseline_sample_with_wall_images():
    """The oracle leg on a walled channel with the image term: the sampled
    first-stage values equal the oracle's full-state computation."""
    from oracle import lbm, vfm
    import tests._cases as cases

    cfg = cases.small_channel(precision="f64", seed=71, n_rings=8, nxy=24, nz=32)
    cfg["vortex"] = dict(cfg["vortex"], wall_images=True)
    base, ref = bench.cpu_baseline(cfg, workers=1, per_worker=40, single=4)
    lat, vp, st = cases.oracle_state(cfg)
    assert vp.wall_images
    _, ub = lbm.bare_velocity(st.f, lat)
    Vs = lbm.mass_balance_superflow(st.f, lat, vp.rho_s_over_rho_n)
    full = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, Vs, lat, vp, want_force=True)
    t = ref["targets"]
    assert t.size > 0
    for k in ("vs", "vn", "sdot", "force"):
        np.testing.assert_allclose(ref[k], full[k][t], rtol=0, atol=1e-14)


def test_cpu_baseline_sample_with_wall_bound_lines():
    """The oracle leg on the closed channel (open lines bound to the end
    walls, wall images on): the sampled first-stage values equal the
    oracle's full-state computation."""
    from oracle import lbm, vfm
    import tests._cases as cases

    cfg = wl.config_closed_channel(nxy=16, nz=24)
    base, ref = bench.cpu_baseline(cfg, workers=1, per_worker=40, single=4)
    lat, vp, st = cases.oracle_state(cfg)
    assert vp.wall_images and not vp.mass_balance
    _, ub = lbm.bare_velocity(st.f, lat)
    full = vfm.line_velocity(st.pos, st.nxt, st.prv, ub, None, lat, vp, want_force=True)
    t = ref["targets"]
    assert t.size > 0 and base["value"] > 0
    for k in ("vs", "vn", "sdot", "force"):
        np.testing.assert_allclose(ref[k], full[k][t], rtol=0, atol=1e-14)


def test_accuracy_crops():
    """The heater channel is checked on a 64^3 crop centred at (64, 64, 256);
    the other workloads on a centred 32^3 crop (at most half the smallest
    extent)."""
    heater = wl.config_heater("f32", n_rings=4)
    assert bench.sample_window(heater, heater["crop_width"]) == ((32, 32, 224), 64)
    tangle = dict(lattice=wl.lattice_preset(256, 256, 256))
    assert bench.sample_window(tangle) == ((112, 112, 112), 32)
    small = dict(lattice=wl.lattice_preset(32, 32, 32))
    assert bench.sample_window(small) == ((8, 8, 8), 16)


def test_point_capacity():
    """1.4 n0 (+ 256) by default, the factor on request."""
    assert bench.point_capacity(104175) == int(104175 * 1.4) + 256
    assert bench.point_capacity(104175, 2.5) == int(104175 * 2.5) + 256
    assert bench.parse_args([]).capacity_factor == 1.4
