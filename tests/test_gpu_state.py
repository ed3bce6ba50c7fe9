"""Checkpoint / resume (vlb_read_state, vlb_write_state with the filament
read and seed) and several runs advanced together (vlb_step_many,
vlb_graph_create_many): every result bit for bit the one of plain
per-run stepping."""

import numpy as np
import pytest

import workloads as wl
from tests._cases import duct, say, small_channel, small_periodic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_04435_amd as vlb  # noqa: E402

D3Q19_W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _snapshot(run):
    buf, step = run.read_state()
    pos, nxt = run.read_filaments()
    return buf.cpu().numpy(), pos, nxt, step


def _assert_same(a, b):
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
    assert a[3] == b[3]


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
@pytest.mark.parametrize("case", ["channel", "periodic", "duct_x_midpoint"])
def test_checkpoint_resume_bitwise(case, precision):
    if case == "channel":
        cfg = small_channel(precision=precision, reconnect=True, seed=51)
    elif case == "duct_x_midpoint":
        # flow and mass balance along x; the midpoint rule in two substeps
        cfg = duct(0, precision=precision, seed=53)
        cfg["vortex"].update(rk_stages=2, vfm_substeps=2, reconnect=True)
    else:
        cfg = small_periodic(precision=precision, seed=52)
    k, m = 5, 6   # odd k: the checkpoint is taken in the swapped AA layout
    say("checkpoint", case, precision, k, m)
    a = vlb.run_from_config(cfg)
    a.step(k)
    a.sync()
    buf, step = a.read_state()
    pos, nxt = a.read_filaments()
    assert step == k
    b = vlb.Run(cfg["lattice"], cfg["vortex"], a.n_cap)
    b.write_state(buf, step)
    b.seed(pos, nxt)
    a.step(m)
    b.step(m)
    a.sync()
    b.sync()
    _assert_same(_snapshot(a), _snapshot(b))
    # and back into the same run: rewinding to step k replays the same steps
    s1 = _snapshot(a)
    a.write_state(buf, step)
    a.seed(pos, nxt)
    a.step(m)
    a.sync()
    _assert_same(_snapshot(a), s1)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_state_is_the_natural_layout(precision):
    """The checkpoint decodes to the populations vlb_read_populations
    reports, at both AA parities."""
    cfg = small_periodic(precision=precision, seed=53)
    run = vlb.run_from_config(cfg)
    dt = {"f64": np.float64, "f32": np.float32, "f16": np.float16}[precision]
    for _ in range(2):
        run.step(1)
        run.sync()
        raw = run.read_state()[0].cpu().numpy().view(dt).reshape((19,) + run.shape)
        if precision == "f16":
            dev = raw.astype(np.float32) * np.float32(1.0 / 1024.0)
        else:
            dev = raw
        f = D3Q19_W[:, None, None, None] + dev.astype(np.float64)
        np.testing.assert_array_equal(f, run.read_populations())
    run.close()


def _runs(streams):
    cfgs = [small_channel(precision="f32", seed=54, reconnect=True),
            small_periodic(precision="f64", seed=55),
            small_channel(precision="f16", seed=56, nxy=20, nz=24),
            wl.config_ring32(precision="f32")]
    runs = []
    for c, s in zip(cfgs, streams):
        with torch.cuda.stream(s):
            r = vlb.Run(c["lattice"], c["vortex"], max(64, int(c["pos"].shape[0] * 1.5) + 64),
                        stream=s)
            r.write_fields(c["rho"], c["u"])
            r.seed(c["pos"], c["nxt"])
            runs.append(r)
    return runs


def test_step_many_equals_single_runs():
    streams = [torch.cuda.Stream() for _ in range(4)]
    together = _runs(streams)
    alone = _runs(streams)
    say("step_many", [r.n_points() for r in together])
    vlb.step_many(together, 7)
    for r in alone:
        r.step(7)
    for r in together + alone:
        r.sync()
    for a, b in zip(together, alone):
        _assert_same(_snapshot(a), _snapshot(b))
    for r in together + alone:
        r.close()


@pytest.mark.skip(reason="multi-run graph capture was taken out: it crashed the host process "
                         "inside the capture call, cause not found")
def test_graph_many_equals_single_runs():
    streams = [torch.cuda.Stream() for _ in range(4)]
    together = _runs(streams)
    alone = _runs(streams)
    g = vlb.GraphMany(together, 4)
    say("graph_many")
    g.launch()
    g.launch()
    # direct steps between launches, on one run's own stream
    together[1].step(2)
    for r in alone:
        r.step(8)
    alone[1].step(2)
    g.launch()
    for r in alone:
        r.step(4)
    for r in together + alone:
        r.sync()
    for a, b in zip(together, alone):
        assert a.get_step() == b.get_step()
        _assert_same(_snapshot(a), _snapshot(b))
    # an odd number of direct steps on one run: the graph refuses
    together[2].step(1)
    with pytest.raises(vlb.VlbError) as ei:
        g.launch()
    assert ei.value.code == vlb.VLB_ESTATE
    g.close()
    for r in together + alone:
        r.close()
