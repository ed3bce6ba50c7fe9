"""Served form: requests of different sizes arrive over time, are admitted
by slot and HBM budget, stepped in graph-captured chunks on separate
streams, and every result equals the same request run alone, bit for bit."""

import numpy as np
import pytest

import workloads as wl
from tests._cases import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2108_04435_amd import serve  # noqa: E402


def _requests():
    reqs = wl.serving_requests(seed=7, n_requests=6, rate=200.0,
                               lattices=((24, 24, 24), (16, 16, 48)),
                               points=(150, 500), steps=(9, 26))
    return reqs


@pytest.mark.parametrize("group", [False, True])
def test_mix_equals_alone_bitwise(group):
    reqs = _requests()
    say("serve mix", group, [(r["rid"], r["steps"], r["cfg"]["pos"].shape[0]) for r in reqs])
    srv = serve.Server(budget_bytes=8 << 30, max_slots=3, chunk=4, keep_fields=True, group=group)
    mix, makespan = srv.serve(reqs)
    summary = serve.summarize(mix, makespan)
    say("summary", summary)
    assert summary["errors"] == 0
    assert [r.rid for r in mix] == [r["rid"] for r in reqs]
    for req, got in zip(reqs, mix):
        alone_req = dict(req, arrival=0.0)
        one = serve.Server(budget_bytes=8 << 30, max_slots=1, chunk=4, keep_fields=True)
        alone, _ = one.serve([alone_req])
        a = alone[0]
        say("request", req["rid"], "points", a.points_start, "->", a.points_end)
        assert a.error == "" and got.error == ""
        np.testing.assert_array_equal(got.nxt, a.nxt)
        np.testing.assert_array_equal(got.pos, a.pos)
        np.testing.assert_array_equal(got.u, a.u)


def test_budget_limits_residency():
    reqs = _requests()[:4]
    fp = max(serve.footprint(r["cfg"], max(4096, int(r["cfg"]["pos"].shape[0] * 6.0) + 256), 1 << 16)
             for r in reqs)
    say("budget", fp)
    srv = serve.Server(budget_bytes=fp + fp // 2, max_slots=4, chunk=4)
    res, makespan = srv.serve(reqs)
    assert all(r.error == "" for r in res)
    # with room for one run at a time, no two runs overlap in time
    spans = sorted((r.admitted, r.finished) for r in res)
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0 - 1e-3


def test_served_results_match_the_oracle_f64():
    """Three short FP64 requests served together: each final state equals
    the oracle's trajectory of the same request (links exact, positions and
    velocity field within 1e-10)."""
    from oracle import coupled, lbm, vfm
    from tests._cases import oracle_state, rel_l2

    reqs = wl.serving_requests(seed=11, n_requests=3, rate=500.0,
                               lattices=((16, 16, 16), (16, 16, 32)),
                               points=(100, 160), steps=(5, 9), precision="f64")
    say("serve vs oracle", [(r["rid"], r["steps"], r["cfg"]["pos"].shape[0]) for r in reqs])
    srv = serve.Server(budget_bytes=8 << 30, max_slots=3, chunk=4, keep_fields=True)
    res, _ = srv.serve(reqs)
    for req, got in zip(reqs, res):
        assert got.error == "", got.error
        lat, vp, st = oracle_state(req["cfg"])
        for _ in range(req["steps"]):
            st = coupled.coupled_step(st, lat, vp)
        say("request", req["rid"], "steps", req["steps"], "points", got.points_end)
        np.testing.assert_array_equal(got.nxt, st.nxt)
        assert np.abs(vfm.min_image(got.pos - st.pos, lat)).max() < 1e-10
        _, u_o = lbm.bare_velocity(st.f, lat)
        assert rel_l2(got.u, u_o) < 1e-10


def test_rejected_request_does_not_stop_the_loop():
    """A request whose seed the library rejects (a non-finite coordinate)
    and one larger than the whole budget are answered with errors; the
    others are served."""
    reqs = _requests()[:3]
    bad = dict(reqs[1], cfg=dict(reqs[1]["cfg"]))
    pos = bad["cfg"]["pos"].copy()
    pos[0, 0] = np.nan
    bad["cfg"]["pos"] = pos
    reqs[1] = bad
    srv = serve.Server(budget_bytes=8 << 30, max_slots=2, chunk=4)
    huge = dict(reqs[2], rid=99, cfg=dict(reqs[2]["cfg"],
                                          lattice=dict(reqs[2]["cfg"]["lattice"],
                                                       nx=1024, ny=1024, nz=1024)))
    res, makespan = srv.serve(reqs + [huge])
    by = {r.rid: r for r in res}
    assert by[reqs[0]["rid"]].error == "" and by[reqs[2]["rid"]].error == ""
    assert by[reqs[1]["rid"]].error != "" and by[99].error != ""
    s = serve.summarize(res, makespan)
    assert s["errors"] == 2 and s["requests"] == 4
