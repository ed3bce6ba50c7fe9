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


def test_mix_equals_alone_bitwise():
    reqs = _requests()
    say("serve mix", [(r["rid"], r["steps"], r["cfg"]["pos"].shape[0]) for r in reqs])
    srv = serve.Server(budget_bytes=8 << 30, max_slots=3, chunk=4, keep_fields=True)
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
