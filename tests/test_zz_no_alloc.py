"""The allocation-free Biot-Savart entry point (vlb_biot_savart_noalloc):
through the C ABI, two calls in a row (the second with fewer points, so
that stale scratch from the first would show) against vlb_biot_savart on a
caller workspace, bit for bit, in FP32 and FP64; sizes above the limit are
refused."""

import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import coupled, vfm
from oracle.lbm import Lattice
from tests._cases import rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_04435_amd as vlb  # noqa: E402


def _lib():
    return vlb.load_library()


def _noalloc(lib, d, pos, nxt):
    p = torch.as_tensor(np.ascontiguousarray(pos)).cuda()
    q = torch.as_tensor(np.ascontiguousarray(nxt, dtype=np.int32)).cuda()
    v = torch.full((pos.shape[0], 3), float("nan"), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    code = lib.vlb_biot_savart_noalloc(ctypes.byref(d), pos.shape[0],
                                       ctypes.c_void_p(p.data_ptr()),
                                       ctypes.c_void_p(q.data_ptr()),
                                       ctypes.c_void_p(v.data_ptr()),
                                       ctypes.c_void_p(s.cuda_stream))
    assert code == vlb.VLB_OK, lib.vlb_last_error(None)
    return v.cpu().numpy()


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("box", ["periodic", "channel"])
def test_noalloc_equals_workspace_call(box, precision):
    lib = _lib()
    dims, walls = {"periodic": ((64, 64, 64), (False,) * 3),
                   "channel": ((40, 40, 72), (True, True, False))}[box]
    big = wl.random_rings(41, 260, 3.0, 10.0, dims, walls, 0.95)
    small = wl.random_rings(42, 17, 2.0, 5.0, dims, walls, 0.95)
    lat = Lattice(*dims, walls=walls)
    d = vlb.bs_desc(dims, walls, kappa=0.1, precision=precision)
    for pos, nxt in (big, small):
        pos = vfm.wrap_positions(pos, lat)
        say("noalloc", box, precision, pos.shape[0], "points")
        assert pos.shape[0] <= 16384
        got = _noalloc(lib, d, pos, nxt)
        want = vlb.biot_savart(pos, nxt, dims, walls, kappa=0.1, precision=precision)
        np.testing.assert_array_equal(got, want)
    # and against the oracle, on the last (small) input
    ref = vfm.biot_savart_nonlocal(pos, nxt, coupled.prev_from_next(nxt), lat, 0.1)
    assert rel_l2(got, ref) <= (1e-10 if precision == "f64" else 1e-5)


def test_noalloc_refuses_sizes_above_the_limit():
    lib = _lib()
    d = vlb.bs_desc((64, 64, 64))
    code = lib.vlb_biot_savart_noalloc(ctypes.byref(d), 16385, None, None, None, None)
    assert code == vlb.VLB_EINVAL
    assert b"16384" in lib.vlb_last_error(None)
    assert lib.vlb_biot_savart_noalloc(ctypes.byref(d), 0, None, None, None, None) == vlb.VLB_OK
