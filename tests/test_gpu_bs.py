"""GPU parity of the stand-alone Biot-Savart sum (vlb_biot_savart) against
the oracle's non-local sum (Sec. II.A, Eq. Biot-Savart): periodic and
walled boxes, several tiles with ragged tails, FP64 and FP32, the empty and
degenerate inputs, and two calls in a row on one workspace."""

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

TOL = {"f64": 1e-10, "f32": 1e-5, "f16": 1e-5}


def _case(seed, n_rings, dims, walls, r=(2.0, 6.0)):
    pos, nxt = wl.random_rings(seed, n_rings, r[0], r[1], dims, walls, 0.95)
    lat = Lattice(*dims, walls=walls)
    return vfm.wrap_positions(pos, lat), nxt, lat


def _oracle(pos, nxt, lat, kappa):
    return vfm.biot_savart_nonlocal(pos, nxt, coupled.prev_from_next(nxt), lat, kappa)


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
@pytest.mark.parametrize("box", ["periodic", "channel", "closed", "odd"])
def test_standalone_matches_oracle(box, precision):
    dims, walls = {"periodic": ((32, 32, 32), (False,) * 3),
                   "channel": ((24, 24, 40), (True, True, False)),
                   "closed": ((20, 28, 24), (True, True, True)),
                   "odd": ((30, 22, 26), (False,) * 3)}[box]
    pos, nxt, lat = _case(31, 40, dims, walls)
    say("standalone", box, precision, pos.shape[0], "points")
    v = vlb.biot_savart(pos, nxt, dims, walls, kappa=0.1, precision=precision)
    ref = _oracle(pos, nxt, lat, 0.1)
    err = rel_l2(v, ref)
    say("rel l2", err)
    assert err <= TOL[precision]


def test_standalone_unwrapped_periodic_positions():
    """On a periodic axis the grid wraps: positions shifted by whole box
    lengths give the same velocities."""
    dims = (32, 32, 32)
    pos, nxt, lat = _case(33, 12, dims, (False,) * 3)
    shift = np.array([32.0, -64.0, 96.0])
    v0 = vlb.biot_savart(pos, nxt, dims, kappa=0.1, precision="f64")
    v1 = vlb.biot_savart(pos + shift, nxt, dims, kappa=0.1, precision="f64")
    np.testing.assert_allclose(v1, v0, rtol=0, atol=1e-12)


def test_standalone_degenerate_inputs():
    # no points; a single loop of 3 (every segment touches every target)
    assert vlb.biot_savart(np.zeros((0, 3)), np.zeros(0, dtype=np.int64), (8, 8, 8)).shape == (0, 3)
    tri = np.array([[1.0, 1.0, 1.0], [2.0, 1.0, 1.0], [1.0, 2.0, 1.0]])
    v = vlb.biot_savart(tri, np.array([1, 2, 0]), (8, 8, 8), precision="f64")
    lat = Lattice(8, 8, 8)
    np.testing.assert_allclose(v, _oracle(tri, np.array([1, 2, 0]), lat, 0.1), atol=1e-15)


def test_standalone_many_points_sampled():
    """About 4e4 points (many chunks and tiles): sampled targets against the
    oracle."""
    dims = (128, 128, 128)
    pos, nxt, lat = _case(35, 700, dims, (False,) * 3, r=(4.0, 12.0))
    n = pos.shape[0]
    say("standalone large", n)
    for precision in ("f64", "f32"):
        v = vlb.biot_savart(pos, nxt, dims, kappa=0.1, precision=precision)
        t = np.random.default_rng(3).choice(n, 48, replace=False)
        ref = vfm.biot_savart_nonlocal(pos, nxt, coupled.prev_from_next(nxt), lat, 0.1, targets=t)
        err = rel_l2(v[t], ref)
        say(precision, err)
        assert err <= TOL[precision]


def test_standalone_two_calls_share_a_workspace():
    """Two calls in a row on one workspace, the second with fewer points:
    each result equals a call on a fresh workspace, bit for bit."""
    lib = vlb.load_library()
    dims = (32, 32, 32)
    a_pos, a_nxt, _ = _case(36, 30, dims, (False,) * 3)
    b_pos, b_nxt, _ = _case(37, 9, dims, (False,) * 3)
    d = vlb.bs_desc(dims, precision="f32")
    nb = ctypes.c_uint64(0)
    assert lib.vlb_biot_savart_workspace(ctypes.byref(d), a_pos.shape[0], ctypes.byref(nb)) == 0
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    outs = []
    for pos, nxt in ((a_pos, a_nxt), (b_pos, b_nxt)):
        p = torch.as_tensor(pos).cuda()
        q = torch.as_tensor(nxt.astype(np.int32)).cuda()
        v = torch.empty((pos.shape[0], 3), dtype=torch.float64, device="cuda")
        s = torch.cuda.current_stream()
        assert lib.vlb_biot_savart(ctypes.byref(d), pos.shape[0], ctypes.c_void_p(p.data_ptr()),
                                   ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), nb,
                                   ctypes.c_void_p(s.cuda_stream)) == 0
        outs.append(v.cpu().numpy())
    np.testing.assert_array_equal(outs[0], vlb.biot_savart(a_pos, a_nxt, dims, precision="f32"))
    np.testing.assert_array_equal(outs[1], vlb.biot_savart(b_pos, b_nxt, dims, precision="f32"))
