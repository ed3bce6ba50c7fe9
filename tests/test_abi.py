"""CPU checks of the C ABI: the library loads, exports every function that
include/vlb.h declares, the ctypes structures match the C layout, and the
host-side argument checks and footprint query work without a GPU."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_2108_04435_amd as vlb
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vlb.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vlb_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_symbols():
    assert _declared() == sorted(vlb.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = vlb.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", vlb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (vlb_[a-z_]+)", out))
    assert set(_declared()) <= exported


def test_struct_layout_matches_c():
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "vlb.h"
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("lat %zu\nvor %zu\n", sizeof(vlb_lattice_desc), sizeof(vlb_vortex_desc));
  O(vlb_lattice_desc, tau); O(vlb_lattice_desc, wall_axes); O(vlb_lattice_desc, plane_u);
  O(vlb_lattice_desc, body_force); O(vlb_vortex_desc, vs_applied); O(vlb_vortex_desc, remesh);
  O(vlb_vortex_desc, n_cap); O(vlb_vortex_desc, recon_cap); O(vlb_vortex_desc, wall_images);
  O(vlb_vortex_desc, ff_cell); O(vlb_vortex_desc, ff_levels); O(vlb_vortex_desc, ff_theta);
  O(vlb_vortex_desc, mass_balance_axis); O(vlb_vortex_desc, rk_stages);
  O(vlb_vortex_desc, vfm_substeps); O(vlb_vortex_desc, reserved2);
  printf("bs %zu\n", sizeof(vlb_bs_desc));
  O(vlb_bs_desc, wall_axes); O(vlb_bs_desc, precision); O(vlb_bs_desc, kappa);
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    vals = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    assert int(vals["lat"]) == ctypes.sizeof(vlb.LatticeDesc)
    assert int(vals["vor"]) == ctypes.sizeof(vlb.VortexDesc)
    assert int(vals["bs"]) == ctypes.sizeof(vlb.BsDesc)
    classes = {"vlb_lattice_desc": vlb.LatticeDesc, "vlb_vortex_desc": vlb.VortexDesc,
               "vlb_bs_desc": vlb.BsDesc}
    for key, v in vals.items():
        if "." in key:
            st, f = key.split(".")
            cls = classes[st]
            assert getattr(cls, f).offset == int(v), key


def _query(lat, vor, n_cap=100, recon_cap=1000):
    lib = vlb.load_library()
    ld = vlb.lattice_desc(lat)
    vd = vlb.vortex_desc(vor, n_cap, recon_cap)
    nb = ctypes.c_uint64(0)
    code = lib.vlb_query_footprint(ctypes.byref(ld), ctypes.byref(vd), ctypes.byref(nb))
    return code, nb.value, lib.vlb_last_error(None).decode()


def test_footprint_grows_with_lattice_and_precision():
    vor = wl.vortex_preset()
    sizes = {}
    for p in ("f64", "f32", "f16"):
        code, nb, _ = _query(wl.lattice_preset(32, 32, 32, precision=p), vor)
        assert code == vlb.VLB_OK
        sizes[p] = nb
    cells = 32 ** 3
    # populations dominate: 19 values per node of 8 / 4 / 2 bytes
    assert sizes["f64"] - sizes["f32"] >= 19 * cells * 4
    assert sizes["f32"] - sizes["f16"] >= 19 * cells * 2
    code, big, _ = _query(wl.lattice_preset(64, 64, 64, precision="f32"), vor)
    assert big > 7 * sizes["f32"]


@pytest.mark.parametrize("bad,msg", [
    (dict(tau=0.5), "tau"),
    (dict(nx=3), ">= 4"),
    (dict(precision="f64", walls=(False, False, True), plane_lo=True), "planes"),
])
def test_invalid_lattice_rejected(bad, msg):
    lat = wl.lattice_preset(16, 16, 16)
    lat.update(bad)
    code, _, err = _query(lat, wl.vortex_preset())
    assert code == vlb.VLB_EINVAL
    assert msg in err


@pytest.mark.parametrize("bad,msg", [
    (dict(dxi_min=1.0, dxi_max=0.9), "dxi_min"),
    (dict(min_loop_pts=2), "min_loop_pts"),
    (dict(kappa=0.0), "kappa"),
    (dict(force_model=2), "force_model"),
])
def test_invalid_vortex_rejected(bad, msg):
    vor = wl.vortex_preset()
    vor.update(bad)
    code, _, err = _query(wl.lattice_preset(16, 16, 16), vor)
    assert code == vlb.VLB_EINVAL
    assert msg in err


@pytest.mark.parametrize("lat_kw,vor_kw,msg", [
    (dict(precision="f64"), dict(ff_cell=4), "FP32"),
    (dict(precision="f32", walls=(False, False, True)), dict(ff_cell=4), "periodic"),
    (dict(precision="f32"), dict(ff_cell=4, wall_images=True), "wall images"),
    (dict(precision="f32"), dict(ff_cell=5), "divide"),
    (dict(precision="f32"), dict(ff_cell=16, ff_levels=2, ff_theta=0.5), "twice"),
    (dict(precision="f16"), dict(ff_cell=4, ff_theta=1.5), "theta"),
    (dict(precision="f32"), dict(ff_cell=-1), "ff_cell"),
])
def test_farfield_run_rejected(lat_kw, vor_kw, msg):
    """A run's far-field switch: FP32 or FP16, a periodic box, no wall
    images, and the stand-alone sum's cell rules."""
    lat = wl.lattice_preset(16, 16, 16, **lat_kw)
    code, _, err = _query(lat, wl.vortex_preset(**vor_kw))
    assert code == vlb.VLB_EINVAL
    assert msg in err


def test_farfield_run_footprint():
    """The far-field switch adds its workspace to a run's footprint."""
    lat = wl.lattice_preset(32, 32, 32, precision="f32")
    _, base, _ = _query(lat, wl.vortex_preset(), n_cap=4096)
    code, ff, _ = _query(lat, wl.vortex_preset(ff_cell=8, ff_levels=2, ff_theta=0.3), n_cap=4096)
    assert code == vlb.VLB_OK and ff > base + 4096 * 600


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mass_balance_needs_a_periodic_flow_axis(axis):
    walls = [True, True, True]
    walls[axis] = False
    lat = wl.lattice_preset(16, 16, 16, walls=tuple(walls))
    code, _, _ = _query(lat, wl.vortex_preset(mass_balance=True, mass_balance_axis=axis))
    assert code == vlb.VLB_OK
    walls = [False, False, False]
    walls[axis] = True
    lat = wl.lattice_preset(16, 16, 16, walls=tuple(walls))
    code, _, err = _query(lat, wl.vortex_preset(mass_balance=True, mass_balance_axis=axis))
    assert code == vlb.VLB_EINVAL and "mass balance" in err


@pytest.mark.parametrize("bad,msg", [
    (dict(mass_balance_axis=3), "mass_balance_axis"),
    (dict(mass_balance_axis=-1), "mass_balance_axis"),
    (dict(rk_stages=3), "rk_stages"),
    (dict(rk_stages=-4), "rk_stages"),
    (dict(vfm_substeps=65), "vfm_substeps"),
    (dict(vfm_substeps=-1), "vfm_substeps"),
])
def test_integration_fields_rejected(bad, msg):
    code, _, err = _query(wl.lattice_preset(16, 16, 16), wl.vortex_preset(**bad))
    assert code == vlb.VLB_EINVAL and msg in err


def test_zero_integration_fields_are_the_defaults():
    """rk_stages 0 and vfm_substeps 0 mean the classical method in one step."""
    lat = wl.lattice_preset(16, 16, 16)
    code0, b0, _ = _query(lat, wl.vortex_preset(rk_stages=0, vfm_substeps=0))
    code1, b1, _ = _query(lat, wl.vortex_preset())
    assert code0 == code1 == vlb.VLB_OK and b0 == b1


def test_zero_capacity_rejected():
    code, _, err = _query(wl.lattice_preset(16, 16, 16), wl.vortex_preset(), n_cap=0)
    assert code == vlb.VLB_EINVAL


def _bs_query(n, **kw):
    lib = vlb.load_library()
    args = dict(dims=(32, 32, 32), walls=(False, False, False), kappa=0.1, precision="f32")
    args.update(kw)
    d = vlb.bs_desc(**args)
    nb = ctypes.c_uint64(0)
    code = lib.vlb_biot_savart_workspace(ctypes.byref(d), n, ctypes.byref(nb))
    return code, nb.value, lib.vlb_last_error(None).decode()


def test_biot_savart_workspace_query():
    code, small, _ = _bs_query(1000)
    assert code == vlb.VLB_OK and small > 0
    code, big, _ = _bs_query(100000)
    assert code == vlb.VLB_OK and big > 50 * small
    code, f64, _ = _bs_query(1000, precision="f64")
    assert f64 > small
    assert _bs_query(0)[:2] == (vlb.VLB_OK, 0)


@pytest.mark.parametrize("kw,n,msg", [
    (dict(kappa=0.0), 10, "kappa"),
    (dict(dims=(0, 8, 8)), 10, "box"),
    (dict(), -1, "n_pts"),
    (dict(), (1 << 26) + 1, "n_pts"),
])
def test_biot_savart_invalid_rejected(kw, n, msg):
    code, _, err = _bs_query(n, **kw)
    assert code == vlb.VLB_EINVAL and msg in err


def test_biot_savart_null_pointers_rejected():
    lib = vlb.load_library()
    d = vlb.bs_desc((8, 8, 8))
    code = lib.vlb_biot_savart(ctypes.byref(d), 10, None, None, None, None, 0, None)
    assert code == vlb.VLB_EINVAL
    assert "null" in lib.vlb_last_error(None).decode()


def _ff_query(n, cell=8, theta=0.5, levels=1, **kw):
    lib = vlb.load_library()
    args = dict(dims=(32, 32, 32), walls=(False, False, False), kappa=0.1, precision="f32")
    args.update(kw)
    d = vlb.bs_desc(**args)
    p = vlb.FfParams(cell, levels, theta)
    nb = ctypes.c_uint64(0)
    code = lib.vlb_biot_savart_farfield_workspace(ctypes.byref(d), ctypes.byref(p), n,
                                                  ctypes.byref(nb))
    return code, nb.value, lib.vlb_last_error(None).decode()


def test_farfield_workspace_query():
    code, small, _ = _ff_query(1000)
    assert code == vlb.VLB_OK and small > 1000 * 600
    code, big, _ = _ff_query(100000)
    assert code == vlb.VLB_OK and big > 50 * small
    # finer cells need more (per-cell records and prefix rows), and so does
    # a second level
    assert _ff_query(1000, cell=2)[1] > small
    assert _ff_query(1000, levels=2)[1] > small
    assert _ff_query(0)[:2] == (vlb.VLB_OK, 0)
    assert ctypes.sizeof(vlb.FfParams) == 16


@pytest.mark.parametrize("kw,msg", [
    (dict(walls=(False, False, True)), "periodic"),
    (dict(precision="f64"), "FP32"),
    (dict(theta=0.0), "theta"),
    (dict(theta=1.0), "theta"),
    (dict(cell=5), "divide"),
    (dict(cell=0), "divide"),
    (dict(cell=1, dims=(256, 256, 128)), "2^22"),
    (dict(kappa=-1.0), "kappa"),
    (dict(levels=3), "levels"),
    (dict(levels=2, cell=8, dims=(32, 32, 24)), "twice"),
])
def test_farfield_invalid_rejected(kw, msg):
    code, _, err = _ff_query(100, **kw)
    assert code == vlb.VLB_EINVAL and msg in err


def test_farfield_null_pointers_rejected():
    lib = vlb.load_library()
    d = vlb.bs_desc((8, 8, 8), precision="f32")
    p = vlb.FfParams(4, 0, 0.5)
    code = lib.vlb_biot_savart_farfield(ctypes.byref(d), ctypes.byref(p), 10, None, None, None,
                                        None, 0, None)
    assert code == vlb.VLB_EINVAL
    assert "null" in lib.vlb_last_error(None).decode()
    code = lib.vlb_biot_savart_farfield(ctypes.byref(d), None, 10, None, None, None, None, 0,
                                        None)
    assert code == vlb.VLB_EINVAL
