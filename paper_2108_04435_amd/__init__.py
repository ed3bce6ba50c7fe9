"""Coupled vortex-filament / lattice-Boltzmann step for superfluid 4He on
AMD gfx950 (S. Inui and M. Tsubota, arXiv:2108.04435, Sec. II).

This package is a thin ctypes binding over the HIP library ``libvlb.so``
(C ABI in ``include/vlb.h``).  It only marshals arguments: device memory
(the run's workspace and field buffers) comes from PyTorch tensors, the
stream is PyTorch's current stream, and every step of the method runs in
the library's kernels.  There is no CPU fallback: if the library is not
built, importing ``Run`` works but creating one raises.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvlb.so")

VLB_OK = 0
VLB_EINVAL = -1
VLB_ENOSPACE = -2
VLB_EDEVICE = -3
VLB_ESTATE = -4
VLB_ECAPACITY = -5
VLB_ENUMERIC = -6

PRECISION = {"f64": 0, "f32": 1, "f16": 2}

# Exported symbols, in the order of include/vlb.h.
SYMBOLS = [
    "vlb_query_footprint", "vlb_create_lattice", "vlb_write_fields", "vlb_seed_vortices",
    "vlb_step", "vlb_step_many", "vlb_sync", "vlb_read_fields", "vlb_read_populations",
    "vlb_read_state", "vlb_write_state", "vlb_read_force",
    "vlb_read_filaments", "vlb_eval_line_velocity", "vlb_apply_topology",
    "vlb_set_friction_profile", "vlb_line_length",
    "vlb_flow_stats", "vlb_read_vorticity", "vlb_vorticity_cylindrical", "vlb_get_step",
    "vlb_set_timing", "vlb_get_timing", "vlb_time_kernel", "vlb_get_work", "vlb_graph_create",
    "vlb_graph_launch", "vlb_graph_destroy", "vlb_biot_savart_workspace", "vlb_biot_savart",
    "vlb_biot_savart_noalloc", "vlb_biot_savart_farfield_workspace", "vlb_biot_savart_farfield",
    "vlb_destroy", "vlb_last_error",
]


class LatticeDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("wall_axes", ctypes.c_uint32),
        ("plane_lo", ctypes.c_int32), ("plane_hi", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("plane_u", ctypes.c_double * 3),
        ("body_force", ctypes.c_double * 3),
    ]


class VortexDesc(ctypes.Structure):
    _fields_ = [
        ("kappa", ctypes.c_double), ("core_a", ctypes.c_double), ("core_c", ctypes.c_double),
        ("alpha", ctypes.c_double), ("alpha_p", ctypes.c_double),
        ("rho_s_over_rho_n", ctypes.c_double),
        ("dxi_min", ctypes.c_double), ("dxi_max", ctypes.c_double),
        ("reconnect_dist", ctypes.c_double),
        ("vs_applied", ctypes.c_double * 3),
        ("remesh", ctypes.c_int32), ("reconnect", ctypes.c_int32),
        ("min_loop_pts", ctypes.c_int32), ("coupling", ctypes.c_int32),
        ("mass_balance", ctypes.c_int32), ("force_model", ctypes.c_int32),
        ("wall_images", ctypes.c_int32), ("mass_balance_axis", ctypes.c_int32),
        ("n_cap", ctypes.c_int64), ("recon_cap", ctypes.c_int64),
        ("ff_cell", ctypes.c_int32), ("ff_levels", ctypes.c_int32),
        ("ff_theta", ctypes.c_double),
        ("rk_stages", ctypes.c_int32), ("vfm_substeps", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
    ]


class BsDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("wall_axes", ctypes.c_uint32), ("precision", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("kappa", ctypes.c_double),
    ]


class FfParams(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("theta", ctypes.c_double)]


class VlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vlb error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path=None):
    """Load libvlb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: build it with `python -m paper_2108_04435_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    dp = ctypes.POINTER(ctypes.c_double)
    lib.vlb_query_footprint.argtypes = [ctypes.POINTER(LatticeDesc), ctypes.POINTER(VortexDesc),
                                        ctypes.POINTER(ctypes.c_uint64)]
    lib.vlb_create_lattice.argtypes = [ctypes.POINTER(LatticeDesc), ctypes.POINTER(VortexDesc),
                                       vp, ctypes.c_uint64, vp, ctypes.POINTER(vp)]
    lib.vlb_write_fields.argtypes = [vp, vp, vp]
    lib.vlb_seed_vortices.argtypes = [vp, i64, vp, vp]
    lib.vlb_step.argtypes = [vp, i64]
    lib.vlb_step_many.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, i64]
    lib.vlb_read_state.argtypes = [vp, vp]
    lib.vlb_write_state.argtypes = [vp, vp, i64]
    lib.vlb_sync.argtypes = [vp]
    lib.vlb_read_fields.argtypes = [vp, vp, vp]
    lib.vlb_read_populations.argtypes = [vp, vp]
    lib.vlb_read_force.argtypes = [vp, vp]
    lib.vlb_set_friction_profile.argtypes = [vp, vp, vp]
    lib.vlb_line_length.argtypes = [vp, vp, vp]
    lib.vlb_flow_stats.argtypes = [vp, vp, vp, vp, vp]
    lib.vlb_read_vorticity.argtypes = [vp, vp, vp]
    lib.vlb_vorticity_cylindrical.argtypes = [vp, vp, vp, vp, vp]
    lib.vlb_read_filaments.argtypes = [vp, i64, vp, vp, ctypes.POINTER(i64)]
    lib.vlb_eval_line_velocity.argtypes = [vp, vp, vp, vp, vp]
    lib.vlb_apply_topology.argtypes = [vp, vp]
    lib.vlb_get_step.argtypes = [vp, ctypes.POINTER(i64)]
    lib.vlb_set_timing.argtypes = [vp, ctypes.c_int32]
    lib.vlb_get_timing.argtypes = [vp, ctypes.c_int32, dp, ctypes.POINTER(i64)]
    lib.vlb_time_kernel.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, dp]
    lib.vlb_get_work.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.vlb_graph_create.argtypes = [vp, i64, ctypes.POINTER(vp)]
    lib.vlb_graph_launch.argtypes = [vp]
    lib.vlb_graph_destroy.argtypes = [vp]
    lib.vlb_biot_savart_workspace.argtypes = [ctypes.POINTER(BsDesc), i64,
                                              ctypes.POINTER(ctypes.c_uint64)]
    lib.vlb_biot_savart.argtypes = [ctypes.POINTER(BsDesc), i64, vp, vp, vp, vp,
                                    ctypes.c_uint64, vp]
    lib.vlb_biot_savart_noalloc.argtypes = [ctypes.POINTER(BsDesc), i64, vp, vp, vp, vp]
    lib.vlb_biot_savart_farfield_workspace.argtypes = [
        ctypes.POINTER(BsDesc), ctypes.POINTER(FfParams), i64, ctypes.POINTER(ctypes.c_uint64)]
    lib.vlb_biot_savart_farfield.argtypes = [ctypes.POINTER(BsDesc), ctypes.POINTER(FfParams),
                                             i64, vp, vp, vp, vp, ctypes.c_uint64, vp]
    lib.vlb_destroy.argtypes = [vp]
    lib.vlb_last_error.argtypes = [vp]
    lib.vlb_last_error.restype = ctypes.c_char_p
    for name in SYMBOLS[:-1]:
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def lattice_desc(lat: dict) -> LatticeDesc:
    d = LatticeDesc()
    d.nx, d.ny, d.nz = int(lat["nx"]), int(lat["ny"]), int(lat["nz"])
    d.precision = PRECISION[lat.get("precision", "f64")]
    d.tau = float(lat.get("tau", 0.8))
    walls = lat.get("walls", (False, False, False))
    d.wall_axes = sum(1 << a for a in range(3) if walls[a])
    d.plane_lo = int(bool(lat.get("plane_lo", False)))
    d.plane_hi = int(bool(lat.get("plane_hi", False)))
    for a in range(3):
        d.plane_u[a] = float(lat.get("plane_u", (0, 0, 0))[a])
        d.body_force[a] = float(lat.get("body_force", (0, 0, 0))[a])
    return d


def vortex_desc(vor: dict, n_cap: int, recon_cap: int = 1 << 16) -> VortexDesc:
    d = VortexDesc()
    for k in ("kappa", "core_a", "core_c", "alpha", "alpha_p", "rho_s_over_rho_n", "dxi_min",
              "dxi_max", "reconnect_dist"):
        setattr(d, k, float(vor[k]))
    for a in range(3):
        d.vs_applied[a] = float(vor.get("vs_applied", (0, 0, 0))[a])
    d.remesh = int(bool(vor.get("remesh", True)))
    d.reconnect = int(bool(vor.get("reconnect", False)))
    d.min_loop_pts = int(vor.get("min_loop_pts", 5))
    d.coupling = int(bool(vor.get("coupling", True)))
    d.mass_balance = int(bool(vor.get("mass_balance", False)))
    d.force_model = int(vor.get("force_model", 0))
    d.wall_images = int(bool(vor.get("wall_images", False)))
    d.mass_balance_axis = int(vor.get("mass_balance_axis", 2))
    d.n_cap = int(n_cap)
    d.recon_cap = int(recon_cap)
    d.ff_cell = int(vor.get("ff_cell", 0))
    d.ff_levels = int(vor.get("ff_levels", 1))
    d.ff_theta = float(vor.get("ff_theta", 0.25))
    d.rk_stages = int(vor.get("rk_stages", 4))
    d.vfm_substeps = int(vor.get("vfm_substeps", 1))
    d.reserved2 = 0
    return d


class Run:
    """One coupled simulation resident on a GPU.

    ``lattice`` / ``vortex`` are plain dicts (keys as in LatticeDesc /
    VortexDesc; ``walls`` is a per-axis bool triple, ``precision`` one of
    "f64", "f32", "f16")."""

    def __init__(self, lattice: dict, vortex: dict, n_cap: int, device=0, recon_cap=1 << 16,
                 stream=None):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.lat = dict(lattice)
        self.ld = lattice_desc(lattice)
        self.vd = vortex_desc(vortex, n_cap, recon_cap)
        self.shape = (self.ld.nz, self.ld.ny, self.ld.nx)
        self.cells = self.ld.nx * self.ld.ny * self.ld.nz
        nbytes = ctypes.c_uint64(0)
        self._check(self.lib.vlb_query_footprint(ctypes.byref(self.ld), ctypes.byref(self.vd),
                                                 ctypes.byref(nbytes)), None)
        self.footprint = int(nbytes.value)
        self.ws = torch.empty(self.footprint + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        self._check(self.lib.vlb_create_lattice(ctypes.byref(self.ld), ctypes.byref(self.vd),
                                                ctypes.c_void_p(self._ws_ptr),
                                                ctypes.c_uint64(self.footprint),
                                                ctypes.c_void_p(self.stream.cuda_stream),
                                                ctypes.byref(h)), None)
        self.h = h
        self.n_cap = int(n_cap)

    # ----------------------------------------------------------- plumbing
    def _check(self, code, h="self"):
        if code != VLB_OK:
            hh = self.h if h == "self" else None
            msg = self.lib.vlb_last_error(hh)
            raise VlbError(code, msg.decode() if msg else "")

    @staticmethod
    def _ptr(t):
        return ctypes.c_void_p(t.data_ptr())

    def _dev(self, arr, shape):
        t = self.torch.as_tensor(np.ascontiguousarray(arr, dtype=np.float64)).reshape(shape)
        return t.to(self.device).contiguous()

    def close(self):
        for g in list(getattr(self, "_graphs", {}).values()):
            self.lib.vlb_graph_destroy(g)
        self._graphs = {}
        if getattr(self, "h", None):
            self.lib.vlb_destroy(self.h)
            self.h = None

    def graph(self, n_steps):
        """Executable graph of n_steps (even) coupled steps captured at the
        run's current step parity (a graph replays only at the parity it was
        captured at), cached per (size, parity)."""
        if not hasattr(self, "_graphs"):
            self._graphs = {}
        key = (int(n_steps), self.get_step() % 2)
        if key not in self._graphs:
            g = ctypes.c_void_p()
            self._check(self.lib.vlb_graph_create(self.h, int(n_steps), ctypes.byref(g)))
            self._graphs[key] = g
        return self._graphs[key]

    def step_graph(self, n_steps):
        """Advance n_steps (even) coupled steps with one graph launch."""
        self._check(self.lib.vlb_graph_launch(self.graph(n_steps)))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- state
    def write_fields(self, rho, u):
        r = self._dev(rho, self.shape)
        v = self._dev(u, (3,) + self.shape)
        self._check(self.lib.vlb_write_fields(self.h, ctypes.c_void_p(r.data_ptr()),
                                              ctypes.c_void_p(v.data_ptr())))

    def seed(self, pos, nxt):
        p = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        n = np.ascontiguousarray(nxt, dtype=np.int32).reshape(-1)
        self._check(self.lib.vlb_seed_vortices(self.h, p.shape[0], p.ctypes.data_as(ctypes.c_void_p),
                                               n.ctypes.data_as(ctypes.c_void_p)))

    def step(self, n=1):
        self._check(self.lib.vlb_step(self.h, int(n)))

    def sync(self):
        self._check(self.lib.vlb_sync(self.h))

    def read_fields(self):
        torch = self.torch
        rho = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.vlb_read_fields(self.h, ctypes.c_void_p(rho.data_ptr()),
                                             ctypes.c_void_p(u.data_ptr())))
        return rho.cpu().numpy(), u.cpu().numpy()

    def read_populations(self):
        f = self.torch.empty((19,) + self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.vlb_read_populations(self.h, ctypes.c_void_p(f.data_ptr())))
        return f.cpu().numpy()

    def state_bytes(self):
        return 19 * self.cells * {0: 8, 1: 4, 2: 2}[self.ld.precision]

    def read_state(self):
        """(stored populations as a device uint8 tensor, step): the run's
        checkpoint together with read_filaments."""
        buf = self.torch.empty(self.state_bytes(), dtype=self.torch.uint8, device=self.device)
        self._check(self.lib.vlb_read_state(self.h, self._ptr(buf)))
        return buf, self.get_step()

    def write_state(self, buf, step):
        if buf.numel() * buf.element_size() != self.state_bytes():
            raise ValueError("state of another size")
        buf = buf.to(self.device).contiguous()
        self._check(self.lib.vlb_write_state(self.h, self._ptr(buf), int(step)))

    def read_force(self):
        F = self.torch.empty((3,) + self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.vlb_read_force(self.h, ctypes.c_void_p(F.data_ptr())))
        return F.cpu().numpy()

    def set_friction_profile(self, alpha_z=None, alpha_p_z=None):
        """alpha(z), alpha'(z) slice profiles (nz each), or None to restore
        the constants."""
        if alpha_z is None and alpha_p_z is None:
            self._check(self.lib.vlb_set_friction_profile(self.h, None, None))
            return
        a = np.ascontiguousarray(alpha_z, dtype=np.float64).reshape(-1)
        b = np.ascontiguousarray(alpha_p_z, dtype=np.float64).reshape(-1)
        if a.shape[0] != self.ld.nz or b.shape[0] != self.ld.nz:
            raise ValueError("friction profiles need nz values each")
        self._check(self.lib.vlb_set_friction_profile(self.h, a.ctypes.data_as(ctypes.c_void_p),
                                                      b.ctypes.data_as(ctypes.c_void_p)))

    def line_length(self):
        """(total line length, length per z slab)."""
        tot = ctypes.c_double(0.0)
        slabs = np.zeros(self.ld.nz)
        self._check(self.lib.vlb_line_length(self.h, ctypes.byref(tot),
                                             slabs.ctypes.data_as(ctypes.c_void_p)))
        return float(tot.value), slabs

    def flow_stats(self):
        """Velocity statistics: slice_mean, slice_rms ((nz, 3)), mean, rms ((3,))."""
        nz = self.ld.nz
        sm, sr, m, r = np.zeros((nz, 3)), np.zeros((nz, 3)), np.zeros(3), np.zeros(3)
        self._check(self.lib.vlb_flow_stats(self.h, *(a.ctypes.data_as(ctypes.c_void_p)
                                                      for a in (sm, sr, m, r))))
        return dict(slice_mean=sm, slice_rms=sr, mean=m, rms=r)

    def read_vorticity(self):
        """(bare velocity, vorticity), each (3, nz, ny, nx)."""
        torch = self.torch
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        w = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.vlb_read_vorticity(self.h, ctypes.c_void_p(u.data_ptr()),
                                                ctypes.c_void_p(w.data_ptr())))
        return u.cpu().numpy(), w.cpu().numpy()

    def vorticity_cylindrical(self, point, direction):
        """(bare velocity, vorticity, cylindrical components of the vorticity
        about the axis through point along direction), each (3, nz, ny, nx)."""
        torch = self.torch
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        w = torch.empty_like(u)
        c = torch.empty_like(u)
        p = np.ascontiguousarray(point, dtype=np.float64)
        d = np.ascontiguousarray(direction, dtype=np.float64)
        self._check(self.lib.vlb_read_vorticity(self.h, ctypes.c_void_p(u.data_ptr()),
                                                ctypes.c_void_p(w.data_ptr())))
        self._check(self.lib.vlb_vorticity_cylindrical(
            self.h, p.ctypes.data_as(ctypes.c_void_p), d.ctypes.data_as(ctypes.c_void_p),
            ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(c.data_ptr())))
        return u.cpu().numpy(), w.cpu().numpy(), c.cpu().numpy()

    def n_points(self):
        n = ctypes.c_int64(0)
        code = self.lib.vlb_read_filaments(self.h, 0, None, None, ctypes.byref(n))
        if code not in (VLB_OK, VLB_ENOSPACE):
            self._check(code)
        return int(n.value)

    def read_filaments(self):
        n = self.n_points()
        pos = np.zeros((n, 3))
        nxt = np.zeros(n, dtype=np.int32)
        m = ctypes.c_int64(0)
        self._check(self.lib.vlb_read_filaments(self.h, n, pos.ctypes.data_as(ctypes.c_void_p),
                                                nxt.ctypes.data_as(ctypes.c_void_p), ctypes.byref(m)))
        return pos, nxt.astype(np.int64)

    def eval_line_velocity(self):
        n = self.n_points()
        out = {k: np.zeros((n, 3)) for k in ("vs", "vn", "sdot", "force")}
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        self._check(self.lib.vlb_eval_line_velocity(self.h, ptr(out["vs"]), ptr(out["vn"]),
                                                    ptr(out["sdot"]), ptr(out["force"])))
        return out

    def apply_topology(self):
        st = np.zeros(4, dtype=np.int64)
        self._check(self.lib.vlb_apply_topology(self.h, st.ctypes.data_as(ctypes.c_void_p)))
        return dict(deleted=int(st[0]), inserted=int(st[1]), reconnections=int(st[2]),
                    loops_removed_pts=int(st[3]))

    def get_step(self):
        s = ctypes.c_int64(0)
        self._check(self.lib.vlb_get_step(self.h, ctypes.byref(s)))
        return int(s.value)

    def set_timing(self, on=True, reserve=0):
        self._check(self.lib.vlb_set_timing(self.h, (max(1, int(reserve)) if on else 0)))

    def timing(self, cls):
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        self._check(self.lib.vlb_get_timing(self.h, int(cls), ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def time_kernel(self, cls, reps=20):
        ms = ctypes.c_double(0)
        self._check(self.lib.vlb_time_kernel(self.h, int(cls), int(reps), ctypes.byref(ms)))
        return float(ms.value)

    def work(self):
        a = ctypes.c_int64(0)
        b = ctypes.c_int64(0)
        self._check(self.lib.vlb_get_work(self.h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)


def _handles(runs):
    arr = (ctypes.c_void_p * len(runs))(*[r.h for r in runs])
    return arr


def step_many(runs, n_steps):
    """Advance several runs by n_steps each (vlb_step_many)."""
    lib = load_library()
    _raise(lib, lib.vlb_step_many(_handles(runs), len(runs), int(n_steps)))


def bs_desc(dims, walls=(False, False, False), kappa=0.1, precision="f64") -> BsDesc:
    d = BsDesc()
    d.nx, d.ny, d.nz = (int(x) for x in dims)
    d.wall_axes = sum(1 << a for a in range(3) if walls[a])
    d.precision = PRECISION[precision]
    d.reserved = 0
    d.kappa = float(kappa)
    return d


def _raise(lib, code):
    if code != VLB_OK:
        msg = lib.vlb_last_error(None)
        raise VlbError(code, msg.decode() if msg else "")


def biot_savart(xyz, nxt, dims, walls=(False, False, False), kappa=0.1, precision="f64",
                device=0):
    """Non-local Biot-Savart velocity of filaments (vlb_biot_savart): closed
    loops, or open lines whose last point links to itself; ``xyz`` (n, 3)
    positions, ``nxt`` (n,) successor links; returns (n, 3)
    velocities as a host array.  Device buffers and the workspace are torch
    tensors; the work runs on torch's current stream."""
    import torch

    lib = load_library()
    dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
    d = bs_desc(dims, walls, kappa, precision)
    p = torch.as_tensor(np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)).to(dev)
    q = torch.as_tensor(np.ascontiguousarray(nxt, dtype=np.int32).reshape(-1)).to(dev)
    n = p.shape[0]
    nb = ctypes.c_uint64(0)
    _raise(lib, lib.vlb_biot_savart_workspace(ctypes.byref(d), n, ctypes.byref(nb)))
    ws = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=dev)
    wp = (ws.data_ptr() + 255) // 256 * 256
    v = torch.empty((n, 3), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    _raise(lib, lib.vlb_biot_savart(ctypes.byref(d), n, ctypes.c_void_p(p.data_ptr()),
                                    ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                    ctypes.c_void_p(wp), ctypes.c_uint64(int(nb.value)),
                                    ctypes.c_void_p(stream.cuda_stream)))
    out = v.cpu().numpy()   # synchronises the stream
    del ws
    return out


class FarField:
    """Far-field approximation of the stand-alone Biot-Savart sum
    (vlb_biot_savart_farfield) for n points in a periodic box ``dims``:
    cells of edge ``cell`` (``levels`` 2: cells of edge 2 cell first),
    opening parameter ``theta``; FP32.  The workspace is allocated once;
    ``run`` enqueues one sum on torch's current stream from device tensors
    (positions (n, 3) float64, links (n,) int32) into ``v`` ((n, 3)
    float64)."""

    def __init__(self, dims, n, cell, theta, kappa=0.1, device=0, levels=1):
        import torch

        self.lib = load_library()
        self.dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.desc = bs_desc(dims, (False, False, False), kappa, "f32")
        self.par = FfParams(int(cell), int(levels), float(theta))
        self.n = int(n)
        nb = ctypes.c_uint64(0)
        _raise(self.lib, self.lib.vlb_biot_savart_farfield_workspace(
            ctypes.byref(self.desc), ctypes.byref(self.par), self.n, ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        self._wp = (self._ws.data_ptr() + 255) // 256 * 256

    def run(self, p, q, v):
        import torch

        for t, shape, dt in ((p, (self.n, 3), torch.float64), (q, (self.n,), torch.int32),
                             (v, (self.n, 3), torch.float64)):
            if tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous() \
                    or t.device != self.dev:
                raise ValueError(f"expected a contiguous {dt} tensor of shape {shape} on {self.dev}")
        stream = torch.cuda.current_stream(self.dev)
        _raise(self.lib, self.lib.vlb_biot_savart_farfield(
            ctypes.byref(self.desc), ctypes.byref(self.par), self.n, ctypes.c_void_p(p.data_ptr()),
            ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(self._wp),
            ctypes.c_uint64(self.ws_bytes), ctypes.c_void_p(stream.cuda_stream)))


def biot_savart_farfield(xyz, nxt, dims, cell, theta, kappa=0.1, device=0, levels=1):
    """Far-field approximation of the non-local velocity (FarField) of
    filaments ``xyz`` (n, 3), ``nxt`` (n,) in a periodic box; returns (n, 3)
    velocities as a host array."""
    import torch

    n = int(np.asarray(nxt).size)
    ff = FarField(dims, max(n, 1), cell, theta, kappa, device, levels)
    if n == 0:
        return np.zeros((0, 3))
    p = torch.as_tensor(np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)).to(ff.dev)
    q = torch.as_tensor(np.ascontiguousarray(nxt, dtype=np.int32).reshape(-1)).to(ff.dev)
    v = torch.empty((n, 3), dtype=torch.float64, device=ff.dev)
    ff.run(p, q, v)
    return v.cpu().numpy()   # synchronises the stream


def run_from_config(cfg: dict, n_cap=None, device=0, recon_cap=1 << 16):
    """Create a run from a workload dict (lattice, vortex, rho, u, pos, nxt)."""
    n = cfg["pos"].shape[0]
    cap = n_cap if n_cap is not None else max(64, int(n * 1.5) + 64)
    r = Run(cfg["lattice"], cfg["vortex"], cap, device=device, recon_cap=recon_cap)
    r.write_fields(cfg["rho"], cfg["u"])
    if n:
        r.seed(cfg["pos"], cfg["nxt"])
    if cfg["vortex"].get("alpha_z") is not None:
        r.set_friction_profile(cfg["vortex"]["alpha_z"], cfg["vortex"]["alpha_p_z"])
    return r
