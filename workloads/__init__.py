"""Seeded synthetic inputs shared by the GPU library's tests/bench and the
oracle.  Holds no arithmetic of the method itself: only initial filament
geometry (rings), initial density/velocity fields, and plain-data workload
presets.  Both sides turn (rho, u) into populations themselves.

Generators use numpy ``Generator(PCG64(seed))``.
"""

import math

import numpy as np

# --------------------------------------------------------------- filaments


def ring(center, radius, normal, n_pts, phase=0.5):
    """Closed ring of ``n_pts`` points at angles 2 pi (j + phase) / n_pts,
    ordered so that the ring's self-induced motion is along +normal.
    Returns (pos (n, 3) float64, nxt (n,) int64)."""
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)
    # e1, e2 with e1 x e2 = n
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(a, n)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    th = 2.0 * np.pi * (np.arange(n_pts) + phase) / n_pts
    pos = (np.asarray(center, dtype=np.float64)[None, :]
           + radius * (np.cos(th)[:, None] * e1[None, :] + np.sin(th)[:, None] * e2[None, :]))
    nxt = (np.arange(n_pts) + 1) % n_pts
    return pos, nxt.astype(np.int64)


def wall_line(foot, axis, n_axis, n_pts, reverse=False, amp=0.0, turns=0.0, phase=0.0):
    """Open vortex line bound to the two walls of a closed axis: ``n_pts``
    points evenly spaced along ``axis`` from the wall plane -1/2 to
    n_axis - 1/2 (both ends exactly on the planes), at transverse position
    ``foot`` (the two other coordinates, in axis order), displaced
    transversally by a helix of amplitude ``amp`` and ``turns`` turns.
    ``reverse`` runs it from the upper wall to the lower one (opposite
    circulation).  The last point links to itself.
    Returns (pos (n, 3) float64, nxt (n,) int64)."""
    t = np.linspace(0.0, 1.0, n_pts)
    if reverse:
        t = t[::-1]
    others = [a for a in range(3) if a != axis]
    pos = np.zeros((n_pts, 3))
    pos[:, axis] = -0.5 + t * float(n_axis)
    pos[0, axis] = n_axis - 0.5 if reverse else -0.5
    pos[-1, axis] = -0.5 if reverse else n_axis - 0.5
    ang = 2.0 * np.pi * (turns * t + phase)
    pos[:, others[0]] = foot[0] + amp * np.cos(ang)
    pos[:, others[1]] = foot[1] + amp * np.sin(ang)
    nxt = np.arange(1, n_pts + 1)
    nxt[-1] = n_pts - 1
    return pos, nxt.astype(np.int64)


def concat_loops(loops):
    """Concatenate (pos, nxt) loops into one point set with global links."""
    if not loops:
        return np.zeros((0, 3)), np.zeros(0, dtype=np.int64)
    pos, nxt, off = [], [], 0
    for p, n in loops:
        pos.append(p)
        nxt.append(n + off)
        off += p.shape[0]
    return np.concatenate(pos, axis=0), np.concatenate(nxt).astype(np.int64)


def random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _too_close(grid, cell, pts, dims, walls, min_sep):
    """Any already placed point within min_sep of one of ``pts``?"""
    for p in pts:
        base = np.floor(p / cell).astype(int)
        for off in np.ndindex(3, 3, 3):
            key = []
            for a in range(3):
                k = base[a] + off[a] - 1
                n = int(math.ceil(dims[a] / cell))
                if not walls[a]:
                    k %= n
                key.append(k)
            for q in grid.get(tuple(key), ()):
                d = q - p
                for a in range(3):
                    if not walls[a]:
                        d[a] -= dims[a] * round(d[a] / dims[a])
                if d @ d < min_sep * min_sep:
                    return True
    return False


def random_rings(seed, n_rings, r_lo, r_hi, dims, walls, dxi_max, margin=1.0, min_sep=0.0,
                 max_tries=200):
    """``n_rings`` rings with radii U[r_lo, r_hi], normals uniform on the
    sphere, centres uniform (kept a radius + margin away from walls);
    ring spacing 2 pi R / ceil(2 pi R / dxi_max) <= dxi_max.  With
    ``min_sep`` > 0 a ring is redrawn while one of its points lies closer
    than min_sep to a point of an earlier ring (no near-intersections at
    the start)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    loops = []
    grid = {}
    cell = max(min_sep, 1e-9)
    for _ in range(n_rings):
        for _try in range(max_tries):
            R = rng.uniform(r_lo, r_hi)
            c = np.empty(3)
            for a in range(3):
                if walls[a]:
                    lo, hi = R + margin - 0.5, dims[a] - 0.5 - R - margin
                    c[a] = rng.uniform(lo, hi) if hi > lo else 0.5 * (dims[a] - 1)
                else:
                    c[a] = rng.uniform(0.0, dims[a])
            nrm = random_unit(rng)
            npts = int(math.ceil(2.0 * math.pi * R / dxi_max))
            lp = ring(c, R, nrm, npts, phase=rng.uniform(0.0, 1.0))
            if min_sep <= 0:
                break
            wrapped = lp[0].copy()
            for a in range(3):
                if not walls[a]:
                    wrapped[:, a] %= dims[a]
            if not _too_close(grid, cell, wrapped, dims, walls, min_sep):
                break
        loops.append(lp)
        if min_sep > 0:
            for p in wrapped:
                key = tuple(int(k) for k in np.floor(p / cell))
                grid.setdefault(key, []).append(p)
    return concat_loops(loops)


# ------------------------------------------------------------ lattice init


def velocity_field(seed, dims, u0, sigma):
    """rho = 1, u = u0 + N(0, sigma^2) per component per node.
    Returns rho (nz, ny, nx), u (3, nz, ny, nx), float64."""
    nx, ny, nz = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.empty((3, nz, ny, nx))
    for a in range(3):
        u[a] = u0[a]
    if sigma > 0:
        u += rng.normal(0.0, sigma, size=u.shape)
    rho = np.ones((nz, ny, nx))
    return rho, u


# ------------------------------------------------------------- presets
# Plain data.  Lattice keys: nx, ny, nz, tau, walls (per axis), plane_lo,
# plane_hi, plane_u, body_force, precision ("f64" | "f32" | "f16").
# Vortex keys mirror the oracle's VortexParams.

VORTEX_DEFAULTS = dict(
    kappa=0.1, core_a=1e-3, core_c=0.5, alpha=0.2, alpha_p=0.01,
    rho_s_over_rho_n=1.35, dxi_min=0.70, dxi_max=0.95, reconnect_dist=0.95,
    remesh=True, reconnect=False, min_loop_pts=5, coupling=True,
    mass_balance=False, mass_balance_axis=2, vs_applied=(0.0, 0.0, 0.0),
    rk_stages=4, vfm_substeps=1,
)


def lattice_preset(nx, ny, nz, tau=0.8, walls=(False, False, False), plane_lo=False,
                   plane_hi=False, plane_u=(0.0, 0.0, 0.0), body_force=(0.0, 0.0, 0.0),
                   precision="f64"):
    return dict(nx=nx, ny=ny, nz=nz, tau=tau, walls=tuple(walls), plane_lo=plane_lo,
                plane_hi=plane_hi, plane_u=tuple(plane_u), body_force=tuple(body_force),
                precision=precision)


def vortex_preset(**kw):
    v = dict(VORTEX_DEFAULTS)
    v.update(kw)
    return v


def config_ring32(precision="f64"):
    """Plain small case: 32^3 periodic, tau 0.8, u = (0,0,0.01) + N(0,1e-4^2),
    one ring R = 8 of 64 points (half-spacing phase), 100 steps."""
    lat = lattice_preset(32, 32, 32, tau=0.8, precision=precision)
    vor = vortex_preset()
    rho, u = velocity_field(1, (32, 32, 32), (0.0, 0.0, 0.01), 1e-4)
    pos, nxt = ring((16.0, 16.0, 16.0), 8.0, (0.0, 0.0, 1.0), 64, phase=0.5)
    return dict(name="ring32", lattice=lat, vortex=vor, rho=rho, u=u, pos=pos, nxt=nxt,
                steps=100)


# Body force for a mean duct velocity of 0.02 in a 64x64 square duct,
# tau = 0.8 (nu = 0.1): G = 28.45 nu U / W^2 (laminar square-duct relation).
COUNTERFLOW_G = 28.45 * 0.1 * 0.02 / (64.0 * 64.0)


def config_counterflow(precision="f32", n_rings=200, nz=256, nxy=64, seed=2):
    """Counterflow channel: 64x64x256, bounce-back walls on x and y, periodic
    z, Guo body force along z for a mean v_n of about 0.02, 200 rings with
    R ~ U[4, 12] placed at least 2 apart, remeshing spacing 1.0
    (dxi_min = 0.737 keeps the paper's 0.70/0.95 ratio), reconnection (part
    of the filament model), mass balance on z, 1000 steps."""
    lat = lattice_preset(nxy, nxy, nz, tau=0.8, walls=(True, True, False),
                         body_force=(0.0, 0.0, COUNTERFLOW_G * (64.0 / nxy) ** 2),
                         precision=precision)
    vor = vortex_preset(dxi_max=1.0, dxi_min=0.70 / 0.95, reconnect_dist=1.0,
                        reconnect=True, mass_balance=True)
    rho, u = velocity_field(seed, (nxy, nxy, nz), (0.0, 0.0, 0.02), 0.0)
    pos, nxt = random_rings(seed, n_rings, 4.0, 12.0, (nxy, nxy, nz), (True, True, False), 1.0,
                            min_sep=2.0)
    return dict(name="counterflow_64x64x256", lattice=lat, vortex=vor, rho=rho, u=u,
                pos=pos, nxt=nxt, steps=1000)


def config_heater(precision="f32", n_rings=1500, nxy=128, nz=512, seed=3):
    """Closed channel with heater: 128x128x512, walls on x and y, velocity
    planes z = 0 / z = nz-1 at v_n = 0.03 z, 1500 rings R ~ U[3, 7.6],
    reconnection on, mass balance on z, 2000 steps."""
    lat = lattice_preset(nxy, nxy, nz, tau=0.8, walls=(True, True, False), plane_lo=True,
                         plane_hi=True, plane_u=(0.0, 0.0, 0.03), precision=precision)
    vor = vortex_preset(reconnect=True, mass_balance=True)
    rho, u = velocity_field(seed, (nxy, nxy, nz), (0.0, 0.0, 0.03), 0.0)
    pos, nxt = random_rings(seed, n_rings, 3.0, 7.6, (nxy, nxy, nz), (True, True, False), 0.95,
                            min_sep=1.5)
    # the accuracy sample's lattice crop: 64^3 centred at (64, 64, 256)
    return dict(name="heater_128x128x512", lattice=lat, vortex=vor, rho=rho, u=u,
                pos=pos, nxt=nxt, steps=2000, crop_width=64)


def config_closed_channel(precision="f64", nxy=48, nz=128, seed=6):
    """Closed channel with lines bound to its end walls (the paper's Sec. IV
    initial condition, synthetic stand-in): walls on z (the streaming axis),
    x and y periodic; normal fluid at rest with N(0, 1e-4^2) noise (the
    heater efflux through the end walls is not among the lattice's
    boundaries); four lines from wall to wall along z (two each way, feet on
    a square of side nxy/2, helical displacement 0.5 with 3 turns) and two
    rings R = nxy/8 beside them; wall images and reconnection on (mass
    balance off: with the fluid at rest it is zero)."""
    rng = np.random.default_rng(seed)
    lat = lattice_preset(nxy, nxy, nz, tau=0.8, walls=(False, False, True), precision=precision)
    vor = vortex_preset(reconnect=True, wall_images=True)
    rho, u = velocity_field(seed, (nxy, nxy, nz), (0.0, 0.0, 0.0), 1e-4)
    # axial spacing <= 0.85: with the helix the segments stay below 0.95
    n_pts = int(math.ceil(nz / 0.85)) + 1
    q = nxy / 4.0
    feet = ((q, q), (3 * q, q), (3 * q, 3 * q), (q, 3 * q))
    loops = [wall_line(f, 2, nz, n_pts, reverse=(i % 2 == 1), amp=0.5, turns=3.0,
                       phase=float(rng.uniform())) for i, f in enumerate(feet)]
    R = nxy / 8.0
    m = int(math.ceil(2.0 * np.pi * R / 0.9))
    loops.append(ring((2 * q, q, nz / 4.0), R, (0.0, 0.0, 1.0), m))
    loops.append(ring((2 * q, 3 * q, 3 * nz / 4.0), R, (0.0, 0.0, -1.0), m))
    pos, nxt = concat_loops(loops)
    return dict(name=f"closed_channel_{nxy}x{nxy}x{nz}", lattice=lat, vortex=vor, rho=rho, u=u,
                pos=pos, nxt=nxt, steps=100)


def config_tangle(precision="f16", n=256, n_rings=2000, seed=4):
    """Precision form: 256^3 periodic, u = 0.02 z + N(0, 1e-4^2), random tangle
    of 2000 rings R ~ U[4, 12] (about 1e5 points), mass balance on z."""
    lat = lattice_preset(n, n, n, tau=0.8, precision=precision)
    vor = vortex_preset(mass_balance=True)
    rho, u = velocity_field(seed, (n, n, n), (0.0, 0.0, 0.02), 1e-4)
    pos, nxt = random_rings(seed, n_rings, 4.0, 12.0, (n, n, n), (False, False, False), 0.95,
                            min_sep=1.5)
    return dict(name="tangle_256", lattice=lat, vortex=vor, rho=rho, u=u, pos=pos, nxt=nxt,
                steps=100)


# ------------------------------------------------------------- serving

SERVE_LATTICES = ((32, 32, 32), (64, 64, 64), (64, 64, 256), (128, 128, 256))


def serving_requests(seed=5, n_requests=64, rate=2.0, lattices=SERVE_LATTICES,
                     points=(1000, 20000), steps=(500, 2000), alpha=(0.1, 0.3),
                     alpha_p=(0.0, 0.02), vn=(0.01, 0.04), precision="f32"):
    """Request stream of counterflow runs: exponential inter-arrival times
    (mean 1/rate s); lattice uniform from ``lattices`` (cubes periodic with
    a uniform initial v_n along z, elongated ones with walls on x, y and a
    Guo body force for a mean v_n); filament points U[points] from rings
    R ~ U[4, min(12, min(dims)/4)]; alpha, alpha', v_n uniform; steps
    U{steps}.  Returns a list of dicts (arrival, steps, cfg)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        dims = lattices[rng.integers(len(lattices))]
        target = int(rng.integers(points[0], points[1] + 1))
        a = rng.uniform(*alpha)
        ap = rng.uniform(*alpha_p)
        v = rng.uniform(*vn)
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        cube = dims[0] == dims[2]
        walls = (False, False, False) if cube else (True, True, False)
        W = float(dims[0])
        body = (0.0, 0.0, 0.0) if cube else (0.0, 0.0, 28.45 * 0.1 * v / (W * W))
        lat = lattice_preset(*dims, tau=0.8, walls=walls, body_force=body, precision=precision)
        vor = vortex_preset(alpha=a, alpha_p=ap, reconnect=True, mass_balance=True)
        r_hi = min(12.0, min(dims) / 4.0)
        r_mean = 0.5 * (4.0 + r_hi)
        per_ring = 2.0 * math.pi * r_mean / 0.95
        n_rings = max(1, int(round(target / per_ring)))
        rho, u = velocity_field(seed * 1000 + rid, dims, (0.0, 0.0, v), 0.0)
        pos, nxt = random_rings(seed * 1000 + rid, n_rings, 4.0, r_hi, dims, walls, 0.95)
        out.append(dict(rid=rid, arrival=t, steps=nsteps,
                        cfg=dict(name=f"req{rid}", lattice=lat, vortex=vor, rho=rho, u=u,
                                 pos=pos, nxt=nxt, steps=nsteps)))
    return out
