"""Vortex filament model and its coupling to the lattice, plain FP64.

Paper Sec. II.A (filaments, Biot-Savart, LIA, Schwarz equation of motion)
and Sec. II.B (mutual-friction force, two-point delta interpolation and
spreading); Sec. III.C (mass-balance superflow).

Filament state: ``pos`` (N, 3) float64 in lattice units (x, y, z), and two
int arrays ``nxt`` / ``prv`` linking every point to its successor and
predecessor (the arc-length parametrisation of Sec. II.A).  Segment k runs
from point k to point nxt[k].  A filament is a closed loop or an open line
bound to the walls (Sec. IV: vortex lines bound to the solid walls; reading
F1b): the last point of an open line links to itself (nxt[e] = e, so its
segment has zero length) and the first point is its own predecessor
(prv[s] = s); both lie on a wall plane of a closed axis.
"""

from dataclasses import dataclass

import numpy as np

from .lbm import Lattice


@dataclass
class VortexParams:
    kappa: float = 0.1          # circulation quantum in lattice units (reading R6)
    core_a: float = 1e-3        # core radius a (Sec. III.A)
    core_c: float = 0.5         # LIA core constant (reading R3)
    alpha: float = 0.2          # mutual friction alpha  (Sec. II.A, Eq. E of M)
    alpha_p: float = 0.01       # mutual friction alpha' (Sec. II.A, Eq. E of M)
    rho_s_over_rho_n: float = 1.35   # rho_s / rho_n (reading R7)
    dxi_min: float = 0.70       # Sec. III: 0.70 dx
    dxi_max: float = 0.95       # Sec. III: 0.95 dx
    reconnect_dist: float = 0.95  # Sec. III.B: within dxi_max (reading R11)
    remesh: bool = True
    reconnect: bool = False
    min_loop_pts: int = 5
    coupling: bool = True       # False: prescribed normal fluid, no back-reaction
    mass_balance: bool = False  # superflow V_s from Eq. (mass cons)
    mass_balance_axis: int = 2  # its flow axis (0, 1, 2 = x, y, z; periodic)
    vs_applied: tuple = (0.0, 0.0, 0.0)  # externally applied v_s,a (Sec. II.A)
    # mutual-friction coefficients varying along z (Sec. IV: temperature
    # dependent alpha, alpha' over the channel; reading D4): nz slice values
    # each, or None for the constants above
    alpha_z: tuple = None
    alpha_p_z: tuple = None
    # reaction on the normal fluid: 0 = Magnus balance (reading R1),
    # 1 = the printed Eq. (f) taken literally (for ablation)
    force_model: int = 0
    # superfluid boundary velocity v_s,b from image vortices in the wall
    # planes (reading F1); False: v_s,b = 0 (reading R13)
    wall_images: bool = False
    # non-local sum: 0 = the direct sum over all segments (Sec. II.A); > 0 =
    # its cell-multipole approximation with cells of this edge (reading F2,
    # oracle/farfield.py), ff_levels levels, opening parameter ff_theta
    ff_cell: int = 0
    ff_levels: int = 1
    ff_theta: float = 0.25
    # time integration of ds/dt over one lattice step (reading R6): an
    # explicit Runge-Kutta method of rk_stages stages (1 forward Euler, 2
    # the midpoint rule, 4 the classical method) applied vfm_substeps times
    # with steps of 1/vfm_substeps
    rk_stages: int = 4
    vfm_substeps: int = 1


# ---------------------------------------------------------------- geometry

def wrap_positions(pos, lat: Lattice):
    """Periodic axes: wrap into [0, L).  Wall axes: a point beyond the wall
    plane at -1/2 or n-1/2 is mirrored back inside (reading R13)."""
    p = np.array(pos, dtype=np.float64, copy=True)
    for a, n in enumerate(lat.dims):
        x = p[:, a]
        if lat.walls[a]:
            lo, hi = -0.5, n - 0.5
            x = np.where(x < lo, 2.0 * lo - x, x)
            x = np.where(x > hi, 2.0 * hi - x, x)
        else:
            L = float(n)
            x = np.where(x < 0.0, x + L, x)
            x = np.where(x >= L, x - L, x)
            x = np.where(x >= L, 0.0, x)  # x + L rounded up to L
        p[:, a] = x
    return p


def min_image(d, lat: Lattice):
    """Nearest periodic image of a separation vector (rows of ``d``): on a
    periodic axis of length L a component with |d| > L/2 is shifted by -+L;
    |d| == L/2 is left alone."""
    d = np.array(d, dtype=np.float64, copy=True)
    for a, n in enumerate(lat.dims):
        if lat.walls[a]:
            continue
        L = float(n)
        x = d[..., a]
        x = np.where(x > 0.5 * L, x - L, x)
        x = np.where(x < -0.5 * L, x + L, x)
        d[..., a] = x
    return d


def norm(v):
    return np.sqrt(v[..., 0] * v[..., 0] + v[..., 1] * v[..., 1] + v[..., 2] * v[..., 2])


def cross(a, b):
    return np.stack(
        [
            a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
            a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
            a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0],
        ],
        axis=-1,
    )


def dot(a, b):
    return a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1] + a[..., 2] * b[..., 2]


def end_walls(pos, nxt, prv, lat: Lattice):
    """The wall an open line's end point is bound to (reading F1b): for every
    point, the first closed axis a (x, y, z order) whose wall plane -1/2
    (side 1) or n - 1/2 (side 2) the point lies on exactly, if the point is
    an end (nxt[k] = k or prv[k] = k); axis -1 otherwise.  Returns
    (axis, side) int arrays."""
    N = pos.shape[0]
    axis = np.full(N, -1, dtype=np.int64)
    side = np.zeros(N, dtype=np.int64)
    ks = np.arange(N)
    end = (np.asarray(nxt) == ks) | (np.asarray(prv) == ks)
    for a in (2, 1, 0):  # lowest axis wins
        if not lat.walls[a]:
            continue
        for sd, w in ((1, -0.5), (2, lat.dims[a] - 0.5)):
            on = end & (pos[:, a] == w)
            axis = np.where(on, a, axis)
            side = np.where(on, sd, side)
    return axis, side


def reflect_except(v, axis):
    """v with every component but the one along ``axis`` negated (per row;
    rows with axis -1 unchanged): the mirror image, in a plane normal to
    that axis, of a vector that crosses the plane."""
    v = np.array(v, dtype=np.float64, copy=True)
    for a in range(3):
        m = (axis >= 0) & (axis != a)
        v[m, a] = -v[m, a]
    return v


def geometry(pos, nxt, prv, lat: Lattice):
    """Local geometry at every point (Sec. II.A; formulas are reading R5).

    d+ = s_{next} - s, d- = s - s_{prev} (nearest image), l+- = |d+-|;
    non-uniform three-point derivatives along the arc length
      s'  = (l-^2 d+ + l+^2 d-) / (l+ l- (l+ + l-)),   then normalised,
      s'' = 2 (l- d+ - l+ d-) / (l+ l- (l+ + l-)).
    At the end of an open line (reading F1b) the line continues into its
    mirror image in the wall: the missing neighbour is the mirror image of
    the existing one, so d+ of a last point is d- reflected in the wall
    plane (normal component kept, the others negated) and d- of a first
    point is d+ reflected; s' is then normal to the wall and s'' lies in it.
    ``lp_real`` / ``lm_real`` are the lengths of the segments that exist
    (0 for the missing one)."""
    dp = min_image(pos[nxt] - pos, lat)
    dm = min_image(pos - pos[prv], lat)
    lp_real = norm(dp)
    lm_real = norm(dm)
    ks = np.arange(pos.shape[0])
    axis, _ = end_walls(pos, nxt, prv, lat)
    last = (np.asarray(nxt) == ks) & (axis >= 0)
    first = (np.asarray(prv) == ks) & (axis >= 0)
    dp = np.where(last[:, None], reflect_except(dm, axis), dp)
    dm = np.where(first[:, None], reflect_except(dp, axis), dm)
    lp = norm(dp)
    lm = norm(dm)
    den = (lp * lm * (lp + lm))[:, None]
    sp = (lm[:, None] ** 2 * dp + lp[:, None] ** 2 * dm) / den
    sp = sp / norm(sp)[:, None]
    spp = 2.0 * (lm[:, None] * dp - lp[:, None] * dm) / den
    return dict(dp=dp, dm=dm, lp=lp, lm=lm, sp=sp, spp=spp, lp_real=lp_real,
                lm_real=lm_real, end_axis=axis)


def lia_velocity(geo, vp: VortexParams):
    """Local (divergent) part of the Biot-Savart integral, computed
    separately (Sec. II.A): beta s' x s'' with
    beta = kappa/(4 pi) ln(2 sqrt(l+ l-) / (e^C a)) (reading R3)."""
    beta = vp.kappa / (4.0 * np.pi) * np.log(
        2.0 * np.sqrt(geo["lp"] * geo["lm"]) / (np.exp(vp.core_c) * vp.core_a)
    )
    return beta[:, None] * cross(geo["sp"], geo["spp"])


# ------------------------------------------------------------ Biot-Savart

def bs_quantised(x, L):
    """Grid index of a coordinate on a periodic axis of length L:
    floor(x * 2^32 / L) mod 2^32 (exact integer, as int64)."""
    q = 4294967296.0 / float(L)
    return np.mod(np.floor(x * q).astype(np.int64), 1 << 32)


def bs_image_offsets(src, tgt, lat: Lattice):
    """Separation R = s_src - r_tgt at the nearest periodic image, for
    broadcastable arrays of source and target positions.

    The paper states periodic boundaries (Sec. III.C) but not how images enter
    the Biot-Savart sum (reading R12).  One image per (target, segment start)
    pair is used, the nearest one, decided on the 32-bit grid
    X = floor(x 2^32/L) mod 2^32: the integer separation is wrapped into
    [-2^31, 2^31) and the shift that wrapping implies is applied to the FP64
    separation.  The decision is therefore exact and reproducible; away from
    separations of exactly L/2 it is the plain nearest image."""
    R = (src - tgt).astype(np.float64)
    for a, n in enumerate(lat.dims):
        if lat.walls[a]:
            continue
        Xs = bs_quantised(src[..., a], n)
        Xt = bs_quantised(tgt[..., a], n)
        raw = Xs - Xt
        wrapped = np.mod(raw + (1 << 31), 1 << 32) - (1 << 31)
        shift = (wrapped - raw) // (1 << 32)
        R[..., a] = R[..., a] + shift.astype(np.float64) * float(n)
    return R


def segment_velocity(R1, R2, kappa):
    """Biot-Savart integral of Sec. II.A, Eq. (Biot-Savart), over one straight
    segment from s1 to s2, seen from r, with R_m = s_m - r (reading R4: the
    segment-wise integral is done exactly for straight segments):
      v = kappa/(4 pi) (R1 x R2) (|R1| + |R2|) / (|R1| |R2| (|R1||R2| + R1.R2))."""
    n1 = norm(R1)
    n2 = norm(R2)
    c = cross(R1, R2)
    fac = (n1 + n2) / (n1 * n2 * (n1 * n2 + dot(R1, R2)))
    return kappa / (4.0 * np.pi) * c * fac[..., None]


def biot_savart_nonlocal(pos, nxt, prv, lat: Lattice, kappa, targets=None, chunk=64):
    """Non-local superfluid velocity at points ``targets`` (default: all):
    sum over every segment k except the two that touch the target
    (k = prv[j] and k = j), of the straight-segment integral.  The two
    excluded segments are the divergent local part, replaced by the LIA
    term (Sec. II.A)."""
    N = pos.shape[0]
    if targets is None:
        targets = np.arange(N)
    targets = np.asarray(targets, dtype=np.int64)
    seg = min_image(pos[nxt] - pos, lat)  # segment vectors d_k
    out = np.zeros((targets.size, 3), dtype=np.float64)
    ks = np.arange(N)
    for c0 in range(0, targets.size, chunk):
        tj = targets[c0:c0 + chunk]
        R1 = bs_image_offsets(pos[None, :, :], pos[tj][:, None, :], lat)
        R2 = R1 + seg[None, :, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            v = segment_velocity(R1, R2, kappa)  # excluded pairs may be 0/0
        keep = (ks[None, :] != tj[:, None]) & (ks[None, :] != prv[tj][:, None])
        v = np.where(keep[:, :, None], v, 0.0)
        out[c0:c0 + chunk] = v.sum(axis=1)
    return out


def image_copies(lat: Lattice):
    """The images of reading F1: for every closed axis the filaments are
    mirrored in its lower wall plane (-1/2) or its upper one (n - 1/2), or
    not at all, independently per axis; every combination but the identity
    is one image copy.  Returns a list of (reflection per axis: 0 none,
    1 lower wall, 2 upper wall; sign (-1)^(number of reflections)).  A
    mirrored filament with the same point order carries circulation
    -kappa per reflection: the mirror image of a vorticity field about a
    plane, with its sign flipped, leaves no flow through that plane."""
    walled = [a for a in range(3) if lat.walls[a]]
    copies = []
    for code in np.ndindex(*([3] * len(walled))):
        if not any(code):
            continue
        refl = [0, 0, 0]
        for a, c in zip(walled, code):
            refl[a] = c
        copies.append((tuple(refl), (-1.0) ** sum(1 for c in code if c)))
    return copies


def mirror(pos, refl, lat: Lattice):
    """Positions mirrored per axis: 1 in the plane -1/2 (x -> 2(-1/2) - x),
    2 in the plane n - 1/2 (x -> 2(n - 1/2) - x)."""
    p = np.array(pos, dtype=np.float64, copy=True)
    for a, n in enumerate(lat.dims):
        if refl[a] == 1:
            p[..., a] = 2.0 * (-0.5) - p[..., a]
        elif refl[a] == 2:
            p[..., a] = 2.0 * (n - 0.5) - p[..., a]
    return p


def biot_savart_images(pos, nxt, prv, lat: Lattice, kappa, targets=None, chunk=64):
    """Boundary superflow v_s,b of Sec. II.A, Eq. (Biot-Savart), from image
    filaments (reading F1): for every image copy (image_copies) the sum over
    all of its segments (mirrored start, mirrored segment vector) of the
    straight-segment integral, times the copy's sign.  On periodic axes each
    image segment is taken at the nearest image of its start, as the real
    ones.  Nothing is excluded except at the end of an open line (reading
    F1b): in the copy mirrored in that end's own wall only, the images of the
    two segments that touch the end (k = prv[j], k = j) meet the target;
    with the real ones they are the local part of the line continued through
    the wall, which the LIA term with the mirrored neighbour replaces."""
    N = pos.shape[0]
    if targets is None:
        targets = np.arange(N)
    targets = np.asarray(targets, dtype=np.int64)
    out = np.zeros((targets.size, 3), dtype=np.float64)
    seg = min_image(pos[nxt] - pos, lat)
    axis, side = end_walls(pos, nxt, prv, lat)
    ks = np.arange(N)
    for refl, sign in image_copies(lat):
        mp = mirror(pos, refl, lat)
        mseg = seg.copy()
        for a in range(3):
            if refl[a]:
                mseg[:, a] = -mseg[:, a]
        # targets whose own wall is this copy's only reflection
        own = np.zeros(N, dtype=bool)
        if sum(1 for r in refl if r) == 1:
            a = [i for i in range(3) if refl[i]][0]
            own = (axis == a) & (side == refl[a])
        for c0 in range(0, targets.size, chunk):
            tj = targets[c0:c0 + chunk]
            R1 = bs_image_offsets(mp[None, :, :], pos[tj][:, None, :], lat)
            R2 = R1 + mseg[None, :, :]
            with np.errstate(divide="ignore", invalid="ignore"):
                v = segment_velocity(R1, R2, kappa)  # excluded pairs may be 0/0
            drop = own[tj][:, None] & ((ks[None, :] == tj[:, None]) | (ks[None, :] == prv[tj][:, None]))
            v = np.where(drop[:, :, None], 0.0, v)
            out[c0:c0 + chunk] += sign * v.sum(axis=1)
    return out


# ------------------------------------------------ interpolation / spreading

def delta2pt(r):
    """Two-point discrete delta (Sec. II.B, Eq. delta_2pt)."""
    r = np.abs(r)
    return np.where(r <= 1.0, 1.0 - r, 0.0)


def _stencil(pos, lat: Lattice):
    """The 8 lattice nodes around each point and their delta_2pt weights.
    Returns (node index triples, valid mask, weight) for the 8 corners.
    Nodes beyond a wall (ghost nodes) are marked invalid (reading R14)."""
    base = np.floor(pos).astype(np.int64)
    out = []
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                o = np.array([ox, oy, oz])
                node = base + o
                w = np.ones(pos.shape[0])
                valid = np.ones(pos.shape[0], dtype=bool)
                idx = []
                for a, n in enumerate(lat.dims):
                    w = w * delta2pt(pos[:, a] - node[:, a])
                    if lat.walls[a]:
                        valid &= (node[:, a] >= 0) & (node[:, a] < n)
                        idx.append(np.clip(node[:, a], 0, n - 1))
                    else:
                        idx.append(np.mod(node[:, a], n))
                out.append((idx, valid, w))
    return out


def interpolate(field, pos, lat: Lattice):
    """v(s) = sum over the 8 surrounding nodes of
    delta_2pt(x - s_x) delta_2pt(y - s_y) delta_2pt(z - s_z) field(node)
    (Sec. II.B).  ``field`` has shape (3, nz, ny, nx); ghost nodes beyond a
    wall contribute 0."""
    v = np.zeros((pos.shape[0], 3))
    for idx, valid, w in _stencil(pos, lat):
        vals = field[:, idx[2], idx[1], idx[0]].T
        v += np.where(valid, w, 0.0)[:, None] * vals
    return v


def spread(g_pts, pos, lat: Lattice):
    """Force density on the lattice from point forces (Sec. II.B: the reaction
    is distributed over the 8 surrounding sites with delta_2pt):
    F(node) = sum_j g_j delta_2pt(...)^3.  Weights on ghost nodes are
    dropped (reading R14)."""
    F = np.zeros((3,) + lat.shape)
    for idx, valid, w in _stencil(pos, lat):
        ww = np.where(valid, w, 0.0)
        for a in range(3):
            np.add.at(F[a], (idx[2], idx[1], idx[0]), ww * g_pts[:, a])
    return F


# -------------------------------------------------- equation of motion

def schwarz_velocity(vs, vn, sp, alpha, alpha_p):
    """Line velocity, Sec. II.A, Eq. (E of M):
    ds/dt = v_s + alpha s' x (v_n - v_s) - alpha' s' x [s' x (v_n - v_s)]."""
    w = vn - vs
    sxw = cross(sp, w)
    return vs + alpha * sxw - alpha_p * cross(sp, sxw)


def mutual_friction_force(sdot, vs, sp, dxi, vp: VortexParams):
    """Reaction of the mutual friction on the normal fluid, per point, in
    lattice units where the LB density 1 stands for rho_n (Sec. II.B; the
    printed relation equates f/(rho_s kappa) with the velocity terms of the
    equation of motion, read as the Magnus balance, reading R1):
      g_j = (rho_s/rho_n) kappa  s' x (ds/dt - v_s)  dxi_j,
    with dxi_j = (l+ + l-)/2 the line length carried by point j (R8).  With
    force_model = 1 the printed relation is taken literally instead: the
    force per length is rho_s kappa times the velocity terms themselves,
      g_j = (rho_s/rho_n) kappa  (ds/dt - v_s)  dxi_j."""
    w = sdot - vs if vp.force_model == 1 else cross(sp, sdot - vs)
    return vp.rho_s_over_rho_n * vp.kappa * w * dxi[:, None]


def superflow_at(Vs, x, n):
    """Mass-balance superflow at points of coordinate x along the flow axis
    (n nodes, periodic): V_s between the slice values at floor(x) and
    floor(x) + 1, delta_2pt-weighted (linear)."""
    ix = np.floor(x).astype(np.int64)
    fx = x - ix
    return (1.0 - fx) * Vs[np.mod(ix, n)] + fx * Vs[np.mod(ix + 1, n)]


def friction_at(vp: VortexParams, z, lat: Lattice):
    """alpha and alpha' at points of height z (reading D4): the constants, or
    the slice profiles interpolated linearly between the slices floor(z) and
    floor(z) + 1 (periodic z wraps; on a wall z axis the end slices' values
    extend to the walls).  Returns two scalars or two (n, 1) arrays."""
    if vp.alpha_z is None:
        return vp.alpha, vp.alpha_p
    nz = lat.nz
    z = np.asarray(z, dtype=np.float64)
    iz = np.floor(z)
    t = z - iz
    i0 = iz.astype(np.int64)
    i1 = i0 + 1
    if lat.walls[2]:
        i0, i1 = np.clip(i0, 0, nz - 1), np.clip(i1, 0, nz - 1)
    else:
        i0, i1 = np.mod(i0, nz), np.mod(i1, nz)
    out = []
    for prof in (vp.alpha_z, vp.alpha_p_z):
        p = np.asarray(prof, dtype=np.float64)
        out.append(((1.0 - t) * p[i0] + t * p[i1])[:, None])
    return out[0], out[1]


def line_velocity(pos, nxt, prv, ub, Vs, lat: Lattice, vp: VortexParams, want_force=False):
    """Everything the equation of motion needs at the current positions:
    v_s = non-local BS + LIA + applied + mass-balance superflow, v_n from the
    lattice, and ds/dt (Sec. II.A).  ``ub`` is the bare normal-fluid velocity
    field; ``Vs`` the slice superflow (or None)."""
    geo = geometry(pos, nxt, prv, lat)
    if vp.ff_cell > 0:
        from .farfield import biot_savart_farfield  # it builds on this module

        nonlocal_v, _ = biot_savart_farfield(pos, nxt, prv, lat, vp.kappa, vp.ff_cell,
                                             vp.ff_theta, levels=max(vp.ff_levels, 1))
    else:
        nonlocal_v = biot_savart_nonlocal(pos, nxt, prv, lat, vp.kappa)
    vs = nonlocal_v + lia_velocity(geo, vp)
    if vp.wall_images:
        vs = vs + biot_savart_images(pos, nxt, prv, lat, vp.kappa)
    vs = vs + np.array(vp.vs_applied, dtype=np.float64)[None, :]
    if Vs is not None:
        a = vp.mass_balance_axis
        vs[:, a] = vs[:, a] + superflow_at(Vs, pos[:, a], lat.dims[a])
    vn = interpolate(ub, pos, lat)
    alpha, alpha_p = friction_at(vp, pos[:, 2], lat)
    sdot = schwarz_velocity(vs, vn, geo["sp"], alpha, alpha_p)
    # an open line's end slides on its wall: no velocity normal to it (F1b)
    ax = geo["end_axis"]
    for a in range(3):
        sdot[ax == a, a] = 0.0
    out = dict(vs=vs, vn=vn, sdot=sdot, geo=geo)
    if want_force:
        # the line length a point carries: half of each segment that exists
        dxi = 0.5 * (geo["lp_real"] + geo["lm_real"])
        out["force"] = mutual_friction_force(sdot, vs, geo["sp"], dxi, vp)
    return out
