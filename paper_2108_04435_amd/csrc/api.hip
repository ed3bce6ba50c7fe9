// C ABI of the vlb library (declared in include/vlb.h): argument checks,
// workspace layout, and the order of device work inside one coupled step.
#include "vlb_internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>
#include <new>

using namespace vlb;

struct vlb_run {
  Run r;
};

struct vlb_graph {
  vlb_run* run = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t n_steps = 0;
  int parity = 0;
  int point_parity = 0;
  bool has_points = false;  // filaments present at capture (else the LBM alone)
};

namespace {

std::mutex g_err_mu;
std::string g_err;

int fail(vlb_run* h, int code, const std::string& msg) {
  if (h) {
    h->r.err = msg;
  } else {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_err = msg;
  }
  return code;
}

int hip_fail(vlb_run* h, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(h, VLB_EDEVICE, m);
}

#define HIP_OR_FAIL(h, call)                       \
  do {                                             \
    hipError_t _e = (call);                        \
    if (_e != hipSuccess) return hip_fail(h, _e, #call); \
  } while (0)

constexpr size_t kAlign = 256;

struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(char* b) : base(b) {}
  void* take(size_t bytes) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

size_t elt_size(int prec) { return prec == VLB_F64 ? 8 : (prec == VLB_F32 ? 4 : 2); }

int check_desc(const vlb_lattice_desc* lat, const vlb_vortex_desc* vor, std::string& msg) {
  if (!lat || !vor) { msg = "null descriptor"; return VLB_EINVAL; }
  if (lat->nx < 4 || lat->ny < 4 || lat->nz < 4) { msg = "every lattice dimension must be >= 4"; return VLB_EINVAL; }
  const double cells = (double)lat->nx * lat->ny * lat->nz;
  if (cells > 1.0e9) { msg = "lattice larger than 1e9 nodes"; return VLB_EINVAL; }
  if (lat->precision < 0 || lat->precision > 2) { msg = "precision must be VLB_F64, VLB_F32 or VLB_F16"; return VLB_EINVAL; }
  if (!(lat->tau > 0.5)) { msg = "tau must exceed 1/2 (positive viscosity)"; return VLB_EINVAL; }
  if (lat->wall_axes & ~7u) { msg = "wall_axes uses bits 0..2 only"; return VLB_EINVAL; }
  if ((lat->plane_lo || lat->plane_hi) && (lat->wall_axes & 4u)) { msg = "velocity planes need a periodic z axis"; return VLB_EINVAL; }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(lat->plane_u[a]) || !std::isfinite(lat->body_force[a])) { msg = "non-finite plane velocity or body force"; return VLB_EINVAL; }
  if (vor->n_cap < 1 || vor->n_cap > (1LL << 28)) { msg = "n_cap must be in [1, 2^28]"; return VLB_EINVAL; }
  if (!(vor->kappa > 0) || !(vor->core_a > 0)) { msg = "kappa and core_a must be positive"; return VLB_EINVAL; }
  if (!(vor->dxi_min > 0) || !(vor->dxi_max > vor->dxi_min)) { msg = "need 0 < dxi_min < dxi_max"; return VLB_EINVAL; }
  if (vor->min_loop_pts < 3) { msg = "min_loop_pts must be >= 3"; return VLB_EINVAL; }
  if (vor->mass_balance_axis < 0 || vor->mass_balance_axis > 2) { msg = "mass_balance_axis must be 0, 1 or 2"; return VLB_EINVAL; }
  if (vor->mass_balance && ((lat->wall_axes >> vor->mass_balance_axis) & 1u)) { msg = "mass balance needs a periodic flow axis"; return VLB_EINVAL; }
  if (vor->rk_stages != 0 && vor->rk_stages != 1 && vor->rk_stages != 2 && vor->rk_stages != 4) { msg = "rk_stages must be 1, 2 or 4 (0: 4)"; return VLB_EINVAL; }
  if (vor->vfm_substeps < 0 || vor->vfm_substeps > 64) { msg = "vfm_substeps must be in [1, 64] (0: 1)"; return VLB_EINVAL; }
  if (vor->reserved2 != 0) { msg = "reserved2 must be 0"; return VLB_EINVAL; }
  if (vor->force_model != 0 && vor->force_model != 1) { msg = "force_model must be 0 or 1"; return VLB_EINVAL; }
  if (vor->wall_images != 0 && vor->wall_images != 1) { msg = "wall_images must be 0 or 1"; return VLB_EINVAL; }
  if (vor->ff_cell < 0) { msg = "ff_cell must be >= 0"; return VLB_EINVAL; }
  if (vor->ff_cell > 0) {
    if (lat->precision == VLB_F64) { msg = "the far-field sum is FP32: precision VLB_F32 or VLB_F16"; return VLB_EINVAL; }
    if (vor->wall_images) { msg = "the far-field sum takes no wall images"; return VLB_EINVAL; }
    vlb_bs_desc bd{lat->nx, lat->ny, lat->nz, lat->wall_axes, VLB_F32, 0, vor->kappa};
    vlb_ff_params fp{vor->ff_cell, vor->ff_levels, vor->ff_theta};
    const int c = ff_check(&bd, &fp, vor->n_cap, msg);
    if (c != VLB_OK) return c;
  }
  if (vor->reconnect) {
    if (!(vor->reconnect_dist > 0)) { msg = "reconnect_dist must be positive"; return VLB_EINVAL; }
    if (vor->recon_cap < 1 || vor->recon_cap > (1LL << 26)) { msg = "recon_cap must be in [1, 2^26]"; return VLB_EINVAL; }
  }
  return VLB_OK;
}

void release_streams(Run& r) {
  hipEvent_t* evs[] = {&r.ev_fork, &r.ev_mom, &r.ev_fin1, &r.ev_join};
  for (hipEvent_t* ev : evs)
    if (*ev) {
      (void)hipEventDestroy(*ev);  // teardown: nothing to report to
      *ev = nullptr;
    }
  if (r.side) {
    (void)hipStreamDestroy(r.side);
    r.side = nullptr;
  }
}

int bits_for(unsigned long long v) {  // smallest b with v < 2^b
  int b = 1;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

// Carve the workspace (base == nullptr: only measure).
size_t layout(Run& r, char* base) {
  Bump B(base);
  const long long cells = r.cells;
  const long long nc = r.ncap;
  const size_t fe = r.prec == VLB_F64 ? 8 : 4;
  r.pops = B.take(19 * cells * elt_size(r.prec));
  r.force = B.take(3 * cells * fe);
  // superflow per cross-section along the flow axis; along x or y also the
  // per-z-slice partial sums of its mean
  const int mba = r.vor.mass_balance_axis;
  const int nmb = mba == 0 ? r.geom.nx : (mba == 1 ? r.geom.ny : r.geom.nz);
  r.Vs = (double*)B.take(nmb * sizeof(double));
  r.Vs_next = (double*)B.take(nmb * sizeof(double));
  r.mbP = (double*)B.take((r.vor.mass_balance && mba != 2 ? (size_t)r.geom.nz * nmb : 0) * sizeof(double));
  r.diag = (double*)B.take((8 + (size_t)kSlabChunks * r.geom.nz) * sizeof(double));
  r.seg = (double*)B.take(3 * (size_t)nc * sizeof(double));
  r.fric = (double*)B.take((2 * (size_t)r.geom.nz + 1) * sizeof(double));
  r.touched = (int32_t*)B.take(8 * nc * sizeof(int32_t));
  double** dbufs[] = {&r.pos, &r.ya, &r.yb, &r.ksum, &r.vs1, &r.vn1, &r.sd1, &r.gpt, &r.pos_t, &r.stage, &r.sfrac};
  for (double** p : dbufs) *p = (double*)B.take(3 * nc * sizeof(double));
  int32_t** ibufs[] = {&r.nxt, &r.prv, &r.nxt_t, &r.prv_t, &r.stage_i, &r.flag_a, &r.flag_b,
                       &r.scan_a, &r.scan_b, &r.used};
  for (int32_t** p : ibufs) *p = (int32_t*)B.take((nc + 1) * sizeof(int32_t));
  const int nco = r.bsax.copies;
  r.bsX = (uint32_t*)B.take((size_t)nco * 3 * nc * sizeof(uint32_t));
  r.bsD = B.take((size_t)nco * (r.prec == VLB_F64 ? 6 : 4) * nc * fe);  // FP64: d (3) and residuals (3)
  size_t pbytes = (size_t)nco * r.bsS * 3 * nc * fe;
  if (r.vor.ff_cell > 0 && (size_t)r.ffS * 3 * nc * fe > pbytes) pbytes = (size_t)r.ffS * 3 * nc * fe;
  r.bsP = B.take(pbytes);
  r.ffws = r.vor.ff_cell > 0 ? B.take(ff_run_bytes(r)) : nullptr;
  r.bsown = nco > 1 ? (int32_t*)B.take(nc * sizeof(int32_t)) : nullptr;
  r.cnt = (int32_t*)B.take(32 * sizeof(int32_t));
  r.marked = (uint32_t*)B.take(nc * sizeof(uint32_t));
  r.keys_a = (uint32_t*)B.take(nc * sizeof(uint32_t));
  r.keys_b = (uint32_t*)B.take(nc * sizeof(uint32_t));
  r.vals_a = (int32_t*)B.take(nc * sizeof(int32_t));
  r.vals_b = (int32_t*)B.take(nc * sizeof(int32_t));
  r.sort_tmp_bytes = sort_tmp_bytes(nc);
  r.sort_tmp = B.take(r.sort_tmp_bytes);
  {
    const long long nw = (nc + 255) / 256 * 4;  // waves of the per-point grids
    r.wmask = (uint64_t*)B.take(nw * sizeof(uint64_t));
    r.wpre = (int32_t*)B.take((nw + 1) * sizeof(int32_t));
  }
  if (r.vor.reconnect) {
    r.rc_head = (int32_t*)B.take((size_t)r.rc_nbins * sizeof(int32_t));
    r.rc_next = (int32_t*)B.take((nc + 1) * sizeof(int32_t));
    r.rc_keyp = (uint32_t*)B.take((nc + 1) * sizeof(uint32_t));
    const long long rc = r.rcap;
    r.rc_i = (int32_t*)B.take(rc * sizeof(int32_t));
    r.rc_j = (int32_t*)B.take(rc * sizeof(int32_t));
    r.rc_idx_a = (int32_t*)B.take(rc * sizeof(int32_t));
    r.rc_key_a = (uint64_t*)B.take(rc * sizeof(uint64_t));
    r.rc_best = (uint64_t*)B.take((nc + 1) * sizeof(uint64_t));
    r.rc_slot_j = (int32_t*)B.take(8 * (nc + 1) * sizeof(int32_t));
    r.rc_slot_k = (uint64_t*)B.take(8 * (nc + 1) * sizeof(uint64_t));
    r.rc_bidx = (int32_t*)B.take((nc + 1) * sizeof(int32_t));
  }
  r.ub = B.take(3 * cells * fe);
  r.ub_next = B.take(3 * cells * fe);
  r.bins = (int32_t*)B.take((size_t)r.nbins_table * sizeof(int32_t));
  return (B.off + kAlign - 1) / kAlign * kAlign;
}

void init_run(Run& r, const vlb_lattice_desc* lat, const vlb_vortex_desc* vor) {
  r.lat = *lat;
  r.vor = *vor;
  if (r.vor.rk_stages == 0) r.vor.rk_stages = 4;
  if (r.vor.vfm_substeps == 0) r.vor.vfm_substeps = 1;
  r.prec = lat->precision;
  r.cells = (long long)lat->nx * lat->ny * lat->nz;
  r.ncap = vor->n_cap;
  r.rcap = vor->reconnect ? vor->recon_cap : 0;
  Geom& g = r.geom;
  g.nx = lat->nx;
  g.ny = lat->ny;
  g.nz = lat->nz;
  for (int a = 0; a < 3; ++a) g.wall[a] = (lat->wall_axes >> a) & 1u;
  g.plane_lo = lat->plane_lo ? 1 : 0;
  g.plane_hi = lat->plane_hi ? 1 : 0;
  g.cells = r.cells;
  for (int a = 0; a < 3; ++a) {
    g.plane_u[a] = lat->plane_u[a];
    g.body[a] = lat->body_force[a];
  }
  g.omega = 1.0 / lat->tau;
  g.fpref = 1.0 - 1.0 / (2.0 * lat->tau);
  for (int a = 0; a < 3; ++a) {
    g.plane_u_f[a] = (float)g.plane_u[a];
    g.body_f[a] = (float)g.body[a];
  }
  g.omega_f = (float)g.omega;
  g.fpref_f = (float)g.fpref;
  const int n[3] = {g.nx, g.ny, g.nz};
  r.bsax = bs_make_axes(n, g.wall, vor->wall_images != 0);
  r.bsS = bs_chunks(r.ncap);
  r.ffS = vor->ff_cell > 0 ? ff_run_chunks(r) : 0;
  // spreading bins: lower stencil corner, n (+1 on wall axes) per axis
  const unsigned long long ext = (unsigned long long)(n[0] + g.wall[0]) * (n[1] + g.wall[1]) * (n[2] + g.wall[2]);
  r.key_bits = bits_for(ext);  // pad key 2^bits - 1 >= ext
  if (r.key_bits > 32) r.key_bits = 32;
  r.nbins_table = (long long)ext;
  // reconnection bins of edge >= reconnect distance
  if (vor->reconnect) {
    const double h0 = vor->reconnect_dist * (1.0 + 1e-9);
    unsigned long long tot = 1;
    for (int a = 0; a < 3; ++a) {
      int nb = (int)std::floor((double)n[a] / h0);
      if (nb < 1) nb = 1;
      r.bin_n[a] = nb;
      r.bin_h[a] = (double)n[a] / nb;
      tot *= (unsigned long long)nb;
    }
    r.rc_nbins = (long long)tot;
  }
}

}  // namespace

namespace vlb {

int fail_global(int code, const std::string& msg) { return fail(nullptr, code, msg); }

// Events come from a pool filled by vlb_set_timing, so that timing a run
// creates no events inside the timed region (the pool grows if it runs dry).
static hipEvent_t take_event(Run& r) {
  if (!r.ev_pool.empty()) {
    hipEvent_t e = r.ev_pool.back();
    r.ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void time_begin(Run& r, int cls, hipEvent_t* b) {
  *b = nullptr;
  (void)cls;
  if (!r.timing) return;
  hipEvent_t e0 = take_event(r);
  if (!e0) return;
  if (hipEventRecord(e0, r.stream) != hipSuccess) {  // the launch then goes untimed
    r.ev_pool.push_back(e0);
    return;
  }
  *b = e0;
}

void time_end(Run& r, int cls, hipEvent_t b) {
  if (!r.timing || !b) return;
  hipEvent_t e1 = take_event(r);
  if (!e1) return;
  if (hipEventRecord(e1, r.stream) != hipSuccess) {  // the launch then goes untimed
    r.ev_pool.push_back(e1);
    r.ev_pool.push_back(b);
    return;
  }
  r.ev_used[cls].emplace_back(b, e1);
}

}  // namespace vlb

namespace {

// Return recorded events to the pool.
void recycle_events(Run& r) {
  for (int c = 0; c < 2; ++c) {
    for (auto& p : r.ev_used[c]) {
      r.ev_pool.push_back(p.first);
      r.ev_pool.push_back(p.second);
    }
    r.ev_used[c].clear();
  }
}

void drop_events(Run& r) {
  recycle_events(r);
  for (hipEvent_t e : r.ev_pool) (void)hipEventDestroy(e);  // teardown
  r.ev_pool.clear();
}

// wrap as in the kernels: periodic into [0, L), walls mirrored
double wrap_host(double x, double L, bool periodic) {
  if (periodic) {
    if (x < 0.0) x = x + L;
    if (x >= L) x = x - L;
    if (x >= L) x = 0.0;
  } else {
    const double lo = -0.5, hi = L - 0.5;
    if (x < lo) x = 2.0 * lo - x;
    if (x > hi) x = 2.0 * hi - x;
  }
  return x;
}

int read_count(vlb_run* h, int32_t* out) {
  Run& r = h->r;
  HIP_OR_FAIL(h, hipMemcpyAsync(out, r.cnt, sizeof(int32_t), hipMemcpyDeviceToHost, r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  return VLB_OK;
}

int latched(vlb_run* h) {
  Run& r = h->r;
  int32_t flags = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(&flags, r.cnt + 7, sizeof(int32_t), hipMemcpyDeviceToHost, r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  if (flags) {
    HIP_OR_FAIL(h, hipMemsetAsync(r.cnt + 7, 0, sizeof(int32_t), r.stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
    if (flags & kFlagNumeric) return fail(h, VLB_ENUMERIC, "non-finite line velocity");
    if (flags & kFlagCapacity) return fail(h, VLB_ECAPACITY, "filament points exceeded n_cap; insertion skipped");
    if (flags & kFlagReconCap)
      return fail(h, VLB_ECAPACITY,
                  "reconnection candidates exceeded recon_cap (or 8 at one point); reconnection skipped");
  }
  return VLB_OK;
}

int copy_soa_to_host(vlb_run* h, const double* dev_soa, int n, double* host_aos) {
  Run& r = h->r;
  std::vector<double> tmp(3 * (size_t)n);
  for (int a = 0; a < 3; ++a)
    HIP_OR_FAIL(h, hipMemcpyAsync(tmp.data() + (size_t)a * n, dev_soa + a * r.ncap,
                                  n * sizeof(double), hipMemcpyDeviceToHost, r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  for (int j = 0; j < n; ++j)
    for (int a = 0; a < 3; ++a) host_aos[3 * (size_t)j + a] = tmp[(size_t)a * n + j];
  return VLB_OK;
}

}  // namespace

extern "C" {

int vlb_query_footprint(const vlb_lattice_desc* lat, const vlb_vortex_desc* vor, uint64_t* bytes) {
  std::string msg;
  const int c = check_desc(lat, vor, msg);
  if (c != VLB_OK) return fail(nullptr, c, msg);
  if (!bytes) return fail(nullptr, VLB_EINVAL, "bytes is NULL");
  Run r;
  init_run(r, lat, vor);
  *bytes = layout(r, nullptr);
  return VLB_OK;
}

int vlb_create_lattice(const vlb_lattice_desc* lat, const vlb_vortex_desc* vor, void* dev_workspace,
                       uint64_t ws_bytes, void* hip_stream, vlb_run** out) {
  std::string msg;
  const int c = check_desc(lat, vor, msg);
  if (c != VLB_OK) return fail(nullptr, c, msg);
  if (!out || !dev_workspace) return fail(nullptr, VLB_EINVAL, "out or workspace is NULL");
  if ((uintptr_t)dev_workspace % kAlign) return fail(nullptr, VLB_EINVAL, "workspace must be 256-byte aligned");
  vlb_run* h = new (std::nothrow) vlb_run();
  if (!h) return fail(nullptr, VLB_EINVAL, "out of host memory");
  Run& r = h->r;
  init_run(r, lat, vor);
  const size_t need = layout(r, nullptr);
  if (ws_bytes < need) {
    delete h;
    return fail(nullptr, VLB_ENOSPACE, "workspace smaller than vlb_query_footprint");
  }
  r.ws = (char*)dev_workspace;
  r.ws_bytes = ws_bytes;
  layout(r, r.ws);
  r.stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&r.device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&r.side, hipStreamNonBlocking);
  hipEvent_t* evs[] = {&r.ev_fork, &r.ev_mom, &r.ev_fin1, &r.ev_join};
  for (hipEvent_t* ev : evs)
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  // populations at rest, no force, no points
  if (e == hipSuccess) e = hipMemsetAsync(r.force, 0, 3 * r.cells * (r.prec == VLB_F64 ? 8 : 4), r.stream);
  if (e == hipSuccess) e = hipMemsetAsync(r.cnt, 0, 32 * sizeof(int32_t), r.stream);
  // no friction profiles: the constants apply
  if (e == hipSuccess) e = hipMemsetAsync(r.fric, 0, (2 * (size_t)r.geom.nz + 1) * sizeof(double), r.stream);
  if (e == hipSuccess) e = hipMemsetAsync(r.pops, 0, 19 * r.cells * elt_size(r.prec), r.stream);
  if (e == hipSuccess) e = hipMemsetAsync(r.bins, 0xFF, (size_t)r.nbins_table * sizeof(int32_t), r.stream);
  if (e == hipSuccess) e = hipMemsetAsync(r.marked, 0xFF, (size_t)r.ncap * sizeof(uint32_t), r.stream);
  if (e == hipSuccess && r.rc_head)
    e = hipMemsetAsync(r.rc_head, 0xFF, (size_t)r.rc_nbins * sizeof(int32_t), r.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(r.stream);
  if (e != hipSuccess) {
    std::string m = std::string("initialising the workspace: ") + hipGetErrorString(e);
    release_streams(r);
    delete h;
    return fail(nullptr, VLB_EDEVICE, m);
  }
  r.parity = 0;
  r.has_fields = true;
  *out = h;
  return VLB_OK;
}

int vlb_write_fields(vlb_run* h, const double* rho_dev, const double* u_dev) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!rho_dev || !u_dev) return fail(h, VLB_EINVAL, "rho and u are required");
  Run& r = h->r;
  HIP_OR_FAIL(h, lbm_init_eq(r, rho_dev, u_dev));
  HIP_OR_FAIL(h, hipMemsetAsync(r.force, 0, 3 * r.cells * (r.prec == VLB_F64 ? 8 : 4), r.stream));
  HIP_OR_FAIL(h, hipMemsetAsync(r.cnt + 1, 0, sizeof(int32_t), r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  r.step = 0;
  r.has_fields = true;
  return VLB_OK;
}

int vlb_seed_vortices(vlb_run* h, int64_t n_pts, const double* xyz, const int32_t* next) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  Run& r = h->r;
  if (n_pts < 0 || n_pts > r.ncap) return fail(h, VLB_EINVAL, "n_pts must be in [0, n_cap]");
  if (n_pts > 0 && (!xyz || !next)) return fail(h, VLB_EINVAL, "xyz and next are required");
  const int n = (int)n_pts;
  // links: at most one predecessor besides itself per point; a point that
  // links to itself is the last point of an open line, one that no other
  // point links to is the first (it keeps itself as its predecessor)
  std::vector<int32_t> prv(n);
  std::vector<uint8_t> has_pred(n, 0);
  for (int j = 0; j < n; ++j) prv[j] = j;
  for (int j = 0; j < n; ++j) {
    const int k = next[j];
    if (k < 0 || k >= n) return fail(h, VLB_EINVAL, "next[] out of range");
    if (k == j) continue;
    if (has_pred[k]) return fail(h, VLB_EINVAL, "next[]: a point has two predecessors");
    has_pred[k] = 1;
    prv[k] = j;
  }
  std::vector<double> soa(3 * (size_t)n);
  const int dims[3] = {r.geom.nx, r.geom.ny, r.geom.nz};
  for (int j = 0; j < n; ++j)
    for (int a = 0; a < 3; ++a) {
      const double x = xyz[3 * (size_t)j + a];
      if (!std::isfinite(x)) return fail(h, VLB_EINVAL, "non-finite position");
      const double L = (double)dims[a];
      const double w = wrap_host(x, L, !r.geom.wall[a]);
      // one wrap (periodic) or one mirror (wall) must bring the point inside
      if (r.geom.wall[a] ? !(w >= -0.5 && w <= L - 0.5) : !(w >= 0.0 && w < L))
        return fail(h, VLB_EINVAL, "position more than one lattice length outside the box");
      soa[(size_t)a * n + j] = w;
    }
  // the ends of open lines lie on a wall plane of a closed axis (the
  // positions as wrapped, exactly)
  for (int j = 0; j < n; ++j) {
    const bool last = next[j] == j, first = !has_pred[j];
    if (!last && !first) continue;
    if (last && first) return fail(h, VLB_EINVAL, "next[]: a one-point line");
    bool on = false;
    for (int a = 0; a < 3; ++a) {
      const double w = soa[(size_t)a * n + j];
      if (r.geom.wall[a] && (w == -0.5 || w == (double)dims[a] - 0.5)) on = true;
    }
    if (!on) return fail(h, VLB_EINVAL, "an open line ends off the wall planes");
  }
  // loops and lines shorter than min_loop_pts are accepted here and removed
  // by the next topology pass
  if (n > 0) {
    for (int a = 0; a < 3; ++a)
      HIP_OR_FAIL(h, hipMemcpyAsync(r.pos + a * r.ncap, soa.data() + (size_t)a * n, n * sizeof(double),
                                    hipMemcpyHostToDevice, r.stream));
    HIP_OR_FAIL(h, hipMemcpyAsync(r.nxt, next, n * sizeof(int32_t), hipMemcpyHostToDevice, r.stream));
    HIP_OR_FAIL(h, hipMemcpyAsync(r.prv, prv.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, r.stream));
  }
  if (n > 0) r.has_points = true;
  int32_t c0 = n;
  HIP_OR_FAIL(h, hipMemcpyAsync(r.cnt, &c0, sizeof(int32_t), hipMemcpyHostToDevice, r.stream));
  // grid coordinates of the seeded positions (FP32 sum of the first step)
  if (n > 0 && r.prec != VLB_F64) HIP_OR_FAIL(h, bs_prep(r, r.pos));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  return VLB_OK;
}

}  // extern "C"

namespace {

// Runs of a many-run call: non-null and distinct.
int check_runs(vlb_run* const* runs, int32_t n) {
  if (!runs || n < 1) return fail(nullptr, VLB_EINVAL, "need at least one run");
  for (int32_t i = 0; i < n; ++i) {
    if (!runs[i]) return fail(nullptr, VLB_EINVAL, "run is NULL");
    for (int32_t k = 0; k < i; ++k)
      if (runs[k] == runs[i]) return fail(nullptr, VLB_EINVAL, "a run appears twice");
  }
  return VLB_OK;
}

// Launchers enqueue on r.stream; this points it at another stream for a
// scope.
struct OnStream {
  Run& r;
  hipStream_t saved;
  OnStream(Run& run, hipStream_t s) : r(run), saved(run.stream) { r.stream = s; }
  ~OnStream() { r.stream = saved; }
};

// One coupled step on two streams.  The caller's stream (main) carries the
// filament part: the four RK4 stages (Biot-Savart sum + finalize) and the
// topology.  The library's side stream carries the lattice part: the
// moments of f^n, the spreading of the stage-1 forces and the LBM update.
// Dependencies (events): finalize 1 needs the moments (velocity field and
// superflow); the spreading needs finalize 1, which leaves it the point
// forces, bin keys, stencil offsets and point count, so the spreading reads
// nothing the later stages or the topology rewrite.  The LBM update follows
// the spreading on the side stream, launched on a narrow grid (two blocks
// per CU) so that it leaves most CU slots to the filament kernels beside
// it.  The next step's moments follow the LBM update on the side stream
// and write the second velocity field (this step's stages read the first;
// the two swap at the end of the step).  The first step of a call forks
// the side stream from main and computes its own moments; the last one
// joins the side stream back, so a call's work is ordered on the caller's
// stream.
int one_step(vlb_run* h, bool first, bool last) {
  Run& r = h->r;
  if (!r.has_points) {  // never seeded: the normal fluid alone
    HIP_OR_FAIL(h, lbm_step(r));
    r.step += 1;
    r.last_nodes += r.cells;
    return VLB_OK;
  }
  hipStream_t M = r.stream, S = r.side;
  if (first) {
    HIP_OR_FAIL(h, hipEventRecord(r.ev_fork, M));
    HIP_OR_FAIL(h, hipStreamWaitEvent(S, r.ev_fork, 0));
    OnStream on(r, S);
    // bare velocity field and mass-balance superflow of f^n
    HIP_OR_FAIL(h, lbm_moments(r));
    HIP_OR_FAIL(h, hipEventRecord(r.ev_mom, S));
  }
  // filament stages: vfm_substeps substeps of the rk_stages-stage method,
  // each from the positions in pos back into pos; stage positions
  // classical: pos -> ya -> yb -> ya -> pos; midpoint: pos -> ya -> pos;
  // Euler: pos -> ya, copied back
  const int K = r.vor.rk_stages;
  const int G = K * r.vor.vfm_substeps;
  double* Ys4[4] = {r.pos, r.ya, r.yb, r.ya};
  double* Yn4[4] = {r.ya, r.yb, r.ya, r.pos};
  double* Ys2[2] = {r.pos, r.ya};
  double* Yn2[2] = {r.ya, r.pos};
  double* Yn1[1] = {r.ya};
  double** Ys = K == 4 ? Ys4 : Ys2;
  double** Yn = K == 4 ? Yn4 : (K == 2 ? Yn2 : Yn1);
  const bool spread = r.vor.coupling != 0;
  // the side stream's work follows the second stage (the first if there is
  // only one)
  const int gside = G > 1 ? 1 : 0;
  for (int gs = 0; gs < G; ++gs) {
    const int s = gs % K;
    // FP32: the grid coordinates of every stage's positions were written by
    // the kernel that wrote the positions (seeding and the topology's copy
    // for the step's first stage, the previous finalize for the others)
    if (r.vor.ff_cell > 0) {
      HIP_OR_FAIL(h, ff_run_sum(r, Ys[s]));
    } else {
      if (r.prec == VLB_F64 || r.bsax.copies > 1) HIP_OR_FAIL(h, bs_prep(r, Ys[s]));
      HIP_OR_FAIL(h, bs_sum(r));
    }
    // the first finalize reads the velocity field and the superflow
    if (gs == 0) HIP_OR_FAIL(h, hipStreamWaitEvent(M, r.ev_mom, 0));
    HIP_OR_FAIL(h, fil_finalize(r, s + 1, gs == 0, gs == G - 1, Ys[s], Yn[s], 0));
    if (K == 1) HIP_OR_FAIL(h, fil_copy_positions(r, r.ya, r.pos));
    // finalize 1 leaves the spreading everything it reads, and it follows
    // the previous step's last reads of the field the next moments overwrite
    if (gs == 0) HIP_OR_FAIL(h, hipEventRecord(r.ev_fin1, M));
    // the side stream's work is enqueued after the main stream's next
    // kernel, so that a graph keeps the main chain on one queue
    if (gs == gside) {
      HIP_OR_FAIL(h, hipStreamWaitEvent(S, r.ev_fin1, 0));
      OnStream on(r, S);
      if (spread) HIP_OR_FAIL(h, fil_spread(r));
      // the LBM update on a narrow grid beside the Biot-Savart sums, then
      // the moments of f^(n+1) into the next step's field (the stages of
      // this step still read the current one)
      r.lbm_narrow = true;
      hipError_t le = lbm_step(r);
      if (le == hipSuccess && !last) {
        std::swap(r.ub, r.ub_next);
        std::swap(r.Vs, r.Vs_next);
        le = lbm_moments(r);
        std::swap(r.ub, r.ub_next);
        std::swap(r.Vs, r.Vs_next);
      }
      r.lbm_narrow = false;
      if (le != hipSuccess) return hip_fail(h, le, "lbm_step / lbm_moments");
      if (!last) HIP_OR_FAIL(h, hipEventRecord(r.ev_mom, S));
    }
  }
  HIP_OR_FAIL(h, topo_update(r, true));
  if (!last) {
    std::swap(r.ub, r.ub_next);
    std::swap(r.Vs, r.Vs_next);
  }
  if (last) {
    HIP_OR_FAIL(h, hipEventRecord(r.ev_join, S));
    HIP_OR_FAIL(h, hipStreamWaitEvent(M, r.ev_join, 0));
  }
  r.step += 1;
  r.last_nodes += r.cells;
  return VLB_OK;
}

}  // namespace

extern "C" {

int vlb_step(vlb_run* h, int64_t n_steps) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (n_steps < 0) return fail(h, VLB_EINVAL, "n_steps must be >= 0");
  for (int64_t s = 0; s < n_steps; ++s) {
    const int c = one_step(h, s == 0, s == n_steps - 1);
    if (c != VLB_OK) return c;
  }
  return VLB_OK;
}

int vlb_step_many(vlb_run* const* runs, int32_t n_runs, int64_t n_steps) {
  int c = check_runs(runs, n_runs);
  if (c != VLB_OK) return c;
  if (n_steps < 0) return fail(nullptr, VLB_EINVAL, "n_steps must be >= 0");
  // step-major: step s of every run is enqueued before step s + 1 of any
  for (int64_t s = 0; s < n_steps; ++s)
    for (int32_t i = 0; i < n_runs; ++i) {
      c = one_step(runs[i], s == 0, s == n_steps - 1);
      if (c != VLB_OK) return c;
    }
  return VLB_OK;
}

int vlb_sync(vlb_run* h) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->r.stream));
  if (h->r.side) HIP_OR_FAIL(h, hipStreamSynchronize(h->r.side));
  return latched(h);
}

int vlb_read_fields(vlb_run* h, double* rho_dev, double* u_dev) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  HIP_OR_FAIL(h, lbm_read_fields(h->r, rho_dev, u_dev));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->r.stream));
  return latched(h);
}

int vlb_read_populations(vlb_run* h, double* f_dev) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!f_dev) return fail(h, VLB_EINVAL, "f is NULL");
  HIP_OR_FAIL(h, lbm_read_pops(h->r, f_dev));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->r.stream));
  return latched(h);
}

int vlb_read_state(vlb_run* h, void* pops_dev) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!pops_dev) return fail(h, VLB_EINVAL, "pops is NULL");
  HIP_OR_FAIL(h, lbm_read_state(h->r, pops_dev));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->r.stream));
  return latched(h);
}

int vlb_write_state(vlb_run* h, const void* pops_dev, int64_t step) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!pops_dev) return fail(h, VLB_EINVAL, "pops is NULL");
  if (step < 0) return fail(h, VLB_EINVAL, "step must be >= 0");
  Run& r = h->r;
  HIP_OR_FAIL(h, hipMemcpyAsync(r.pops, pops_dev, 19 * (size_t)r.cells * elt_size(r.prec),
                                hipMemcpyDeviceToDevice, r.stream));
  HIP_OR_FAIL(h, hipMemsetAsync(r.force, 0, 3 * r.cells * (r.prec == VLB_F64 ? 8 : 4), r.stream));
  HIP_OR_FAIL(h, hipMemsetAsync(r.cnt + 1, 0, sizeof(int32_t), r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  r.parity = 0;
  r.step = step;
  r.has_fields = true;
  return VLB_OK;
}

int vlb_read_force(vlb_run* h, double* force_dev) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!force_dev) return fail(h, VLB_EINVAL, "force is NULL");
  HIP_OR_FAIL(h, lbm_read_force(h->r, force_dev));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->r.stream));
  return latched(h);
}

int vlb_read_filaments(vlb_run* h, int64_t cap, double* xyz, int32_t* next, int64_t* n_pts) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!n_pts) return fail(h, VLB_EINVAL, "n_pts is NULL");
  int32_t n = 0;
  int c = read_count(h, &n);
  if (c != VLB_OK) return c;
  *n_pts = n;
  if (n > cap) return fail(h, VLB_ENOSPACE, "more points than cap");
  if (n > 0) {
    if (xyz) {
      c = copy_soa_to_host(h, h->r.pos, n, xyz);
      if (c != VLB_OK) return c;
    }
    if (next) {
      HIP_OR_FAIL(h, hipMemcpyAsync(next, h->r.nxt, n * sizeof(int32_t), hipMemcpyDeviceToHost, h->r.stream));
      HIP_OR_FAIL(h, hipStreamSynchronize(h->r.stream));
    }
  }
  return latched(h);
}

int vlb_eval_line_velocity(vlb_run* h, double* vs, double* vn, double* sdot, double* force) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  Run& r = h->r;
  HIP_OR_FAIL(h, lbm_moments(r));
  if (r.vor.ff_cell > 0) {
    HIP_OR_FAIL(h, ff_run_sum(r, r.pos));
  } else {
    HIP_OR_FAIL(h, bs_prep(r, r.pos));
    HIP_OR_FAIL(h, bs_sum(r));
  }
  HIP_OR_FAIL(h, fil_finalize(r, 1, 1, 1, r.pos, r.ya, 1));
  if (r.vor.coupling) HIP_OR_FAIL(h, fil_spread(r));
  int32_t n = 0;
  int c = read_count(h, &n);
  if (c != VLB_OK) return c;
  const double* src[4] = {r.vs1, r.vn1, r.sd1, r.gpt};
  double* dst[4] = {vs, vn, sdot, force};
  for (int k = 0; k < 4; ++k)
    if (dst[k] && n > 0) {
      c = copy_soa_to_host(h, src[k], n, dst[k]);
      if (c != VLB_OK) return c;
    }
  return latched(h);
}

int vlb_apply_topology(vlb_run* h, int64_t* stats) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  Run& r = h->r;
  HIP_OR_FAIL(h, topo_update(r, false));
  int32_t c[8];
  HIP_OR_FAIL(h, hipMemcpyAsync(c, r.cnt, sizeof(c), hipMemcpyDeviceToHost, r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  if (stats) {
    stats[0] = c[3];
    stats[1] = c[2];
    stats[2] = c[4];
    stats[3] = c[5];
  }
  return latched(h);
}

int vlb_set_friction_profile(vlb_run* h, const double* alpha_z, const double* alpha_p_z) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if ((alpha_z == nullptr) != (alpha_p_z == nullptr))
    return fail(h, VLB_EINVAL, "give both profiles or neither");
  Run& r = h->r;
  const int nz = r.geom.nz;
  std::vector<double> buf(2 * (size_t)nz + 1, 0.0);
  if (alpha_z) {
    for (int z = 0; z < nz; ++z) {
      if (!std::isfinite(alpha_z[z]) || !std::isfinite(alpha_p_z[z]))
        return fail(h, VLB_EINVAL, "non-finite friction coefficient");
      buf[z] = alpha_z[z];
      buf[nz + z] = alpha_p_z[z];
    }
    buf[2 * (size_t)nz] = 1.0;
  }
  // ordered after the work already on the run's stream; later steps (and
  // graph launches) read the new values
  HIP_OR_FAIL(h, hipMemcpyAsync(r.fric, buf.data(), buf.size() * sizeof(double),
                                hipMemcpyHostToDevice, r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  return VLB_OK;
}

int vlb_line_length(vlb_run* h, double* total, double* per_slab) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!total && !per_slab) return fail(h, VLB_EINVAL, "total and per_slab are both NULL");
  Run& r = h->r;
  const int nz = r.geom.nz;
  HIP_OR_FAIL(h, diag_line_length(r, total ? r.diag : nullptr, per_slab ? r.diag + 8 : nullptr));
  if (total)
    HIP_OR_FAIL(h, hipMemcpyAsync(total, r.diag, sizeof(double), hipMemcpyDeviceToHost, r.stream));
  std::vector<double> part(per_slab ? (size_t)kSlabChunks * nz : 0);
  if (per_slab)
    HIP_OR_FAIL(h, hipMemcpyAsync(part.data(), r.diag + 8, part.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  if (per_slab)  // the chunks' parts of each slab, added in chunk order
    for (int z = 0; z < nz; ++z) {
      double t = 0.0;
      for (int c = 0; c < kSlabChunks; ++c) t += part[(size_t)c * nz + z];
      per_slab[z] = t;
    }
  return latched(h);
}

int vlb_flow_stats(vlb_run* h, double* slice_mean, double* slice_rms, double* mean, double* rms) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  Run& r = h->r;
  const int nz = r.geom.nz;
  HIP_OR_FAIL(h, lbm_flow_stats(r, r.diag + 8));
  std::vector<double> st(6 * (size_t)nz);
  HIP_OR_FAIL(h, hipMemcpyAsync(st.data(), r.diag + 8, st.size() * sizeof(double),
                                hipMemcpyDeviceToHost, r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  // slices hold the same number of nodes: the lattice mean is the mean of
  // the slice means, and the lattice sum of squared deviations adds each
  // slice's own and its mean's offset from the lattice mean
  const double ns = (double)r.geom.nx * r.geom.ny;
  double m[3] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0};
  for (int z = 0; z < nz; ++z)
    for (int a = 0; a < 3; ++a) m[a] += st[6 * z + a];
  for (int a = 0; a < 3; ++a) m[a] /= nz;
  for (int z = 0; z < nz; ++z)
    for (int a = 0; a < 3; ++a) {
      const double dm = st[6 * z + a] - m[a];
      q[a] += st[6 * z + 3 + a] + ns * dm * dm;
      if (slice_mean) slice_mean[3 * z + a] = st[6 * z + a];
      if (slice_rms) slice_rms[3 * z + a] = std::sqrt(st[6 * z + 3 + a] / ns);
    }
  for (int a = 0; a < 3; ++a) {
    if (mean) mean[a] = m[a];
    if (rms) rms[a] = std::sqrt(q[a] / (ns * nz));
  }
  return latched(h);
}

int vlb_read_vorticity(vlb_run* h, double* u_dev, double* omega_dev) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!u_dev || !omega_dev) return fail(h, VLB_EINVAL, "u and omega are required");
  Run& r = h->r;
  HIP_OR_FAIL(h, lbm_read_fields(r, nullptr, u_dev));
  HIP_OR_FAIL(h, diag_curl(r, u_dev, omega_dev));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  return latched(h);
}

int vlb_vorticity_cylindrical(vlb_run* h, const double* point, const double* direction,
                              const double* omega_dev, double* out_dev) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!point || !direction || !omega_dev || !out_dev) return fail(h, VLB_EINVAL, "null argument");
  double a[3] = {direction[0], direction[1], direction[2]};
  const double nn = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  if (!(nn > 0.0) || !std::isfinite(nn) || !std::isfinite(point[0]) || !std::isfinite(point[1]) ||
      !std::isfinite(point[2]))
    return fail(h, VLB_EINVAL, "need a finite point and a non-zero finite direction");
  for (double& v : a) v /= nn;
  HIP_OR_FAIL(h, diag_cylindrical(h->r, point, a, omega_dev, out_dev));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->r.stream));
  return latched(h);
}

int vlb_get_step(vlb_run* h, int64_t* step) {
  if (!h || !step) return fail(h, VLB_EINVAL, "null argument");
  *step = h->r.step;
  return VLB_OK;
}

int vlb_set_timing(vlb_run* h, int32_t enable) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  Run& r = h->r;
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  recycle_events(r);
  r.timing = enable != 0;
  // enable > 1 pre-creates that many events
  while (enable > 1 && (int64_t)r.ev_pool.size() < enable) {
    hipEvent_t e = nullptr;
    HIP_OR_FAIL(h, hipEventCreate(&e));
    r.ev_pool.push_back(e);
  }
  r.last_nodes = 0;
  r.last_pairs = 0;
  HIP_OR_FAIL(h, hipMemsetAsync(r.cnt + 16, 0, 8 * sizeof(int32_t), r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  return VLB_OK;
}

int vlb_get_timing(vlb_run* h, int32_t cls, double* total_ms, int64_t* launches) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (cls < 0 || cls > 1 || !total_ms || !launches) return fail(h, VLB_EINVAL, "bad timing query");
  Run& r = h->r;
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  double tot = 0.0;
  for (auto& p : r.ev_used[cls]) {
    float ms = 0.f;
    HIP_OR_FAIL(h, hipEventElapsedTime(&ms, p.first, p.second));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)r.ev_used[cls].size();
  return VLB_OK;
}

int vlb_time_kernel(vlb_run* h, int32_t cls, int32_t reps, double* avg_ms) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (cls < 0 || cls > 1 || reps < 1 || !avg_ms) return fail(h, VLB_EINVAL, "bad kernel timing request");
  Run& r = h->r;
  // the events and the timing flag are restored on every exit
  struct Guard {
    Run& r;
    bool was;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Guard() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      r.timing = was;
    }
  } gd{r, r.timing};
  r.timing = false;
  HIP_OR_FAIL(h, hipEventCreate(&gd.e0));
  HIP_OR_FAIL(h, hipEventCreate(&gd.e1));
  const bool ff = cls == 0 && r.vor.ff_cell > 0;
  if (cls == 0 && !ff) HIP_OR_FAIL(h, bs_prep(r, r.pos));
  HIP_OR_FAIL(h, hipEventRecord(gd.e0, r.stream));
  for (int k = 0; k < reps; ++k) {
    if (ff)
      HIP_OR_FAIL(h, ff_run_sum(r, r.pos));
    else if (cls == 0)
      HIP_OR_FAIL(h, bs_sum(r));
    else
      HIP_OR_FAIL(h, lbm_step(r));
  }
  HIP_OR_FAIL(h, hipEventRecord(gd.e1, r.stream));
  HIP_OR_FAIL(h, hipEventSynchronize(gd.e1));
  float ms = 0.f;
  HIP_OR_FAIL(h, hipEventElapsedTime(&ms, gd.e0, gd.e1));
  *avg_ms = (double)ms / reps;
  return latched(h);
}

int vlb_get_work(vlb_run* h, int64_t* node_updates, int64_t* bs_pairs) {
  if (!h || !node_updates || !bs_pairs) return fail(h, VLB_EINVAL, "null argument");
  Run& r = h->r;
  long long acc = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(&acc, r.cnt + 16, sizeof(long long), hipMemcpyDeviceToHost, r.stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(r.stream));
  *node_updates = r.last_nodes;
  *bs_pairs = acc;
  return VLB_OK;
}

int vlb_graph_create(vlb_run* h, int64_t n_steps, vlb_graph** out) {
  if (!h) return fail(nullptr, VLB_EINVAL, "run is NULL");
  if (!out || n_steps < 2 || (n_steps & 1)) return fail(h, VLB_EINVAL, "n_steps must be even and >= 2");
  Run& r = h->r;
  if (!r.stream) return fail(h, VLB_EINVAL, "graph capture needs a non-null stream");
  const int64_t step0 = r.step, nodes0 = r.last_nodes;
  const int parity0 = r.parity;
  const int pparity0 = r.point_parity;
  const bool timing0 = r.timing;
  // velocity fields: every call (and so every launch) starts with fresh
  // moments into the current one, so only the host's choice is restored
  void* const ub0 = r.ub;
  void* const ubn0 = r.ub_next;
  double* const vs0 = r.Vs;
  double* const vsn0 = r.Vs_next;
  r.timing = false;
  HIP_OR_FAIL(h, hipStreamBeginCapture(r.stream, hipStreamCaptureModeRelaxed));
  int code = VLB_OK;
  for (int64_t k = 0; k < n_steps && code == VLB_OK; ++k) code = one_step(h, k == 0, k == n_steps - 1);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(r.stream, &graph);
  r.step = step0;
  r.last_nodes = nodes0;
  r.parity = parity0;
  r.timing = timing0;
  r.ub = ub0;
  r.ub_next = ubn0;
  r.Vs = vs0;
  r.Vs_next = vsn0;
  if (r.point_parity != pparity0) {  // an odd number of compactions was captured
    std::swap(r.pos, r.pos_t);
    std::swap(r.nxt, r.nxt_t);
    std::swap(r.prv, r.prv_t);
    r.point_parity = pparity0;
  }
  if (code != VLB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return code;
  }
  if (ec != hipSuccess) return hip_fail(h, ec, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return hip_fail(h, ei, "hipGraphInstantiate");
  vlb_graph* g = new (std::nothrow) vlb_graph();
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    return fail(h, VLB_EINVAL, "out of host memory");
  }
  g->run = h;
  g->exec = exec;
  g->n_steps = n_steps;
  g->parity = parity0;
  g->point_parity = pparity0;
  g->has_points = r.has_points;
  *out = g;
  return VLB_OK;
}

int vlb_graph_launch(vlb_graph* g) {
  if (!g || !g->run) return fail(nullptr, VLB_EINVAL, "graph is NULL");
  vlb_run* h = g->run;
  Run& r = h->r;
  if (r.parity != g->parity || r.point_parity != g->point_parity)
    return fail(h, VLB_ESTATE, "run parity differs from the captured one");
  if (r.has_points != g->has_points)
    return fail(h, VLB_ESTATE, "filaments were seeded after the graph was captured");
  HIP_OR_FAIL(h, hipGraphLaunch(g->exec, r.stream));
  r.step += g->n_steps;
  r.last_nodes += g->n_steps * r.cells;
  return VLB_OK;
}

int vlb_graph_destroy(vlb_graph* g) {
  if (!g) return VLB_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  delete g;
  return VLB_OK;
}

int vlb_destroy(vlb_run* h) {
  if (!h) return VLB_OK;
  // teardown: a device error has nowhere to go any more (vlb_sync reports it)
  (void)hipStreamSynchronize(h->r.stream);
  if (h->r.side) (void)hipStreamSynchronize(h->r.side);
  drop_events(h->r);
  release_streams(h->r);
  delete h;
  return VLB_OK;
}

int vlb_biot_savart_workspace(const vlb_bs_desc* d, int64_t n_pts, uint64_t* bytes) {
  std::string msg;
  const int c = bs_check_desc(d, n_pts, msg);
  if (c != VLB_OK) return fail(nullptr, c, msg);
  if (!bytes) return fail(nullptr, VLB_EINVAL, "bytes is NULL");
  *bytes = n_pts > 0 ? (uint64_t)bs_solo_layout(d->precision, n_pts, nullptr, nullptr) : 0;
  return VLB_OK;
}

int vlb_biot_savart(const vlb_bs_desc* d, int64_t n_pts, const double* xyz_dev,
                    const int32_t* next_dev, double* v_dev, void* dev_workspace,
                    uint64_t ws_bytes, void* hip_stream) {
  std::string msg;
  const int c = bs_check_desc(d, n_pts, msg);
  if (c != VLB_OK) return fail(nullptr, c, msg);
  if (n_pts == 0) return VLB_OK;
  if (!xyz_dev || !next_dev || !v_dev || !dev_workspace)
    return fail(nullptr, VLB_EINVAL, "null device pointer");
  if ((uintptr_t)dev_workspace % 256) return fail(nullptr, VLB_EINVAL, "workspace not 256-byte aligned");
  BsSolo b;
  const size_t need = bs_solo_layout(d->precision, n_pts, (char*)dev_workspace, &b);
  if (ws_bytes < need) return fail(nullptr, VLB_ENOSPACE, "workspace smaller than vlb_biot_savart_workspace");
  const int n[3] = {d->nx, d->ny, d->nz};
  const int wall[3] = {(int)(d->wall_axes & 1u), (int)((d->wall_axes >> 1) & 1u),
                       (int)((d->wall_axes >> 2) & 1u)};
  const hipError_t e = bs_solo(bs_make_axes(n, wall, false), d->precision, n_pts, xyz_dev, next_dev,
                               d->kappa, v_dev, b, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "vlb_biot_savart");
  return VLB_OK;
}

int vlb_biot_savart_farfield_workspace(const vlb_bs_desc* d, const vlb_ff_params* p,
                                       int64_t n_pts, uint64_t* bytes) {
  std::string msg;
  const int c = ff_check(d, p, n_pts, msg);
  if (c != VLB_OK) return fail(nullptr, c, msg);
  if (!bytes) return fail(nullptr, VLB_EINVAL, "bytes is NULL");
  *bytes = n_pts > 0 ? (uint64_t)ff_workspace(d, p, n_pts) : 0;
  return VLB_OK;
}

int vlb_biot_savart_farfield(const vlb_bs_desc* d, const vlb_ff_params* p, int64_t n_pts,
                             const double* xyz_dev, const int32_t* next_dev, double* v_dev,
                             void* dev_workspace, uint64_t ws_bytes, void* hip_stream) {
  std::string msg;
  const int c = ff_check(d, p, n_pts, msg);
  if (c != VLB_OK) return fail(nullptr, c, msg);
  if (n_pts == 0) return VLB_OK;
  if (!xyz_dev || !next_dev || !v_dev || !dev_workspace)
    return fail(nullptr, VLB_EINVAL, "null device pointer");
  if ((uintptr_t)dev_workspace % 256) return fail(nullptr, VLB_EINVAL, "workspace not 256-byte aligned");
  if (ws_bytes < ff_workspace(d, p, n_pts))
    return fail(nullptr, VLB_ENOSPACE, "workspace smaller than vlb_biot_savart_farfield_workspace");
  const hipError_t e = ff_solo(d, p, n_pts, xyz_dev, next_dev, v_dev, dev_workspace,
                               (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "vlb_biot_savart_farfield");
  return VLB_OK;
}

const char* vlb_last_error(const vlb_run* h) {
  if (h) return h->r.err.c_str();
  std::lock_guard<std::mutex> lk(g_err_mu);
  return g_err.c_str();
}

}  // extern "C"
