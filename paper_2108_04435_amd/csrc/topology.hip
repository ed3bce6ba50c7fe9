// Filament topology (paper Sec. II.A: segment lengths kept between dxi_min
// and dxi_max; Sec. II.A / III.B: legs of two vortices exchanged when they
// come within the resolution), made data-parallel and deterministic:
//  * remeshing: of the points whose incoming segment is shorter than
//    dxi_min and whose removal leaves a chord no longer than dxi_max, every
//    other one along each run is deleted; every remaining
//    segment longer than dxi_max gets its midpoint, appended after the old
//    points in ascending segment order;
//  * reconnection: candidate pairs (i < j, more than two links apart,
//    closer than the reconnection distance, exchange not lengthening the
//    line) are found through a cell binning and taken greedily in ascending
//    (d^2, i, j), each point at most once;
//  * loops with fewer than min_loop_pts points are removed, and the point
//    arrays are compacted in index order.
// All decisions compare FP64 squared distances summed as dx*dx + dy*dy +
// dz*dz with no fused multiply-add, so the integer outcome is a fixed
// function of the positions.
#include <utility>

#include "vlb_internal.h"

#pragma clang fp contract(off)

namespace vlb {

namespace {

struct TopoGeom {
  double L[3];
  int periodic[3];
};

__device__ inline double sq3(const double d[3]) {
  return __dadd_rn(__dadd_rn(__dmul_rn(d[0], d[0]), __dmul_rn(d[1], d[1])), __dmul_rn(d[2], d[2]));
}

// d = s_j - s_i at the nearest periodic image
__device__ inline void sep(const double* __restrict__ pos, long long nc, int i, int j,
                           const TopoGeom& tg, double d[3]) {
  for (int a = 0; a < 3; ++a) {
    double x = __dsub_rn(pos[a * nc + j], pos[a * nc + i]);
    if (tg.periodic[a]) {
      if (x > 0.5 * tg.L[a])
        x = __dsub_rn(x, tg.L[a]);
      else if (x < -0.5 * tg.L[a])
        x = __dadd_rn(x, tg.L[a]);
    }
    d[a] = x;
  }
}

// the same from loaded positions: d = b - a at the nearest periodic image
__device__ inline void sep_v(const double a[3], const double b[3], const TopoGeom& tg,
                             double d[3]) {
  for (int k = 0; k < 3; ++k) {
    double x = __dsub_rn(b[k], a[k]);
    if (tg.periodic[k]) {
      if (x > 0.5 * tg.L[k])
        x = __dsub_rn(x, tg.L[k]);
      else if (x < -0.5 * tg.L[k])
        x = __dadd_rn(x, tg.L[k]);
    }
    d[k] = x;
  }
}

__device__ inline void load3(const double* __restrict__ pos, long long nc, int i, double y[3]) {
  y[0] = pos[i];
  y[1] = pos[nc + i];
  y[2] = pos[2 * nc + i];
}

// Index for loads issued before the point count is known: every slot below
// the capacity is read, stale links are clamped into the arrays, and only
// live points use what was read.
__device__ inline int clamp_index(long long x, long long nc) {
  return (int)(x < 0 ? 0 : (x >= nc ? nc - 1 : x));
}

__device__ inline double wrap1(double x, double L, int periodic) {
  if (periodic) {
    if (x < 0.0) x = __dadd_rn(x, L);
    if (x >= L) x = __dsub_rn(x, L);
    if (x >= L) x = 0.0;
  } else {
    const double lo = -0.5, hi = L - 0.5;
    if (x < lo) x = __dsub_rn(2.0 * lo, x);
    if (x > hi) x = __dsub_rn(2.0 * hi, x);
  }
  return x;
}

// ---- ranks of flagged points without a separate scan kernel.  Every wave
// stores the ballot of its flags and their count; the last block of the
// grid to arrive (integer ticket, reset by that block) turns the per-wave
// counts into exclusive prefixes.  The rank of a flagged point x is then
// pre[x / 64] + the flags below it in its wave.
constexpr int kBlock = 256;

__device__ inline uint64_t lanes_below(int lane) {
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__device__ inline int flag_rank(const uint64_t* __restrict__ mask, const int32_t* __restrict__ pre,
                                int x) {
  const int w = x >> 6;
  return pre[w] + __popcll(mask[w] & lanes_below(x & 63));
}

// Exclusive scan of a[0..n) in place by one block of kBlock threads.
__device__ void block_scan_inplace(int32_t* a, int n, int32_t* total) {
  __shared__ int32_t wsum[kBlock / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += 4 * kBlock) {
    const int k0 = base + 4 * t;
    int v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (k0 + q < n) ? a[k0 + q] : 0;
    const int mine = v[0] + v[1] + v[2] + v[3];
    int x = mine;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int before = 0, all = 0;
    for (int u = 0; u < kBlock / 64; ++u) {
      before += u < w ? wsum[u] : 0;
      all += wsum[u];
    }
    int run = carry + before + x - mine;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (k0 + q < n) a[k0 + q] = run;
      run += v[q];
    }
    carry += all;
    __syncthreads();
  }
  if (t == 0) *total = carry;
}

// Called by every thread of every block of a one-dimensional grid of kBlock
// threads (no thread may have returned before).
__device__ void wave_scan_commit(bool flag, uint64_t* __restrict__ mask, int32_t* __restrict__ pre,
                                 int32_t* ticket, int32_t* total) {
  __shared__ int s_last;
  const int t = threadIdx.x;
  const int w = (blockIdx.x * kBlock + t) >> 6;
  const uint64_t m = __ballot(flag);
  if ((t & 63) == 0) {
    mask[w] = m;
    pre[w] = __popcll(m);
  }
  // one device-scope fence per block, after the barrier that orders the
  // block's stores before it (the fence writes back the L2 as a whole)
  __syncthreads();
  if (t == 0) {
    __threadfence();
    s_last = atomicAdd(ticket, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  block_scan_inplace(pre, gridDim.x * (kBlock / 64), total);
  if (t == 0) *ticket = 0;
}

__global__ void k_reset_stats(int32_t* cnt) {
  if (threadIdx.x == 0) cnt[2] = cnt[3] = cnt[4] = cnt[5] = cnt[6] = 0;
}

// Deletion candidate (the test written out in k_rm_mark): not an end of an
// open line (those stay on their walls), the incoming segment is shorter
// than dxi_min, and the chord from the predecessor to the successor, which
// would replace the point's two segments, is not longer than dxi_max.

// Along each run of consecutive deletion candidates every other point is
// deleted: candidate j goes when the number c of candidates directly before
// it (walking back to the first point of the run, however long the run) is
// even; a loop made only of candidates is counted from its lowest index and
// keeps its last point when its length is odd.  No two neighbours are
// deleted, and every run is thinned in one pass.  Candidacy of the points
// walked over is evaluated on the way; a walk takes one round of loads per
// point, so its latency grows with the length of the run (runs are a few
// points long unless the input is over-resolved, and each pass halves
// them).  Block 0 also clears the step's statistics counters.

__global__ __launch_bounds__(kBlock) void k_rm_mark(const double* __restrict__ pos,
                                                    const int32_t* __restrict__ nxt,
                                                    const int32_t* __restrict__ prv,
                                                    int32_t* __restrict__ cnt, long long nc,
                                                    TopoGeom tg, double mn2, double mx2,
                                                    int32_t* __restrict__ del) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  // the point's links and the three positions of its candidacy test are
  // loaded before the point count arrives
  const int jc = clamp_index(j, nc);
  const int p0 = clamp_index(prv[jc], nc), q0 = clamp_index(nxt[jc], nc);
  double yj[3], yp[3], yq[3];
  load3(pos, nc, jc, yj);
  load3(pos, nc, p0, yp);
  load3(pos, nc, q0, yq);
  const int n = cnt[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[2] = cnt[3] = cnt[4] = cnt[5] = cnt[6] = 0;
  if (j >= n) return;
  int dd = 0;
  double d[3], c3[3];
  sep_v(yp, yj, tg, d);
  sep_v(yp, yq, tg, c3);
  const bool end = p0 == j || q0 == j;  // the first or the last point of an open line
  if (!end && sq3(d) < mn2 && sq3(c3) <= mx2) {  // j is a deletion candidate
    // walk back over the candidates before j: the candidacy of point p
    // needs the positions of its predecessor r, of p and of its successor
    // (the point walked from); r's predecessor is loaded together with r's
    // position, so every step costs one round of loads
    int c = 0, p = p0;
    double yc[3] = {yp[0], yp[1], yp[2]};  // position of p
    double ys[3] = {yj[0], yj[1], yj[2]};  // position of p's successor
    int r = clamp_index(prv[p], nc);
    // (a valid loop brings the walk back to j within n steps; the bound
    // only guarantees termination on corrupted links)
    while (p != j && c < n) {
      if (r == p) break;  // p is the first point of an open line: no candidate
      const int rr = clamp_index(prv[r], nc);
      double yr[3], e[3], f[3];
      load3(pos, nc, r, yr);
      sep_v(yr, yc, tg, e);
      sep_v(yr, ys, tg, f);
      if (!(sq3(e) < mn2 && sq3(f) <= mx2)) break;  // p is no deletion candidate
      ++c;
      for (int a = 0; a < 3; ++a) {
        ys[a] = yc[a];
        yc[a] = yr[a];
      }
      p = r;
      r = rr;
    }
    if (p == j) {
      const int L = c + 1;
      int m = j, tm = 0, q = j;
      for (int t = 1; t < L; ++t) {
        q = nxt[q];
        if (q < m) {
          m = q;
          tm = t;
        }
      }
      const int ps = (L - tm) % L;
      dd = ((ps & 1) == 0 && !(ps == L - 1 && (L & 1))) ? 1 : 0;
    } else {
      dd = (c & 1) == 0 ? 1 : 0;
    }
  }
  del[j] = dd;
}

// Deleted points are unlinked; every kept point whose segment (to its
// successor after the unlinking) is longer than dxi_max is flagged for a
// midpoint, and the flags are ranked.  A kept point may read its successor
// link before or after the deleted successor rewrote it: both lead to the
// same new successor, since deleted points have kept neighbours.
__global__ __launch_bounds__(kBlock) void k_rm_link(const double* __restrict__ pos,
                                                    int32_t* __restrict__ nxt,
                                                    int32_t* __restrict__ prv,
                                                    int32_t* __restrict__ cnt, long long nc,
                                                    TopoGeom tg, double mx2,
                                                    const int32_t* __restrict__ del,
                                                    uint64_t* __restrict__ imask,
                                                    int32_t* __restrict__ ipre,
                                                    int32_t* ticket) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  // loads before the point count arrives.  A deleted point's own links are
  // not rewritten here (its neighbours are kept); a kept point's successor
  // link may be read before or after a deleted successor rewrote it, and
  // both lead to the same new successor.
  const int jc = clamp_index(j, nc);
  const int dj0 = del[jc];
  const int p0 = prv[jc];
  const int s0 = __hip_atomic_load(&nxt[jc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double yj[3];
  load3(pos, nc, jc, yj);
  const int n = cnt[0];
  const bool valid = j < n;
  const int dj = valid ? dj0 : 0;
  bool ins = false;
  if (valid) {
    if (dj) {
      __hip_atomic_store(&nxt[p0], s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      prv[s0] = p0;
    } else {
      // the successor's flag, link and position in one round of loads; a
      // deleted successor's link is stable, a kept one's is not used
      const int ds = del[s0];
      const int ns = clamp_index(
          __hip_atomic_load(&nxt[s0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), nc);
      double ys[3], d[3];
      load3(pos, nc, s0, ys);
      if (ds) load3(pos, nc, ns, ys);
      sep_v(yj, ys, tg, d);
      ins = sq3(d) > mx2;
    }
  }
  const uint64_t dm = __ballot(dj != 0);
  if ((threadIdx.x & 63) == 0 && dm) atomicAdd(&cnt[3], (int)__popcll(dm));
  wave_scan_commit(ins, imask, ipre, ticket, cnt + 2);
}

// Midpoints of the flagged segments, appended at n + rank in ascending
// segment order; all or none (capacity).
__global__ __launch_bounds__(kBlock) void k_rm_insert(double* __restrict__ pos,
                                                      int32_t* __restrict__ nxt,
                                                      int32_t* __restrict__ prv,
                                                      int32_t* __restrict__ cnt, long long nc,
                                                      TopoGeom tg, int32_t* __restrict__ del,
                                                      const uint64_t* __restrict__ imask,
                                                      const int32_t* __restrict__ ipre) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  // loads before the point count arrives (only this thread rewrites the
  // successor link of point j here)
  const int jc = clamp_index(j, nc);
  const uint64_t mw = imask[jc >> 6];
  const int pw = ipre[jc >> 6];
  const int k = clamp_index(nxt[jc], nc);
  double yj[3], yk[3];
  load3(pos, nc, jc, yj);
  load3(pos, nc, k, yk);
  const int n = cnt[0];
  const int M = cnt[2];
  const bool fits = (long long)n + M <= nc;
  if (j == 0) {
    cnt[9] = fits ? n + M : n;
    if (!fits && M > 0) atomicOr(&cnt[7], kFlagCapacity);
  }
  if (j >= n || !fits || !((mw >> (j & 63)) & 1ull)) return;
  const int q = n + pw + __popcll(mw & lanes_below(j & 63));
  if (q >= nc) return;
  double d[3];
  sep_v(yj, yk, tg, d);
  for (int a = 0; a < 3; ++a)
    pos[a * nc + q] = wrap1(__dadd_rn(yj[a], 0.5 * d[a]), tg.L[a], tg.periodic[a]);
  nxt[j] = q;
  prv[q] = j;
  nxt[q] = k;
  prv[k] = q;
  del[q] = 0;
}

// ---- reconnection bins
struct BinGeom {
  int nb[3];
  double h[3];
  double off[3];  // 0.5 on wall axes (range starts at -1/2), 0 on periodic
  int periodic[3];
};

__device__ inline int bin_of(double x, const BinGeom& bg, int a) {
  int b = (int)floor((x + bg.off[a]) / bg.h[a]);
  if (b < 0) b = 0;
  if (b >= bg.nb[a]) b = bg.nb[a] - 1;
  return b;
}

// Small-loop pass over the points below the bound: a point is alive when
// it is kept (not deleted / alive before) and its filament has at least
// min_pts points (a closed loop, or an open line counted from its first to
// its last point).  Optionally the alive points are pushed on per-bin lists
// for the reconnection search (integer exchange on the bin head; the order
// inside a list is irrelevant, every consumer sorts what it collects), or
// the lists of an earlier pass are cleared, or the alive points are ranked
// for the compaction.
struct SmallArgs {
  const double* pos;
  const int32_t* nxt;
  const int32_t* prv;
  int32_t* cnt;
  long long nc;
  int bound9;               // 1: bound = cnt[9]; 0: bound = cnt[0], and cnt[9] := bound
  const int32_t* dead_in;   // 1 = deleted (or null)
  const int32_t* alive_in;  // 1 = alive before this pass (or null)
  int32_t* alive_out;       // or null
  int min_pts;
  int rc_mode;              // 0: none, 1: push on bin lists (and zero the
                            // candidate counts), 2: clear bin heads
  int32_t* rc_count;
  BinGeom bg;
  int32_t* rc_head;
  int32_t* rc_next;
  uint32_t* rc_key;
  uint64_t* mask;           // ranks of the alive points (null: none)
  int32_t* pre;
  int32_t* ticket;
};

__global__ __launch_bounds__(kBlock) void k_small_pass(SmallArgs A) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  const long long nc = A.nc;
  // the flags and the first links are loaded before the bound arrives
  const int jc = clamp_index(j, nc);
  const int dead0 = A.dead_in ? A.dead_in[jc] : 0;
  const int alive0 = A.alive_in ? A.alive_in[jc] : 1;
  const int f1 = A.nxt[jc], b1 = A.prv[jc];
  double yj[3] = {0.0, 0.0, 0.0};
  if (A.rc_mode == 1) load3(A.pos, nc, jc, yj);
  const uint32_t key0 = A.rc_mode == 2 ? A.rc_key[jc] : 0u;
  const int bound = A.bound9 ? A.cnt[9] : A.cnt[0];
  if (!A.bound9 && j == 0) A.cnt[9] = bound;
  const bool valid = j < bound;
  const bool in = valid && dead0 == 0 && alive0 != 0;
  bool alive = false;
  if (in) {
    // A loop is shorter than min_pts iff nxt^k(j) = j for some k <=
    // min_pts - 1: walking i links forward (f) and back (b) together,
    // f == prv^(i-1)(j) tests k = 2i - 1 and f == b tests k = 2i.  An open
    // line is shorter iff fe + be + 1 <= min_pts - 1, with fe (be) the
    // number of links from j to its last (first) point; a walk stops at the
    // end it reaches.  The walk ends once every loop length up to
    // min_pts - 1 has been tested and the line is known to be long enough.
    const int m1 = A.min_pts - 1;
    int f = j, b = j, fe = -1, be = -1;
    bool small = false;
    for (int i = 1; i <= m1 && !small; ++i) {
      const int bp = b;
      const int fn = fe >= 0 ? f : (i == 1 ? f1 : A.nxt[f]);
      const int bn = be >= 0 ? b : (i == 1 ? b1 : A.prv[b]);
      if (fe < 0 && fn == f) fe = i - 1;  // f is the last point of an open line
      if (be < 0 && bn == b) be = i - 1;  // b is the first point
      f = fn;
      b = bn;
      if (fe >= 0 && be >= 0)
        small = fe + be + 1 <= m1;
      else if (fe < 0 && be < 0 && 2 * i - 1 <= m1)
        small = f == bp || (2 * i <= m1 && f == b);
      const int lf = fe >= 0 ? fe : i, lb = be >= 0 ? be : i;
      if (2 * i >= m1 && lf + lb + 1 > m1) break;
    }
    alive = !small;
  }
  if (valid && A.alive_out) A.alive_out[j] = alive ? 1 : 0;
  if (valid && A.rc_mode == 1) A.rc_count[j] = 0;
  const uint64_t dm = __ballot(in && !alive);
  if ((threadIdx.x & 63) == 0 && dm) atomicAdd(&A.cnt[5], (int)__popcll(dm));
  if (A.rc_mode == 1 && alive) {
    const int bx = bin_of(yj[0], A.bg, 0);
    const int by = bin_of(yj[1], A.bg, 1);
    const int bz = bin_of(yj[2], A.bg, 2);
    const uint32_t key = (uint32_t)(((long long)bz * A.bg.nb[1] + by) * A.bg.nb[0] + bx);
    A.rc_key[j] = key;
    A.rc_next[j] = atomicExch(&A.rc_head[key], j);
  }
  if (A.rc_mode == 2 && in) A.rc_head[key0] = -1;
  if (A.mask) wave_scan_commit(alive, A.mask, A.pre, A.ticket, A.cnt + 8);
}

// Stable compaction of the alive points into the other point arrays, links
// renumbered through the ranks.  In a step the two sets of point arrays
// then swap roles (no copy back); the standalone topology call copies back.
// With X non-null the grid coordinates of the compacted positions are
// written for the FP32 Biot-Savart sum of the next step, and the point
// count is set (when no copy follows).
__device__ inline uint32_t grid_coord(double y, const BsAxes& ax, int a) {
  const double g = floor((y + ax.off[a]) * ax.q[a]);
  return ax.periodic[a] ? (uint32_t)(long long)g : (uint32_t)(int)(long long)g;
}

__global__ __launch_bounds__(kBlock) void k_compact_scatter(const double* __restrict__ pos,
                                                            const int32_t* __restrict__ nxt,
                                                            const int32_t* __restrict__ prv,
                                                            int32_t* __restrict__ cnt,
                                                            long long nc,
                                                            const uint64_t* __restrict__ mask,
                                                            const int32_t* __restrict__ pre,
                                                            double* __restrict__ pos_t,
                                                            int32_t* __restrict__ nxt_t,
                                                            int32_t* __restrict__ prv_t,
                                                            int set_count,
                                                            uint32_t* __restrict__ X, BsAxes ax) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  // loads before the bound arrives
  const int jc = clamp_index(j, nc);
  const uint64_t mw = mask[jc >> 6];
  const int pw = pre[jc >> 6];
  const int nj = clamp_index(nxt[jc], nc), pj = clamp_index(prv[jc], nc);
  double y[3];
  load3(pos, nc, jc, y);
  if (set_count && j == 0) cnt[0] = cnt[8];
  if (j >= cnt[9] || !((mw >> (j & 63)) & 1ull)) return;
  const int q = pw + __popcll(mw & lanes_below(j & 63));
  if (q >= nc) return;
  for (int a = 0; a < 3; ++a) {
    pos_t[a * nc + q] = y[a];
    if (X) X[a * nc + q] = grid_coord(y[a], ax, a);
  }
  nxt_t[q] = flag_rank(mask, pre, nj);
  prv_t[q] = flag_rank(mask, pre, pj);
}

// The copy also writes the 32-bit grid coordinates of the new positions
// for the FP32 Biot-Savart sum of the next step (X non-null).
__global__ __launch_bounds__(kBlock) void k_compact_copy(double* __restrict__ pos,
                                                         int32_t* __restrict__ nxt,
                                                         int32_t* __restrict__ prv,
                                                         int32_t* __restrict__ cnt, long long nc,
                                                         const double* __restrict__ pos_t,
                                                         const int32_t* __restrict__ nxt_t,
                                                         const int32_t* __restrict__ prv_t,
                                                         uint32_t* __restrict__ X, BsAxes ax) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  const int nn = cnt[8];
  if (q == 0) cnt[0] = nn;
  if (q >= nn) return;
  for (int a = 0; a < 3; ++a) {
    const double y = pos_t[a * nc + q];
    pos[a * nc + q] = y;
    if (X) X[a * nc + q] = grid_coord(y, ax, a);
  }
  nxt[q] = nxt_t[q];
  prv[q] = prv_t[q];
}

// ---- reconnection search
// Offsets of the neighbouring bins along one axis (no duplicates when the
// periodic axis has fewer than 3 bins).
__device__ inline int bin_offsets(const BinGeom& bg, int a, int b, int out[3]) {
  int m = 0;
  for (int o = -1; o <= 1; ++o) {
    int c = b + o;
    if (bg.periodic[a]) {
      if (bg.nb[a] == 1 && o != 0) continue;
      if (bg.nb[a] == 2 && o == -1) continue;
      c = (c + bg.nb[a]) % bg.nb[a];
    } else if (c < 0 || c >= bg.nb[a]) {
      continue;
    }
    out[m++] = c;
  }
  return m;
}

// One thread per (alive point i, neighbouring bin q): every alive j > i in
// bin q, more than two links away, closer than the reconnection distance,
// whose exchange does not lengthen the line, takes the next of i's slots
// (integer add on i's count) with the bits of d^2 as its key.  The slot
// order depends on timing; the matching kernel orders each point's slots
// by j, so the candidate list is a fixed function of the positions.  A
// point with more candidates than slots latches the reconnection-capacity
// flag and the step skips reconnection (the candidate set must be
// complete).  The counts start at zero (first small-loop pass); the q = 0
// thread clears the point's `used` flag.
constexpr int kSlots = 8;

__global__ __launch_bounds__(kBlock) void k_rc_find(const double* __restrict__ pos,
                                                    const int32_t* __restrict__ nxt,
                                                    const int32_t* __restrict__ prv,
                                                    const int32_t* __restrict__ head,
                                                    const int32_t* __restrict__ lnext,
                                                    const int32_t* __restrict__ alive,
                                                    int32_t* __restrict__ cnt, long long nc,
                                                    TopoGeom tg, BinGeom bg, double d2max,
                                                    int32_t* __restrict__ count,
                                                    int32_t* __restrict__ slot_j,
                                                    uint64_t* __restrict__ slot_k,
                                                    int32_t* __restrict__ used) {
  const long long id = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int i = (int)(id / 27), q = (int)(id % 27);
  // the point's flag, position and links are loaded before the bound arrives
  const int ic = clamp_index(i, nc);
  const int alive0 = alive[ic];
  double yi[3];
  load3(pos, nc, ic, yi);
  const int ni0 = clamp_index(nxt[ic], nc), pi0 = clamp_index(prv[ic], nc);
  if (i >= cnt[9]) return;
  if (q == 0) used[i] = 0;
  // the last point of an open line has no segment to exchange
  if (!alive0 || ni0 == i) return;
  const int b[3] = {bin_of(yi[0], bg, 0), bin_of(yi[1], bg, 1), bin_of(yi[2], bg, 2)};
  int ox[3], oy[3], oz[3];
  const int mx = bin_offsets(bg, 0, b[0], ox);
  const int my = bin_offsets(bg, 1, b[1], oy);
  const int mz = bin_offsets(bg, 2, b[2], oz);
  const int ix = q % 3, iy = (q / 3) % 3, iz = q / 9;
  if (ix >= mx || iy >= my || iz >= mz) return;
  const long long key = ((long long)oz[iz] * bg.nb[1] + oy[iy]) * bg.nb[0] + ox[ix];
  int j = head[key];
  if (j < 0) return;
  const int ni = ni0, nni = nxt[ni], pi = pi0, ppi = prv[pi];
  const int bound = cnt[9];
  for (int guard = 0; j >= 0 && guard < bound; ++guard) {  // bounded by the point count
    const int jc = j;
    j = lnext[jc];
    if (jc <= i || jc == ni || jc == nni || jc == pi || jc == ppi) continue;
    double d[3];
    sep(pos, nc, i, jc, tg, d);
    const double d2 = sq3(d);
    if (!(d2 < d2max)) continue;
    const int nj = nxt[jc];
    if (nj == jc) continue;  // the last point of an open line
    double ea[3], eb[3], ec[3], ee[3];
    sep(pos, nc, i, ni, tg, ea);
    sep(pos, nc, jc, nj, tg, eb);
    sep(pos, nc, i, nj, tg, ec);
    sep(pos, nc, jc, ni, tg, ee);
    const double before = __dadd_rn(sqrt(sq3(ea)), sqrt(sq3(eb)));
    const double after = __dadd_rn(sqrt(sq3(ec)), sqrt(sq3(ee)));
    if (!(after <= before)) continue;
    const int slot = atomicAdd(&count[i], 1);
    if (slot < kSlots) {
      slot_j[(long long)i * kSlots + slot] = jc;
      slot_k[(long long)i * kSlots + slot] = (uint64_t)__double_as_longlong(d2);
    } else {
      atomicOr(&cnt[7], kFlagReconCap);
      atomicOr(&cnt[10], 1);
    }
  }
}

// Greedy matching in ascending (d^2, i, j), one workgroup.  First the
// per-point slots are gathered into one list in (i, j) order (a block scan
// of the counts); a slot overflow or a list longer than its capacity
// leaves the list empty.  Then rounds: a live candidate whose key is the
// smallest among the live candidates at both of its points is taken (the
// globally smallest one always is, and no candidate of smaller key can
// claim its points later), its points are used, and every candidate
// touching a used point dies.  The set taken is exactly the one of the
// sequential greedy pass.  Taken exchanges are disjoint, so their link
// updates do not interact.  Values that atomics update are read and
// written with device-scope atomics.
constexpr int kMatchPer = 16;  // points per thread in the slot gather of k_rc_match

__global__ __launch_bounds__(1024) void k_rc_match(int32_t* __restrict__ nxt,
                                                   int32_t* __restrict__ prv,
                                                   int32_t* __restrict__ cnt, long long rcap,
                                                   const int32_t* __restrict__ count,
                                                   const int32_t* __restrict__ slot_j,
                                                   const uint64_t* __restrict__ slot_k,
                                                   int32_t* __restrict__ ci,
                                                   int32_t* __restrict__ cj,
                                                   uint64_t* __restrict__ ckey,
                                                   int32_t* __restrict__ live,
                                                   uint64_t* __restrict__ bkey,
                                                   int32_t* __restrict__ bidx,
                                                   int32_t* __restrict__ used) {
  __shared__ int32_t wsum[16];
  __shared__ int s_live;
  __shared__ int s_taken;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int n = cnt[9];
  const bool overflow = cnt[10] != 0;
  // gather the slots in (i, j) order: exclusive scan of the counts,
  // kMatchPer points per thread (one round up to 16384 points, vector loads
  // where the round is full); a point's slots go to their rank by j
  int carry = 0;
  for (int base = 0; base < n; base += kMatchPer * 1024) {
    const int k0 = base + kMatchPer * t;
    int v[kMatchPer];
    if (k0 + kMatchPer <= n) {
      const int4* p = reinterpret_cast<const int4*>(count + k0);
#pragma unroll
      for (int q = 0; q < kMatchPer / 4; ++q) {
        const int4 c4 = p[q];
        v[4 * q] = c4.x;
        v[4 * q + 1] = c4.y;
        v[4 * q + 2] = c4.z;
        v[4 * q + 3] = c4.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < kMatchPer; ++q) v[q] = (k0 + q < n) ? count[k0 + q] : 0;
    }
    int mine = 0;
#pragma unroll
    for (int q = 0; q < kMatchPer; ++q) {
      v[q] = min(v[q], kSlots);
      mine += v[q];
    }
    int x = mine;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int before = 0, all = 0;
    for (int u = 0; u < 16; ++u) {
      before += u < w ? wsum[u] : 0;
      all += wsum[u];
    }
    int run = carry + before + x - mine;
    if (!overflow) {
#pragma unroll
      for (int q = 0; q < kMatchPer; ++q) {
        const int32_t* sj = slot_j + (long long)(k0 + q) * kSlots;
        for (int m = 0; m < v[q]; ++m) {
          const int jm = sj[m];
          int rk = 0;
          for (int u = 0; u < v[q]; ++u) rk += sj[u] < jm ? 1 : 0;
          const int o = run + rk;
          if (o < rcap) {
            ci[o] = k0 + q;
            cj[o] = jm;
            ckey[o] = slot_k[(long long)(k0 + q) * kSlots + m];
          }
        }
        run += v[q];
      }
    }
    carry += all;
    __syncthreads();
  }
  if (t == 0) {
    cnt[6] = carry;
    if (carry > rcap) atomicOr(&cnt[7], kFlagReconCap);
  }
  const int tot = (overflow || carry > rcap) ? 0 : carry;
  for (int c = t; c < tot; c += blockDim.x) live[c] = 1;
  if (t == 0) s_taken = 0;
  __syncthreads();
  for (int round = 0; round <= tot; ++round) {
    for (int c = t; c < tot; c += blockDim.x)
      if (live[c]) {
        __hip_atomic_store(&bkey[ci[c]], ~(uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&bkey[cj[c]], ~(uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&bidx[ci[c]], 0x7fffffff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&bidx[cj[c]], 0x7fffffff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    __syncthreads();
    for (int c = t; c < tot; c += blockDim.x)
      if (live[c]) {
        atomicMin((unsigned long long*)&bkey[ci[c]], (unsigned long long)ckey[c]);
        atomicMin((unsigned long long*)&bkey[cj[c]], (unsigned long long)ckey[c]);
      }
    __syncthreads();
    for (int c = t; c < tot; c += blockDim.x)
      if (live[c]) {
        const uint64_t k = ckey[c];
        if (__hip_atomic_load(&bkey[ci[c]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == k)
          atomicMin(&bidx[ci[c]], c);
        if (__hip_atomic_load(&bkey[cj[c]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == k)
          atomicMin(&bidx[cj[c]], c);
      }
    __syncthreads();
    for (int c = t; c < tot; c += blockDim.x)
      if (live[c]) {
        const int i = ci[c], j = cj[c];
        if (__hip_atomic_load(&bidx[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == c &&
            __hip_atomic_load(&bidx[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == c) {
          const int a = nxt[i], b = nxt[j];
          nxt[i] = b;
          prv[b] = i;
          nxt[j] = a;
          prv[a] = j;
          used[i] = 1;
          used[j] = 1;
          live[c] = 0;
          atomicAdd(&s_taken, 1);
        }
      }
    if (t == 0) s_live = 0;
    __syncthreads();
    int mine = 0;
    for (int c = t; c < tot; c += blockDim.x)
      if (live[c]) {
        if (used[ci[c]] || used[cj[c]])
          live[c] = 0;
        else
          ++mine;
      }
    if (mine) atomicAdd(&s_live, mine);
    __syncthreads();
    if (s_live == 0) break;
    __syncthreads();
  }
  if (t == 0) {
    cnt[4] = s_taken;
    cnt[10] = 0;
  }
}

inline int nb_of(long long n, int b) { return (int)((n + b - 1) / b); }

TopoGeom topo_geom(const Run& r) {
  TopoGeom tg;
  const int n[3] = {r.geom.nx, r.geom.ny, r.geom.nz};
  for (int a = 0; a < 3; ++a) {
    tg.L[a] = (double)n[a];
    tg.periodic[a] = !r.geom.wall[a];
  }
  return tg;
}

BinGeom bin_geom(const Run& r) {
  BinGeom bg;
  for (int a = 0; a < 3; ++a) {
    bg.nb[a] = r.bin_n[a];
    bg.h[a] = r.bin_h[a];
    bg.periodic[a] = !r.geom.wall[a];
    bg.off[a] = r.geom.wall[a] ? 0.5 : 0.0;
  }
  return bg;
}

}  // namespace

// Topology of one step: remeshing (mark, unlink + rank the midpoints,
// insert), then the small-loop pass, the reconnection search and matching
// and a second small-loop pass, and one compaction.  The reconnection runs
// on the uncompacted arrays: deleted points and removed small loops are
// unlinked from the alive ones, and renumbering by a stable compaction
// keeps the (d^2, i, j) order of every candidate pair, so the outcome is
// the one of compacting before reconnecting.
hipError_t topo_update(Run& r, bool swap) {
  const TopoGeom tg = topo_geom(r);
  const int nb = nb_of(r.ncap, kBlock);
  int32_t* del = r.flag_b;
  int32_t* ticket = r.cnt + 12;
  if (r.vor.remesh) {
    const double mn2 = r.vor.dxi_min * r.vor.dxi_min;
    const double mx2 = r.vor.dxi_max * r.vor.dxi_max;
    hipLaunchKernelGGL(k_rm_mark, dim3(nb), dim3(kBlock), 0, r.stream, r.pos, r.nxt, r.prv, r.cnt,
                       r.ncap, tg, mn2, mx2, del);
    hipLaunchKernelGGL(k_rm_link, dim3(nb), dim3(kBlock), 0, r.stream, r.pos, r.nxt, r.prv, r.cnt,
                       r.ncap, tg, mx2, del, r.wmask, r.wpre, ticket);
    hipLaunchKernelGGL(k_rm_insert, dim3(nb), dim3(kBlock), 0, r.stream, r.pos, r.nxt, r.prv,
                       r.cnt, r.ncap, tg, del, r.wmask, r.wpre);
  } else {
    hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(64), 0, r.stream, r.cnt);
  }
  SmallArgs A{};
  A.pos = r.pos;
  A.nxt = r.nxt;
  A.prv = r.prv;
  A.cnt = r.cnt;
  A.nc = r.ncap;
  A.bound9 = r.vor.remesh ? 1 : 0;
  A.dead_in = r.vor.remesh ? del : nullptr;
  A.min_pts = r.vor.min_loop_pts;
  A.ticket = ticket;
  if (r.vor.reconnect) {
    const BinGeom bg = bin_geom(r);
    A.bg = bg;
    A.rc_head = r.rc_head;
    A.rc_next = r.rc_next;
    A.rc_key = r.rc_keyp;
    A.rc_count = r.scan_a;
    A.alive_out = r.flag_a;
    A.rc_mode = 1;
    hipLaunchKernelGGL(k_small_pass, dim3(nb), dim3(kBlock), 0, r.stream, A);
    const double d2max = r.vor.reconnect_dist * r.vor.reconnect_dist;
    hipLaunchKernelGGL(k_rc_find, dim3(nb_of(27 * r.ncap, kBlock)), dim3(kBlock), 0, r.stream, r.pos, r.nxt, r.prv,
                       r.rc_head, r.rc_next, r.flag_a, r.cnt, r.ncap, tg, bg, d2max, r.scan_a,
                       r.rc_slot_j, r.rc_slot_k, r.used);
    hipLaunchKernelGGL(k_rc_match, dim3(1), dim3(1024), 0, r.stream, r.nxt, r.prv, r.cnt, r.rcap,
                       r.scan_a, r.rc_slot_j, r.rc_slot_k, r.rc_i, r.rc_j, r.rc_key_a,
                       r.rc_idx_a, r.rc_best, r.rc_bidx, r.used);
    SmallArgs B = A;
    B.bound9 = 1;
    B.dead_in = nullptr;
    B.alive_in = r.flag_a;
    B.alive_out = nullptr;
    B.rc_mode = 2;
    B.mask = r.wmask;
    B.pre = r.wpre;
    hipLaunchKernelGGL(k_small_pass, dim3(nb), dim3(kBlock), 0, r.stream, B);
  } else {
    A.mask = r.wmask;
    A.pre = r.wpre;
    hipLaunchKernelGGL(k_small_pass, dim3(nb), dim3(kBlock), 0, r.stream, A);
  }
  uint32_t* X = r.prec == VLB_F64 ? nullptr : r.bsX;
  if (swap) {
    hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(kBlock), 0, r.stream, r.pos, r.nxt, r.prv,
                       r.cnt, r.ncap, r.wmask, r.wpre, r.pos_t, r.nxt_t, r.prv_t, 1, X, r.bsax);
    std::swap(r.pos, r.pos_t);
    std::swap(r.nxt, r.nxt_t);
    std::swap(r.prv, r.prv_t);
    r.point_parity ^= 1;
  } else {
    hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(kBlock), 0, r.stream, r.pos, r.nxt, r.prv,
                       r.cnt, r.ncap, r.wmask, r.wpre, r.pos_t, r.nxt_t, r.prv_t, 0, nullptr,
                       r.bsax);
    hipLaunchKernelGGL(k_compact_copy, dim3(nb), dim3(kBlock), 0, r.stream, r.pos, r.nxt, r.prv,
                       r.cnt, r.ncap, r.pos_t, r.nxt_t, r.prv_t, X, r.bsax);
  }
  return hipGetLastError();
}

}  // namespace vlb
