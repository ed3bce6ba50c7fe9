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

// ---- single-workgroup exclusive scan of n ints (n read from *np): tiles
// of 4096 values, 4 consecutive values per thread, wave prefix sums with
// shuffles, wave totals combined in LDS, a running carry between tiles.
__global__ __launch_bounds__(1024) void k_scan_excl(const int32_t* __restrict__ in,
                                                    int32_t* __restrict__ out,
                                                    const int32_t* __restrict__ np, int nconst,
                                                    int32_t* __restrict__ total) {
  __shared__ int32_t wsum[16];
  const int n = np ? *np : nconst;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += 4096) {
    const int k0 = base + 4 * t;
    int v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (k0 + q < n) ? in[k0 + q] : 0;
    const int mine = v[0] + v[1] + v[2] + v[3];
    int x = mine;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
      int s = lane < 16 ? wsum[lane] : 0;
      for (int off = 1; off < 16; off <<= 1) {
        const int y = __shfl_up(s, off, 64);
        if (lane >= off) s += y;
      }
      if (lane < 16) wsum[lane] = s;
    }
    __syncthreads();
    int run = carry + (w > 0 ? wsum[w - 1] : 0) + x - mine;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (k0 + q < n) out[k0 + q] = run;
      run += v[q];
    }
    carry += wsum[15];
    __syncthreads();
  }
  if (t == 0) *total = carry;
}

__global__ void k_reset_stats(int32_t* cnt) {
  if (threadIdx.x == 0) {
    cnt[2] = cnt[3] = cnt[4] = cnt[5] = cnt[6] = 0;
    cnt[9] = cnt[0];
  }
}

// Deletion candidate: incoming segment shorter than dxi_min, and the chord
// that would replace the point's two segments not longer than dxi_max.
__global__ void k_rm_cand(const double* __restrict__ pos, const int32_t* __restrict__ nxt,
                          const int32_t* __restrict__ prv, const int32_t* __restrict__ cnt,
                          long long nc, TopoGeom tg, double mn2, double mx2,
                          int32_t* __restrict__ cand) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt[0]) return;
  double d[3], c[3];
  sep(pos, nc, prv[j], j, tg, d);
  sep(pos, nc, prv[j], nxt[j], tg, c);
  cand[j] = (sq3(d) < mn2 && sq3(c) <= mx2) ? 1 : 0;
}

// Along each run of consecutive deletion candidates every other point is
// deleted: candidate j goes when the number c of candidates directly before
// it (walking back, at most kChainLimit) is even and below the limit; a
// loop made only of candidates is counted from its lowest index and keeps
// its last point when its length is odd.  No two neighbours are deleted.
constexpr int kChainLimit = 32;

__global__ void k_rm_del(const int32_t* __restrict__ nxt, const int32_t* __restrict__ prv,
                         int32_t* __restrict__ cnt, const int32_t* __restrict__ cand,
                         int32_t* __restrict__ del) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt[0]) return;
  int dd = 0;
  if (cand[j]) {
    int c = 0, p = prv[j];
    while (c < kChainLimit && cand[p] && p != j) {
      ++c;
      p = prv[p];
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
      const int pos = (L - tm) % L;
      dd = ((pos & 1) == 0 && !(pos == L - 1 && (L & 1))) ? 1 : 0;
    } else {
      dd = (c < kChainLimit && (c & 1) == 0) ? 1 : 0;
    }
  }
  del[j] = dd;
  if (dd) atomicAdd(&cnt[3], 1);
}

__global__ void k_rm_relink(int32_t* __restrict__ nxt, int32_t* __restrict__ prv,
                            const int32_t* __restrict__ cnt, const int32_t* __restrict__ del) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt[0] || !del[j]) return;
  const int p = prv[j], q = nxt[j];
  nxt[p] = q;
  prv[q] = p;
}

__global__ void k_rm_insmark(const double* __restrict__ pos, const int32_t* __restrict__ nxt,
                             const int32_t* __restrict__ cnt, long long nc, TopoGeom tg,
                             double mx2, const int32_t* __restrict__ del, int32_t* __restrict__ ins) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt[0]) return;
  int v = 0;
  if (!del[j]) {
    double d[3];
    sep(pos, nc, j, nxt[j], tg, d);
    v = sq3(d) > mx2 ? 1 : 0;
  }
  ins[j] = v;
}

__global__ void k_rm_insert(double* __restrict__ pos, int32_t* __restrict__ nxt,
                            int32_t* __restrict__ prv, int32_t* __restrict__ cnt, long long nc,
                            TopoGeom tg, int32_t* __restrict__ del, const int32_t* __restrict__ ins,
                            const int32_t* __restrict__ rank) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = cnt[0];
  const int M = cnt[2];
  const bool fits = (long long)n + M <= nc;
  if (j == 0) {
    cnt[9] = fits ? n + M : n;
    if (!fits && M > 0) atomicOr(&cnt[7], kFlagCapacity);
  }
  if (j >= n || !fits || !ins[j]) return;
  const int q = n + rank[j];
  const int k = nxt[j];
  double d[3];
  sep(pos, nc, j, k, tg, d);
  for (int a = 0; a < 3; ++a)
    pos[a * nc + q] = wrap1(__dadd_rn(pos[a * nc + j], 0.5 * d[a]), tg.L[a], tg.periodic[a]);
  nxt[j] = q;
  prv[q] = j;
  nxt[q] = k;
  prv[k] = q;
  del[q] = 0;
}

// alive = not deleted and not on a loop with fewer than min_pts points
__global__ void k_small(const int32_t* __restrict__ nxt, int32_t* __restrict__ cnt,
                        const int32_t* __restrict__ del, int min_pts, int32_t* __restrict__ alive) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt[9]) return;
  if (del[j]) {
    alive[j] = 0;
    return;
  }
  int p = nxt[j];
  int steps = 1;
  while (p != j && steps < min_pts) {
    p = nxt[p];
    ++steps;
  }
  const int dead = (p == j && steps < min_pts) ? 1 : 0;
  alive[j] = 1 - dead;
  if (dead) atomicAdd(&cnt[5], 1);
}

__global__ void k_compact_scatter(const double* __restrict__ pos, const int32_t* __restrict__ nxt,
                                  const int32_t* __restrict__ prv, const int32_t* __restrict__ cnt,
                                  long long nc, const int32_t* __restrict__ alive,
                                  const int32_t* __restrict__ idx, double* __restrict__ pos_t,
                                  int32_t* __restrict__ nxt_t, int32_t* __restrict__ prv_t) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt[9] || !alive[j]) return;
  const int q = idx[j];
  for (int a = 0; a < 3; ++a) pos_t[a * nc + q] = pos[a * nc + j];
  nxt_t[q] = idx[nxt[j]];
  prv_t[q] = idx[prv[j]];
}

__global__ void k_compact_copy(double* __restrict__ pos, int32_t* __restrict__ nxt,
                               int32_t* __restrict__ prv, int32_t* __restrict__ cnt, long long nc,
                               const double* __restrict__ pos_t, const int32_t* __restrict__ nxt_t,
                               const int32_t* __restrict__ prv_t) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int nn = cnt[8];
  if (q == 0) cnt[0] = nn;
  if (q >= nn) return;
  for (int a = 0; a < 3; ++a) pos[a * nc + q] = pos_t[a * nc + q];
  nxt[q] = nxt_t[q];
  prv[q] = prv_t[q];
}

__global__ void k_fill(int32_t* __restrict__ p, long long n, int32_t v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- reconnection
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

__global__ void k_rc_keys(const double* __restrict__ pos, const int32_t* __restrict__ cnt,
                          long long nc, BinGeom bg, uint32_t pad, uint32_t* __restrict__ keys,
                          int32_t* __restrict__ vals) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  uint32_t k = pad;
  if (j < cnt[0]) {
    const int bx = bin_of(pos[j], bg, 0);
    const int by = bin_of(pos[nc + j], bg, 1);
    const int bz = bin_of(pos[2 * nc + j], bg, 2);
    k = (uint32_t)(((long long)bz * bg.nb[1] + by) * bg.nb[0] + bx);
  }
  keys[j] = k;
  vals[j] = j;
}

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

// Visit every candidate partner j > i of point i; calls f(j, d2).  The 27
// neighbouring bins are looked up first (independent loads), then walked.
template <class Fn>
__device__ inline void rc_visit(int i, const double* __restrict__ pos,
                                const int32_t* __restrict__ nxt, const int32_t* __restrict__ prv,
                                const uint32_t* __restrict__ skey, const int32_t* __restrict__ sval,
                                const int32_t* __restrict__ bins,
                                int n, long long nc, const TopoGeom& tg, const BinGeom& bg,
                                double d2max, Fn f) {
  const int b[3] = {bin_of(pos[i], bg, 0), bin_of(pos[nc + i], bg, 1), bin_of(pos[2 * nc + i], bg, 2)};
  int ox[3], oy[3], oz[3];
  const int mx = bin_offsets(bg, 0, b[0], ox);
  const int my = bin_offsets(bg, 1, b[1], oy);
  const int mz = bin_offsets(bg, 2, b[2], oz);
  uint32_t kk[27];
  int first[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const int ix = q % 3, iy = (q / 3) % 3, iz = q / 9;
    const bool ok = ix < mx && iy < my && iz < mz;
    kk[q] = ok ? (uint32_t)(((long long)oz[ok ? iz : 0] * bg.nb[1] + oy[ok ? iy : 0]) * bg.nb[0] +
                            ox[ok ? ix : 0])
               : 0u;
    first[q] = ok ? bins[kk[q]] : -1;
  }
  const int ni = nxt[i], nni = nxt[ni], pi = prv[i], ppi = prv[pi];
  for (int q = 0; q < 27; ++q) {
    if (first[q] < 0) continue;
    const uint32_t k = kk[q];
    for (int t = first[q]; t < n && skey[t] == k; ++t) {
      const int j = sval[t];
      if (j <= i || j == ni || j == nni || j == pi || j == ppi) continue;
      double d[3];
      sep(pos, nc, i, j, tg, d);
      const double d2 = sq3(d);
      if (!(d2 < d2max)) continue;
      const int nj = nxt[j];
      double ea[3], eb[3], ec[3], ee[3];
      sep(pos, nc, i, ni, tg, ea);
      sep(pos, nc, j, nj, tg, eb);
      sep(pos, nc, i, nj, tg, ec);
      sep(pos, nc, j, ni, tg, ee);
      const double before = __dadd_rn(sqrt(sq3(ea)), sqrt(sq3(eb)));
      const double after = __dadd_rn(sqrt(sq3(ec)), sqrt(sq3(ee)));
      if (after <= before) f(j, d2);
    }
  }
}

// One search per point: candidates j > i go into the point's own slots
// (at most kSlots, kept sorted by j), with their count; a point with more
// candidates than slots latches the reconnection-capacity flag, and the
// step then skips reconnection (the candidate set must be complete).  The
// kernel also clears the point's `used` flag for the matching.
constexpr int kSlots = 8;

__global__ void k_rc_find(const double* __restrict__ pos, const int32_t* __restrict__ nxt,
                          const int32_t* __restrict__ prv, const uint32_t* __restrict__ skey,
                          const int32_t* __restrict__ sval, const int32_t* __restrict__ bins,
                          int32_t* __restrict__ cnt, long long nc, TopoGeom tg, BinGeom bg,
                          double d2max, int32_t* __restrict__ count, int32_t* __restrict__ slot_j,
                          uint64_t* __restrict__ slot_k, int32_t* __restrict__ used) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = cnt[0];
  if (i >= n) return;
  used[i] = 0;
  int m = 0;
  int32_t* sj = slot_j + (long long)i * kSlots;
  uint64_t* sk = slot_k + (long long)i * kSlots;
  rc_visit(i, pos, nxt, prv, skey, sval, bins, n, nc, tg, bg, d2max, [&](int j, double d2) {
    if (m < kSlots) {
      int p = m;
      while (p > 0 && sj[p - 1] > j) {
        sj[p] = sj[p - 1];
        sk[p] = sk[p - 1];
        --p;
      }
      sj[p] = j;
      sk[p] = (uint64_t)__double_as_longlong(d2);
    }
    ++m;
  });
  if (m > kSlots) {
    atomicOr(&cnt[7], kFlagReconCap);
    atomicOr(&cnt[10], 1);
  }
  count[i] = m < kSlots ? m : kSlots;
}

// Candidates in (i, j) order into the compact list; overflow of the list or
// of a point's slots leaves the list empty (reconnection skipped).
__global__ void k_rc_compact(const int32_t* __restrict__ count, const int32_t* __restrict__ off,
                             const int32_t* __restrict__ slot_j, const uint64_t* __restrict__ slot_k,
                             int32_t* __restrict__ cnt, long long rcap, int32_t* __restrict__ ci,
                             int32_t* __restrict__ cj, uint64_t* __restrict__ ckey) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = cnt[0];
  const bool skip = cnt[10] != 0 || cnt[6] > rcap;
  if (i == 0 && cnt[6] > rcap) atomicOr(&cnt[7], kFlagReconCap);
  if (i >= n || skip) return;
  const int o = off[i];
  for (int m = 0; m < count[i]; ++m) {
    ci[o + m] = i;
    cj[o + m] = slot_j[(long long)i * kSlots + m];
    ckey[o + m] = slot_k[(long long)i * kSlots + m];
  }
}

// Greedy matching in ascending (d^2, i, j), computed in rounds: a live
// candidate whose key is the smallest among the live candidates at both of
// its points is taken (the globally smallest one always is, and no
// candidate of smaller key can claim its points later), its points are
// used, and every candidate touching a used point dies.  The set taken is
// exactly the one of the sequential greedy pass.  Taken exchanges are
// disjoint, so their link updates do not interact.  One workgroup; values
// that atomics update are read and written with device-scope atomics.
__global__ __launch_bounds__(1024) void k_rc_match(int32_t* __restrict__ nxt,
                                                   int32_t* __restrict__ prv,
                                                   int32_t* __restrict__ cnt, long long rcap,
                                                   const int32_t* __restrict__ ci,
                                                   const int32_t* __restrict__ cj,
                                                   const uint64_t* __restrict__ ckey,
                                                   int32_t* __restrict__ live,
                                                   uint64_t* __restrict__ bkey,
                                                   int32_t* __restrict__ bidx,
                                                   int32_t* __restrict__ used,
                                                   int32_t* __restrict__ del_out) {
  __shared__ int s_live;
  __shared__ int s_taken;
  const int t = threadIdx.x;
  const int n = cnt[0];
  // prepare the small-loop pass that follows: nothing deleted, bound n
  for (int j = t; j < n; j += blockDim.x) del_out[j] = 0;
  if (t == 0) cnt[9] = n;
  const int tot = (cnt[10] != 0 || cnt[6] > rcap) ? 0 : cnt[6];
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
  const int n[3] = {r.geom.nx, r.geom.ny, r.geom.nz};
  for (int a = 0; a < 3; ++a) {
    bg.nb[a] = r.bin_n[a];
    bg.h[a] = r.bin_h[a];
    bg.periodic[a] = !r.geom.wall[a];
    bg.off[a] = r.geom.wall[a] ? 0.5 : 0.0;
    (void)n;
  }
  return bg;
}

hipError_t small_and_compact(Run& r, int32_t* del) {
  const int nb = nb_of(r.ncap, 256);
  hipLaunchKernelGGL(k_small, dim3(nb), dim3(256), 0, r.stream, r.nxt, r.cnt, del,
                     r.vor.min_loop_pts, r.scan_a);
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, r.stream, r.scan_a, r.scan_b, r.cnt + 9, 0, r.cnt + 8);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(256), 0, r.stream, r.pos, r.nxt, r.prv,
                     r.cnt, r.ncap, r.scan_a, r.scan_b, r.pos_t, r.nxt_t, r.prv_t);
  hipLaunchKernelGGL(k_compact_copy, dim3(nb), dim3(256), 0, r.stream, r.pos, r.nxt, r.prv, r.cnt,
                     r.ncap, r.pos_t, r.nxt_t, r.prv_t);
  return hipGetLastError();
}

}  // namespace

hipError_t scan_excl(Run& r, const int32_t* in, int32_t* out, const int32_t* np, int n,
                     int32_t* total) {
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, r.stream, in, out, np, n, total);
  return hipGetLastError();
}

hipError_t topo_update(Run& r) {
  const TopoGeom tg = topo_geom(r);
  const int nb = nb_of(r.ncap, 256);
  hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(64), 0, r.stream, r.cnt);
  int32_t* del = r.flag_b;
  if (r.vor.remesh) {
    const double mn2 = r.vor.dxi_min * r.vor.dxi_min;
    const double mx2 = r.vor.dxi_max * r.vor.dxi_max;
    hipLaunchKernelGGL(k_rm_cand, dim3(nb), dim3(256), 0, r.stream, r.pos, r.nxt, r.prv, r.cnt, r.ncap, tg, mn2, mx2, r.flag_a);
    hipLaunchKernelGGL(k_rm_del, dim3(nb), dim3(256), 0, r.stream, r.nxt, r.prv, r.cnt, r.flag_a, del);
    hipLaunchKernelGGL(k_rm_relink, dim3(nb), dim3(256), 0, r.stream, r.nxt, r.prv, r.cnt, del);
    hipLaunchKernelGGL(k_rm_insmark, dim3(nb), dim3(256), 0, r.stream, r.pos, r.nxt, r.cnt, r.ncap, tg, mx2, del, r.scan_a);
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, r.stream, r.scan_a, r.scan_b, r.cnt, 0, r.cnt + 2);
    hipLaunchKernelGGL(k_rm_insert, dim3(nb), dim3(256), 0, r.stream, r.pos, r.nxt, r.prv, r.cnt,
                       r.ncap, tg, del, r.scan_a, r.scan_b);
  } else {
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, r.stream, del, r.ncap, 0);
  }
  hipError_t e = small_and_compact(r, del);
  if (e != hipSuccess) return e;

  if (r.vor.reconnect) {
    const BinGeom bg = bin_geom(r);
    const double d2max = r.vor.reconnect_dist * r.vor.reconnect_dist;
    const uint32_t pad = (r.bin_bits >= 32) ? 0xFFFFFFFFu : ((1u << r.bin_bits) - 1u);
    hipLaunchKernelGGL(k_rc_keys, dim3(nb), dim3(256), 0, r.stream, r.pos, r.cnt, r.ncap, bg, pad, r.keys_a, r.vals_a);
    uint32_t* sk = nullptr;
    int32_t* sv = nullptr;
    e = sort_pairs(r, r.bin_bits, &sk, &sv);
    if (e != hipSuccess) return e;
    e = bins_mark(r, sk, 1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rc_find, dim3(nb), dim3(256), 0, r.stream, r.pos, r.nxt, r.prv, sk, sv,
                       r.bins, r.cnt, r.ncap, tg, bg, d2max, r.scan_a, r.rc_slot_j, r.rc_slot_k,
                       r.used);
    e = bins_mark(r, sk, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, r.stream, r.scan_a, r.scan_b, r.cnt, 0, r.cnt + 6);
    hipLaunchKernelGGL(k_rc_compact, dim3(nb), dim3(256), 0, r.stream, r.scan_a, r.scan_b,
                       r.rc_slot_j, r.rc_slot_k, r.cnt, r.rcap, r.rc_i, r.rc_j, r.rc_key_a);
    hipLaunchKernelGGL(k_rc_match, dim3(1), dim3(1024), 0, r.stream, r.nxt, r.prv, r.cnt, r.rcap,
                       r.rc_i, r.rc_j, r.rc_key_a, r.rc_idx_a, r.rc_best, r.rc_bidx, r.used, del);
    e = small_and_compact(r, del);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace vlb
