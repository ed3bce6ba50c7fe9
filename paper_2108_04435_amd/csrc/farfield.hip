// Far-field approximation of the non-local Biot-Savart sum (an extension of
// Sec. II.A, Eq. Biot-Savart, for large tangles): periodic box, uniform
// cells of edge h, monopole to quadrupole moments of each cell's segment
// vorticity about its centre, evaluated per (target, cell) where the cell
// is far, the exact straight-segment integral where it is near.
//
// Definitions (the decisions are those of the FP64 reference of the same
// approximation, taken in FP64 and on the 32-bit position grid):
//  * positions are reduced into [0, L) per axis; segment k belongs to the
//    cell of its midpoint; y_k = m_k - c at the nearest image, d_k the
//    segment vector at the nearest image; rad = max_k (|y_k| + |d_k| / 2);
//  * per target r, each segment sits at the image of its start that the
//    direct sum takes (the wrapped difference of 32-bit grid coordinates);
//    with delta_k = X(s_k) - X(c) (wrapped, small) and u = X(c) - X(r),
//    the segment's image places the centre at (c - r) + K L with
//    K = (wrap(u + delta_k) - delta_k - (X(c) - X(r))) / 2^32, so the class
//    of a cell's segments changes only where u + delta crosses 2^31 (the
//    plane half a box from the target);
//  * one class: far when |R|^2 theta^2 >= rad^2 at R = (c - r) + K L;
//    classes differing on one axis (delta_min and delta_max on opposite
//    sides): split when both images pass, the class below the crossing
//    taking the prefix moments of the cell's segments sorted by delta on
//    that axis, the other the rest; otherwise direct;
//  * with two levels the cells of edge 2h are classified first and an
//    opened one (neither far nor split) hands its 8 children of edge h to
//    the same rule, the lanes that opened it taking part.
//
// Layout (workspace, all per call):
//  * per point: wrapped FP64 positions, grid coordinates, links, y and d
//    (FP64), cell key;
//  * segments sorted by cell (stable radix sort, so ascending index inside
//    a cell; with two levels the key is coarse cell * 8 + child, so each
//    coarse cell's children are consecutive), one 32-byte record each for
//    the direct loop;
//  * one 256-byte record per cell (range, rad^2, centre, grid centre,
//    delta extremes, 36 moments), read with scalar loads;
//  * per axis: each cell's deltas in ascending order and the prefix sums of
//    the 36 moment components over that order (cnt + 1 rows per cell);
//  * the evaluation grid: blockIdx.x picks 64 targets (consecutive in the
//    cell order, so a wave's targets are close), blockIdx.y one of S cell
//    chunks; the 4 waves of a block take interleaved cells of the coarsest
//    level (c = 4 y + w modulo 4 S) and add their sums in LDS in a fixed
//    order; the chunk partials are added in FP64 in chunk order (bitwise
//    reproducible).
#include "vlb_internal.h"

#include <cmath>

namespace vlb {

namespace {

constexpr int kMom = 36;       // moment components per cell or class
constexpr int kFfTargets = 64;

// Moment components (no kappa: the caller scales the sum): 0..2 M0_n = d_n;
// 3..5 A = d x y (the antisymmetric part of M1, eps_mnp M1_np); 6..14
// M1_np = d_n y_p; 15..32 M2_njk = d_n (y_j y_k + d_j d_k / 12) for
// jk = 00 01 02 11 12 22; 33..35 tr_n = d_n (|y|^2 + |d|^2 / 12).
__device__ inline double comp_value(int comp, const double* y, const double* d) {
#pragma clang fp contract(off)
  if (comp < 3) return d[comp];
  if (comp < 6) {
    const int m = comp - 3;
    const int a = (m + 1) % 3, b = (m + 2) % 3;
    return d[a] * y[b] - d[b] * y[a];
  }
  if (comp < 15) {
    const int i = comp - 6;
    return d[i / 3] * y[i % 3];
  }
  if (comp < 33) {
    const int i = comp - 15;
    const int nn = i / 6, jk = i % 6;
    const int j = jk < 3 ? 0 : (jk < 5 ? 1 : 2);
    const int k = jk < 3 ? jk : (jk < 5 ? jk - 2 : 2);
    return d[nn] * (y[j] * y[k] + d[j] * d[k] / 12.0);
  }
  const int nn = comp - 33;
  return d[nn] * ((y[0] * y[0] + y[1] * y[1] + y[2] * y[2]) +
                  (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) / 12.0);
}

struct FfAxes {
  double L[3], q[3], th2;
  double h[2];   // cell edge per level (level 0 the finest)
  float iqf[3];  // lattice units per grid step
  float qf;      // one grid step count per lattice unit when uniform
  int nc[2][3];  // cells per axis per level
  int C[2];      // cells per level
  int levels;    // 1 or 2
  int uniform;
};

// Cell coordinates at a level from its record index: one level, x fastest;
// two levels, the coarse cell x fastest and, at the fine level, index =
// coarse * 8 + child with child bits x | y << 1 | z << 2.
__device__ inline void ff_coords(const FfAxes& ax, int level, int idx, int* ci) {
  if (ax.levels == 1 || level == 1) {
    const int* nc = ax.nc[level];
    ci[0] = idx % nc[0];
    ci[1] = (idx / nc[0]) % nc[1];
    ci[2] = idx / (nc[0] * nc[1]);
  } else {
    const int t = idx >> 3, ch = idx & 7;
    const int* nc = ax.nc[1];
    ci[0] = 2 * (t % nc[0]) + (ch & 1);
    ci[1] = 2 * ((t / nc[0]) % nc[1]) + ((ch >> 1) & 1);
    ci[2] = 2 * (t / (nc[0] * nc[1])) + ((ch >> 2) & 1);
  }
}

__device__ inline double ff_min_image(double x, double L) {
#pragma clang fp contract(off)
  if (x > 0.5 * L) return x - L;
  if (x < -0.5 * L) return x + L;
  return x;
}

struct __align__(256) FfCell {
  int32_t start, count;      // range in the sorted order
  double rad2;               // rad * rad
  double c[3];               // centre
  uint32_t xc[3];            // centre on the 32-bit grid
  int32_t dmin[3], dmax[3];  // extremes of the wrapped grid offset start - centre
  int32_t pad;
  float m[kMom];
};

struct __align__(32) FfSeg {
  uint32_t x[3];  // start on the grid
  float d[3];     // segment vector: wrapped grid difference (uniform) or lattice units
  float dq;       // |d|^2
  int32_t idx;    // segment (point) index
};

__device__ inline double ff_wrap(double x, double L) {
#pragma clang fp contract(off)
  if (x < 0.0) x = x + L;
  if (x >= L) x = x - L;
  if (x >= L) x = 0.0;  // x + L rounded up to L
  return x;
}

__global__ void k_ff_init(int32_t* __restrict__ prv, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) prv[j] = j;
}

// Point j with successor k (positions y_j, y_k): wrapped position, grid
// coordinate, segment vector, midpoint and the sort key of its finest cell.
__device__ inline void ff_point(const double* yj, const double* yk, int j, long long nc,
                                const FfAxes& ax, double* __restrict__ P,
                                uint32_t* __restrict__ X, double* __restrict__ M,
                                double* __restrict__ D, uint32_t* __restrict__ keys,
                                int32_t* __restrict__ kidx, int32_t* __restrict__ vals) {
#pragma clang fp contract(off)
  int idx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double L = ax.L[a];
    const double p = ff_wrap(yj[a], L);
    const double pk = ff_wrap(yk[a], L);
    P[(long long)a * nc + j] = p;
    X[(long long)a * nc + j] = (uint32_t)(long long)floor(p * ax.q[a]);
    const double d = ff_min_image(pk - p, L);
    double mid = p + 0.5 * d;
    mid = mid - L * floor(mid / L);
    int i = (int)floor(mid / ax.h[0]);
    idx[a] = min(max(i, 0), ax.nc[0][a] - 1);
    M[(long long)a * nc + j] = mid;
    D[(long long)a * nc + j] = d;
  }
  int key;
  if (ax.levels == 1) {
    key = (idx[2] * ax.nc[0][1] + idx[1]) * ax.nc[0][0] + idx[0];
  } else {
    const int t = ((idx[2] >> 1) * ax.nc[1][1] + (idx[1] >> 1)) * ax.nc[1][0] + (idx[0] >> 1);
    key = t * 8 + ((idx[0] & 1) | ((idx[1] & 1) << 1) | ((idx[2] & 1) << 2));
  }
  keys[j] = (uint32_t)key;
  kidx[j] = key;
  vals[j] = j;
}

// Stand-alone sum: links sanitised from the caller's (clamped into
// [0, n), inverted into prv, which k_ff_init set to self), positions
// [n][3]; thread 0 writes the point count.
__global__ void k_ff_prep(const double* __restrict__ xyz, const int32_t* __restrict__ next, int n,
                          FfAxes ax, int32_t* __restrict__ cnt, double* __restrict__ P,
                          uint32_t* __restrict__ X, int32_t* __restrict__ nxt,
                          int32_t* __restrict__ prv, double* __restrict__ M,
                          double* __restrict__ D, uint32_t* __restrict__ keys,
                          int32_t* __restrict__ kidx, int32_t* __restrict__ vals) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) {
    cnt[0] = n;
    for (int i = 1; i < 32; ++i) cnt[i] = 0;
  }
  if (j >= n) return;
  const int k = min(max(next[j], 0), n - 1);
  nxt[j] = k;
  if (k != j) prv[k] = j;
  const double yj[3] = {xyz[3LL * j], xyz[3LL * j + 1], xyz[3LL * j + 2]};
  const double yk[3] = {xyz[3LL * k], xyz[3LL * k + 1], xyz[3LL * k + 2]};
  ff_point(yj, yk, j, n, ax, P, X, M, D, keys, kidx, vals);
}

// In a run: positions Y (3 x nc, SoA) and the run's links, the live count
// cnt[0]; slots beyond it get the largest key (they sort last).
__global__ void k_ff_prep_run(const double* __restrict__ Y, const int32_t* __restrict__ nxt,
                              const int32_t* __restrict__ cnt, long long nc, FfAxes ax,
                              double* __restrict__ P, uint32_t* __restrict__ X,
                              double* __restrict__ M, double* __restrict__ D,
                              uint32_t* __restrict__ keys, int32_t* __restrict__ kidx,
                              int32_t* __restrict__ vals) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  if (j >= cnt[0]) {
    keys[j] = 0xffffffffu;
    kidx[j] = 0;
    vals[j] = j;
    return;
  }
  const int k = nxt[j];
  const double yj[3] = {Y[j], Y[nc + j], Y[2 * nc + j]};
  const double yk[3] = {Y[k], Y[nc + k], Y[2 * nc + k]};
  ff_point(yj, yk, j, nc, ax, P, X, M, D, keys, kidx, vals);
}

// Cell ranges in the sorted keys (binary search; empty cells get count 0).
__device__ inline int lower_bound_u32(const uint32_t* a, int n, uint32_t v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Level records cover the sorted keys [c << shift, (c + 1) << shift).
__global__ void k_ff_bounds(const uint32_t* __restrict__ sk, int n, int C, int shift,
                            FfCell* __restrict__ cells) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int lo = lower_bound_u32(sk, n, (uint32_t)c << shift);
  const int hi = lower_bound_u32(sk, n, ((uint32_t)c + 1u) << shift);
  cells[c].start = lo;
  cells[c].count = hi - lo;
}

// Per sorted position: the direct loop's segment record.
__global__ void k_ff_seg(const int32_t* __restrict__ so, const uint32_t* __restrict__ X,
                         const int32_t* __restrict__ nxt, const int32_t* __restrict__ cntp,
                         long long nc, FfAxes ax, FfSeg* __restrict__ recs) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= cntp[0]) return;
  const int k = so[p];
  const int kn = nxt[k];
  FfSeg r;
  float dq = 0.f;
  for (int a = 0; a < 3; ++a) {
    const uint32_t x0 = X[(long long)a * nc + k];
    float e = (float)(int)(X[(long long)a * nc + kn] - x0);
    if (!ax.uniform) e *= ax.iqf[a];
    r.x[a] = x0;
    r.d[a] = e;
  }
  dq = r.d[0] * r.d[0] + r.d[1] * r.d[1] + r.d[2] * r.d[2];
  r.dq = dq;
  r.idx = k;
  recs[p] = r;
}

__device__ inline double ff_lane_d(double x, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), k);
  return __hiloint2double(hi, lo);
}

// Per segment, at one level: the 36 moment components about its cell's
// centre (FP64, row k of comps) and |y| + |d| / 2 (srad).
__global__ void k_ff_comps(const double* __restrict__ M, const double* __restrict__ D,
                           const int32_t* __restrict__ kidx, const int32_t* __restrict__ cntp,
                           long long nc, FfAxes ax, int level, double* __restrict__ comps,
                           double* __restrict__ srad) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cntp[0]) return;
  int ci[3];
  ff_coords(ax, level, kidx[k] >> (3 * level), ci);
  double y[3], d[3];
  for (int b = 0; b < 3; ++b) {
    y[b] = ff_min_image(M[(long long)b * nc + k] - ((double)ci[b] + 0.5) * ax.h[level], ax.L[b]);
    d[b] = D[(long long)b * nc + k];
  }
  double* row = comps + (long long)k * kMom;
#pragma unroll
  for (int i = 0; i < kMom; ++i) row[i] = comp_value(i, y, d);
  const double ny = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
  const double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  srad[k] = ny + 0.5 * nd;
}

// One wave (a block of 64) per (cell of a level, axis): the cell's start
// offsets on the axis in ascending order (ties by sorted position) with
// their segment indices (sdel, sidx), the prefix sums of the 36 moment
// components over that order (FP64 sums stored FP32, rows
// a (nc + C) + start + c + i for i = 0 .. count, row 0 zero; nc the
// capacity of the point arrays), and the
// record's fields for the axis (centre, grid centre, offset extremes); the
// axis-0 wave also writes the radius and the moments (its prefix totals).
// The ranks compare offsets held in registers (64 at a time, broadcast
// with readlane); the prefix sums add the components of k_ff_comps, one
// lane per component.
__global__ __launch_bounds__(64) void k_ff_order(const int32_t* __restrict__ so,
                                                 const double* __restrict__ comps,
                                                 const double* __restrict__ srad,
                                                 const uint32_t* __restrict__ X, long long nc,
                                                 FfAxes ax,
                                                 int level, FfCell* __restrict__ cells,
                                                 int32_t* __restrict__ sdel,
                                                 int32_t* __restrict__ sidx,
                                                 float* __restrict__ pre) {
#pragma clang fp contract(off)
  const int c = blockIdx.x / 3, a = blockIdx.x - 3 * (blockIdx.x / 3);
  const int lane = threadIdx.x;
  const int C = ax.C[level];
  const int s = cells[c].start, cnt = cells[c].count;
  int ci[3];
  ff_coords(ax, level, c, ci);
  double cen[3];
  for (int b = 0; b < 3; ++b) cen[b] = ((double)ci[b] + 0.5) * ax.h[level];
  const uint32_t xc = (uint32_t)(long long)floor(cen[a] * ax.q[a]);
  const uint32_t* Xa = X + (long long)a * nc;
  int32_t* sd = sdel + (long long)a * nc + s;
  int32_t* si = sidx + (long long)a * nc + s;
  int dmn = 0x7fffffff, dmx = -0x7fffffff - 1;
  for (int b0 = 0; b0 < cnt; b0 += 64) {
    const int i = b0 + lane;
    const bool vi = i < cnt;
    const int ki = vi ? so[s + i] : 0;
    const int di = vi ? (int)(Xa[ki] - xc) : 0;
    if (vi) {
      dmn = min(dmn, di);
      dmx = max(dmx, di);
    }
    int rank = 0;
    for (int j0 = 0; j0 < cnt; j0 += 64) {
      const int jj = j0 + lane;
      const int dj = jj < cnt ? (int)(Xa[so[s + jj]] - xc) : 0;
      const int m = min(64, cnt - j0);
      for (int k = 0; k < m; ++k) {
        const int dk = __builtin_amdgcn_readlane(dj, k);
        rank += (dk < di || (dk == di && j0 + k < i)) ? 1 : 0;
      }
    }
    if (vi) {
      sd[rank] = di;
      si[rank] = ki;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    dmn = min(dmn, __shfl_xor(dmn, off));
    dmx = max(dmx, __shfl_xor(dmx, off));
  }
  __syncthreads();  // the sorted order, written above, is read below
  float* row = pre + ((long long)a * (nc + C) + s + c) * kMom;
  double acc = 0.0, rad = 0.0;
  for (int i = lane; i < cnt; i += 64) rad = fmax(rad, srad[so[s + i]]);
  if (lane < kMom) {
    row[lane] = 0.f;
#pragma unroll 8
    for (int i = 0; i < cnt; ++i) {
      acc = acc + comps[(long long)si[i] * kMom + lane];
      row[(long long)(i + 1) * kMom + lane] = (float)acc;
    }
  }
  for (int off = 32; off > 0; off >>= 1) rad = fmax(rad, __shfl_xor(rad, off));
  FfCell& o = cells[c];
  if (lane == 0) {
    o.c[a] = cen[a];
    o.xc[a] = xc;
    o.dmin[a] = cnt > 0 ? dmn : 0;
    o.dmax[a] = cnt > 0 ? dmx : 0;
    if (a == 0) {
      o.rad2 = rad * rad;
      o.pad = 0;
    }
  }
  if (a == 0 && lane < kMom) o.m[lane] = (float)acc;
}

// Moments: one array, or the difference of two (the upper class of a split
// cell: the cell's totals minus the prefix of the lower class).
struct MomA {
  const float* p;
  __device__ float operator()(int i) const { return p[i]; }
};
struct MomD {
  const float* t;
  const float* p;
  __device__ float operator()(int i) const { return t[i] - p[i]; }
};

template <class M>
__device__ inline void m2p_f32(float Rx, float Ry, float Rz, const M& m, float& vx, float& vy,
                               float& vz) {
  const float r2 = fmaf(Rx, Rx, fmaf(Ry, Ry, Rz * Rz));
  const float ir = __builtin_amdgcn_rsqf(r2);
  const float i2 = ir * ir;
  const float r3 = ir * i2;
  const float r5 = r3 * i2;
  const float r7h = 7.5f * (r5 * i2);
  float S[3][3], W[3];
#pragma unroll
  for (int nn = 0; nn < 3; ++nn) {
    const int q = 15 + 6 * nn;
    const float q0 = m(q), q1 = m(q + 1), q2 = m(q + 2), q3 = m(q + 3), q4 = m(q + 4),
                q5 = m(q + 5);
    S[nn][0] = fmaf(q0, Rx, fmaf(q1, Ry, q2 * Rz));
    S[nn][1] = fmaf(q1, Rx, fmaf(q3, Ry, q4 * Rz));
    S[nn][2] = fmaf(q2, Rx, fmaf(q4, Ry, q5 * Rz));
    const float Q = fmaf(Rx, S[nn][0], fmaf(Ry, S[nn][1], Rz * S[nn][2]));
    const float a = fmaf(m(6 + 3 * nn), Rx, fmaf(m(7 + 3 * nn), Ry, m(8 + 3 * nn) * Rz));
    W[nn] = fmaf(r5, fmaf(3.0f, a, -1.5f * m(33 + nn)), r7h * Q);
  }
  const float B0 = S[1][2] - S[2][1];
  const float B1 = S[2][0] - S[0][2];
  const float B2 = S[0][1] - S[1][0];
  const float m0 = m(0), m1 = m(1), m2 = m(2);
  const float V0 = fmaf(m1, Rz, -fmaf(m2, Ry, m(3)));
  const float V1 = fmaf(m2, Rx, -fmaf(m0, Rz, m(4)));
  const float V2 = fmaf(m0, Ry, -fmaf(m1, Rx, m(5)));
  const float t5 = 3.0f * r5;
  vx = fmaf(r3, V0, vx + fmaf(W[1], Rz, -fmaf(W[2], Ry, t5 * B0)));
  vy = fmaf(r3, V1, vy + fmaf(W[2], Rx, -fmaf(W[0], Rz, t5 * B1)));
  vz = fmaf(r3, V2, vz + fmaf(W[0], Ry, -fmaf(W[1], Rx, t5 * B2)));
}

// One (target, segment) pair of the exact straight-segment integral, as in
// the direct FP32 sum: R1 = s - r from the wrapped grid difference, R2 =
// R1 + d, v += (R1 x d) (i1 + i2) i1 i2 / (1 + (R1.R2) i1 i2).
template <bool kUniform>
__device__ inline void ff_pair(const FfSeg& g, uint32_t xt, uint32_t yt, uint32_t zt,
                               const FfAxes& ax, float& vx, float& vy, float& vz, bool zero) {
  float r1x = (float)(int)(g.x[0] - xt);
  float r1y = (float)(int)(g.x[1] - yt);
  float r1z = (float)(int)(g.x[2] - zt);
  if (!kUniform) {
    r1x *= ax.iqf[0];
    r1y *= ax.iqf[1];
    r1z *= ax.iqf[2];
  }
  const float ex = g.d[0], ey = g.d[1], ez = g.d[2];
  const float t = fmaf(r1x, ex, fmaf(r1y, ey, r1z * ez));
  const float n1 = fmaf(r1x, r1x, fmaf(r1y, r1y, r1z * r1z));
  const float n2 = fmaf(2.0f, t, n1 + g.dq);
  const float i1 = __builtin_amdgcn_rsqf(n1);
  const float i2 = __builtin_amdgcn_rsqf(n2);
  const float crx = fmaf(r1y, ez, -r1z * ey);
  const float cry = fmaf(r1z, ex, -r1x * ez);
  const float crz = fmaf(r1x, ey, -r1y * ex);
  const float a = i1 * i2;
  const float den = fmaf(n1 + t, a, 1.0f);
  float f = (i1 + i2) * a * __builtin_amdgcn_rcpf(den);
  f = zero ? 0.0f : f;
  vx = fmaf(f, crx, vx);
  vy = fmaf(f, cry, vy);
  vz = fmaf(f, crz, vz);
}

// The decision fields of a cell record, loaded one cell ahead.
struct FfHead {
  int32_t start, count;
  double rad2;
  double c[3];
  uint32_t xc[3];
  int32_t dmin[3], dmax[3];
};

__device__ inline void ff_head(const FfCell* __restrict__ cm, FfHead& h) {
  h.start = cm->start;
  h.count = cm->count;
  h.rad2 = cm->rad2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h.c[a] = cm->c[a];
    h.xc[a] = cm->xc[a];
    h.dmin[a] = cm->dmin[a];
    h.dmax[a] = cm->dmax[a];
  }
}

// Per-lane decision for one cell (FP64 and integers, no contraction).
struct FfDecision {
  double R0[3];  // (c - r) + K L of the class of the smallest start offset
  int ncross;    // axes on which the start offsets cross the half-box plane
  int axis;      // the crossed axis (ncross == 1)
  int kc;        // K of that class on the crossed axis
  bool ok0;      // R0 passes the opening test
};

__device__ inline void ff_decide(const FfHead* cm, const double* r, const uint32_t* xt,
                                 const FfAxes& ax, FfDecision& o) {
#pragma clang fp contract(off)
  o.ncross = 0;
  o.axis = 0;
  o.kc = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t xc = cm->xc[a];
    const int dmin = cm->dmin[a], dmax = cm->dmax[a];
    const uint32_t u = xc - xt[a];
    const int wmin = (int)(u + (uint32_t)dmin);
    const int wmax = (int)(u + (uint32_t)dmax);
    const long long rawc = (long long)xc - (long long)xt[a];
    const int k = (int)(((long long)wmin - (long long)dmin - rawc) >> 32);
    const bool cr = wmax < wmin;
    o.ncross += cr ? 1 : 0;
    o.axis = cr ? a : o.axis;
    o.kc = cr ? k : o.kc;
    o.R0[a] = (cm->c[a] - r[a]) + (double)k * ax.L[a];
  }
  const double d2 = (o.R0[0] * o.R0[0] + o.R0[1] * o.R0[1]) + o.R0[2] * o.R0[2];
  o.ok0 = d2 * ax.th2 >= cm->rad2;
}

// The class of the largest offset on the crossed axis: its wrapped offset
// dropped by 2^32 at the crossing, so its K there is one less.  Returns
// whether that image passes the opening test.
__device__ inline bool ff_other(const FfHead* cm, const FfDecision& o, const double* r,
                                const FfAxes& ax, double* R1) {
#pragma clang fp contract(off)
#pragma unroll
  for (int a = 0; a < 3; ++a)
    R1[a] = a == o.axis ? (cm->c[a] - r[a]) + (double)(o.kc - 1) * ax.L[a] : o.R0[a];
  const double d2 = (R1[0] * R1[0] + R1[1] * R1[1]) + R1[2] * R1[2];
  return d2 * ax.th2 >= cm->rad2;
}

// Far and split contributions of one cell for the active lanes; returns
// whether this lane opens the cell (active, neither far nor split).
__device__ inline bool ff_cell_eval(const FfHead& hc, const FfCell* __restrict__ cm, int c,
                                    const int32_t* __restrict__ sdel,
                                    const float* __restrict__ pre, long long nc, int C,
                                    bool active,
                                    const double* r, const uint32_t* xt, const FfAxes& ax,
                                    float& fx, float& fy, float& fz) {
  FfDecision dc;
  ff_decide(&hc, r, xt, ax, dc);
  const bool far = active && dc.ncross == 0 && dc.ok0;
  bool split = false;
  double R1[3] = {0.0, 0.0, 0.0};
  if (active && dc.ncross == 1 && dc.ok0) split = ff_other(&hc, dc, r, ax, R1);
  if (__any(far)) {
    if (far)
      m2p_f32((float)-dc.R0[0], (float)-dc.R0[1], (float)-dc.R0[2], MomA{cm->m}, fx, fy, fz);
  }
  if (__any(split)) {
    if (split) {
      // offsets below the crossing: u + delta < 2^31
      const int a = dc.axis;
      const uint32_t u = hc.xc[a] - xt[a];
      const int db = (int)(0x80000000u - u);
      const int32_t* dl = sdel + (long long)a * nc + hc.start;
      int lo = 0, hi = hc.count;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (dl[mid] < db)
          lo = mid + 1;
        else
          hi = mid;
      }
      const float* pr = pre + ((long long)a * (nc + C) + hc.start + c + lo) * kMom;
      m2p_f32((float)-dc.R0[0], (float)-dc.R0[1], (float)-dc.R0[2], MomA{pr}, fx, fy, fz);
      m2p_f32((float)-R1[0], (float)-R1[1], (float)-R1[2], MomD{cm->m, pr}, fx, fy, fz);
    }
  }
  return active && !far && !split;
}

// The exact pairs of a finest cell for the lanes in `near`; the target's
// own two segments excluded where the cell holds them (kCheck).  The
// cell's records are staged 64 at a time in the wave's own LDS slots
// (lds, 64 records) and read back with broadcast LDS loads, so the loop
// waits on no scalar load.
template <bool kUniform, bool kCheck>
__device__ inline void ff_direct_loop(int s0, int e, const FfSeg* __restrict__ recs,
                                      FfSeg* lds, bool near, int jj, int pj, const uint32_t* xt,
                                      const FfAxes& ax, float& dx, float& dy, float& dz) {
  const int lane = threadIdx.x & 63;
  for (int c0 = s0; c0 < e; c0 += 64) {
    const int m = min(64, e - c0);
    if (lane < m) lds[lane] = recs[c0 + lane];
    __builtin_amdgcn_wave_barrier();
    for (int k = 0; k < m; ++k) {
      const FfSeg g = lds[k];
      if (near)
        ff_pair<kUniform>(g, xt[0], xt[1], xt[2], ax, dx, dy, dz,
                          kCheck && (g.idx == jj || g.idx == pj));
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <bool kUniform>
__device__ inline void ff_direct(const FfHead& hc, int c, const FfSeg* __restrict__ recs,
                                 FfSeg* lds, bool near, int kj, int kp, int jj, int pj,
                                 const uint32_t* xt, const FfAxes& ax, float& dx, float& dy,
                                 float& dz) {
  const int s0 = hc.start, e = hc.start + hc.count;
  if (__any(kj == c || kp == c))
    ff_direct_loop<kUniform, true>(s0, e, recs, lds, near, jj, pj, xt, ax, dx, dy, dz);
  else
    ff_direct_loop<kUniform, false>(s0, e, recs, lds, near, jj, pj, xt, ax, dx, dy, dz);
}

template <bool kUniform, int kLevels>
__global__ __launch_bounds__(256) void k_ff_eval(
    const FfCell* __restrict__ cells0, const FfCell* __restrict__ cells1,
    const FfSeg* __restrict__ recs, const int32_t* __restrict__ so,
    const int32_t* __restrict__ kidx, const int32_t* __restrict__ prv,
    const double* __restrict__ Pw, const uint32_t* __restrict__ X,
    const int32_t* __restrict__ sdel0, const int32_t* __restrict__ sdel1,
    const float* __restrict__ pre0, const float* __restrict__ pre1,
    const int32_t* __restrict__ cntp, long long nc, int S, FfAxes ax, float* __restrict__ Pout) {
  const int n = cntp[0];
  if (blockIdx.x * kFfTargets >= n) return;  // whole block beyond the live points
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = blockIdx.x * kFfTargets + lane;
  const bool valid = t < n;
  const int j = valid ? so[t] : 0;
  double r[3];
  uint32_t xt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = Pw[(long long)a * nc + j];
    xt[a] = X[(long long)a * nc + j];
  }
  const int pj = valid ? prv[j] : -1;
  const int jj = valid ? j : -1;
  const int kj = valid ? kidx[j] : -1;
  const int kp = valid ? kidx[pj] : -1;
  float fx = 0.f, fy = 0.f, fz = 0.f;  // expansions (lattice units)
  float dx = 0.f, dy = 0.f, dz = 0.f;  // direct pairs (grid units when uniform)
  const FfCell* __restrict__ top = kLevels == 2 ? cells1 : cells0;
  const int32_t* __restrict__ sdt = kLevels == 2 ? sdel1 : sdel0;
  const float* __restrict__ prt = kLevels == 2 ? pre1 : pre0;
  const int Ct = ax.C[kLevels - 1];
  const int step = 4 * S;
  __shared__ FfSeg stage[4][64];  // each wave's staged segment records
  FfSeg* lds = stage[w];
  int c = blockIdx.y * 4 + w;
  FfHead hc;
  if (c < Ct) ff_head(top + c, hc);
  for (; c < Ct; c += step) {
    // the next cell's decision fields are loaded while this one is summed
    FfHead hn;
    if (c + step < Ct) ff_head(top + c + step, hn);
    if (hc.count > 0) {
      const bool open =
          ff_cell_eval(hc, top + c, c, sdt, prt, nc, Ct, valid, r, xt, ax, fx, fy, fz);
      if (kLevels == 1) {
        if (__any(open))
          ff_direct<kUniform>(hc, c, recs, lds, open, kj, kp, jj, pj, xt, ax, dx, dy, dz);
      } else if (__any(open)) {
        // the children, each child's decision fields loaded one child ahead
        FfHead hf;
        ff_head(cells0 + c * 8, hf);
        for (int ch = 0; ch < 8; ++ch) {
          const int f = c * 8 + ch;
          FfHead hfn;
          if (ch < 7) ff_head(cells0 + f + 1, hfn);
          if (hf.count > 0) {
            const bool near = ff_cell_eval(hf, cells0 + f, f, sdel0, pre0, nc, ax.C[0], open, r,
                                           xt, ax, fx, fy, fz);
            if (__any(near))
              ff_direct<kUniform>(hf, f, recs, lds, near, kj, kp, jj, pj, xt, ax, dx, dy, dz);
          }
          hf = hfn;
        }
      }
    }
    hc = hn;
  }
  if (kUniform) {
    fx = fmaf(dx, ax.qf, fx);
    fy = fmaf(dy, ax.qf, fy);
    fz = fmaf(dz, ax.qf, fz);
  } else {
    fx += dx;
    fy += dy;
    fz += dz;
  }
  __shared__ float red[3][3][kFfTargets];
  if (w > 0) {
    red[w - 1][0][lane] = fx;
    red[w - 1][1][lane] = fy;
    red[w - 1][2][lane] = fz;
  }
  __syncthreads();
  if (w == 0 && valid) {
    float* out = Pout + (long long)blockIdx.y * 3 * nc;
    out[j] = ((fx + red[0][0][lane]) + red[1][0][lane]) + red[2][0][lane];
    out[nc + j] = ((fy + red[0][1][lane]) + red[1][1][lane]) + red[2][1][lane];
    out[2 * nc + j] = ((fz + red[0][2][lane]) + red[1][2][lane]) + red[2][2][lane];
  }
}

// v[j][a] = scale * (sum over the S chunk partials of target j, in chunk
// order, in FP64).
__global__ void k_ff_sum(const float* __restrict__ P, int S, int n, double scale,
                         double* __restrict__ v) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double t = 0.0;
    for (int c = 0; c < S; ++c) t += (double)P[((long long)c * 3 + a) * n + j];
    v[3LL * j + a] = t * scale;
  }
}

FfAxes ff_axes(const vlb_bs_desc* d, const vlb_ff_params* p) {
  FfAxes ax{};
  const int nn[3] = {d->nx, d->ny, d->nz};
  ax.levels = p->levels == 2 ? 2 : 1;
  bool uniform = true;
  for (int a = 0; a < 3; ++a) {
    ax.L[a] = (double)nn[a];
    ax.q[a] = 4294967296.0 / (double)nn[a];
    ax.iqf[a] = (float)((double)nn[a] / 4294967296.0);
    ax.nc[0][a] = nn[a] / p->cell;
    ax.nc[1][a] = ax.levels == 2 ? nn[a] / (2 * p->cell) : 0;
    uniform = uniform && nn[a] == nn[0];
  }
  // one grid step for all axes: equal power-of-two lengths
  int ex = 0;
  uniform = uniform && std::frexp((double)nn[0], &ex) == 0.5;
  ax.uniform = uniform ? 1 : 0;
  ax.qf = (float)ax.q[0];
  ax.h[0] = (double)p->cell;
  ax.h[1] = 2.0 * p->cell;
  ax.th2 = p->theta * p->theta;
  for (int l = 0; l < 2; ++l) ax.C[l] = ax.nc[l][0] * ax.nc[l][1] * ax.nc[l][2];
  return ax;
}

// Chunks of the coarsest cells: about 32768 blocks over the target blocks
// (a 256^3 tangle of 1e5 points: 15 in a run, whose launch is sized by the
// capacity, 21 stand-alone; 4 chunks measured 10% slower per coupled step),
// at least 4 cells per chunk, at most 64 chunks.
int ff_chunks(long long n, int Ctop) {
  const long long tb = (n + kFfTargets - 1) / kFfTargets;
  long long S = (32768 + tb - 1) / tb;
  if (S > Ctop / 4) S = Ctop / 4;
  if (S > 64) S = 64;
  if (S < 1) S = 1;
  return (int)S;
}

struct FfBufs {
  int32_t* cnt;
  double* Pw;
  uint32_t* X;
  int32_t* nxt;
  int32_t* prv;
  double* M;
  double* D;
  uint32_t* ka;
  uint32_t* kb;
  int32_t* va;
  int32_t* vb;
  int32_t* kidx;
  void* stmp;
  FfSeg* recs;
  double* comps;  // per segment, one level at a time
  double* srad;
  FfCell* cells[2];
  int32_t* sdel[2];
  int32_t* sidx[2];
  float* pre[2];
  float* P;
  int S;
};

// Workspace of the sum for n points (the capacity in a run).  solo: the
// stand-alone call, which also needs the sanitised links, the point count
// and its own chunk partials (a run has its own and writes into its
// Biot-Savart partials).
size_t ff_layout(long long n, const FfAxes& ax, bool solo, char* base, FfBufs* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    off = (off + 255) / 256 * 256;
    void* q = base ? base + off : nullptr;
    off += bytes;
    return q;
  };
  FfBufs s{};
  s.S = ff_chunks(n, ax.C[ax.levels - 1]);
  if (solo) {
    s.cnt = (int32_t*)take(32 * sizeof(int32_t));
    s.nxt = (int32_t*)take((size_t)n * sizeof(int32_t));
    s.prv = (int32_t*)take((size_t)n * sizeof(int32_t));
  }
  s.Pw = (double*)take(3 * (size_t)n * sizeof(double));
  s.X = (uint32_t*)take(3 * (size_t)n * sizeof(uint32_t));
  s.M = (double*)take(3 * (size_t)n * sizeof(double));
  s.D = (double*)take(3 * (size_t)n * sizeof(double));
  s.ka = (uint32_t*)take((size_t)n * sizeof(uint32_t));
  s.kb = (uint32_t*)take((size_t)n * sizeof(uint32_t));
  s.va = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.vb = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.kidx = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.stmp = take(sort_tmp_bytes(n));
  s.recs = (FfSeg*)take((size_t)n * sizeof(FfSeg));
  s.comps = (double*)take((size_t)n * kMom * sizeof(double));
  s.srad = (double*)take((size_t)n * sizeof(double));
  for (int l = 0; l < ax.levels; ++l) {
    const size_t C = (size_t)ax.C[l];
    s.cells[l] = (FfCell*)take(C * sizeof(FfCell));
    s.sdel[l] = (int32_t*)take(3 * (size_t)n * sizeof(int32_t));
    s.sidx[l] = (int32_t*)take(3 * (size_t)n * sizeof(int32_t));
    s.pre[l] = (float*)take(3 * ((size_t)n + C) * kMom * sizeof(float));
  }
  if (ax.levels == 1) {
    s.cells[1] = s.cells[0];
    s.sdel[1] = s.sdel[0];
    s.sidx[1] = s.sidx[0];
    s.pre[1] = s.pre[0];
  }
  if (solo) s.P = (float*)take((size_t)s.S * 3 * n * sizeof(float));
  if (b) *b = s;
  return (off + 255) / 256 * 256;
}

}  // namespace

int ff_check(const vlb_bs_desc* d, const vlb_ff_params* p, int64_t n, std::string& msg) {
  const int c = bs_check_desc(d, n, msg);
  if (c != VLB_OK) return c;
  if (!p) { msg = "null far-field parameters"; return VLB_EINVAL; }
  if (d->wall_axes != 0) { msg = "the far-field sum needs a periodic box (wall_axes 0)"; return VLB_EINVAL; }
  if (d->precision != VLB_F32) { msg = "the far-field sum is FP32 (precision VLB_F32)"; return VLB_EINVAL; }
  if (!(p->theta > 0.0 && p->theta < 1.0)) { msg = "theta must lie in (0, 1)"; return VLB_EINVAL; }
  if (p->levels < 0 || p->levels > 2) { msg = "levels must be 0, 1 or 2"; return VLB_EINVAL; }
  const int top = p->levels == 2 ? 2 * p->cell : p->cell;
  if (p->cell < 1 || d->nx % top || d->ny % top || d->nz % top) {
    msg = p->levels == 2 ? "the cell edge must be >= 1 and twice the cell edge divide nx, ny and nz"
                         : "the cell edge must be >= 1 and divide nx, ny and nz";
    return VLB_EINVAL;
  }
  const long long C = (long long)(d->nx / p->cell) * (d->ny / p->cell) * (d->nz / p->cell);
  if (C > (1LL << 22)) { msg = "more than 2^22 cells"; return VLB_EINVAL; }
  return VLB_OK;
}

size_t ff_workspace(const vlb_bs_desc* d, const vlb_ff_params* p, long long n) {
  return ff_layout(n, ff_axes(d, p), true, nullptr, nullptr);
}

hipError_t ff_solo(const vlb_bs_desc* d, const vlb_ff_params* p, long long n, const double* xyz,
                   const int32_t* next, double* v, void* ws, hipStream_t stream) {
  const FfAxes ax = ff_axes(d, p);
  FfBufs b;
  ff_layout(n, ax, true, (char*)ws, &b);
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_ff_init, dim3(nb), dim3(256), 0, stream, b.prv, (int)n);
  hipLaunchKernelGGL(k_ff_prep, dim3(nb), dim3(256), 0, stream, xyz, next, (int)n, ax, b.cnt, b.Pw,
                     b.X, b.nxt, b.prv, b.M, b.D, b.ka, b.kidx, b.va);
  int bits = 1;
  while ((1LL << bits) < ax.C[0]) ++bits;
  uint32_t* sk = nullptr;
  int32_t* so = nullptr;
  hipError_t e = sort_pairs_raw(n, bits, 0, b.stmp, b.ka, b.kb, b.va, b.vb, stream, &sk, &so);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ff_seg, dim3(nb), dim3(256), 0, stream, so, b.X, b.nxt, b.cnt, n, ax,
                     b.recs);
  for (int l = 0; l < ax.levels; ++l) {
    const int C = ax.C[l];
    hipLaunchKernelGGL(k_ff_bounds, dim3((C + 255) / 256), dim3(256), 0, stream, sk, (int)n, C,
                       3 * l, b.cells[l]);
    hipLaunchKernelGGL(k_ff_comps, dim3(nb), dim3(256), 0, stream, b.M, b.D, b.kidx, b.cnt, n,
                       ax, l, b.comps, b.srad);
    hipLaunchKernelGGL(k_ff_order, dim3((unsigned)(3 * C)), dim3(64), 0, stream, so, b.comps,
                       b.srad, b.X, n, ax, l, b.cells[l], b.sdel[l], b.sidx[l], b.pre[l]);
  }
  const dim3 grid((unsigned)((n + kFfTargets - 1) / kFfTargets), b.S);
#define FF_EVAL(U, LV)                                                                         \
  hipLaunchKernelGGL((k_ff_eval<U, LV>), grid, dim3(256), 0, stream, b.cells[0], b.cells[1],   \
                     b.recs, so, b.kidx, b.prv, b.Pw, b.X, b.sdel[0], b.sdel[1], b.pre[0],     \
                     b.pre[1], b.cnt, n, b.S, ax, b.P)
  if (ax.uniform) {
    if (ax.levels == 2) FF_EVAL(true, 2); else FF_EVAL(true, 1);
  } else {
    if (ax.levels == 2) FF_EVAL(false, 2); else FF_EVAL(false, 1);
  }
#undef FF_EVAL
  hipLaunchKernelGGL(k_ff_sum, dim3(nb), dim3(256), 0, stream, b.P, b.S, (int)n,
                     d->kappa / (4.0 * M_PI), v);
  return hipGetLastError();
}

namespace {

FfAxes ff_run_axes(const Run& r) {
  const vlb_bs_desc bd{r.lat.nx, r.lat.ny, r.lat.nz, 0u, VLB_F32, 0, r.vor.kappa};
  const vlb_ff_params fp{r.vor.ff_cell, r.vor.ff_levels, r.vor.ff_theta};
  return ff_axes(&bd, &fp);
}

}  // namespace

size_t ff_run_bytes(const Run& r) {
  return ff_layout(r.ncap, ff_run_axes(r), false, nullptr, nullptr);
}

int ff_run_chunks(const Run& r) {
  const FfAxes ax = ff_run_axes(r);
  return ff_chunks(r.ncap, ax.C[ax.levels - 1]);
}

hipError_t ff_run_sum(Run& r, const double* Y) {
  const FfAxes ax = ff_run_axes(r);
  const long long nc = r.ncap;
  hipStream_t stream = r.stream;
  FfBufs b;
  ff_layout(nc, ax, false, (char*)r.ffws, &b);
  hipEvent_t t0 = nullptr;
  time_begin(r, 0, &t0);
  const int nb = (int)((nc + 255) / 256);
  hipLaunchKernelGGL(k_ff_prep_run, dim3(nb), dim3(256), 0, stream, Y, r.nxt, r.cnt, nc, ax, b.Pw,
                     b.X, b.M, b.D, b.ka, b.kidx, b.va);
  int bits = 1;
  while ((1LL << bits) < ax.C[0]) ++bits;
  uint32_t* sk = nullptr;
  int32_t* so = nullptr;
  hipError_t e = sort_pairs_raw(nc, bits, 0, b.stmp, b.ka, b.kb, b.va, b.vb, stream, &sk, &so);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ff_seg, dim3(nb), dim3(256), 0, stream, so, b.X, r.nxt, r.cnt, nc, ax,
                     b.recs);
  for (int l = 0; l < ax.levels; ++l) {
    const int C = ax.C[l];
    hipLaunchKernelGGL(k_ff_bounds, dim3((C + 255) / 256), dim3(256), 0, stream, sk, (int)nc, C,
                       3 * l, b.cells[l]);
    hipLaunchKernelGGL(k_ff_comps, dim3(nb), dim3(256), 0, stream, b.M, b.D, b.kidx, r.cnt, nc,
                       ax, l, b.comps, b.srad);
    hipLaunchKernelGGL(k_ff_order, dim3((unsigned)(3 * C)), dim3(64), 0, stream, so, b.comps,
                       b.srad, b.X, nc, ax, l, b.cells[l], b.sdel[l], b.sidx[l], b.pre[l]);
  }
  const dim3 grid((unsigned)((nc + kFfTargets - 1) / kFfTargets), r.ffS);
#define FF_EVAL(U, LV)                                                                         \
  hipLaunchKernelGGL((k_ff_eval<U, LV>), grid, dim3(256), 0, stream, b.cells[0], b.cells[1],   \
                     b.recs, so, b.kidx, r.prv, b.Pw, b.X, b.sdel[0], b.sdel[1], b.pre[0],     \
                     b.pre[1], r.cnt, nc, r.ffS, ax, (float*)r.bsP)
  if (ax.uniform) {
    if (ax.levels == 2) FF_EVAL(true, 2); else FF_EVAL(true, 1);
  } else {
    if (ax.levels == 2) FF_EVAL(false, 2); else FF_EVAL(false, 1);
  }
#undef FF_EVAL
  time_end(r, 0, t0);
  return hipGetLastError();
}

}  // namespace vlb
