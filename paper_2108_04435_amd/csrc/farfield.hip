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
//    that axis, the other the rest; otherwise direct.
//
// Layout (workspace, all per call):
//  * per point: wrapped FP64 positions, grid coordinates, links, y and d
//    (FP64), cell key;
//  * segments sorted by cell (stable radix sort, so ascending index inside
//    a cell), one 32-byte record each for the direct loop;
//  * one 256-byte record per cell (range, rad^2, centre, grid centre,
//    delta extremes, 36 moments), read with scalar loads;
//  * per axis: each cell's deltas in ascending order and the prefix sums of
//    the 36 moment components over that order (cnt + 1 rows per cell);
//  * the evaluation grid: blockIdx.x picks 64 targets (consecutive in the
//    cell order, so a wave's targets are close), blockIdx.y one of S cell
//    chunks; the 4 waves of a block take interleaved cells (c = 4 y + w
//    modulo 4 S) and add their sums in LDS in a fixed order; the chunk
//    partials are added in FP64 in chunk order (bitwise reproducible).
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
  double L[3], q[3], h, th2;
  float iqf[3];  // lattice units per grid step
  float qf;      // one grid step count per lattice unit when uniform
  int nc[3];
  int C;
  int uniform;
};

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

// Per point: wrapped position, grid coordinate, links, segment vector,
// midpoint cell, y; sort keys (cell) and values (index).
__global__ void k_ff_prep(const double* __restrict__ xyz, const int32_t* __restrict__ next, int n,
                          FfAxes ax, int32_t* __restrict__ cnt, double* __restrict__ P,
                          uint32_t* __restrict__ X, int32_t* __restrict__ nxt,
                          int32_t* __restrict__ prv, double* __restrict__ Y,
                          double* __restrict__ D, uint32_t* __restrict__ keys,
                          int32_t* __restrict__ kidx, int32_t* __restrict__ vals) {
#pragma clang fp contract(off)
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) {
    cnt[0] = n;
    for (int i = 1; i < 32; ++i) cnt[i] = 0;
  }
  if (j >= n) return;
  const int k = min(max(next[j], 0), n - 1);
  nxt[j] = k;
  if (k != j) prv[k] = j;
  int idx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double L = ax.L[a];
    const double p = ff_wrap(xyz[3LL * j + a], L);
    const double pk = ff_wrap(xyz[3LL * k + a], L);
    P[(long long)a * n + j] = p;
    X[(long long)a * n + j] = (uint32_t)(long long)floor(p * ax.q[a]);
    double d = pk - p;
    if (d > 0.5 * L)
      d = d - L;
    else if (d < -0.5 * L)
      d = d + L;
    double mid = p + 0.5 * d;
    mid = mid - L * floor(mid / L);
    int i = (int)floor(mid / ax.h);
    i = min(max(i, 0), ax.nc[a] - 1);
    idx[a] = i;
    double y = mid - ((double)i + 0.5) * ax.h;
    if (y > 0.5 * L)
      y = y - L;
    else if (y < -0.5 * L)
      y = y + L;
    Y[(long long)a * n + j] = y;
    D[(long long)a * n + j] = d;
  }
  const int key = (idx[2] * ax.nc[1] + idx[1]) * ax.nc[0] + idx[0];
  keys[j] = (uint32_t)key;
  kidx[j] = key;
  vals[j] = j;
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

__global__ void k_ff_bounds(const uint32_t* __restrict__ sk, int n, int C,
                            FfCell* __restrict__ cells) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int lo = lower_bound_u32(sk, n, (uint32_t)c);
  const int hi = lower_bound_u32(sk, n, (uint32_t)c + 1u);
  cells[c].start = lo;
  cells[c].count = hi - lo;
}

// One thread per cell: radius, grid centre and the extremes of the start
// offsets (the moments come from the prefix sums).
__global__ void k_ff_cell(const int32_t* __restrict__ so, const double* __restrict__ Y,
                          const double* __restrict__ D, const uint32_t* __restrict__ X, int n,
                          FfAxes ax, FfCell* __restrict__ cells) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ax.C) return;
  const int s = cells[c].start, e = s + cells[c].count;
  const int ci[3] = {c % ax.nc[0], (c / ax.nc[0]) % ax.nc[1], c / (ax.nc[0] * ax.nc[1])};
  double cen[3];
  uint32_t xc[3];
  for (int a = 0; a < 3; ++a) {
    cen[a] = ((double)ci[a] + 0.5) * ax.h;
    xc[a] = (uint32_t)(long long)floor(cen[a] * ax.q[a]);
  }
  double rad = 0.0;
  int dmin[3] = {0, 0, 0}, dmax[3] = {0, 0, 0};
  for (int p = s; p < e; ++p) {
    const int k = so[p];
    double y[3], d[3];
    for (int a = 0; a < 3; ++a) {
      y[a] = Y[(long long)a * n + k];
      d[a] = D[(long long)a * n + k];
      const int dl = (int)(X[(long long)a * n + k] - xc[a]);
      dmin[a] = p == s ? dl : min(dmin[a], dl);
      dmax[a] = p == s ? dl : max(dmax[a], dl);
    }
    const double ny = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    const double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    rad = fmax(rad, ny + 0.5 * nd);
  }
  FfCell& o = cells[c];
  o.rad2 = rad * rad;
  for (int a = 0; a < 3; ++a) {
    o.c[a] = cen[a];
    o.xc[a] = xc[a];
    o.dmin[a] = dmin[a];
    o.dmax[a] = dmax[a];
  }
  o.pad = 0;
}

// Per sorted position: the direct loop's segment record.
__global__ void k_ff_seg(const int32_t* __restrict__ so, const uint32_t* __restrict__ X,
                         const int32_t* __restrict__ nxt, int n, FfAxes ax,
                         FfSeg* __restrict__ recs) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int k = so[p];
  const int kn = nxt[k];
  FfSeg r;
  float dq = 0.f;
  for (int a = 0; a < 3; ++a) {
    const uint32_t x0 = X[(long long)a * n + k];
    float e = (float)(int)(X[(long long)a * n + kn] - x0);
    if (!ax.uniform) e *= ax.iqf[a];
    r.x[a] = x0;
    r.d[a] = e;
  }
  dq = r.d[0] * r.d[0] + r.d[1] * r.d[1] + r.d[2] * r.d[2];
  r.dq = dq;
  r.idx = k;
  recs[p] = r;
}

// Per (sorted position, axis): rank of the segment's start offset inside
// its cell (ties by position), giving each cell's segments in ascending
// offset order: sdel (the offsets) and sidx (the segment indices).
__global__ void k_ff_rank(const uint32_t* __restrict__ sk, const int32_t* __restrict__ so,
                          const uint32_t* __restrict__ X, const FfCell* __restrict__ cells,
                          int n, int32_t* __restrict__ sdel, int32_t* __restrict__ sidx) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3LL * n) return;
  const int a = (int)(t / n), p = (int)(t - (long long)a * n);
  const int c = (int)sk[p];
  const int s = cells[c].start, e = s + cells[c].count;
  const uint32_t xc = cells[c].xc[a];
  const uint32_t* Xa = X + (long long)a * n;
  const int dp = (int)(Xa[so[p]] - xc);
  int rank = 0;
  for (int q = s; q < e; ++q) {
    const int dq = (int)(Xa[so[q]] - xc);
    rank += (dq < dp || (dq == dp && q < p)) ? 1 : 0;
  }
  sdel[(long long)a * n + s + rank] = dp;
  sidx[(long long)a * n + s + rank] = so[p];
}

// Per (cell, axis, component): prefix sums (FP64, stored FP32) of the
// component over the cell's segments in ascending offset order on the
// axis; rows a (n + C) + start + c + i for i = 0..count (row 0 is zero).
// The axis-0 totals are the cell's moments.
__global__ void k_ff_prefix(FfCell* __restrict__ cells, const int32_t* __restrict__ sidx,
                            const double* __restrict__ Y, const double* __restrict__ D, int n,
                            int C, float* __restrict__ pre) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3LL * kMom * C) return;
  const int comp = (int)(t % kMom);
  const long long ca = t / kMom;
  const int a = (int)(ca % 3), c = (int)(ca / 3);
  const int s = cells[c].start, cnt = cells[c].count;
  float* row = pre + ((long long)a * (n + C) + s + c) * kMom + comp;
  double acc = 0.0;
  row[0] = 0.f;
  for (int i = 0; i < cnt; ++i) {
    const int k = sidx[(long long)a * n + s + i];
    double y[3], d[3];
    for (int b = 0; b < 3; ++b) {
      y[b] = Y[(long long)b * n + k];
      d[b] = D[(long long)b * n + k];
    }
    acc = acc + comp_value(comp, y, d);
    row[(long long)(i + 1) * kMom] = (float)acc;
  }
  if (a == 0) cells[c].m[comp] = (float)acc;
}

// Velocity times 4 pi (no kappa) at R = target - centre of the moments m
// (module comment), accumulated into v:
//   v += (M0 x R - A) / r^3 + W x R - 3 B / r^5,
//   W_n = (3 (M1 R)_n - 3/2 tr_n) / r^5 + 15/2 (R M2_n R) / r^7,
//   B_m = eps_mnp (M2_n R)_p.
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

template <bool kUniform>
__global__ __launch_bounds__(256) void k_ff_eval(
    const FfCell* __restrict__ cells, const FfSeg* __restrict__ recs,
    const int32_t* __restrict__ so, const int32_t* __restrict__ kidx,
    const int32_t* __restrict__ prv, const double* __restrict__ Pw,
    const uint32_t* __restrict__ X, const int32_t* __restrict__ sdel,
    const float* __restrict__ pre, int n, int S, FfAxes ax, float* __restrict__ Pout) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = blockIdx.x * kFfTargets + lane;
  const bool valid = t < n;
  const int j = valid ? so[t] : 0;
  double r[3];
  uint32_t xt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = Pw[(long long)a * n + j];
    xt[a] = X[(long long)a * n + j];
  }
  const int pj = valid ? prv[j] : -1;
  const int jj = valid ? j : -1;
  const int kj = valid ? kidx[j] : -1;
  const int kp = valid ? kidx[pj] : -1;
  float fx = 0.f, fy = 0.f, fz = 0.f;  // far part (lattice units)
  float dx = 0.f, dy = 0.f, dz = 0.f;  // direct part (grid units when uniform)
  const int C = ax.C;
  const int step = 4 * S;
  int c = blockIdx.y * 4 + w;
  FfHead hc;
  if (c < C) ff_head(cells + c, hc);
  for (; c < C; c += step) {
    // the next cell's decision fields are loaded while this one is summed
    FfHead hn;
    if (c + step < C) ff_head(cells + c + step, hn);
    const FfCell* __restrict__ cm = cells + c;
    const int cnt = hc.count;
    if (cnt > 0) {
      FfDecision dc;
      ff_decide(&hc, r, xt, ax, dc);
      const bool far = valid && dc.ncross == 0 && dc.ok0;
      bool split = false;
      double R1[3] = {0.0, 0.0, 0.0};
      if (valid && dc.ncross == 1 && dc.ok0) split = ff_other(&hc, dc, r, ax, R1);
      const bool near = valid && !far && !split;
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
          const int32_t* dl = sdel + (long long)a * n + hc.start;
          int lo = 0, hi = cnt;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (dl[mid] < db)
              lo = mid + 1;
            else
              hi = mid;
          }
          const float* pr = pre + ((long long)a * (n + C) + hc.start + c + lo) * kMom;
          m2p_f32((float)-dc.R0[0], (float)-dc.R0[1], (float)-dc.R0[2], MomA{pr}, fx, fy, fz);
          m2p_f32((float)-R1[0], (float)-R1[1], (float)-R1[2], MomD{cm->m, pr}, fx, fy, fz);
        }
      }
      if (__any(near)) {
        const int s0 = hc.start;
        const bool own = __any(kj == c || kp == c);
        if (own) {
          for (int p = s0; p < s0 + cnt; ++p) {
            const FfSeg g = recs[p];
            if (near)
              ff_pair<kUniform>(g, xt[0], xt[1], xt[2], ax, dx, dy, dz, g.idx == jj || g.idx == pj);
          }
        } else {
          for (int p = s0; p < s0 + cnt; ++p) {
            const FfSeg g = recs[p];
            if (near) ff_pair<kUniform>(g, xt[0], xt[1], xt[2], ax, dx, dy, dz, false);
          }
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
    float* out = Pout + (long long)blockIdx.y * 3 * n;
    out[j] = ((fx + red[0][0][lane]) + red[1][0][lane]) + red[2][0][lane];
    out[n + j] = ((fy + red[0][1][lane]) + red[1][1][lane]) + red[2][1][lane];
    out[2LL * n + j] = ((fz + red[0][2][lane]) + red[1][2][lane]) + red[2][2][lane];
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
  bool uniform = true;
  for (int a = 0; a < 3; ++a) {
    ax.L[a] = (double)nn[a];
    ax.q[a] = 4294967296.0 / (double)nn[a];
    ax.iqf[a] = (float)((double)nn[a] / 4294967296.0);
    ax.nc[a] = nn[a] / p->cell;
    uniform = uniform && nn[a] == nn[0];
  }
  // one grid step for all axes: equal power-of-two lengths
  int ex = 0;
  uniform = uniform && std::frexp((double)nn[0], &ex) == 0.5;
  ax.uniform = uniform ? 1 : 0;
  ax.qf = (float)ax.q[0];
  ax.h = (double)p->cell;
  ax.th2 = p->theta * p->theta;
  ax.C = ax.nc[0] * ax.nc[1] * ax.nc[2];
  return ax;
}

int ff_chunks(long long n, int C) {
  const long long tb = (n + kFfTargets - 1) / kFfTargets;
  long long S = (8192 + tb - 1) / tb;
  if (S > C / 4) S = C / 4;
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
  double* Y;
  double* D;
  uint32_t* ka;
  uint32_t* kb;
  int32_t* va;
  int32_t* vb;
  int32_t* kidx;
  void* stmp;
  FfCell* cells;
  FfSeg* recs;
  int32_t* sdel;
  int32_t* sidx;
  float* pre;
  float* P;
  int S;
};

size_t ff_layout(long long n, int C, char* base, FfBufs* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    off = (off + 255) / 256 * 256;
    void* q = base ? base + off : nullptr;
    off += bytes;
    return q;
  };
  FfBufs s{};
  s.S = ff_chunks(n, C);
  s.cnt = (int32_t*)take(32 * sizeof(int32_t));
  s.Pw = (double*)take(3 * (size_t)n * sizeof(double));
  s.X = (uint32_t*)take(3 * (size_t)n * sizeof(uint32_t));
  s.nxt = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.prv = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.Y = (double*)take(3 * (size_t)n * sizeof(double));
  s.D = (double*)take(3 * (size_t)n * sizeof(double));
  s.ka = (uint32_t*)take((size_t)n * sizeof(uint32_t));
  s.kb = (uint32_t*)take((size_t)n * sizeof(uint32_t));
  s.va = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.vb = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.kidx = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.stmp = take(sort_tmp_bytes(n));
  s.cells = (FfCell*)take((size_t)C * sizeof(FfCell));
  s.recs = (FfSeg*)take((size_t)n * sizeof(FfSeg));
  s.sdel = (int32_t*)take(3 * (size_t)n * sizeof(int32_t));
  s.sidx = (int32_t*)take(3 * (size_t)n * sizeof(int32_t));
  s.pre = (float*)take(3 * ((size_t)n + C) * kMom * sizeof(float));
  s.P = (float*)take((size_t)s.S * 3 * n * sizeof(float));
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
  if (p->cell < 1 || d->nx % p->cell || d->ny % p->cell || d->nz % p->cell) {
    msg = "the cell edge must be >= 1 and divide nx, ny and nz";
    return VLB_EINVAL;
  }
  const long long C = (long long)(d->nx / p->cell) * (d->ny / p->cell) * (d->nz / p->cell);
  if (C > (1LL << 22)) { msg = "more than 2^22 cells"; return VLB_EINVAL; }
  return VLB_OK;
}

size_t ff_workspace(const vlb_bs_desc* d, const vlb_ff_params* p, long long n) {
  const int C = (d->nx / p->cell) * (d->ny / p->cell) * (d->nz / p->cell);
  return ff_layout(n, C, nullptr, nullptr);
}

hipError_t ff_solo(const vlb_bs_desc* d, const vlb_ff_params* p, long long n, const double* xyz,
                   const int32_t* next, double* v, void* ws, hipStream_t stream) {
  const FfAxes ax = ff_axes(d, p);
  FfBufs b;
  ff_layout(n, ax.C, (char*)ws, &b);
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_ff_init, dim3(nb), dim3(256), 0, stream, b.prv, (int)n);
  hipLaunchKernelGGL(k_ff_prep, dim3(nb), dim3(256), 0, stream, xyz, next, (int)n, ax, b.cnt, b.Pw,
                     b.X, b.nxt, b.prv, b.Y, b.D, b.ka, b.kidx, b.va);
  int bits = 1;
  while ((1LL << bits) < ax.C) ++bits;
  uint32_t* sk = nullptr;
  int32_t* so = nullptr;
  hipError_t e = sort_pairs_raw(n, bits, 0, b.stmp, b.ka, b.kb, b.va, b.vb, stream, &sk, &so);
  if (e != hipSuccess) return e;
  const int cb = (ax.C + 255) / 256;
  hipLaunchKernelGGL(k_ff_bounds, dim3(cb), dim3(256), 0, stream, sk, (int)n, ax.C, b.cells);
  hipLaunchKernelGGL(k_ff_cell, dim3(cb), dim3(256), 0, stream, so, b.Y, b.D, b.X, (int)n, ax,
                     b.cells);
  hipLaunchKernelGGL(k_ff_seg, dim3(nb), dim3(256), 0, stream, so, b.X, b.nxt, (int)n, ax, b.recs);
  const long long nr = 3LL * n;
  hipLaunchKernelGGL(k_ff_rank, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, stream, sk, so,
                     b.X, b.cells, (int)n, b.sdel, b.sidx);
  const long long np = 3LL * kMom * ax.C;
  hipLaunchKernelGGL(k_ff_prefix, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, stream,
                     b.cells, b.sidx, b.Y, b.D, (int)n, ax.C, b.pre);
  const dim3 grid((unsigned)((n + kFfTargets - 1) / kFfTargets), b.S);
  if (ax.uniform)
    hipLaunchKernelGGL(k_ff_eval<true>, grid, dim3(256), 0, stream, b.cells, b.recs, so, b.kidx,
                       b.prv, b.Pw, b.X, b.sdel, b.pre, (int)n, b.S, ax, b.P);
  else
    hipLaunchKernelGGL(k_ff_eval<false>, grid, dim3(256), 0, stream, b.cells, b.recs, so, b.kidx,
                       b.prv, b.Pw, b.X, b.sdel, b.pre, (int)n, b.S, ax, b.P);
  hipLaunchKernelGGL(k_ff_sum, dim3(nb), dim3(256), 0, stream, b.P, b.S, (int)n,
                     d->kappa / (4.0 * M_PI), v);
  return hipGetLastError();
}

}  // namespace vlb
