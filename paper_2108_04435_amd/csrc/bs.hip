// Biot-Savart non-local superfluid velocity (paper Sec. II.A, Eq.
// Biot-Savart): every target point j sums the exact straight-segment
// integral over all segments k = (s_k, s_next(k)) except the two that touch
// it (k = prev(j) and k = j; their divergent contribution is the LIA term).
//
// Layout and decomposition:
//  * per point: 32-bit grid coordinates X (3 x u32, SoA); the segment
//    vector d_k = s_next(k) - s_k is the wrapped grid difference in the FP32
//    sum and an FP64 nearest-image vector in the FP64 sum;
//  * a 2-D grid: blockIdx.x picks 64 consecutive targets (one per lane of
//    every wave), blockIdx.y one contiguous chunk of sources; the chunk is
//    staged through LDS in tiles of 256 sources, each of the block's 4
//    waves walks its own quarter of the tile, and the 4 wave sums are added
//    in LDS in a fixed order at the end (fewer, longer chunks than with one
//    wave per target, so fewer partial sums to write and to add);
//  * the separation R1 = s_k - r is the wrapped integer difference of the
//    grid coordinates, converted to floating point: exact nearest periodic
//    image and a relative (not absolute) rounding error for near pairs;
//  * each chunk writes one partial sum per target; the finalize kernel adds
//    the chunks in a fixed order (no atomics, bitwise reproducible).
#include "vlb_internal.h"

#include <cmath>

namespace vlb {

namespace {

constexpr int kTile = 256;
constexpr int kTargets = 64;  // targets per block, one per lane of each wave

// Quarter of a staged tile of cnt sources walked by wave w: [lo, hi) (empty
// when lo >= hi), lo a multiple of 4 so that the unrolled loop reads the
// tile with 16-byte loads.
__device__ inline void wave_range(int cnt, int w, int& lo, int& hi) {
  const int q = (((cnt + 3) >> 2) + 3) & ~3;
  lo = w * q;
  hi = __builtin_amdgcn_readfirstlane(min(cnt, lo + q));
}

// Grid coordinates of the points at positions Y, and for the FP64 path the
// segment vectors (nearest image, lattice units) and the residuals
// rho = (y + off) - X / q of the positions below their grid value (taken
// with the unwrapped grid value), so that y_s - y_t of the image the grid
// difference chooses is (X_s - X_t) / q + rho_s - rho_t.  The FP32 sum
// takes each segment vector as the wrapped grid difference to the successor.
//
// With image copies (own non-null), own[j] is the copy mirrored in the wall
// that point j is bound to when j is an end of an open line (the lowest
// closed axis whose wall plane it lies on; nothing else reflected), else 0:
// in that copy the images of j's two segments meet j and are excluded, as
// the real ones are in copy 0.
template <class T>
__global__ void k_prep(const double* __restrict__ Y, const int32_t* __restrict__ nxt,
                       const int32_t* __restrict__ prv, const int32_t* __restrict__ cnt,
                       long long ncap, BsAxes ax, uint32_t* __restrict__ X, T* __restrict__ D,
                       int32_t* __restrict__ own) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = cnt[0];
  if (j >= n) return;
  const int k = nxt[j];
  double y[3], d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    y[a] = Y[a * ncap + j];
    d[a] = Y[a * ncap + k] - y[a];
    if (ax.periodic[a]) {
      if (d[a] > 0.5 * ax.L[a])
        d[a] = d[a] - ax.L[a];
      else if (d[a] < -0.5 * ax.L[a])
        d[a] = d[a] + ax.L[a];
    }
  }
  if (own) {
    int oc = 0;
    if (k == j || prv[j] == j) {
      int ea = -1, es = 0;
      for (int a = 2; a >= 0; --a)
        if (!ax.periodic[a] && (y[a] == -0.5 || y[a] == ax.L[a] - 0.5)) {
          ea = a;
          es = y[a] == -0.5 ? 1 : 2;
        }
      if (ea >= 0)
        for (int c = 1; c < ax.copies; ++c) {
          bool only = true;
          for (int a = 0; a < 3; ++a) only = only && ax.refl[c][a] == (a == ea ? es : 0);
          if (only) oc = c;
        }
    }
    own[j] = oc;
  }
  // copy 0: the point itself; copies 1..: its images in the wall planes
  for (int c = 0; c < ax.copies; ++c) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int m = ax.refl[c][a];
      const double yc = m == 0 ? y[a] : (m == 1 ? 2.0 * (-0.5) - y[a] : 2.0 * (ax.L[a] - 0.5) - y[a]);
      const double s = floor((yc + ax.off[a]) * ax.q[a]);
      X[((long long)c * 3 + a) * ncap + j] =
          ax.periodic[a] ? (uint32_t)(long long)s : (uint32_t)(int)(long long)s;
      if (sizeof(T) == 8) {
        D[((long long)c * 6 + a) * ncap + j] = (T)(m == 0 ? d[a] : -d[a]);
        D[((long long)c * 6 + 3 + a) * ncap + j] = (T)((yc + ax.off[a]) - s * ax.invq_d[a]);
      }
    }
  }
}

// FP32 pair sum.  Per pair, with R1 = s_k - r (from the grid difference)
// and d = s_next(k) - s_k:
//   R1 x R2 = R1 x d,  R1.R2 = |R1|^2 + R1.d,  |R2|^2 = |R1|^2 + 2 R1.d + |d|^2,
//   v = (R1 x R2) (i1 + i2) i1 i2 / (1 + (R1.R2) i1 i2),  i_m = 1/|R_m|,
// the closed form (|R1| + |R2|) / (|R1||R2| (|R1||R2| + R1.R2)) rewritten with
// inverse norms.  Uniform grid: R1 stays in grid units and the result is
// rescaled once per target (v is homogeneous of degree -1 in R).
template <bool kCheck, bool kUniform>
__device__ inline void bs_tile_f32(const uint32_t* sx, const uint32_t* sy, const uint32_t* sz,
                                   const float* dx, const float* dy, const float* dz,
                                   const float* dq, int cnt, int t0, uint32_t xt, uint32_t yt,
                                   uint32_t zt, float iqx, float iqy, float iqz, int jj, int pj,
                                   float& ax, float& ay, float& az) {
  // unrolled twice: 52 VGPRs, 8 waves per SIMD (four ways: 79 VGPRs and 6
  // waves, 2.6% slower although a quarter instruction per pair shorter)
#pragma unroll 2
  for (int s = 0; s < cnt; ++s) {
    float r1x = (float)(int)(sx[s] - xt);
    float r1y = (float)(int)(sy[s] - yt);
    float r1z = (float)(int)(sz[s] - zt);
    if (!kUniform) {
      r1x *= iqx;
      r1y *= iqy;
      r1z *= iqz;
    }
    const float ex = dx[s], ey = dy[s], ez = dz[s];
    const float t = r1x * ex + r1y * ey + r1z * ez;
    const float n1 = r1x * r1x + r1y * r1y + r1z * r1z;
    const float n2 = fmaf(2.0f, t, n1 + dq[s]);
    const float i1 = __builtin_amdgcn_rsqf(n1);
    const float i2 = __builtin_amdgcn_rsqf(n2);
    const float crx = r1y * ez - r1z * ey;
    const float cry = r1z * ex - r1x * ez;
    const float crz = r1x * ey - r1y * ex;
    const float a = i1 * i2;
    const float den = fmaf(n1 + t, a, 1.0f);
    float f = (i1 + i2) * a * __builtin_amdgcn_rcpf(den);
    if (kCheck) {
      const int k = t0 + s;
      f = (k == jj || k == pj) ? 0.0f : f;
    }
    ax = fmaf(f, crx, ax);
    ay = fmaf(f, cry, ay);
    az = fmaf(f, crz, az);
  }
}

// Grid y: S chunks of every source copy (copy 0 the filaments, the others
// their wall images, which take no exclusion and carry the copy's sign).
template <bool kUniform>
__global__ __launch_bounds__(256) void k_bs_f32(const uint32_t* __restrict__ X,
                                               const int32_t* __restrict__ nxt,
                                               const int32_t* __restrict__ prv,
                                               int32_t* __restrict__ cntp, long long ncap,
                                               int S, float iqx, float iqy, float iqz,
                                               float* __restrict__ P, BsAxes bx,
                                               const int32_t* __restrict__ own) {
  const int n = cntp[0];
  // work counter: (target, segment) pairs of this sum
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && n > 2)
    *(long long*)(cntp + 16) += (long long)n * (n - 2) + (long long)(bx.copies - 1) * n * n;
  const int j0 = blockIdx.x * kTargets;
  if (j0 >= n) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int j = j0 + lane;
  const bool valid = j < n;
  const int copy = blockIdx.y / S;
  const uint32_t* __restrict__ Xs = X + (long long)copy * 3 * ncap;  // this copy's sources
  const int per = (n + S - 1) / S;
  const int kb = (blockIdx.y - copy * S) * per;
  const int ke = min(n, kb + per);
  const uint32_t xt = valid ? X[j] : 0u;
  const uint32_t yt = valid ? X[ncap + j] : 0u;
  const uint32_t zt = valid ? X[2 * ncap + j] : 0u;
  // the target's own two segments are excluded in copy 0 and, for the end
  // of an open line, in the copy mirrored in its wall
  const int oc = (valid && own) ? own[j] : 0;
  const bool exl = valid && (copy == 0 || copy == oc);
  const int pj = exl ? prv[j] : -1;
  const int jj = exl ? j : -1;
  __shared__ __align__(16) uint32_t sx[kTile], sy[kTile], sz[kTile];
  __shared__ __align__(16) float dx[kTile], dy[kTile], dz[kTile], dq[kTile];
  __shared__ float red[3][3][kTargets];  // sums of waves 1..3
  float ax = 0.f, ay = 0.f, az = 0.f;
  for (int t0 = kb; t0 < ke; t0 += kTile) {
    const int k = t0 + threadIdx.x;
    if (k < ke) {
      // segment vector: wrapped grid difference to the successor
      const int kn = nxt[k];
      const uint32_t ax0 = Xs[k], ay0 = Xs[ncap + k], az0 = Xs[2 * ncap + k];
      float ex = (float)(int)(Xs[kn] - ax0);
      float ey = (float)(int)(Xs[ncap + kn] - ay0);
      float ez = (float)(int)(Xs[2 * ncap + kn] - az0);
      if (!kUniform) {
        ex *= iqx;
        ey *= iqy;
        ez *= iqz;
      }
      sx[threadIdx.x] = ax0;
      sy[threadIdx.x] = ay0;
      sz[threadIdx.x] = az0;
      dx[threadIdx.x] = ex;
      dy[threadIdx.x] = ey;
      dz[threadIdx.x] = ez;
      dq[threadIdx.x] = ex * ex + ey * ey + ez * ez;
    }
    __syncthreads();
    int lo, hi;
    wave_range(min(kTile, ke - t0), w, lo, hi);
    if (lo < hi) {
      const int s0 = t0 + lo, s1 = t0 + hi;
      const bool hit = exl && ((jj >= s0 && jj < s1) || (pj >= s0 && pj < s1));
      if (__any(hit))
        bs_tile_f32<true, kUniform>(sx + lo, sy + lo, sz + lo, dx + lo, dy + lo, dz + lo, dq + lo,
                                    hi - lo, s0, xt, yt, zt, iqx, iqy, iqz, jj, pj, ax, ay, az);
      else
        bs_tile_f32<false, kUniform>(sx + lo, sy + lo, sz + lo, dx + lo, dy + lo, dz + lo, dq + lo,
                                     hi - lo, s0, xt, yt, zt, iqx, iqy, iqz, jj, pj, ax, ay, az);
    }
    __syncthreads();
  }
  if (w > 0) {
    red[w - 1][0][lane] = ax;
    red[w - 1][1][lane] = ay;
    red[w - 1][2][lane] = az;
  }
  __syncthreads();
  if (w == 0 && valid) {
    const float sg = bx.sign[copy];
    float* out = P + (long long)blockIdx.y * 3 * ncap;
    out[j] = sg * (((ax + red[0][0][lane]) + red[1][0][lane]) + red[2][0][lane]);
    out[ncap + j] = sg * (((ay + red[0][1][lane]) + red[1][1][lane]) + red[2][1][lane]);
    out[2 * ncap + j] = sg * (((az + red[0][2][lane]) + red[1][2][lane]) + red[2][2][lane]);
  }
}

// FP64 pair sum (plain path).  R1 = (X_s - X_t) / q + (rho_s - rho_t): the
// wrapped grid difference picks the image (the same decision as the FP32
// sum), the residuals restore the FP64 separation of that image to
// rounding; R2 = R1 + d enters through |R2|^2 = |R1|^2 + 2 R1.d + |d|^2 and
// R1.R2 = |R1|^2 + R1.d, as in the FP32 sum.  The closed form is evaluated
// with the inverse norms and the reciprocal of the hardware approximations
// (relative error up to about 5e-8), each refined by one Newton step (which
// squares it: at most 4.1e-15 for the inverse root and 2.1e-15 for the
// reciprocal over 1e6 arguments from 1e-8 to 1e22, measured against
// long-double references), and the same checked / unchecked tile split as
// the FP32 sum.
__device__ inline double rsq_nr(double n) {
  const double y = __builtin_amdgcn_rsq(n);
  const double e = fma(-(n * y), y, 1.0);  // 1 - n y^2
  return fma(0.5 * y, e, y);
}

__device__ inline double rcp_nr(double d) {
  const double q = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, q, 1.0);
  return fma(q, e, q);
}

template <bool kCheck>
__device__ inline void bs_tile_f64(const uint32_t* sx, const uint32_t* sy, const uint32_t* sz,
                                   const double* rx, const double* ry, const double* rz,
                                   const double* dx, const double* dy, const double* dz,
                                   const double* dq, int cnt,
                                   int t0, uint32_t xt, uint32_t yt, uint32_t zt, double rtx,
                                   double rty, double rtz, double gx, double gy, double gz, int jj,
                                   int pj, double& ax, double& ay, double& az) {
#pragma unroll 2
  for (int s = 0; s < cnt; ++s) {
    const double r1x = fma((double)(int)(sx[s] - xt), gx, rx[s] - rtx);
    const double r1y = fma((double)(int)(sy[s] - yt), gy, ry[s] - rty);
    const double r1z = fma((double)(int)(sz[s] - zt), gz, rz[s] - rtz);
    const double ex = dx[s], ey = dy[s], ez = dz[s];
    const double t = r1x * ex + r1y * ey + r1z * ez;
    const double n1 = r1x * r1x + r1y * r1y + r1z * r1z;
    const double n2 = fma(2.0, t, n1 + dq[s]);
    const double u = n1 + t;
    const double crx = r1y * ez - r1z * ey;
    const double cry = r1z * ex - r1x * ez;
    const double crz = r1x * ey - r1y * ex;
    const double i1 = rsq_nr(n1);
    const double i2 = rsq_nr(n2);
    const double a = i1 * i2;
    double f = (i1 + i2) * a * rcp_nr(fma(u, a, 1.0));
    if (kCheck) {
      const int k = t0 + s;
      f = (k == jj || k == pj) ? 0.0 : f;
    }
    ax = fma(f, crx, ax);
    ay = fma(f, cry, ay);
    az = fma(f, crz, az);
  }
}

__global__ __launch_bounds__(256) void k_bs_f64(const uint32_t* __restrict__ X,
                                               const double* __restrict__ D,
                                               const int32_t* __restrict__ prv,
                                               int32_t* __restrict__ cntp, long long ncap,
                                               int S, double gx, double gy, double gz,
                                               double* __restrict__ P, BsAxes bx,
                                               const int32_t* __restrict__ own) {
  const int n = cntp[0];
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && n > 2)
    *(long long*)(cntp + 16) += (long long)n * (n - 2) + (long long)(bx.copies - 1) * n * n;
  const int j0 = blockIdx.x * kTargets;
  if (j0 >= n) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int j = j0 + lane;
  const bool valid = j < n;
  const int copy = blockIdx.y / S;
  const uint32_t* __restrict__ Xs = X + (long long)copy * 3 * ncap;  // this copy's sources
  const double* __restrict__ Ds = D + (long long)copy * 6 * ncap;
  const int per = (n + S - 1) / S;
  const int kb = (blockIdx.y - copy * S) * per;
  const int ke = min(n, kb + per);
  const uint32_t xt = valid ? X[j] : 0u;
  const uint32_t yt = valid ? X[ncap + j] : 0u;
  const uint32_t zt = valid ? X[2 * ncap + j] : 0u;
  const double rtx = valid ? D[3 * ncap + j] : 0.0;
  const double rty = valid ? D[4 * ncap + j] : 0.0;
  const double rtz = valid ? D[5 * ncap + j] : 0.0;
  const int oc = (valid && own) ? own[j] : 0;
  const bool exl = valid && (copy == 0 || copy == oc);
  const int pj = exl ? prv[j] : -1;
  const int jj = exl ? j : -1;
  __shared__ __align__(16) uint32_t sx[kTile], sy[kTile], sz[kTile];
  __shared__ __align__(16) double rx[kTile], ry[kTile], rz[kTile];
  __shared__ __align__(16) double dx[kTile], dy[kTile], dz[kTile], dq[kTile];
  __shared__ double red[3][3][kTargets];  // sums of waves 1..3
  double ax = 0.0, ay = 0.0, az = 0.0;
  for (int t0 = kb; t0 < ke; t0 += kTile) {
    const int k = t0 + threadIdx.x;
    if (k < ke) {
      sx[threadIdx.x] = Xs[k];
      sy[threadIdx.x] = Xs[ncap + k];
      sz[threadIdx.x] = Xs[2 * ncap + k];
      const double ex = Ds[k], ey = Ds[ncap + k], ez = Ds[2 * ncap + k];
      dx[threadIdx.x] = ex;
      dy[threadIdx.x] = ey;
      dz[threadIdx.x] = ez;
      dq[threadIdx.x] = ex * ex + ey * ey + ez * ez;
      rx[threadIdx.x] = Ds[3 * ncap + k];
      ry[threadIdx.x] = Ds[4 * ncap + k];
      rz[threadIdx.x] = Ds[5 * ncap + k];
    }
    __syncthreads();
    int lo, hi;
    wave_range(min(kTile, ke - t0), w, lo, hi);
    if (lo < hi) {
      const int s0 = t0 + lo, s1 = t0 + hi;
      const bool hit = exl && ((jj >= s0 && jj < s1) || (pj >= s0 && pj < s1));
      if (__any(hit))
        bs_tile_f64<true>(sx + lo, sy + lo, sz + lo, rx + lo, ry + lo, rz + lo, dx + lo, dy + lo,
                          dz + lo, dq + lo, hi - lo, s0, xt, yt, zt, rtx, rty, rtz, gx, gy, gz, jj,
                          pj, ax, ay, az);
      else
        bs_tile_f64<false>(sx + lo, sy + lo, sz + lo, rx + lo, ry + lo, rz + lo, dx + lo, dy + lo,
                           dz + lo, dq + lo, hi - lo, s0, xt, yt, zt, rtx, rty, rtz, gx, gy, gz, jj,
                           pj, ax, ay, az);
    }
    __syncthreads();
  }
  if (w > 0) {
    red[w - 1][0][lane] = ax;
    red[w - 1][1][lane] = ay;
    red[w - 1][2][lane] = az;
  }
  __syncthreads();
  if (w == 0 && valid) {
    const double sg = (double)bx.sign[copy];
    double* out = P + (long long)blockIdx.y * 3 * ncap;
    out[j] = sg * (((ax + red[0][0][lane]) + red[1][0][lane]) + red[2][0][lane]);
    out[ncap + j] = sg * (((ay + red[0][1][lane]) + red[1][1][lane]) + red[2][1][lane]);
    out[2 * ncap + j] = sg * (((az + red[0][2][lane]) + red[1][2][lane]) + red[2][2][lane]);
  }
}

// ---- standalone sum (positions and links from the caller, no run)

// Links and grid data of a caller's filaments: next is clamped into [0, n)
// (an invalid permutation gives meaningless velocities, never an access out
// of bounds) and inverted into prev; grid coordinates and, for the FP64
// sum, segment vectors and residuals as k_prep, from [n][3] positions.
// Thread 0 writes the point count and clears the pair counter.
// prv[j] = j: the first point of an open line keeps it (no real link to it)
__global__ void k_solo_init(int32_t* __restrict__ prv, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) prv[j] = j;
}

template <class T>
__global__ void k_solo_prep(const double* __restrict__ xyz, const int32_t* __restrict__ next,
                            int n, BsAxes ax, int32_t* __restrict__ cnt,
                            uint32_t* __restrict__ X, T* __restrict__ D,
                            int32_t* __restrict__ nxt, int32_t* __restrict__ prv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) {
    cnt[0] = n;
    for (int i = 1; i < 32; ++i) cnt[i] = 0;
  }
  if (j >= n) return;
  const int k = min(max(next[j], 0), n - 1);
  nxt[j] = k;
  if (k != j) prv[k] = j;  // the last point of an open line links to itself
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double y = xyz[3LL * j + a];
    const double s = floor((y + ax.off[a]) * ax.q[a]);
    X[(long long)a * n + j] = ax.periodic[a] ? (uint32_t)(long long)s
                                             : (uint32_t)(int)(long long)s;
    if (sizeof(T) == 8) {
      double d = xyz[3LL * k + a] - y;
      if (ax.periodic[a]) {
        if (d > 0.5 * ax.L[a])
          d = d - ax.L[a];
        else if (d < -0.5 * ax.L[a])
          d = d + ax.L[a];
      }
      D[(long long)a * n + j] = (T)d;
      D[(long long)(3 + a) * n + j] = (T)((y + ax.off[a]) - s * ax.invq_d[a]);
    }
  }
}

// v[j][a] = scale * (sum over the S chunk partials of target j, in chunk
// order, in FP64).
template <class PT>
__global__ void k_solo_sum(const PT* __restrict__ P, int S, int n, double scale,
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

}  // namespace

// Grid of the Biot-Savart sum on a box of n[a] nodes per axis (wall[a]: the
// axis is closed, positions in [-1/2, n - 1/2]; else periodic of length
// n[a]): periodic axes map [0, L) onto the whole 32-bit range, so that
// separations wrap exactly; wall axes use a power-of-two step with room
// for [-1, n + 1).
BsAxes bs_make_axes(const int n[3], const int wall[3], bool images) {
  BsAxes ax{};
  for (int a = 0; a < 3; ++a) {
    ax.L[a] = (double)n[a];
    ax.periodic[a] = !wall[a];
    if (ax.periodic[a]) {
      ax.q[a] = 4294967296.0 / (double)n[a];
      ax.off[a] = 0.0;
      ax.invq_d[a] = (double)n[a] / 4294967296.0;
    } else {
      // [-1, n + 1), or with wall images [-n - 1, 2n + 1)
      const double span = images ? 3.0 * n[a] + 2.0 : n[a] + 2.0;
      int k = 0;
      while (span * std::ldexp(1.0, k + 1) <= 2147483648.0) ++k;
      ax.q[a] = std::ldexp(1.0, k);
      ax.off[a] = images ? n[a] + 1.0 : 1.0;
      ax.invq_d[a] = std::ldexp(1.0, -k);
    }
    ax.invq_f[a] = (float)ax.invq_d[a];
  }
  {
    // one power-of-two grid step for all axes when every periodic axis has
    // the same power-of-two length and the wall axes fit that step
    double q = 0.0;
    for (int a = 0; a < 3; ++a)
      if (ax.periodic[a]) q = ax.q[a];
    if (q == 0.0)
      for (int a = 0; a < 3; ++a) q = (q == 0.0 || ax.q[a] < q) ? ax.q[a] : q;
    int ex = 0;
    bool ok = std::frexp(q, &ex) == 0.5;
    for (int a = 0; a < 3 && ok; ++a) {
      if (ax.periodic[a])
        ok = ax.q[a] == q;
      else
        ok = (images ? 3.0 * n[a] + 2.0 : n[a] + 2.0) * q <= 2147483648.0;
    }
    ax.uniform = ok ? 1 : 0;
    if (ok)
      for (int a = 0; a < 3; ++a) {
        ax.q[a] = q;
        ax.invq_d[a] = 1.0 / q;
        ax.invq_f[a] = (float)ax.invq_d[a];
      }
  }
  // source copies: every combination of no / lower / upper reflection on
  // the closed axes (the identity first)
  ax.copies = 0;
  for (int cz = 0; cz < 3; ++cz)
    for (int cy = 0; cy < 3; ++cy)
      for (int cx = 0; cx < 3; ++cx) {
        const int code[3] = {cx, cy, cz};
        bool ok = true;
        int refl = 0;
        for (int a = 0; a < 3; ++a) {
          if (code[a] && (!images || !wall[a])) ok = false;
          if (code[a]) ++refl;
        }
        if (!ok) continue;
        for (int a = 0; a < 3; ++a) ax.refl[ax.copies][a] = (int8_t)code[a];
        ax.sign[ax.copies] = (refl & 1) ? -1.0f : 1.0f;
        ++ax.copies;
      }
  return ax;
}

// Source chunks S: about 16384 blocks over the target blocks, or up to
// 32768 while every chunk keeps at least 1024 sources (large point counts:
// the launch's tail shortens), at least 256 sources per chunk (64 per
// wave), at most 256 chunks; the chunk partials are added by the finalize
// kernel.  (At 1.2e4 points 512 and 1024 sources per chunk measured 1.5%
// and 6% slower per step, 128 and 192 no faster; at 1.0e5 points 14 chunks
// instead of 7 measured 1.1% faster, at 5e4 points 28 instead of 14 0.9%.)
int bs_chunks(long long ncap) {
  const long long tb = (ncap + kTargets - 1) / kTargets;
  const long long t = tb > 0 ? tb : 1;
  long long S = 16384 / t;
  const long long wide = std::min(32768 / t, ncap / 1024);
  if (wide > S) S = wide;
  const long long maxS = ncap / 256;
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  if (S > 256) S = 256;
  return (int)S;
}

hipError_t bs_prep(Run& r, const double* Y) {
  const int nb = (int)((r.ncap + 255) / 256);
  int32_t* own = r.bsax.copies > 1 ? r.bsown : nullptr;
  if (r.prec == VLB_F64)
    hipLaunchKernelGGL(k_prep<double>, dim3(nb), dim3(256), 0, r.stream, Y, r.nxt, r.prv, r.cnt,
                       r.ncap, r.bsax, r.bsX, (double*)r.bsD, own);
  else
    hipLaunchKernelGGL(k_prep<float>, dim3(nb), dim3(256), 0, r.stream, Y, r.nxt, r.prv, r.cnt,
                       r.ncap, r.bsax, r.bsX, (float*)r.bsD, own);
  return hipGetLastError();
}

hipError_t bs_sum(Run& r) {
  const int tb = (int)((r.ncap + kTargets - 1) / kTargets);
  dim3 grid(tb, r.bsS * r.bsax.copies);
  hipEvent_t b = nullptr;
  time_begin(r, 0, &b);
  const int32_t* own = r.bsax.copies > 1 ? r.bsown : nullptr;
  if (r.prec == VLB_F64)
    hipLaunchKernelGGL(k_bs_f64, grid, dim3(256), 0, r.stream, r.bsX, (const double*)r.bsD,
                       r.prv, r.cnt, r.ncap, r.bsS, r.bsax.invq_d[0], r.bsax.invq_d[1],
                       r.bsax.invq_d[2], (double*)r.bsP, r.bsax, own);
  else if (r.bsax.uniform)
    hipLaunchKernelGGL(k_bs_f32<true>, grid, dim3(256), 0, r.stream, r.bsX, r.nxt,
                       r.prv, r.cnt, r.ncap, r.bsS, r.bsax.invq_f[0], r.bsax.invq_f[1],
                       r.bsax.invq_f[2], (float*)r.bsP, r.bsax, own);
  else
    hipLaunchKernelGGL(k_bs_f32<false>, grid, dim3(256), 0, r.stream, r.bsX, r.nxt,
                       r.prv, r.cnt, r.ncap, r.bsS, r.bsax.invq_f[0], r.bsax.invq_f[1],
                       r.bsax.invq_f[2], (float*)r.bsP, r.bsax, own);
  time_end(r, 0, b);
  return hipGetLastError();
}

int bs_check_desc(const vlb_bs_desc* d, int64_t n, std::string& msg) {
  if (!d) { msg = "null descriptor"; return VLB_EINVAL; }
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > (1 << 24) || d->ny > (1 << 24) ||
      d->nz > (1 << 24)) { msg = "box dimensions must be in [1, 2^24]"; return VLB_EINVAL; }
  if (d->wall_axes & ~7u) { msg = "wall_axes uses bits 0..2 only"; return VLB_EINVAL; }
  if (d->precision < 0 || d->precision > 2) { msg = "precision must be VLB_F64, VLB_F32 or VLB_F16"; return VLB_EINVAL; }
  if (!(d->kappa > 0) || !std::isfinite(d->kappa)) { msg = "kappa must be positive and finite"; return VLB_EINVAL; }
  if (n < 0 || n > kSoloMaxPoints) { msg = "n_pts must be in [0, 2^26]"; return VLB_EINVAL; }
  return VLB_OK;
}

// Standalone sum: the chunk count, scratch layout and launches.  The
// chunks are capped at kSoloChunks, so that the scratch of the largest
// allocation-free call stays small.
constexpr int kSoloChunks = 8;

int bs_solo_chunks(long long n) {
  const int S = bs_chunks(n);
  return S < kSoloChunks ? S : kSoloChunks;
}

size_t bs_solo_layout(int prec, long long n, char* base, BsSolo* b) {
  const size_t fe = prec == VLB_F64 ? 8 : 4;
  const int S = bs_solo_chunks(n);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    off = (off + 255) / 256 * 256;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  BsSolo s{};
  s.cnt = (int32_t*)take(32 * sizeof(int32_t));
  s.X = (uint32_t*)take(3 * (size_t)n * sizeof(uint32_t));
  s.D = take((prec == VLB_F64 ? 6 : 1) * (size_t)n * fe);
  s.nxt = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.prv = (int32_t*)take((size_t)n * sizeof(int32_t));
  s.P = take((size_t)S * 3 * n * fe);
  s.S = S;
  if (b) *b = s;
  return (off + 255) / 256 * 256;
}

hipError_t bs_solo(const BsAxes& ax, int prec, long long n, const double* xyz,
                   const int32_t* next, double kappa, double* v, const BsSolo& b,
                   hipStream_t stream) {
  const int nb = (int)((n + 255) / 256);
  const int tb = (int)((n + kTargets - 1) / kTargets);
  const dim3 grid(tb, b.S);
  const double s = kappa / (4.0 * M_PI);
  hipLaunchKernelGGL(k_solo_init, dim3(nb), dim3(256), 0, stream, b.prv, (int)n);
  if (prec == VLB_F64) {
    hipLaunchKernelGGL(k_solo_prep<double>, dim3(nb), dim3(256), 0, stream, xyz, next, (int)n,
                       ax, b.cnt, b.X, (double*)b.D, b.nxt, b.prv);
    hipLaunchKernelGGL(k_bs_f64, grid, dim3(256), 0, stream, b.X, (const double*)b.D, b.prv,
                       b.cnt, n, b.S, ax.invq_d[0], ax.invq_d[1], ax.invq_d[2], (double*)b.P, ax,
                       nullptr);
    hipLaunchKernelGGL(k_solo_sum<double>, dim3(nb), dim3(256), 0, stream, (const double*)b.P,
                       b.S, (int)n, s, v);
  } else {
    hipLaunchKernelGGL(k_solo_prep<float>, dim3(nb), dim3(256), 0, stream, xyz, next, (int)n,
                       ax, b.cnt, b.X, (float*)b.D, b.nxt, b.prv);
    if (ax.uniform)
      hipLaunchKernelGGL(k_bs_f32<true>, grid, dim3(256), 0, stream, b.X, b.nxt, b.prv, b.cnt,
                         n, b.S, ax.invq_f[0], ax.invq_f[1], ax.invq_f[2], (float*)b.P, ax,
                         nullptr);
    else
      hipLaunchKernelGGL(k_bs_f32<false>, grid, dim3(256), 0, stream, b.X, b.nxt, b.prv, b.cnt,
                         n, b.S, ax.invq_f[0], ax.invq_f[1], ax.invq_f[2], (float*)b.P, ax,
                         nullptr);
    hipLaunchKernelGGL(k_solo_sum<float>, dim3(nb), dim3(256), 0, stream, (const float*)b.P,
                       b.S, (int)n, ax.uniform ? s * ax.q[0] : s, v);
  }
  return hipGetLastError();
}

}  // namespace vlb
