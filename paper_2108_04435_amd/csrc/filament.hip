// Per-point filament kernels (paper Sec. II.A and II.B):
//  * finalize: sum of the Biot-Savart partials, local geometry and LIA term,
//    mass-balance superflow, two-point-delta interpolation of the normal
//    fluid, Schwarz line velocity, mutual-friction force and the RK4
//    bookkeeping of one stage;
//  * spreading of the point forces onto the lattice, without atomics on
//    the forces: points are binned by the cell of their stencil's lower
//    corner with the library's stable radix sort; each touched node is then
//    owned by exactly one bin and gathers the contributions of the (at most
//    8) bins around it in a fixed order.
#include "vlb_internal.h"

namespace vlb {

namespace {

// Spreading bins: the lattice cell of the stencil's lower corner.
struct SpreadGeom {
  int n[3];
  int wall[3];
  int ext[3];  // bins per axis: n (periodic) or n + 1 (wall: lower corner -1..n-1)
};

// floor of a coordinate as an int; 0 for a non-finite or absurd value, so
// that a position that blew up still yields an index inside the lattice
// (the non-finite line velocity is reported by its own flag)
__device__ inline int ifloor_safe(double x) {
  const double f = floor(x);
  return (f > -1.0e9 && f < 1.0e9) ? (int)f : 0;
}

__device__ inline uint32_t base_key(const SpreadGeom& sg, const double p[3], int b[3]) {
  for (int a = 0; a < 3; ++a) {
    int c = ifloor_safe(p[a]);
    if (sg.wall[a]) {
      c += 1;  // lower corner -1 .. n-1 -> 0 .. n
      c = c < 0 ? 0 : (c > sg.n[a] ? sg.n[a] : c);
    } else {
      c = ((c % sg.n[a]) + sg.n[a]) % sg.n[a];
    }
    b[a] = c;
  }
  return (uint32_t)(((long long)b[2] * sg.ext[1] + b[1]) * sg.ext[0] + b[0]);
}

SpreadGeom spread_geom(const Run& r) {
  SpreadGeom sg;
  const int n[3] = {r.geom.nx, r.geom.ny, r.geom.nz};
  for (int a = 0; a < 3; ++a) {
    sg.n[a] = n[a];
    sg.wall[a] = r.geom.wall[a];
    sg.ext[a] = n[a] + (r.geom.wall[a] ? 1 : 0);
  }
  return sg;
}

struct FinArgs {
  const void* ub;  // bare normal-fluid velocity field of the step
  Geom g;
  const double* Y;
  double* Ynext;
  double* pos;
  double* ksum;
  const int32_t* nxt;
  const int32_t* prv;
  int32_t* cnt;
  const void* P;
  int S;
  long long ncap;
  const double* Vs;
  int mass_balance;
  int mb_axis;      // flow axis of the superflow
  int stage;        // stage of the Runge-Kutta method, 1..rk
  int rk;           // stages of the method: 1, 2 or 4
  int first;        // first stage of the step's first substep: stage-1 outputs
  double h, hh;     // substep length 1/m and half of it
  int eval_only;
  int coupling;
  int force_model;  // 0: s' x (ds/dt - v_s) (Magnus balance); 1: ds/dt - v_s
  double kappa;
  double bs_scale;    // kappa / (4 pi)
  double nl_scale;    // kappa / (4 pi) times the grid step when the sum ran in grid units
  double ln2_ea;      // ln(2 / (e^C a))
  double alpha, alpha_p;
  // mutual-friction profiles along z: alpha at [0, nz), alpha' at
  // [nz, 2 nz), and at [2 nz] 1.0 when they replace the constants (read at
  // run time, so that a captured graph follows the current setting)
  const double* fric;
  double rs_rn;
  double vs_app[3];
  double* vs1;
  double* vn1;
  double* sd1;
  double* gpt;
  uint32_t* X;      // grid coordinates of the next stage's positions (FP32 sum), or null
  BsAxes ax;
  // stage 1 with spreading: per point, the bin key and the fractional
  // stencil offsets of the step's positions, and the point count
  SpreadGeom sg;
  uint32_t* skeys;  // or null
  double* sfrac;
};

// Nearest-image separation on the filament axes (wall axes: plain).
__device__ inline double mimg(double d, double L, int periodic) {
  if (periodic) {
    if (d > 0.5 * L)
      d = d - L;
    else if (d < -0.5 * L)
      d = d + L;
  }
  return d;
}

// Periodic axes wrap into [0, L); wall axes mirror a point that crossed
// the wall plane at -1/2 or n - 1/2.
__device__ inline double wrap_coord(double x, double L, int periodic) {
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

// Normal-fluid velocity at a point: delta_2pt weights on the 8 surrounding
// nodes of the step's bare-velocity field; nodes beyond a wall carry zero.
template <class UT>
__device__ void interp_vn(const UT* __restrict__ ub, const Geom& g, double px, double py,
                          double pz, double v[3]) {
  const double b[3] = {floor(px), floor(py), floor(pz)};
  const double fr[3] = {px - b[0], py - b[1], pz - b[2]};
  const int ib[3] = {ifloor_safe(px), ifloor_safe(py), ifloor_safe(pz)};
  const int n[3] = {g.nx, g.ny, g.nz};
  v[0] = v[1] = v[2] = 0.0;
  for (int o = 0; o < 8; ++o) {
    const int off[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
    int node[3];
    double w = 1.0;
    bool ghost = false;
    for (int a = 0; a < 3; ++a) {
      int c = ib[a] + off[a];
      w *= off[a] ? fr[a] : 1.0 - fr[a];
      if (c < 0 || c >= n[a]) {
        if (g.wall[a])
          ghost = true;
        else
          c = ((c % n[a]) + n[a]) % n[a];
      }
      node[a] = c;
    }
    if (ghost) continue;
    const long long c = ((long long)node[2] * g.ny + node[1]) * g.nx + node[0];
    v[0] += w * (double)ub[c];
    v[1] += w * (double)ub[g.cells + c];
    v[2] += w * (double)ub[2 * g.cells + c];
  }
}

// 64 points per block of kFinWaves waves.  The waves add the Biot-Savart
// chunk partials of the block's points (wave g takes chunks g, g + kFinWaves,
// ..., eight chunks' loads in flight at a time); before its share, wave 1
// interpolates the normal-fluid velocity, wave 2 evaluates the local
// geometry and the LIA term and wave 3 loads the RK4 state, so that these
// load chains overlap.  Wave 0 then combines the parts in a fixed order and
// does the rest per point.
constexpr int kFinPts = 64;
constexpr int kFinWaves = 4;

template <class UT, class PT>
__global__ __launch_bounds__(kFinWaves * 64) void k_finalize(FinArgs A) {
  __shared__ double red[kFinWaves - 1][3][kFinPts];  // chunk sums of waves 1..kFinWaves-1
  __shared__ double s_vn[3][kFinPts];    // wave 1: normal-fluid velocity
  __shared__ double s_geo[8][kFinPts];   // wave 2: s' (3), LIA (3), real l+, l-
  __shared__ int s_end[kFinPts];         // wave 2: wall axis of an open line's end, or -1
  __shared__ double s_rk[9][kFinPts];    // wave 3: s^n (3), ksum (3), superflow, alpha, alpha'
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int j = blockIdx.x * kFinPts + lane;
  const int n = A.cnt[0];
  const bool live = j < n;
  const long long nc = A.ncap;
  // The loads do not wait for the point count: every slot below the
  // capacity is read (indices clamped into the arrays, non-finite values
  // harmless), and only live points write.
  const bool slot = j < nc;
  // the first batch of this wave's Biot-Savart chunk partials (chunks grp,
  // grp + kFinWaves, ..., up to 8 of them; beyond S they read as zero, which
  // adds nothing), loaded before the wave's own work so that the latencies
  // overlap
  const PT* __restrict__ P = (const PT*)A.P;
  const long long jc = slot ? j : 0;  // in-bounds index for the unconditional loads
  PT v0[8][3];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const bool ok = slot && grp + kFinWaves * u < A.S;
    const long long c = ok ? grp + kFinWaves * u : 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const PT x = P[(c * 3 + a) * nc + jc];
      v0[u][a] = ok ? x : (PT)0;
    }
  }
  const Geom& g = A.g;
  const double L[3] = {(double)g.nx, (double)g.ny, (double)g.nz};
  const int per[3] = {!g.wall[0], !g.wall[1], !g.wall[2]};

  if (slot && grp == 1) {
    const double p[3] = {A.Y[j], A.Y[nc + j], A.Y[2 * nc + j]};
    double vn[3];
    interp_vn<UT>((const UT*)A.ub, g, p[0], p[1], p[2], vn);
    for (int a = 0; a < 3; ++a) s_vn[a][lane] = vn[a];
    if (live && A.skeys) {
      int b[3];
      A.skeys[j] = base_key(A.sg, p, b);
      for (int a = 0; a < 3; ++a) A.sfrac[a * nc + j] = p[a] - floor(p[a]);
    }
  }
  if (A.skeys && blockIdx.x == 0 && threadIdx.x == 0) A.cnt[11] = n;
  if (slot && grp == 2) {
    // local geometry (three-point derivatives on a non-uniform arc length)
    const int jn = min(max(A.nxt[j], 0), (int)nc - 1), jp = min(max(A.prv[j], 0), (int)nc - 1);
    double dp[3], dm[3], pj[3];
    for (int a = 0; a < 3; ++a) {
      const double pa = A.Y[a * nc + j];
      pj[a] = pa;
      dp[a] = mimg(A.Y[a * nc + jn] - pa, L[a], per[a]);
      dm[a] = mimg(pa - A.Y[a * nc + jp], L[a], per[a]);
    }
    // the lengths of the segments that exist (the line length carried)
    const double lp_real = sqrt(dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2]);
    const double lm_real = sqrt(dm[0] * dm[0] + dm[1] * dm[1] + dm[2] * dm[2]);
    // An end of an open line lies on a wall plane (the lowest such closed
    // axis); the line continues into its mirror image there, so the
    // missing neighbour is the mirrored existing one: the missing segment
    // vector is the existing one with its components along the wall negated.
    int ea = -1;
    if (jn == j || jp == j)
      for (int a = 2; a >= 0; --a)
        if (!per[a] && (pj[a] == -0.5 || pj[a] == L[a] - 0.5)) ea = a;
    if (ea >= 0) {
      if (jn == j) {
        for (int a = 0; a < 3; ++a) dp[a] = a == ea ? dm[a] : -dm[a];
      } else {
        for (int a = 0; a < 3; ++a) dm[a] = a == ea ? dp[a] : -dp[a];
      }
    }
    s_end[lane] = ea;
    const double lp = sqrt(dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2]);
    const double lm = sqrt(dm[0] * dm[0] + dm[1] * dm[1] + dm[2] * dm[2]);
    const double iden = 1.0 / (lp * lm * (lp + lm));
    double sp[3], spp[3];
    for (int a = 0; a < 3; ++a) {
      sp[a] = (lm * lm * dp[a] + lp * lp * dm[a]) * iden;
      spp[a] = 2.0 * (lm * dp[a] - lp * dm[a]) * iden;
    }
    const double isn = 1.0 / sqrt(sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2]);
    for (int a = 0; a < 3; ++a) sp[a] *= isn;
    // LIA: beta s' x s'', beta = kappa/(4 pi) ln(2 sqrt(l+ l-) / (e^C a))
    //                          = kappa/(4 pi) (ln(l+ l-) / 2 + ln(2 / (e^C a)))
    const double beta = A.bs_scale * fma(0.5, log(lp * lm), A.ln2_ea);
    s_geo[3][lane] = beta * (sp[1] * spp[2] - sp[2] * spp[1]);
    s_geo[4][lane] = beta * (sp[2] * spp[0] - sp[0] * spp[2]);
    s_geo[5][lane] = beta * (sp[0] * spp[1] - sp[1] * spp[0]);
    for (int a = 0; a < 3; ++a) s_geo[a][lane] = sp[a];
    s_geo[6][lane] = lp_real;
    s_geo[7][lane] = lm_real;
  }
  if (slot && grp == 3) {
    if (!A.eval_only)
      for (int a = 0; a < 3; ++a) {
        s_rk[a][lane] = A.pos[a * nc + j];
        s_rk[3 + a][lane] = A.stage > 1 ? A.ksum[a * nc + j] : 0.0;
      }
    if (A.mass_balance) {
      const int ma = A.mb_axis;
      const int nm = ma == 0 ? g.nx : (ma == 1 ? g.ny : g.nz);
      const double pz = A.Y[ma * nc + j];
      const double fz = floor(pz);
      const double t = pz - fz;
      int i0 = ifloor_safe(pz), i1 = i0 + 1;
      i0 = ((i0 % nm) + nm) % nm;
      i1 = ((i1 % nm) + nm) % nm;
      s_rk[6][lane] = (1.0 - t) * A.Vs[i0] + t * A.Vs[i1];
    }
    // mutual-friction coefficients at the point's height: the constants,
    // or the slice profiles linear between floor(z) and floor(z) + 1
    // (periodic z wraps; a wall z axis extends its end values)
    double al = A.alpha, alp = A.alpha_p;
    if (A.fric[2 * g.nz] != 0.0) {
      const double pz = A.Y[2 * nc + j];
      const double t = pz - floor(pz);
      int i0 = ifloor_safe(pz), i1 = i0 + 1;
      if (g.wall[2]) {
        i0 = min(max(i0, 0), g.nz - 1);
        i1 = min(max(i1, 0), g.nz - 1);
      } else {
        i0 = ((i0 % g.nz) + g.nz) % g.nz;
        i1 = ((i1 % g.nz) + g.nz) % g.nz;
      }
      al = (1.0 - t) * A.fric[i0] + t * A.fric[i1];
      alp = (1.0 - t) * A.fric[g.nz + i0] + t * A.fric[g.nz + i1];
    }
    s_rk[7][lane] = al;
    s_rk[8][lane] = alp;
  }

  // non-local Biot-Savart: chunk partials added in a fixed order
  double vs[3] = {0.0, 0.0, 0.0};
  if (slot) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int a = 0; a < 3; ++a) vs[a] += (double)v0[u][a];
    for (int s = grp + 8 * kFinWaves; s < A.S; s += 8 * kFinWaves) {
      PT v[8][3];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool ok = s + kFinWaves * u < A.S;
        const long long c = ok ? s + kFinWaves * u : 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const PT x = P[(c * 3 + a) * nc + j];
          v[u][a] = ok ? x : (PT)0;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int a = 0; a < 3; ++a) vs[a] += (double)v[u][a];
    }
  }
  if (grp > 0)
    for (int a = 0; a < 3; ++a) red[grp - 1][a][lane] = vs[a];
  __syncthreads();
  if (grp > 0 || !live) return;
  for (int a = 0; a < 3; ++a) {
    double t = vs[a];
#pragma unroll
    for (int w = 0; w < kFinWaves - 1; ++w) t += red[w][a][lane];
    vs[a] = t * A.nl_scale;
  }

  double sp[3];
  for (int a = 0; a < 3; ++a) {
    sp[a] = s_geo[a][lane];
    vs[a] += s_geo[3 + a][lane];
  }
  const double lp = s_geo[6][lane], lm = s_geo[7][lane];
  for (int a = 0; a < 3; ++a) vs[a] += A.vs_app[a];
  if (A.mass_balance) vs[A.mb_axis] += s_rk[6][lane];

  // normal-fluid velocity at the point
  const double vn[3] = {s_vn[0][lane], s_vn[1][lane], s_vn[2][lane]};

  // Schwarz equation of motion (Sec. II.A, Eq. E of M)
  const double w[3] = {vn[0] - vs[0], vn[1] - vs[1], vn[2] - vs[2]};
  const double sxw[3] = {sp[1] * w[2] - sp[2] * w[1], sp[2] * w[0] - sp[0] * w[2],
                         sp[0] * w[1] - sp[1] * w[0]};
  const double ssw[3] = {sp[1] * sxw[2] - sp[2] * sxw[1], sp[2] * sxw[0] - sp[0] * sxw[2],
                         sp[0] * sxw[1] - sp[1] * sxw[0]};
  const double al = s_rk[7][lane], alp = s_rk[8][lane];
  double sd[3];
  for (int a = 0; a < 3; ++a) sd[a] = vs[a] + al * sxw[a] - alp * ssw[a];
  // an open line's end slides on its wall: no velocity normal to it
  const int ea = s_end[lane];
  if (ea >= 0) sd[ea] = 0.0;
  if (!(isfinite(sd[0]) && isfinite(sd[1]) && isfinite(sd[2])))
    atomicOr(&A.cnt[7], kFlagNumeric);

  if (A.first) {
    for (int a = 0; a < 3; ++a) {
      A.vs1[a * nc + j] = vs[a];
      A.vn1[a * nc + j] = vn[a];
      A.sd1[a * nc + j] = sd[a];
    }
    // reaction on the normal fluid (Magnus balance), per point, with the
    // line length (l+ + l-)/2 carried by the point (the real segments)
    const double r[3] = {sd[0] - vs[0], sd[1] - vs[1], sd[2] - vs[2]};
    const double sxr[3] = {sp[1] * r[2] - sp[2] * r[1], sp[2] * r[0] - sp[0] * r[2],
                           sp[0] * r[1] - sp[1] * r[0]};
    const double dxi = 0.5 * (lp + lm);
    for (int a = 0; a < 3; ++a) {
      const double w = A.force_model ? r[a] : sxr[a];  // literal reading: for ablation
      A.gpt[a * nc + j] = A.coupling ? A.rs_rn * A.kappa * w * dxi : 0.0;
    }
  }
  if (A.eval_only) return;

  // Runge-Kutta over a substep of length h from s0 (the substep's start):
  // classical (4 stages): ksum = k1 + 2 k2 + 2 k3 + k4, stage positions
  // s0 + (h/2) k1, s0 + (h/2) k2, s0 + h k3, result s0 + h ksum / 6;
  // midpoint (2): s0 + (h/2) k1, result s0 + h k2; Euler (1): s0 + h k1
  for (int a = 0; a < 3; ++a) {
    const double s0 = s_rk[a][lane];
    const double kp = s_rk[3 + a][lane];
    double ks = sd[a];
    double y;
    if (A.rk == 4) {
      switch (A.stage) {
        case 1:
          y = s0 + A.hh * sd[a];
          break;
        case 2:
          ks = kp + 2.0 * sd[a];
          y = s0 + A.hh * sd[a];
          break;
        case 3:
          ks = kp + 2.0 * sd[a];
          y = s0 + A.h * sd[a];
          break;
        default:
          ks = kp + sd[a];
          y = s0 + A.h * (ks / 6.0);
          break;
      }
    } else if (A.rk == 2 && A.stage == 1) {
      y = s0 + A.hh * sd[a];
    } else {
      y = s0 + A.h * sd[a];
    }
    A.ksum[a * nc + j] = ks;
    const double yw = wrap_coord(y, L[a], per[a]);
    A.Ynext[a * nc + j] = yw;
    if (A.X) {
      const double sgrid = floor((yw + A.ax.off[a]) * A.ax.q[a]);
      A.X[a * nc + j] = A.ax.periodic[a] ? (uint32_t)(long long)sgrid : (uint32_t)(int)(long long)sgrid;
    }
  }
}

// ----------------------------------------------------------- spreading

// Spreading preparation, one launch with two roles by block:
//  * blocks [0, ntiles): a tile of the binning keys (written by the
//    stage-1 finalize for the live points, padded here with the largest
//    key beyond them) and the tile's digit counts for the first pass of
//    the sort;
//  * the other blocks: zero the force at the nodes the previous spreading
//    wrote, and clear the previous spreading's bin marks.
template <class FT>
__global__ __launch_bounds__(kSortThreads) void k_spread_prepare(
    const int32_t* __restrict__ cnt, long long ncap, uint32_t pad, int dbits, int ntiles, uint32_t* __restrict__ keys, int32_t* __restrict__ vals,
    int32_t* __restrict__ counts, FT* __restrict__ F, long long cells,
    const int32_t* __restrict__ touched, const uint32_t* __restrict__ marked,
    int32_t* __restrict__ bins) {
  __shared__ int32_t hist[kSortMaxBins];
  if ((int)blockIdx.x < ntiles) {
    const int j = blockIdx.x * kSortThreads + threadIdx.x;
    const int n = cnt[11];
    uint32_t k = pad;
    if (j < n) k = keys[j];
    if (j < ncap) {
      keys[j] = k;
      vals[j] = j;
    }
    sort_tile_count(k, j < ncap, 0, dbits, ntiles, blockIdx.x, hist, counts);
    return;
  }
  const long long s = (long long)(blockIdx.x - ntiles) * kSortThreads + threadIdx.x;
  if (s < cnt[1]) {
    const int node = touched[s];
    if (node >= 0) {
      F[node] = FT(0);
      F[cells + node] = FT(0);
      F[2 * cells + node] = FT(0);
    }
  }
  if (s < ncap) {
    const uint32_t mk = marked[s];
    if (mk != 0xFFFFFFFFu) bins[mk] = -1;
  }
}

// Dense bin table: bins[key] = first sorted entry of that bin, -1 if empty.
// The marked keys are listed so that the next spreading clears them.
__global__ void k_bin_mark(const uint32_t* __restrict__ skey, const int32_t* __restrict__ cnt,
                           long long ncap, int32_t* __restrict__ bins,
                           uint32_t* __restrict__ marked) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ncap) return;
  const bool head = r < cnt[11] && (r == 0 || skey[r - 1] != skey[r]);
  if (head) bins[skey[r]] = r;
  marked[r] = head ? skey[r] : 0xFFFFFFFFu;
}

// One thread per (sorted entry, stencil corner).  Only the first entry of
// each bin acts: the node at that corner of the bin's stencil is written by
// the occupied bin of smallest key among the (up to 8) bins whose stencils
// contain it, which gathers those bins' points in a fixed order.
template <class FT>
__global__ void k_spread_gather(const uint32_t* __restrict__ skey, const int32_t* __restrict__ sval,
                                const int32_t* __restrict__ bins,
                                const double* __restrict__ sfrac, const double* __restrict__ gpt,
                                int32_t* __restrict__ cnt, long long ncap, SpreadGeom sg,
                                long long cells, FT* __restrict__ F, int32_t* __restrict__ touched) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = cnt[11];
  if (id == 0) cnt[1] = 8 * n;
  const int r = (int)(id >> 3);
  const int o = (int)(id & 7);
  if (r >= n) return;
  const uint32_t me = skey[r];
  if (r > 0 && skey[r - 1] == me) {
    touched[id] = -1;
    return;
  }
  int b[3];
  b[0] = (int)(me % (uint32_t)sg.ext[0]);
  b[1] = (int)((me / (uint32_t)sg.ext[0]) % (uint32_t)sg.ext[1]);
  b[2] = (int)(me / ((uint32_t)sg.ext[0] * (uint32_t)sg.ext[1]));
  const int off[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
  int e[3];    // node in bin coordinates
  int lat[3];  // node in lattice coordinates
  bool ghost = false;
  for (int a = 0; a < 3; ++a) {
    e[a] = b[a] + off[a];
    if (sg.wall[a]) {
      lat[a] = e[a] - 1;
      if (lat[a] < 0 || lat[a] >= sg.n[a]) ghost = true;
    } else {
      if (e[a] >= sg.n[a]) e[a] -= sg.n[a];
      lat[a] = e[a];
    }
  }
  if (ghost) {
    touched[id] = -1;
    return;
  }
  // the bins whose stencil contains this node: e - o' for o' in {0,1}^3
  uint32_t kq[8];
  int lo[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int oq[3] = {q & 1, (q >> 1) & 1, (q >> 2) & 1};
    int c[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
      c[a] = e[a] - oq[a];
      if (sg.wall[a]) {
        if (c[a] < 0) ok = false;
      } else if (c[a] < 0) {
        c[a] += sg.n[a];
      }
    }
    kq[q] = (uint32_t)(((long long)c[2] * sg.ext[1] + c[1]) * sg.ext[0] + c[0]);
    lo[q] = ok ? bins[kq[q]] : -1;
  }
  bool owner = true;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (lo[q] >= 0 && kq[q] < me) owner = false;
  if (!owner) {
    touched[id] = -1;
    return;
  }
  double f[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 8; ++q) {
    if (lo[q] < 0) continue;
    const int oq[3] = {q & 1, (q >> 1) & 1, (q >> 2) & 1};
    for (int t = lo[q]; t < n && skey[t] == kq[q]; ++t) {
      const int pidx = sval[t];
      double w = 1.0;
      for (int a = 0; a < 3; ++a) {
        const double fr = sfrac[a * ncap + pidx];
        w *= oq[a] ? fr : 1.0 - fr;
      }
      for (int a = 0; a < 3; ++a) f[a] += w * gpt[a * ncap + pidx];
    }
  }
  const long long node = ((long long)lat[2] * sg.n[1] + lat[1]) * sg.n[0] + lat[0];
  F[node] = (FT)f[0];
  F[cells + node] = (FT)f[1];
  F[2 * cells + node] = (FT)f[2];
  touched[id] = (int32_t)node;
}

inline int nblocks(long long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t fil_finalize(Run& r, int stage, int first, int last, const double* Y, double* Ynext,
                        int eval_only) {
  FinArgs A;
  A.ub = r.ub;
  A.g = r.geom;
  A.Y = Y;
  A.Ynext = Ynext;
  A.pos = r.pos;
  A.ksum = r.ksum;
  A.nxt = r.nxt;
  A.prv = r.prv;
  A.cnt = r.cnt;
  A.P = r.bsP;
  A.S = r.vor.ff_cell > 0 ? r.ffS : r.bsS * r.bsax.copies;
  A.ncap = r.ncap;
  A.Vs = r.Vs;
  A.mass_balance = r.vor.mass_balance;
  A.mb_axis = r.vor.mass_balance_axis;
  A.stage = stage;
  A.rk = r.vor.rk_stages;
  A.first = first;
  A.h = 1.0 / r.vor.vfm_substeps;
  A.hh = 0.5 * A.h;
  A.eval_only = eval_only;
  A.coupling = r.vor.coupling;
  A.kappa = r.vor.kappa;
  A.bs_scale = r.vor.kappa / (4.0 * M_PI);
  // the direct FP32 sum on a uniform grid leaves grid units; the far-field
  // sum lattice units
  A.nl_scale = (r.prec != VLB_F64 && r.bsax.uniform && r.vor.ff_cell <= 0)
                   ? A.bs_scale * r.bsax.q[0]
                   : A.bs_scale;
  A.ln2_ea = log(2.0 / (exp(r.vor.core_c) * r.vor.core_a));
  A.alpha = r.vor.alpha;
  A.alpha_p = r.vor.alpha_p;
  A.fric = r.fric;
  A.force_model = r.vor.force_model;
  A.rs_rn = r.vor.rho_s_over_rho_n;
  for (int a = 0; a < 3; ++a) A.vs_app[a] = r.vor.vs_applied[a];
  A.vs1 = r.vs1;
  A.vn1 = r.vn1;
  A.sd1 = r.sd1;
  A.gpt = r.gpt;
  // the FP32 sum of the next stage reads grid coordinates written here
  A.X = (r.prec != VLB_F64 && !last && !eval_only) ? r.bsX : nullptr;
  A.ax = r.bsax;
  A.sg = spread_geom(r);
  A.skeys = (first && r.vor.coupling) ? r.keys_a : nullptr;
  A.sfrac = r.sfrac;
  const int nb = nblocks(r.ncap, kFinPts);
  switch (r.prec) {
    case VLB_F64: hipLaunchKernelGGL((k_finalize<double, double>), dim3(nb), dim3(kFinWaves * 64), 0, r.stream, A); break;
    default: hipLaunchKernelGGL((k_finalize<float, float>), dim3(nb), dim3(kFinWaves * 64), 0, r.stream, A); break;
  }
  return hipGetLastError();
}

// Positions copied slot by slot (3 n_cap values): forward Euler writes its
// result beside the positions it reads and copies it back.
__global__ void k_copy_pos(const double* __restrict__ src, double* __restrict__ dst, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t fil_copy_positions(Run& r, const double* src, double* dst) {
  const long long n = 3 * r.ncap;
  hipLaunchKernelGGL(k_copy_pos, dim3(nblocks(n, 256)), dim3(256), 0, r.stream, src, dst, n);
  return hipGetLastError();
}

hipError_t fil_spread(Run& r) {
  const SpreadGeom sg = spread_geom(r);
  const uint32_t pad = (r.key_bits >= 32) ? 0xFFFFFFFFu : ((1u << r.key_bits) - 1u);
  const int ntiles = sort_tiles(r.ncap);
  int dbits = 0;
  sort_first_digit(r.key_bits, &dbits);
  const int nclear = nblocks(8 * r.ncap, kSortThreads);
  if (r.prec == VLB_F64)
    hipLaunchKernelGGL(k_spread_prepare<double>, dim3(ntiles + nclear), dim3(kSortThreads), 0,
                       r.stream, r.cnt, r.ncap, pad, dbits, ntiles, r.keys_a, r.vals_a,
                       sort_counts(r), (double*)r.force, r.cells, r.touched, r.marked, r.bins);
  else
    hipLaunchKernelGGL(k_spread_prepare<float>, dim3(ntiles + nclear), dim3(kSortThreads), 0,
                       r.stream, r.cnt, r.ncap, pad, dbits, ntiles, r.keys_a, r.vals_a,
                       sort_counts(r), (float*)r.force, r.cells, r.touched, r.marked, r.bins);
  uint32_t* sk = nullptr;
  int32_t* sv = nullptr;
  hipError_t e = sort_pairs(r, r.key_bits, 1, &sk, &sv);
  if (e != hipSuccess) return e;
  const int nb = nblocks(r.ncap, 256);
  hipLaunchKernelGGL(k_bin_mark, dim3(nb), dim3(256), 0, r.stream, sk, r.cnt, r.ncap, r.bins,
                     r.marked);
  const int nb8 = nblocks(8 * r.ncap, 256);
  if (r.prec == VLB_F64)
    hipLaunchKernelGGL(k_spread_gather<double>, dim3(nb8), dim3(256), 0, r.stream, sk, sv,
                       r.bins, r.sfrac, r.gpt, r.cnt, r.ncap, sg, r.cells, (double*)r.force, r.touched);
  else
    hipLaunchKernelGGL(k_spread_gather<float>, dim3(nb8), dim3(256), 0, r.stream, sk, sv,
                       r.bins, r.sfrac, r.gpt, r.cnt, r.ncap, sg, r.cells, (float*)r.force, r.touched);
  return hipGetLastError();
}

}  // namespace vlb
