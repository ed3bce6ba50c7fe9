// Internal declarations of the vlb library: run state, workspace layout,
// D3Q19 tables and the population access rules shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vlb.h"

namespace vlb {

// ------------------------------------------------------------------ D3Q19
// Velocity set of the paper's Table I (Sec. II.B): index 0 rest, 1-6 the
// axis neighbours (weight 1/18), 7-18 the face diagonals (weight 1/36).
// Opposite pairs are (2k-1, 2k) for k >= 1.
__host__ __device__ constexpr int cx(int i) {
  constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return t[i];
}
__host__ __device__ constexpr int cy(int i) {
  constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return t[i];
}
__host__ __device__ constexpr int cz(int i) {
  constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return t[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double wq(int i) {
  return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// FP16 storage keeps deviations scaled by 2^10 (exact power-of-two scale).
constexpr float kHalfScale = 1024.0f;
constexpr float kHalfInvScale = 1.0f / 1024.0f;

// Storage traits: memory holds deviations d_i = f_i - w_i (rho0 = 1).
// Population storage; the _nt forms carry the non-temporal hint, for
// lattices far larger than the last-level cache (every value is read once
// and written once per update).
template <class S> struct Store;
template <> struct Store<double> {
  using T = double;
  __device__ static T ld(const double* p) { return *p; }
  __device__ static void st(double* p, T v) { *p = v; }
  __device__ static T ld_nt(const double* p) { return __builtin_nontemporal_load(p); }
  __device__ static void st_nt(double* p, T v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<float> {
  using T = float;
  __device__ static T ld(const float* p) { return *p; }
  __device__ static void st(float* p, T v) { *p = v; }
  __device__ static T ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
  __device__ static void st_nt(float* p, T v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<__half> {
  using T = float;
  __device__ static T ld(const __half* p) { return __half2float(*p) * kHalfInvScale; }
  __device__ static void st(__half* p, T v) { *p = __float2half_rn(v * kHalfScale); }
  __device__ static T ld_nt(const __half* p) {
    const unsigned short u = __builtin_nontemporal_load((const unsigned short*)p);
    return __half2float(__ushort_as_half(u)) * kHalfInvScale;
  }
  __device__ static void st_nt(__half* p, T v) {
    __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v * kHalfScale)), (unsigned short*)p);
  }
};
template <class S, bool NT>
__device__ inline typename Store<S>::T pop_ld(const S* p) {
  return NT ? Store<S>::ld_nt(p) : Store<S>::ld(p);
}
template <class S, bool NT>
__device__ inline void pop_st(S* p, typename Store<S>::T v) {
  if (NT)
    Store<S>::st_nt(p, v);
  else
    Store<S>::st(p, v);
}

// Stored values as they are kept (FP16: the deviation times 2^10; otherwise
// the deviation itself) and that scale: deviation = raw / kScale.  The
// non-temporal choice is a template argument: as a run-time flag, the two
// forms of an access merge into one plain access and the hint is lost.
template <class S> struct Raw;
template <> struct Raw<double> {
  static constexpr double kScale = 1.0;
  template <bool NT> __device__ static double ld(const double* p) { return pop_ld<double, NT>(p); }
  template <bool NT> __device__ static void st(double* p, double v) { pop_st<double, NT>(p, v); }
  __device__ static double enc(double v) { return v; }
  template <bool NT> __device__ static void st_enc(double* p, double v) { pop_st<double, NT>(p, v); }
};
template <> struct Raw<float> {
  static constexpr float kScale = 1.0f;
  template <bool NT> __device__ static float ld(const float* p) { return pop_ld<float, NT>(p); }
  template <bool NT> __device__ static void st(float* p, float v) { pop_st<float, NT>(p, v); }
  __device__ static float enc(float v) { return v; }
  template <bool NT> __device__ static void st_enc(float* p, float v) { pop_st<float, NT>(p, v); }
};
template <> struct Raw<__half> {
  static constexpr float kScale = kHalfScale;
  template <bool NT> __device__ static float ld(const __half* p) {
    if (NT) return __half2float(__ushort_as_half(__builtin_nontemporal_load((const unsigned short*)p)));
    return __half2float(*p);
  }
  template <bool NT> __device__ static void st(__half* p, float v) {
    if (NT)
      __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v)), (unsigned short*)p);
    else
      *p = __float2half_rn(v);
  }
  // the stored value, rounded to nearest
  __device__ static __half enc(float v) { return __float2half_rn(v); }
  template <bool NT> __device__ static void st_enc(__half* p, __half h) {
    if (NT)
      __builtin_nontemporal_store(__half_as_ushort(h), (unsigned short*)p);
    else
      *p = h;
  }
};

// Population array as a raw buffer (I32 lattices: fewer than 4 GiB): an
// access names a per-lane byte offset (VGPR) and a uniform one (SGPR), so
// that a slot at a uniform distance from a lane's node costs no vector
// arithmetic.  Cache policy 2 is the non-temporal hint.
typedef unsigned int vlb_u32x2 __attribute__((ext_vector_type(2)));
template <class S>
__device__ inline __amdgpu_buffer_rsrc_t pop_rsrc(S* M, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(M, 0, (int)bytes, 0x00020000);
}
template <class S> struct Buf;
template <> struct Buf<double> {
  template <bool NT> __device__ static double ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, NT ? 2 : 0));
  }
  template <bool NT> __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(vlb_u32x2, v), r, vo, so, NT ? 2 : 0);
  }
};
template <> struct Buf<float> {
  template <bool NT> __device__ static float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, NT ? 2 : 0));
  }
  template <bool NT> __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, vo, so, NT ? 2 : 0);
  }
};
template <> struct Buf<__half> {
  template <bool NT> __device__ static float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, NT ? 2 : 0)));
  }
  template <bool NT> __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, __half h) {
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(h), r, vo, so, NT ? 2 : 0);
  }
};


// Lattice description as passed to kernels.
struct Geom {
  int nx, ny, nz;
  int wall[3];
  int plane_lo, plane_hi;
  long long cells;
  double plane_u[3];
  double body[3];
  double omega;       // 1/tau
  double fpref;       // 1 - 1/(2 tau)
  // the same parameters rounded to FP32 once, for the FP32 arithmetic
  float plane_u_f[3];
  float body_f[3];
  float omega_f;
  float fpref_f;
};

// Geometry parameters in the arithmetic type T.
template <class T>
__device__ inline void geom_params(const Geom& g, T& om, T& pref, T body[3], T plane[3]) {
  if constexpr (sizeof(T) == 4) {
    om = g.omega_f;
    pref = g.fpref_f;
    for (int a = 0; a < 3; ++a) {
      body[a] = g.body_f[a];
      plane[a] = g.plane_u_f[a];
    }
  } else {
    om = g.omega;
    pref = g.fpref;
    for (int a = 0; a < 3; ++a) {
      body[a] = g.body[a];
      plane[a] = g.plane_u[a];
    }
  }
}

// c_i . (x, y, z) summed over the nonzero components of c_i only (they are
// +-1), so that no product with a zero component is evaluated.
template <class T>
__device__ __forceinline__ T cdot(int i, T x, T y, T z) {
  const int a = cx(i), b = cy(i), c = cz(i);
  T r = T(0);
  bool any = false;
  if (a != 0) {
    r = a > 0 ? x : -x;
    any = true;
  }
  if (b != 0) {
    const T v = b > 0 ? y : -y;
    r = any ? r + v : v;
    any = true;
  }
  if (c != 0) {
    const T v = c > 0 ? z : -z;
    r = any ? r + v : v;
  }
  return r;
}

// Quotient by a divisor d >= 1 fixed for a launch, by multiplication
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, Fig. 4.1): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, t / d = (h + ((t - h) >> s1)) >> s2
// for h = mulhi(m, t), s1 = min(l, 1), s2 = max(l - 1, 0); exact for every
// 32-bit t.  Uniform operands keep it on the scalar unit.
struct FastDiv {
  uint32_t d, m;
  int s1, s2;
};
inline FastDiv make_fastdiv(uint32_t d) {
  int l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  const uint32_t m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
  return FastDiv{d, m, l < 1 ? l : 1, l > 1 ? l - 1 : 0};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t t, const FastDiv& f) {
  const uint32_t h = __umulhi(f.m, t);
  return (h + ((t - h) >> f.s1)) >> f.s2;
}

// Index of node (x, y, z) + (dx, dy, dz), or -1 when that node lies beyond
// a wall (periodic axes wrap).
__device__ inline long long neighbour(const Geom& g, int x, int y, int z, int dx, int dy, int dz) {
  int xx = x + dx, yy = y + dy, zz = z + dz;
  if (xx < 0 || xx >= g.nx) {
    if (g.wall[0]) return -1;
    xx = xx < 0 ? xx + g.nx : xx - g.nx;
  }
  if (yy < 0 || yy >= g.ny) {
    if (g.wall[1]) return -1;
    yy = yy < 0 ? yy + g.ny : yy - g.ny;
  }
  if (zz < 0 || zz >= g.nz) {
    if (g.wall[2]) return -1;
    zz = zz < 0 ? zz + g.nz : zz - g.nz;
  }
  return ((long long)zz * g.ny + yy) * g.nx + xx;
}

// Offsets of the 3 x 3 x 3 neighbourhood of one node, per axis: index of
// the node (x+dx, y+dy, z+dz) is zo[dz+1] + yo[dy+1] + xo[dx+1], negative
// when that node lies beyond a wall (periodic axes wrap).
struct Nbr {
  long long zo[3], yo[3], xo[3];
};
constexpr long long kBeyond = -(1LL << 40);

__device__ inline void make_nbr(const Geom& g, int x, int y, int z, Nbr& nb) {
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    int xx = x + d, yy = y + d, zz = z + d;
    bool vx = true, vy = true, vz = true;
    if (xx < 0 || xx >= g.nx) {
      if (g.wall[0]) vx = false;
      xx = xx < 0 ? xx + g.nx : xx - g.nx;
    }
    if (yy < 0 || yy >= g.ny) {
      if (g.wall[1]) vy = false;
      yy = yy < 0 ? yy + g.ny : yy - g.ny;
    }
    if (zz < 0 || zz >= g.nz) {
      if (g.wall[2]) vz = false;
      zz = zz < 0 ? zz + g.nz : zz - g.nz;
    }
    nb.xo[d + 1] = vx ? (long long)xx : kBeyond;
    nb.yo[d + 1] = vy ? (long long)yy * g.nx : kBeyond;
    nb.zo[d + 1] = vz ? (long long)zz * g.ny * g.nx : kBeyond;
  }
}

__device__ inline long long nbr_index(const Nbr& nb, int dx, int dy, int dz) {
  return nb.zo[dz + 1] + nb.yo[dy + 1] + nb.xo[dx + 1];
}

// The same in 32-bit integers, for lattices of fewer than 2^29 nodes whose
// population array spans less than 4 GiB (a node beyond a wall gives a
// negative index: one or two of the three terms are -2^29, the others sum
// to less than 2^29).
struct Nbr32 {
  int zo[3], yo[3], xo[3];
};
constexpr int kBeyond32 = -(1 << 29);

__device__ inline void make_nbr32(const Geom& g, int x, int y, int z, Nbr32& nb) {
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    int xx = x + d, yy = y + d, zz = z + d;
    bool vx = true, vy = true, vz = true;
    if (xx < 0 || xx >= g.nx) {
      if (g.wall[0]) vx = false;
      xx = xx < 0 ? xx + g.nx : xx - g.nx;
    }
    if (yy < 0 || yy >= g.ny) {
      if (g.wall[1]) vy = false;
      yy = yy < 0 ? yy + g.ny : yy - g.ny;
    }
    if (zz < 0 || zz >= g.nz) {
      if (g.wall[2]) vz = false;
      zz = zz < 0 ? zz + g.nz : zz - g.nz;
    }
    nb.xo[d + 1] = vx ? xx : kBeyond32;
    nb.yo[d + 1] = vy ? yy * g.nx : kBeyond32;
    nb.zo[d + 1] = vz ? zz * g.ny * g.nx : kBeyond32;
  }
}

__device__ inline int nbr_index32(const Nbr32& nb, int dx, int dy, int dz) {
  return nb.zo[dz + 1] + nb.yo[dy + 1] + nb.xo[dx + 1];
}

// Element i of M at a 32-bit byte offset from the (wave-uniform) base, so
// that loads and stores take the base from scalar registers and one vector
// register per address.
template <class S>
__device__ inline S* at_byte(S* M, uint32_t byte_off) {
  return reinterpret_cast<S*>(reinterpret_cast<char*>(M) + byte_off);
}
template <class S>
__device__ inline const S* at_byte(const S* M, uint32_t byte_off) {
  return reinterpret_cast<const S*>(reinterpret_cast<const char*>(M) + byte_off);
}

// Deviations of the populations at node (x, y, z) at a time whose storage
// parity is P (0: natural layout, population i of node x in slot i of x;
// 1: the AA-swapped layout written by an even step: population i of x sits
// in slot opp(i) of x - c_i, or in slot i of x itself when x - c_i is
// beyond a wall -- the halfway bounce-back).
template <class S>
__device__ inline void load_node(const S* __restrict__ M, const Geom& g, int parity, int x, int y,
                                 int z, typename Store<S>::T d[19]) {
  const long long c = ((long long)z * g.ny + y) * g.nx + x;
  if (parity == 0) {
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = Store<S>::ld(M + (long long)i * g.cells + c);
  } else {
    Nbr nb;
    make_nbr(g, x, y, z, nb);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const long long s = nbr_index(nb, -cx(i), -cy(i), -cz(i));
      d[i] = (s >= 0) ? Store<S>::ld(M + (long long)opp(i) * g.cells + s)
                      : Store<S>::ld(M + (long long)i * g.cells + c);
    }
  }
}

__device__ inline bool is_plane(const Geom& g, int z) {
  return (g.plane_lo && z == 0) || (g.plane_hi && z == g.nz - 1);
}

// Equilibrium deviation f^eq_i(rho, u) - w_i for rho = 1 + drho.
template <class T>
__device__ inline T eq_dev(int i, T drho, T rho, T ux, T uy, T uz) {
  const T cu = cdot<T>(i, ux, uy, uz);
  const T uu = ux * ux + uy * uy + uz * uz;
  return T(wq(i)) * (drho + rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu));
}

// Density deviation and momentum of a node's deviations.
template <class T>
__device__ inline void moments(const T d[19], T& drho, T& jx, T& jy, T& jz) {
  // each sum starts from its first term (no addition of a zero)
  T r = d[0], a = T(0), b = T(0), c = T(0);
  bool ha = false, hb = false, hc = false;
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    r += d[i];
    if (cx(i)) {
      const T v = cx(i) > 0 ? d[i] : -d[i];
      a = ha ? a + v : v;
      ha = true;
    }
    if (cy(i)) {
      const T v = cy(i) > 0 ? d[i] : -d[i];
      b = hb ? b + v : v;
      hb = true;
    }
    if (cz(i)) {
      const T v = cz(i) > 0 ? d[i] : -d[i];
      c = hc ? c + v : v;
      hc = true;
    }
  }
  drho = r;
  jx = a;
  jy = b;
  jz = c;
}

// Map a hardware workgroup id to a logical tile id so that the workgroups
// one XCD receives (hardware ids k, k+8, k+16, ... go round-robin to the 8
// XCDs) cover one contiguous range of tiles, which keeps stencil halos
// inside that XCD's L2.
__device__ inline int xcd_remap(int hw, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int k = hw & 7, j = hw >> 3;
  return (k < r) ? k * (q + 1) + j : r * (q + 1) + (k - r) * q + j;
}

// Biot-Savart grid: a coordinate is represented by a 32-bit integer so that
// periodic separations wrap exactly in two's complement.
struct BsAxes {
  double q[3];      // grid steps per lattice unit
  double off[3];    // added before scaling (1 on wall axes, 0 on periodic)
  float invq_f[3];  // lattice units per grid step, FP32
  double invq_d[3];
  double L[3];
  int periodic[3];
  int uniform;      // 1: one grid step q for all axes (FP32 sum in grid units)
  // source copies of the sum: copy 0 the filaments, copies 1.. their
  // images in the wall planes (refl per axis: 0 none, 1 the plane -1/2,
  // 2 the plane n - 1/2; sign (-1)^(reflections))
  int copies;
  int8_t refl[27][3];
  float sign[27];
};

// Radix-sort tiles: one key per thread, one tile per block.
constexpr int kSortThreads = 1024;
constexpr int kSortMaxBits = 11;
constexpr int kSortMaxBins = 1 << kSortMaxBits;

// Lanes of this wave whose (valid) digit equals this lane's digit.
__device__ inline uint64_t sort_peer_mask(uint32_t d, bool valid, int bits) {
  uint64_t m = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t x = __ballot(valid && bit);
    m &= bit ? x : ~x;
  }
  return m;
}

// Digit histogram of one tile (one key per thread of a kSortThreads block;
// every thread calls it): LDS integer adds by the lowest lane of each digit
// group; counts[d * ntiles + tile] receives the tile's count of digit d.
__device__ inline void sort_tile_count(uint32_t key, bool valid, int shift, int bits, int ntiles,
                                       int tile, int32_t* hist, int32_t* __restrict__ counts) {
  const int t = threadIdx.x, lane = t & 63;
  const int nbins = 1 << bits;
  for (int e = t; e < nbins; e += kSortThreads) hist[e] = 0;
  __syncthreads();
  const uint32_t d = (key >> shift) & (uint32_t)(nbins - 1);
  const uint64_t m = sort_peer_mask(d, valid, bits);
  if (valid && (int)(__ffsll((unsigned long long)m) - 1) == lane) atomicAdd(&hist[d], (int)__popcll(m));
  __syncthreads();
  for (int e = t; e < nbins; e += kSortThreads) counts[(long long)e * ntiles + tile] = hist[e];
}

// Workspace-resident state of a run.
struct Run {
  vlb_lattice_desc lat;
  vlb_vortex_desc vor;
  hipStream_t stream = nullptr;  // the caller's stream: every call's work joins it
  hipStream_t side = nullptr;    // library stream for the lattice part of a step
  hipEvent_t ev_fork = nullptr, ev_mom = nullptr, ev_fin1 = nullptr, ev_join = nullptr;
  int device = 0;
  char* ws = nullptr;
  uint64_t ws_bytes = 0;
  Geom geom;
  BsAxes bsax;
  int prec = 0;
  long long cells = 0;
  long long ncap = 0;

  // lattice
  void* pops = nullptr;   // 19 * cells storage values (deviations)
  void* force = nullptr;  // 3 * cells (double for F64, float otherwise)
  int32_t* touched = nullptr;  // 8 * ncap node indices written by spreading
  double* Vs = nullptr;        // superflow per cross-section along the flow axis
  void* ub = nullptr;          // 3 * cells bare velocity of the current step
  // the same for the next step: its moments are taken right after the LBM
  // update while the stages of this step still read ub (swapped at the
  // end of the step)
  double* Vs_next = nullptr;
  double* mbP = nullptr;       // flow along x or y: per (z, cross-section) partial sums of the mass balance
  double* diag = nullptr;      // diagnostics results (8 + kSlabChunks nz doubles)
  double* seg = nullptr;       // diagnostics: z extent and length per segment (3 n_cap doubles)
  double* fric = nullptr;      // alpha(z), alpha'(z) profiles and their on flag (2 nz + 1 doubles)
  void* ub_next = nullptr;
  int32_t* bins = nullptr;     // spreading: dense bin -> first sorted entry (-1 = empty)
  uint32_t* marked = nullptr;  // per sorted entry: the bin it marked (all ones: none)
  long long nbins_table = 0;

  // filaments
  double* pos = nullptr;   // 3 * ncap, SoA
  double* ya = nullptr;
  double* yb = nullptr;
  double* ksum = nullptr;
  double* vs1 = nullptr;
  double* vn1 = nullptr;
  double* sd1 = nullptr;
  double* gpt = nullptr;
  double* sfrac = nullptr;  // 3 * ncap stencil offsets of the spread positions
  int32_t* nxt = nullptr;
  int32_t* prv = nullptr;
  double* pos_t = nullptr;  // the other point-array set (compaction target)
  int32_t* nxt_t = nullptr;
  int32_t* prv_t = nullptr;

  // Biot-Savart
  uint32_t* bsX = nullptr;  // 3 * ncap grid coordinates
  void* bsD = nullptr;      // 3 * ncap segment vectors (float or double)
  void* bsP = nullptr;      // S * 3 * ncap partial sums
  int32_t* bsown = nullptr;
  // far-field approximation of the non-local sum (vor.ff_cell > 0): its
  // workspace and chunk count (its partials go to bsP)
  void* ffws = nullptr;
  int ffS = 0; // ncap, with image copies: the copy mirrored in an end's own wall
  int bsS = 1;

  // counters on the device: [0] n points, [1] n touched slots,
  // [2] inserted, [3] deleted, [4] reconnections, [5] small-loop points,
  // [6] candidates, [7] error flags, [8] compacted count, [9] bound of the
  // small-loop pass, [10] candidate-slot overflow, [11] points of the
  // spreading in flight, [12] last-block ticket (zero between kernels),
  // [16..17] pair counter
  int32_t* cnt = nullptr;

  // sorting / scans
  uint32_t* keys_a = nullptr;
  uint32_t* keys_b = nullptr;
  int32_t* vals_a = nullptr;
  int32_t* vals_b = nullptr;
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  int key_bits = 32;
  int32_t* flag_a = nullptr;  // per point int flags
  int32_t* flag_b = nullptr;
  int32_t* scan_a = nullptr;
  int32_t* scan_b = nullptr;
  uint64_t* wmask = nullptr;  // per-wave flag ballots
  int32_t* wpre = nullptr;    // per-wave exclusive prefix counts

  // reconnection
  long long rcap = 0;
  int bin_n[3] = {1, 1, 1};
  double bin_h[3] = {1, 1, 1};
  long long rc_nbins = 0;
  int32_t* rc_head = nullptr;    // per bin: last point pushed (-1 = empty)
  int32_t* rc_next = nullptr;    // per point: next point of its bin list
  uint32_t* rc_keyp = nullptr;   // per point: its bin
  int32_t* rc_i = nullptr;
  int32_t* rc_j = nullptr;
  uint64_t* rc_key_a = nullptr;  // candidate keys (bits of d^2)
  int32_t* rc_idx_a = nullptr;   // candidate liveness during matching
  int32_t* rc_slot_j = nullptr;  // per point: up to 8 candidate partners
  uint64_t* rc_slot_k = nullptr; // per point: their keys
  uint64_t* rc_best = nullptr;   // per point: smallest live key
  int32_t* rc_bidx = nullptr;    // per point: smallest live candidate of that key
  int32_t* used = nullptr;

  // staging for host <-> device filament copies
  double* stage = nullptr;  // 3 * ncap doubles
  int32_t* stage_i = nullptr;

  int64_t step = 0;
  int parity = 0;
  int point_parity = 0;     // which of the two point-array sets is current
  bool lbm_narrow = false;  // LBM update launched beside the filament kernels
  bool has_fields = false;
  bool has_points = false;  // set once filaments were seeded

  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[2];

  int64_t last_nodes = 0;
  int64_t last_pairs = 0;

  std::string err;
};

// error flag bits in cnt[7]
constexpr int kFlagCapacity = 1;
constexpr int kFlagNumeric = 2;
constexpr int kFlagReconCap = 4;

// ---- launchers (one per .hip file)
hipError_t lbm_init_eq(Run& r, const double* rho, const double* u);
hipError_t lbm_step(Run& r);
hipError_t lbm_read_fields(Run& r, double* rho, double* u);
hipError_t lbm_read_pops(Run& r, double* f);
hipError_t lbm_read_state(Run& r, void* out);
hipError_t lbm_read_force(Run& r, double* out);
hipError_t lbm_moments(Run& r);
hipError_t lbm_flow_stats(Run& r, double* out);

// The per-slab line length is added over this many chunks of the segments.
constexpr int kSlabChunks = 8;
hipError_t diag_line_length(Run& r, double* total, double* slabs);
hipError_t diag_curl(Run& r, const double* u, double* w);
hipError_t diag_cylindrical(Run& r, const double point[3], const double unit_dir[3],
                            const double* w, double* out);

BsAxes bs_make_axes(const int n[3], const int wall[3], bool images);

// Scratch of the standalone Biot-Savart sum (vlb_biot_savart*): point
// count and pair counter, grid coordinates, FP64 segment data, sanitised
// links, chunk partials.
struct BsSolo {
  int32_t* cnt;
  uint32_t* X;
  void* D;
  int32_t* nxt;
  int32_t* prv;
  void* P;
  int S;
};
constexpr long long kSoloMaxPoints = 1LL << 26;
int bs_check_desc(const vlb_bs_desc* d, int64_t n, std::string& msg);
int bs_solo_chunks(long long n);
size_t bs_solo_layout(int prec, long long n, char* base, BsSolo* b);
hipError_t bs_solo(const BsAxes& ax, int prec, long long n, const double* xyz,
                   const int32_t* next, double kappa, double* v, const BsSolo& b,
                   hipStream_t stream);
// Error message of a call without a run (vlb_last_error(NULL)); returns code.
int fail_global(int code, const std::string& msg);
// Far-field approximation of the non-local sum inside a run: workspace
// bytes and chunk count for the run's capacity, and the sum of one stage's
// positions Y (3 x n_cap, SoA) into the run's chunk partials bsP (lattice
// units, FP32), with the live point count on the device.
size_t ff_run_bytes(const Run& r);
int ff_run_chunks(const Run& r);
hipError_t ff_run_sum(Run& r, const double* Y);
// Far-field approximation of the standalone sum (vlb_biot_savart_farfield).
int ff_check(const vlb_bs_desc* d, const vlb_ff_params* p, int64_t n, std::string& msg);
size_t ff_workspace(const vlb_bs_desc* d, const vlb_ff_params* p, long long n);
hipError_t ff_solo(const vlb_bs_desc* d, const vlb_ff_params* p, long long n, const double* xyz,
                   const int32_t* next, double* v, void* ws, hipStream_t stream);
hipError_t bs_prep(Run& r, const double* Y);
hipError_t bs_sum(Run& r);
int bs_chunks(long long ncap);

// One finalize of a filament stage: stage of the Runge-Kutta method (1..rk),
// first = the first stage of the step's first substep (leaves the stage-1
// velocities, forces and spreading keys), last = the step's last stage (no
// grid coordinates for a next sum).
hipError_t fil_finalize(Run& r, int stage, int first, int last, const double* Y, double* Ynext,
                        int eval_only);
hipError_t fil_copy_positions(Run& r, const double* src, double* dst);
hipError_t fil_spread(Run& r);
hipError_t fil_seed(Run& r, long long n);

// swap: compact into the other point arrays and swap them (steps); else
// compact and copy back (the standalone call)
hipError_t topo_update(Run& r, bool swap);

size_t sort_tmp_bytes(long long n);
int sort_tiles(long long n);
void sort_first_digit(int bits, int* dbits);
int32_t* sort_counts(Run& r);
hipError_t sort_pairs(Run& r, int bits, int first_counted, uint32_t** kres, int32_t** vres);
hipError_t sort_pairs_raw(long long n, int bits, int first_counted, void* tmp, uint32_t* ka,
                          uint32_t* kb, int32_t* va, int32_t* vb, hipStream_t stream,
                          uint32_t** kres, int32_t** vres);

// timing helpers (api.cpp)
void time_begin(Run& r, int cls, hipEvent_t* b);
void time_end(Run& r, int cls, hipEvent_t b);

}  // namespace vlb
