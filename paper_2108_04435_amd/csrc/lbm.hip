// Normal fluid on the D3Q19 lattice (paper Sec. II.B): forced BGK
// collision and streaming in one pass, AA access pattern in a single
// structure-of-arrays population array.
//
// Memory holds deviations d_i = f_i - w_i.  An even pass reads the
// populations of a node from its own slots and writes the post-collision
// values into the opposite slots of the same node; an odd pass reads
// population i of x from slot opp(i) of x - c_i and writes the new
// population i to slot i of x + c_i, which restores the natural layout.  A
// neighbour beyond a wall is replaced by the node itself with the reflected
// slot (halfway bounce-back).  Each node's 19 slots are read and written by
// that node's thread only, so the update is in place and race-free.
#include "vlb_internal.h"

// Multiplies and adds fuse only within one source expression, so that every
// variant of a kernel (even or odd pass, any addressing) rounds the same
// arithmetic the same way, whatever the surrounding control flow: a run
// resumed in the natural layout continues bit for bit.
#pragma clang fp contract(on)

namespace vlb {

namespace {

// The forced BGK collision of one node (Sec. II.B, Eqs. LBM 1-3 collapsed)
// from its 19 raw stored values D (deviations times kScale; overwritten on a
// velocity plane) and the spread force (fx, fy, fz) when has_f: the 19
// post-collision values in the storage format.  Every kernel variant calls
// this one function, so every variant rounds the update identically.
template <class S>
__device__ __forceinline__ void collide_values(typename Store<S>::T* D, bool has_f,
                                               typename Store<S>::T fx,
                                               typename Store<S>::T fy,
                                               typename Store<S>::T fz, const Geom& g,
                                               bool on_plane, S* En) {
  using T = typename Store<S>::T;
  const T kS = T(Raw<S>::kScale);
  const T kInvS = T(1) / kS;  // a power of two: exact
  T om, pref, body[3], plane[3];
  geom_params<T>(g, om, pref, body, plane);
  if (on_plane) {
#pragma unroll
    for (int i = 0; i < 19; ++i) D[i] = kS * eq_dev<T>(i, T(0), T(1), plane[0], plane[1], plane[2]);
  }
  T gx = body[0], gy = body[1], gz = body[2];
  if (has_f) {
    gx += fx;
    gy += fy;
    gz += fz;
  }
  T sD, sx, sy, sz;
  moments<T>(D, sD, sx, sy, sz);
  const T drho = kInvS * sD;
  const T rho = T(1) + drho;
  T inv;
  if constexpr (sizeof(T) == 4) {
    // hardware reciprocal refined by one Newton step (within an ulp of 1/rho)
    const T r0 = __builtin_amdgcn_rcpf(rho);
    inv = fmaf(r0, fmaf(-rho, r0, 1.0f), r0);
  } else {
    inv = T(1) / rho;
  }
  const T ux = (kInvS * sx + T(0.5) * gx) * inv;
  const T uy = (kInvS * sy + T(0.5) * gy) * inv;
  const T uz = (kInvS * sz + T(0.5) * gz) * inv;
  const T ug = ux * gx + uy * gy + uz * gz;
  // Post-collision value f - (f - f^eq)/tau + F_i with f^eq and the
  // Cheng-Li/Guo term F_i built from rho and u = (sum c f + g/2)/rho
  // (Sec. II.B, Eqs. LBM 1-3 collapsed).  It is (1 - 1/tau) d_i +
  // [d^eq_i/tau + F_i], and the bracket splits into parts even and odd in
  // c_i, shared by each pair (i, opp(i)): with cu = c_i.u and cg = c_i.g it
  // is w_i (P + Q) for i and w_i (P - Q) for opp(i),
  //   P = om (drho - 1.5 rho u.u) - 3 pref u.g + cu (4.5 om rho cu + 9 pref cg),
  //   Q = 3 om rho cu + 3 pref cg,
  // all of it times kScale, the storage scale.  Half the directional terms
  // of the direct form; it matters with FP16 storage, where the arithmetic
  // is a large share of the update.
  T Dn[19];
  {
    const T uu = ux * ux + uy * uy + uz * uz;
    const T om1 = T(1) - om;
    const T Kp = om * (drho - T(1.5) * rho * uu) - T(3) * pref * ug;
    const T a1 = T(4.5) * om * rho, a2 = T(9) * pref;
    const T b1 = T(3) * om * rho, b2 = T(3) * pref;
    Dn[0] = fma(om1, D[0], (T(wq(0)) * kS) * Kp);
#pragma unroll
    for (int k = 1; k <= 9; ++k) {
      const int i = 2 * k - 1;  // i and opp(i) = i + 1
      const T ws = T(wq(i)) * kS;
      const T cu = cdot<T>(i, ux, uy, uz);
      const T cg = cdot<T>(i, gx, gy, gz);
      const T Pk = ws * fma(cu, fma(a1, cu, a2 * cg), Kp);
      const T Qk = ws * fma(b1, cu, b2 * cg);
      Dn[i] = fma(om1, D[i], Pk + Qk);
      Dn[i + 1] = fma(om1, D[i + 1], Pk - Qk);
    }
  }
  // Values in the storage format, encoded here, before the passes'
  // addressing branches: a conversion to FP16 that the compiler fuses with
  // the last multiply-add rounds once, and it must do so in every variant.
#pragma unroll
  for (int i = 0; i < 19; ++i) En[i] = Raw<S>::enc(Dn[i]);
}

// Post-collision deviation (Sec. II.B, Eqs. LBM 1-3 collapsed):
// f''' = f - (f - f^eq)/tau + F, with f^eq and the Cheng-Li/Guo term F built
// from rho and u = (sum c f + g/2)/rho.
//
// I32: the lattice has fewer than 2^29 nodes and its population array
// spans less than 4 GiB, so a slot has a 32-bit byte offset.  With FP16
// storage, where the vector arithmetic is a large share of the update, the
// array is accessed as a raw buffer: a slot's byte offset is a per-lane part
// plus a uniform part.  Even passes use the node's own offset for all 38
// accesses and the slot's slab as the uniform part.  Odd passes of a tile
// that is periodic in x and y and has both z neighbours (a tile is one z
// slice: the choice is uniform) use nine per-lane offsets, one per (dx, dy)
// in {-1, 0, 1}^2, and the slab plus the neighbour slice as the uniform
// part, so that no access costs vector arithmetic (256^3: odd pass 626 ->
// 395 VALU instructions per wave, 308 -> 247 us).  Other tiles, and FP32
// and FP64 storage (bound by HBM, and 1-3% faster with plain global
// accesses), find each neighbour's slot (or the bounce-back slot) per lane
// from one base.
template <class S, int P, bool NT, bool I32>
__device__ __forceinline__ void collide_node(S* __restrict__ M,
                                             const typename Store<S>::T* __restrict__ F,
                                             const Geom& g, int x, int y, int z) {
  using T = typename Store<S>::T;
  const long long c = ((long long)z * g.ny + y) * g.nx + x;
  const uint32_t c32 = (uint32_t)c;
  const uint32_t cells32 = (uint32_t)g.cells;
  constexpr uint32_t kSz = sizeof(S);
  constexpr bool kBuf = I32 && sizeof(S) == 2;
  const bool fast = P == 1 && kBuf && !g.wall[0] && !g.wall[1] &&
                    (!g.wall[2] || (z > 0 && z < g.nz - 1));
  __amdgpu_buffer_rsrc_t rs;
  if (kBuf) rs = pop_rsrc(M, (uint32_t)(19ull * g.cells * kSz));

  // raw stored values (deviations times kScale)
  T D[19];
  Nbr nb;
  Nbr32 nb32;
  uint32_t off[3][3];  // [dy + 1][dx + 1]: byte offset of (x + dx, y + dy) in a slice
  uint32_t zo[3];      // [dz + 1]: byte offset of slice z + dz (periodic)
  if (P == 1 && fast) {
    const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny, nz = (uint32_t)g.nz;
    const uint32_t ux = (uint32_t)x, uy = (uint32_t)y, uz = (uint32_t)z;
    const uint32_t xo[3] = {ux == 0 ? nx - 1 : ux - 1, ux, ux + 1 == nx ? 0u : ux + 1};
    const uint32_t yo[3] = {(uy == 0 ? ny - 1 : uy - 1) * nx, uy * nx,
                            (uy + 1 == ny ? 0u : uy + 1) * nx};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) off[a][b] = (yo[a] + xo[b]) * kSz;
    const uint32_t sl = nx * ny * kSz;
    zo[0] = (uz == 0 ? nz - 1 : uz - 1) * sl;
    zo[1] = uz * sl;
    zo[2] = (uz + 1 == nz ? 0u : uz + 1) * sl;
  } else if (P == 1) {
    if (I32)
      make_nbr32(g, x, y, z, nb32);
    else
      make_nbr(g, x, y, z, nb);
  }
  if (P == 0 && kBuf) {
    const uint32_t vo = c32 * kSz;
#pragma unroll
    for (int i = 0; i < 19; ++i) D[i] = Buf<S>::template ld<NT>(rs, vo, (uint32_t)i * cells32 * kSz);
  } else if (P == 0) {
#pragma unroll
    for (int i = 0; i < 19; ++i) D[i] = Raw<S>::template ld<NT>(M + (long long)i * g.cells + c);
  } else if (fast) {
    // slot opp(i) of x - c_i
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const uint32_t o = off[1 - cy(i)][1 - cx(i)];
      const uint32_t so = (uint32_t)opp(i) * cells32 * kSz + zo[1 - cz(i)];
      // FP64: the x-shifted loads (a wave spans five lines instead of
      // four) go through L2, where the neighbouring wave finds the shared
      // line (256^3: 0.940 -> 0.932 ms per update; no gain for FP32/FP16)
      if (NT && (sizeof(S) < 8 || cx(i) == 0))
        D[i] = Buf<S>::template ld<true>(rs, o, so);
      else
        D[i] = Buf<S>::template ld<false>(rs, o, so);
    }
  } else if (I32) {
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const int s = nbr_index32(nb32, -cx(i), -cy(i), -cz(i));
      const uint32_t e = (s >= 0) ? (uint32_t)opp(i) * cells32 + (uint32_t)s
                                  : (uint32_t)i * cells32 + c32;
      if (NT && (sizeof(S) < 8 || cx(i) == 0))
        D[i] = Raw<S>::template ld<true>(at_byte(M, e * kSz));
      else
        D[i] = Raw<S>::template ld<false>(at_byte(M, e * kSz));
    }
  } else {
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const long long s = nbr_index(nb, -cx(i), -cy(i), -cz(i));
      D[i] = (s >= 0) ? Raw<S>::template ld<NT>(M + (long long)opp(i) * g.cells + s)
                      : Raw<S>::template ld<NT>(M + (long long)i * g.cells + c);
    }
  }
  T fxv = T(0), fyv = T(0), fzv = T(0);
  if (F) {
    if (I32) {
      const uint32_t fo = c32 * (uint32_t)sizeof(T);
      fxv = *at_byte(F, fo);
      fyv = *at_byte(F + g.cells, fo);
      fzv = *at_byte(F + 2 * g.cells, fo);
    } else {
      fxv = F[c];
      fyv = F[g.cells + c];
      fzv = F[2 * g.cells + c];
    }
  }
  S En[19];
  collide_values<S>(D, F != nullptr, fxv, fyv, fzv, g, is_plane(g, z), En);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const S dn = En[i];
    // Odd passes store to the neighbours' slots: a direction with an x
    // component stores each wave's values one element off the cache lines,
    // and those partial lines must meet their other part in L2, so only the
    // directions without an x component bypass it with non-temporal stores
    // (256^3 FP32: 7% fewer bytes written, odd pass 537 -> 460 us).
    const bool nt_st = NT && (P == 0 || cx(i) == 0);
    if (P == 0 && kBuf) {
      Buf<S>::template st<NT>(rs, c32 * kSz, (uint32_t)opp(i) * cells32 * kSz, dn);
    } else if (P == 0) {
      Raw<S>::template st_enc<NT>(M + (long long)opp(i) * g.cells + c, dn);
    } else if (fast) {
      // slot i of x + c_i
      const uint32_t o = off[1 + cy(i)][1 + cx(i)];
      const uint32_t so = (uint32_t)i * cells32 * kSz + zo[1 + cz(i)];
      if (nt_st)
        Buf<S>::template st<true>(rs, o, so, dn);
      else
        Buf<S>::template st<false>(rs, o, so, dn);
    } else if (I32) {
      const int s = nbr_index32(nb32, cx(i), cy(i), cz(i));
      const uint32_t e = (s >= 0) ? (uint32_t)i * cells32 + (uint32_t)s
                                  : (uint32_t)opp(i) * cells32 + c32;
      if (nt_st)
        Raw<S>::template st_enc<true>(at_byte(M, e * kSz), dn);
      else
        Raw<S>::template st_enc<false>(at_byte(M, e * kSz), dn);
    } else {
      const long long s = nbr_index(nb, cx(i), cy(i), cz(i));
      S* p = (s >= 0) ? M + (long long)i * g.cells + s : M + (long long)opp(i) * g.cells + c;
      if (nt_st)
        Raw<S>::template st_enc<true>(p, dn);
      else
        Raw<S>::template st_enc<false>(p, dn);
    }
  }
}

// Tiles of (bx, 256 / bx) nodes (x, y) of one z slice; hardware blocks are mapped
// so that the blocks of one XCD cover one contiguous range of tiles.  The
// grid may be smaller than the tile count (a multiple of 8): each block
// then walks tiles b, b + grid, ..., which stay on its XCD's range.  The
// tile id splits into (x tile, y tile, z) by divisions by the launch's
// tile counts.
template <class S, int P, bool NT, bool I32>
__global__ __launch_bounds__(256) void k_collide_stream(S* __restrict__ M,
                                                        const typename Store<S>::T* __restrict__ F,
                                                        Geom g, FastDiv fbx, FastDiv fby, int nblk) {
  for (int it = blockIdx.x; it < nblk; it += gridDim.x) {
    const uint32_t t = (uint32_t)xcd_remap(it, nblk);
    const uint32_t rr = fdiv(t, fbx);
    const uint32_t zq = fdiv(rr, fby);
    const int bxi = (int)(t - rr * fbx.d);
    const int byi = (int)(rr - zq * fby.d);
    const int z = (int)zq;
    const int x = bxi * blockDim.x + threadIdx.x;
    const int y = byi * blockDim.y + threadIdx.y;
    if (x < g.nx && y < g.ny) collide_node<S, P, NT, I32>(M, F, g, x, y, z);
  }
}

// FP16 storage on rows of exactly 256 nodes, periodic in x and y: one wave
// per row (z, y), four x-consecutive nodes per lane, every slot of the
// four read or written with one aligned 8-byte buffer access (2-byte
// accesses cap the pattern at about 0.71 of the HBM peak, 8-byte ones at
// about 0.77: pure-memory probes on this chip).  The lane's byte offset in
// a row is the same for all 38 accesses; rows and slabs are uniform.  The
// x-shifted directions of odd passes move one node across lanes: the
// element entering from the previous lane (or, for -x, from the next) comes
// with a one-lane rotation of the whole wave, which also wraps x
// periodically (lane 0 takes lane 63's last node).  Each slot is still read
// and written by its own node's lane only.  Odd passes of the slices next
// to z walls take the per-node path (collide_node) for the lane's four
// nodes.
__device__ inline uint32_t rot_prev(uint32_t v) {  // lane L gets lane L - 1's value (wave_ror:1)
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x13C, 0xF, 0xF, false);
}
__device__ inline uint32_t rot_next(uint32_t v) {  // lane L gets lane L + 1's value (wave_rol:1)
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x134, 0xF, 0xF, false);
}
// The lane's four nodes (halves e0..e3 in lo/hi of .x, .y) as seen one
// node to the left: [e3 of lane L - 1, e0, e1, e2]; and to the right:
// [e1, e2, e3, e0 of lane L + 1].
__device__ inline vlb_u32x2 shift_in_prev(vlb_u32x2 g) {
  const uint32_t p3 = rot_prev(g.y) >> 16;
  vlb_u32x2 o;
  o.x = (g.x << 16) | p3;
  o.y = (g.y << 16) | (g.x >> 16);
  return o;
}
__device__ inline vlb_u32x2 shift_in_next(vlb_u32x2 g) {
  const uint32_t n0 = rot_next(g.x) & 0xffffu;
  vlb_u32x2 o;
  o.x = (g.x >> 16) | (g.y << 16);
  o.y = (g.y >> 16) | (n0 << 16);
  return o;
}

template <int P, bool NT>
__global__ __launch_bounds__(256) void k_collide_rows4(__half* __restrict__ M,
                                                       const float* __restrict__ F, Geom g,
                                                       int nblk) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows = g.ny * g.nz;
  const uint32_t cells32 = (uint32_t)g.cells;
  const uint32_t slab = cells32 * 2u;
  const __amdgpu_buffer_rsrc_t rs = pop_rsrc(M, 19u * slab);
  const uint32_t vo = (uint32_t)lane * 8u;  // byte offset of the lane's nodes in a row
  for (int it = blockIdx.x; it < nblk; it += gridDim.x) {
    const int row = __builtin_amdgcn_readfirstlane(xcd_remap(it, nblk) * 4 + w);
    if (row >= rows) continue;
    const int z = row / g.ny, y = row - z * g.ny;
    if (P == 1 && g.wall[2] && (z == 0 || z == g.nz - 1)) {
#pragma unroll 1
      for (int k = 0; k < 4; ++k) collide_node<__half, 1, NT, true>(M, F, g, 4 * lane + k, y, z);
      continue;
    }
    // byte offsets of the rows (y + dy, z + dz), periodic
    uint32_t ro[3][3];  // [dz + 1][dy + 1]
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        int zz = z + dz, yy = y + dy;
        zz = zz < 0 ? zz + g.nz : (zz >= g.nz ? zz - g.nz : zz);
        yy = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
        ro[dz + 1][dy + 1] = (uint32_t)(zz * g.ny + yy) * 512u;
      }
    vlb_u32x2 G[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      if (P == 0) {
        G[i] = __builtin_bit_cast(vlb_u32x2, __builtin_amdgcn_raw_buffer_load_b64(
                                                 rs, vo, (uint32_t)i * slab + ro[1][1], NT ? 2 : 0));
      } else {
        // slot opp(i) of x - c_i
        const vlb_u32x2 v = __builtin_bit_cast(
            vlb_u32x2, __builtin_amdgcn_raw_buffer_load_b64(
                           rs, vo, (uint32_t)opp(i) * slab + ro[1 - cz(i)][1 - cy(i)], NT ? 2 : 0));
        G[i] = cx(i) == 1 ? shift_in_prev(v) : (cx(i) == -1 ? shift_in_next(v) : v);
      }
    }
    const long long fo = (long long)row * 256 + 4 * lane;  // the lane's first node
    const bool pl = is_plane(g, z);
    vlb_u32x2 O[19];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float D[19];
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const uint32_t word = (k < 2) ? G[i].x : G[i].y;
        const unsigned short h = (unsigned short)((k & 1) ? (word >> 16) : (word & 0xffffu));
        D[i] = __half2float(__ushort_as_half(h));
      }
      float fx = 0.f, fy = 0.f, fz = 0.f;
      if (F) {
        fx = F[fo + k];
        fy = F[g.cells + fo + k];
        fz = F[2 * g.cells + fo + k];
      }
      __half En[19];
      collide_values<__half>(D, F != nullptr, fx, fy, fz, g, pl, En);
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const uint32_t h = (uint32_t)__half_as_ushort(En[i]);
        if (k == 0) O[i].x = h;
        else if (k == 1) O[i].x |= h << 16;
        else if (k == 2) O[i].y = h;
        else O[i].y |= h << 16;
      }
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      if (P == 0) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(vlb_u32x2, O[i]), rs, vo,
                                              (uint32_t)opp(i) * slab + ro[1][1], NT ? 2 : 0);
      } else {
        // slot i of x + c_i: the lane's group holds the values of the nodes
        // one to the left (+x) or right (-x)
        const vlb_u32x2 v = cx(i) == 1 ? shift_in_prev(O[i]) : (cx(i) == -1 ? shift_in_next(O[i]) : O[i]);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(vlb_u32x2, v), rs, vo,
                                              (uint32_t)i * slab + ro[1 + cz(i)][1 + cy(i)],
                                              NT ? 2 : 0);
      }
    }
  }
}

template <class S>
__global__ void k_init_eq(S* __restrict__ M, const double* __restrict__ rho,
                          const double* __restrict__ u, Geom g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.cells) return;
  const double r = rho[c];
  const double ux = u[c], uy = u[g.cells + c], uz = u[2 * g.cells + c];
  const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const double cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
    const double feq = wq(i) * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    Store<S>::st(M + (long long)i * g.cells + c, (typename Store<S>::T)(feq - wq(i)));
  }
}

// Effective density and bare velocity of node c (velocity planes applied).
template <class S>
__device__ inline void node_rho_u(const S* M, const Geom& g, int parity, int x, int y, int z,
                                  double& rho, double& ux, double& uy, double& uz) {
  using T = typename Store<S>::T;
  if (is_plane(g, z)) {
    rho = 1.0;
    ux = g.plane_u[0];
    uy = g.plane_u[1];
    uz = g.plane_u[2];
    return;
  }
  T d[19];
  load_node<S>(M, g, parity, x, y, z, d);
  T drho, jx, jy, jz;
  moments<T>(d, drho, jx, jy, jz);
  rho = 1.0 + (double)drho;
  ux = (double)jx / rho;
  uy = (double)jy / rho;
  uz = (double)jz / rho;
}

template <class S>
__global__ void k_read_fields(const S* __restrict__ M, Geom g, int parity, double* rho_out,
                              double* u_out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.cells) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  double rho, ux, uy, uz;
  node_rho_u<S>(M, g, parity, x, y, z, rho, ux, uy, uz);
  if (rho_out) rho_out[c] = rho;
  if (u_out) {
    u_out[c] = ux;
    u_out[g.cells + c] = uy;
    u_out[2 * g.cells + c] = uz;
  }
}

template <class S>
__global__ void k_read_pops(const S* __restrict__ M, Geom g, int parity, double* f) {
  using T = typename Store<S>::T;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.cells) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  T d[19];
  load_node<S>(M, g, parity, x, y, z, d);
#pragma unroll
  for (int i = 0; i < 19; ++i) f[(long long)i * g.cells + c] = wq(i) + (double)d[i];
}

// The stored values (deviations in the storage format) of every node's
// populations in natural layout (population i of node c in slot i of c),
// gathered from the current AA layout.
template <class S>
__global__ void k_read_state(const S* __restrict__ M, Geom g, int parity, S* __restrict__ out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.cells) return;
  if (parity == 0) {
#pragma unroll
    for (int i = 0; i < 19; ++i) out[(long long)i * g.cells + c] = M[(long long)i * g.cells + c];
    return;
  }
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  Nbr nb;
  make_nbr(g, x, y, z, nb);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const long long s = nbr_index(nb, -cx(i), -cy(i), -cz(i));
    out[(long long)i * g.cells + c] = (s >= 0) ? M[(long long)opp(i) * g.cells + s]
                                               : M[(long long)i * g.cells + c];
  }
}

template <class T>
__global__ void k_read_force(const T* __restrict__ F, long long n, double* out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) out[c] = F ? (double)F[c] : 0.0;
}

// Bare normal-fluid velocity u_b = sum(c f)/sum(f) of every node (velocity
// planes applied), written once per step for the interpolation onto the
// filaments, fused (flow along z) with the mean of u_z over each z slice
// that the mass-balance superflow needs (Sec. III.C, Eq. mass cons): one
// block per slice walks the slice in tiles (x fastest), each thread adds
// its nodes' u_z in order, the block adds the threads' sums in a fixed
// tree, and Vs[z] = scale * sum.  Vs is null otherwise.
template <class S, class UT>
__global__ __launch_bounds__(1024) void k_moments(const S* __restrict__ M, Geom g, int parity,
                                                 UT* __restrict__ ub, double scale,
                                                 double* __restrict__ Vs) {
  const int z = blockIdx.x;
  double uzv = 0.0;
  for (int y0 = 0; y0 < g.ny; y0 += blockDim.y)
    for (int x0 = 0; x0 < g.nx; x0 += blockDim.x) {
      const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
      if (x < g.nx && y < g.ny) {
        double rho, ux, uy, uz;
        node_rho_u<S>(M, g, parity, x, y, z, rho, ux, uy, uz);
        const long long c = ((long long)z * g.ny + y) * g.nx + x;
        ub[c] = (UT)ux;
        ub[g.cells + c] = (UT)uy;
        ub[2 * g.cells + c] = (UT)uz;
        uzv += uz;
      }
    }
  if (!Vs) return;
  __shared__ double red[1024];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nt = blockDim.x * blockDim.y;
  red[tid] = uzv;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s && tid + s < nt) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) Vs[z] = scale * red[0];
}

// Mass balance along x or y (flow axis a): for each z slice and each node
// position i along a, the sum of u_a over the slice's other axis in
// ascending order (one thread per (i, z)); then for each i the slice sums
// in ascending z, Vs[i] = scale * total.  u_a is the bare velocity the
// moments kernel wrote.
template <class UT>
__global__ void k_mb_partial(const UT* __restrict__ ua, Geom g, int axis, double* __restrict__ P) {
  const int z = blockIdx.y;
  const int n = axis == 0 ? g.nx : g.ny;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long slice = (long long)z * g.ny * g.nx;
  double s = 0.0;
  if (axis == 0)
    for (int y = 0; y < g.ny; ++y) s += (double)ua[slice + (long long)y * g.nx + i];
  else
    for (int x = 0; x < g.nx; ++x) s += (double)ua[slice + (long long)i * g.nx + x];
  P[(long long)z * n + i] = s;
}

__global__ void k_mb_total(const double* __restrict__ P, int nz, int n, double scale,
                           double* __restrict__ Vs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += P[(long long)z * n + i];
  Vs[i] = scale * s;
}

// Sum of v[0..2] over the 1024 threads of a block in a fixed tree; every
// thread returns the three totals.
__device__ inline void block_sum3_1024(double v[3], double (*red)[1024]) {
  const int t = threadIdx.x;
  for (int a = 0; a < 3; ++a) red[a][t] = v[a];
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s)
      for (int a = 0; a < 3; ++a) red[a][t] += red[a][t + s];
    __syncthreads();
  }
  for (int a = 0; a < 3; ++a) v[a] = red[a][0];
  __syncthreads();
}

// Statistics of the bare velocity over each z slice (diagnostics of the
// mean flow and its fluctuations, Sec. III.C): one block of 1024 threads
// per slice; the slice mean of each component, then the sum of the squared
// deviations from that mean (the nodes' velocities are recomputed from the
// populations in the second pass).  Each thread adds its nodes in order,
// the block adds the threads in a fixed tree.  out[6 z + a] = mean of
// component a, out[6 z + 3 + a] = sum of squared deviations.
template <class S>
__global__ __launch_bounds__(1024) void k_flow_stats(const S* __restrict__ M, Geom g, int parity,
                                                    double* __restrict__ out) {
  __shared__ double red[3][1024];
  const int z = blockIdx.x;
  const long long ns = (long long)g.nx * g.ny;
  double v[3] = {0.0, 0.0, 0.0};
  for (long long k = threadIdx.x; k < ns; k += 1024) {
    double rho, u[3];
    node_rho_u<S>(M, g, parity, (int)(k % g.nx), (int)(k / g.nx), z, rho, u[0], u[1], u[2]);
    for (int a = 0; a < 3; ++a) v[a] += u[a];
  }
  block_sum3_1024(v, red);
  const double m[3] = {v[0] / (double)ns, v[1] / (double)ns, v[2] / (double)ns};
  double q[3] = {0.0, 0.0, 0.0};
  for (long long k = threadIdx.x; k < ns; k += 1024) {
    double rho, u[3];
    node_rho_u<S>(M, g, parity, (int)(k % g.nx), (int)(k / g.nx), z, rho, u[0], u[1], u[2]);
    for (int a = 0; a < 3; ++a) q[a] += (u[a] - m[a]) * (u[a] - m[a]);
  }
  block_sum3_1024(q, red);
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) {
      out[6 * z + a] = m[a];
      out[6 * z + 3 + a] = q[a];
    }
}

inline int blocks_for(long long n, int b) { return (int)((n + b - 1) / b); }

// Population arrays above this size are streamed with non-temporal hints
// (the last-level cache is 256 MB; smaller lattices stay resident in it
// from one step to the next).
constexpr double kStreamBytes = 192.0 * (1 << 20);

template <class S>
hipError_t launch_collide(Run& r) {
  using T = typename Store<S>::T;
  const Geom& g = r.geom;
  // one x row of up to 256 nodes per block: the x-shifted accesses of odd
  // passes stay inside the block's row (measured 4% faster than 64 x 4)
  const int bx = g.nx < 256 ? g.nx : 256;
  const int by = 256 / bx;
  const int nbx = (g.nx + bx - 1) / bx;
  const int nby = (g.ny + by - 1) / by;
  const int nblk = nbx * nby * g.nz;
  // the spread force field exists once filaments were seeded into a coupled run
  const T* F = (r.vor.coupling && r.has_points) ? (const T*)r.force : nullptr;
  dim3 blk(bx, by);
  // beside the filament kernels the update runs on a narrow grid (two
  // blocks per CU), leaving most CU slots to the other stream
  int grid = nblk;
  if (r.lbm_narrow && grid > 512) grid = 512;
  // populations far above the last-level cache: non-temporal accesses
  const bool nt = 19.0 * (double)g.cells * sizeof(S) > kStreamBytes;
  // odd passes: 32-bit slot offsets when the population array spans less than 4 GiB
  const bool i32 = g.cells < (1LL << 29) && 19.0 * (double)g.cells * sizeof(S) < 4294967296.0;
  if constexpr (sizeof(S) == 2) {
    // rows of 256 nodes periodic in x and y: four nodes per lane
    if (i32 && g.nx == 256 && !g.wall[0] && !g.wall[1]) {
      const int nrb = (g.ny * g.nz + 3) / 4;  // blocks of four rows
      int grid4 = nrb;
      if (r.lbm_narrow && grid4 > 512) grid4 = 512;
      auto k4 = r.parity == 0 ? (nt ? k_collide_rows4<0, true> : k_collide_rows4<0, false>)
                              : (nt ? k_collide_rows4<1, true> : k_collide_rows4<1, false>);
      hipLaunchKernelGGL(k4, dim3(grid4), dim3(256), 0, r.stream, (__half*)r.pops, (const float*)F,
                         g, nrb);
      return hipGetLastError();
    }
  }
  auto kern = r.parity == 0
                  ? (i32 ? (nt ? k_collide_stream<S, 0, true, true> : k_collide_stream<S, 0, false, true>)
                         : (nt ? k_collide_stream<S, 0, true, false> : k_collide_stream<S, 0, false, false>))
                  : (i32 ? (nt ? k_collide_stream<S, 1, true, true> : k_collide_stream<S, 1, false, true>)
                         : (nt ? k_collide_stream<S, 1, true, false> : k_collide_stream<S, 1, false, false>));
  hipLaunchKernelGGL(kern, dim3(grid), blk, 0, r.stream, (S*)r.pops, F, g, make_fastdiv(nbx),
                     make_fastdiv(nby), nblk);
  return hipGetLastError();
}

}  // namespace

hipError_t lbm_step(Run& r) {
  hipEvent_t b = nullptr;
  time_begin(r, 1, &b);
  hipError_t e;
  switch (r.prec) {
    case VLB_F64: e = launch_collide<double>(r); break;
    case VLB_F32: e = launch_collide<float>(r); break;
    default: e = launch_collide<__half>(r); break;
  }
  time_end(r, 1, b);
  r.parity ^= 1;
  return e;
}

hipError_t lbm_init_eq(Run& r, const double* rho, const double* u) {
  const int nb = blocks_for(r.cells, 256);
  switch (r.prec) {
    case VLB_F64:
      hipLaunchKernelGGL(k_init_eq<double>, dim3(nb), dim3(256), 0, r.stream, (double*)r.pops, rho, u, r.geom);
      break;
    case VLB_F32:
      hipLaunchKernelGGL(k_init_eq<float>, dim3(nb), dim3(256), 0, r.stream, (float*)r.pops, rho, u, r.geom);
      break;
    default:
      hipLaunchKernelGGL(k_init_eq<__half>, dim3(nb), dim3(256), 0, r.stream, (__half*)r.pops, rho, u, r.geom);
      break;
  }
  r.parity = 0;
  return hipGetLastError();
}

hipError_t lbm_read_fields(Run& r, double* rho, double* u) {
  const int nb = blocks_for(r.cells, 256);
  switch (r.prec) {
    case VLB_F64:
      hipLaunchKernelGGL(k_read_fields<double>, dim3(nb), dim3(256), 0, r.stream, (const double*)r.pops, r.geom, r.parity, rho, u);
      break;
    case VLB_F32:
      hipLaunchKernelGGL(k_read_fields<float>, dim3(nb), dim3(256), 0, r.stream, (const float*)r.pops, r.geom, r.parity, rho, u);
      break;
    default:
      hipLaunchKernelGGL(k_read_fields<__half>, dim3(nb), dim3(256), 0, r.stream, (const __half*)r.pops, r.geom, r.parity, rho, u);
      break;
  }
  return hipGetLastError();
}

hipError_t lbm_read_pops(Run& r, double* f) {
  const int nb = blocks_for(r.cells, 256);
  switch (r.prec) {
    case VLB_F64:
      hipLaunchKernelGGL(k_read_pops<double>, dim3(nb), dim3(256), 0, r.stream, (const double*)r.pops, r.geom, r.parity, f);
      break;
    case VLB_F32:
      hipLaunchKernelGGL(k_read_pops<float>, dim3(nb), dim3(256), 0, r.stream, (const float*)r.pops, r.geom, r.parity, f);
      break;
    default:
      hipLaunchKernelGGL(k_read_pops<__half>, dim3(nb), dim3(256), 0, r.stream, (const __half*)r.pops, r.geom, r.parity, f);
      break;
  }
  return hipGetLastError();
}

hipError_t lbm_read_state(Run& r, void* out) {
  const int nb = blocks_for(r.cells, 256);
  switch (r.prec) {
    case VLB_F64:
      hipLaunchKernelGGL(k_read_state<double>, dim3(nb), dim3(256), 0, r.stream, (const double*)r.pops, r.geom, r.parity, (double*)out);
      break;
    case VLB_F32:
      hipLaunchKernelGGL(k_read_state<float>, dim3(nb), dim3(256), 0, r.stream, (const float*)r.pops, r.geom, r.parity, (float*)out);
      break;
    default:
      hipLaunchKernelGGL(k_read_state<__half>, dim3(nb), dim3(256), 0, r.stream, (const __half*)r.pops, r.geom, r.parity, (__half*)out);
      break;
  }
  return hipGetLastError();
}

hipError_t lbm_flow_stats(Run& r, double* out) {
  const int nz = r.geom.nz;
  switch (r.prec) {
    case VLB_F64:
      hipLaunchKernelGGL(k_flow_stats<double>, dim3(nz), dim3(1024), 0, r.stream, (const double*)r.pops, r.geom, r.parity, out);
      break;
    case VLB_F32:
      hipLaunchKernelGGL(k_flow_stats<float>, dim3(nz), dim3(1024), 0, r.stream, (const float*)r.pops, r.geom, r.parity, out);
      break;
    default:
      hipLaunchKernelGGL(k_flow_stats<__half>, dim3(nz), dim3(1024), 0, r.stream, (const __half*)r.pops, r.geom, r.parity, out);
      break;
  }
  return hipGetLastError();
}

hipError_t lbm_read_force(Run& r, double* out) {
  const long long n = 3 * r.cells;
  const int nb = blocks_for(n, 256);
  if (r.prec == VLB_F64)
    hipLaunchKernelGGL(k_read_force<double>, dim3(nb), dim3(256), 0, r.stream, (const double*)r.force, n, out);
  else
    hipLaunchKernelGGL(k_read_force<float>, dim3(nb), dim3(256), 0, r.stream, (const float*)r.force, n, out);
  return hipGetLastError();
}

hipError_t lbm_moments(Run& r) {
  const Geom& g = r.geom;
  const int bx = g.nx < 64 ? g.nx : 64;
  // beside the filament kernels: 256 threads per slice block, else 1024
  int by = (r.lbm_narrow ? 256 : 1024) / bx;
  if (by < 1) by = 1;
  if (by > g.ny) by = g.ny;
  dim3 blk(bx, by);
  // flow along z: the slice means come with the moments (one block per z
  // slice); along x or y: two small passes over u_a afterwards
  const int axis = r.vor.mass_balance_axis;
  const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
  double* Vs = (r.vor.mass_balance && axis == 2) ? r.Vs : nullptr;
  const double scale = -(1.0 / r.vor.rho_s_over_rho_n) / ((double)g.cells / n);
  switch (r.prec) {
    case VLB_F64:
      hipLaunchKernelGGL((k_moments<double, double>), dim3(g.nz), blk, 0, r.stream, (const double*)r.pops, g, r.parity, (double*)r.ub, scale, Vs);
      break;
    case VLB_F32:
      hipLaunchKernelGGL((k_moments<float, float>), dim3(g.nz), blk, 0, r.stream, (const float*)r.pops, g, r.parity, (float*)r.ub, scale, Vs);
      break;
    default:
      hipLaunchKernelGGL((k_moments<__half, float>), dim3(g.nz), blk, 0, r.stream, (const __half*)r.pops, g, r.parity, (float*)r.ub, scale, Vs);
      break;
  }
  if (r.vor.mass_balance && axis != 2) {
    const dim3 pg((n + 63) / 64, g.nz);
    if (r.prec == VLB_F64)
      hipLaunchKernelGGL(k_mb_partial<double>, pg, dim3(64), 0, r.stream, (const double*)r.ub + (long long)axis * g.cells, g, axis, r.mbP);
    else
      hipLaunchKernelGGL(k_mb_partial<float>, pg, dim3(64), 0, r.stream, (const float*)r.ub + (long long)axis * g.cells, g, axis, r.mbP);
    hipLaunchKernelGGL(k_mb_total, dim3((n + 63) / 64), dim3(64), 0, r.stream, (const double*)r.mbP, g.nz, n, scale, r.Vs);
  }
  return hipGetLastError();
}

}  // namespace vlb
