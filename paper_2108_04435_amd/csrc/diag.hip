// Diagnostics of the coupled state (paper Sec. III.A, III.C, IV): the
// vortex line length, in total and per slab along z (the line density the
// paper follows in time and along the channel), and the vorticity of the
// normal fluid.  (The velocity statistics of the mean flow and its
// fluctuations are a lattice pass and live with the other lattice kernels.)
//
// Every sum runs in FP64 in a fixed order (per-thread strided sums, then a
// fixed tree), so the results are bitwise reproducible.
#include "vlb_internal.h"

namespace vlb {

namespace {

// Segment j -> nxt[j] at the nearest periodic image; a separation of
// exactly half the period is left alone.
__device__ inline void segment(const double* __restrict__ pos, const int32_t* __restrict__ nxt,
                               long long nc, const Geom& g, int j, double d[3], double& z0) {
  const int k = nxt[j];
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    const double p = pos[a * nc + j];
    double x = pos[a * nc + k] - p;
    if (!g.wall[a]) {
      const double L = (double)n[a];
      if (x > 0.5 * L)
        x -= L;
      else if (x < -0.5 * L)
        x += L;
    }
    d[a] = x;
    if (a == 2) z0 = p;
  }
}

template <int B>
__device__ inline double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = B / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  return red[0];
}

// Per segment j (one thread each): the ends of its z extent, lo and hi
// (unwrapped: s_j and s_j + d at the nearest image), and its length.
__global__ __launch_bounds__(256) void k_line_segs(const double* __restrict__ pos,
                                                   const int32_t* __restrict__ nxt,
                                                   const int32_t* __restrict__ cnt, long long nc,
                                                   Geom g, double* __restrict__ seg) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt[0]) return;
  double d[3], a;
  segment(pos, nxt, nc, g, j, d, a);
  const double b = a + d[2];
  seg[j] = fmin(a, b);
  seg[nc + j] = fmax(a, b);
  seg[2 * nc + j] = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

// Total length: one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_line_total(const double* __restrict__ seg,
                                                     const int32_t* __restrict__ cnt, long long nc,
                                                     double* __restrict__ out) {
  __shared__ double red[1024];
  const int n = cnt[0];
  double acc = 0.0;
#pragma unroll 8
  for (int j = threadIdx.x; j < n; j += 1024) acc += seg[2 * nc + j];
  const double tot = block_sum<1024>(acc, red);
  if (threadIdx.x == 0) out[0] = tot;
}

// Length inside slab z = [z - 1/2, z + 1/2) along z (periodic z wraps): the
// block (z, c) walks chunk c of the segments (chunks of the segment range,
// kSlabChunks of them) and adds the part of each length in proportion to
// the overlap of its z extent with the slab (its three periodic images on a
// periodic z axis); a segment with no z extent belongs to the slab of its
// start point.  out[c * nz + z] receives the chunk's part; the caller adds
// the chunks in order.
__global__ __launch_bounds__(256) void k_line_slabs(const double* __restrict__ seg,
                                                    const int32_t* __restrict__ cnt, long long nc,
                                                    Geom g, double* __restrict__ out) {
  __shared__ double red[256];
  const int z = blockIdx.x;
  const int n = cnt[0];
  const int nz = g.nz;
  const bool periodic = !g.wall[2];
  const int per = (n + kSlabChunks - 1) / kSlabChunks;
  const int j0 = blockIdx.y * per, j1 = min(n, j0 + per);
  double acc = 0.0;
  for (int j = j0 + threadIdx.x; j < j1; j += 256) {
    const double lo = seg[j], hi = seg[nc + j], ell = seg[2 * nc + j];
    if (hi == lo) {
      int k = (int)floor(lo + 0.5);
      k = periodic ? ((k % nz) + nz) % nz : min(max(k, 0), nz - 1);
      if (k == z) acc += ell;
    } else {
      for (int img = periodic ? -1 : 0; img <= (periodic ? 1 : 0); ++img) {
        const double s_lo = (double)z - 0.5 + (double)img * nz;
        const double s_hi = s_lo + 1.0;
        const double ov = fmin(hi, s_hi) - fmax(lo, s_lo);
        if (ov > 0.0) acc += ell * ov / (hi - lo);  // (no overlap adds nothing)
      }
    }
  }
  const double tot = block_sum<256>(acc, red);
  if (threadIdx.x == 0) out[(long long)blockIdx.y * nz + z] = tot;
}

// Component comp of u at node (x, y, z) + s e_axis: periodic axes wrap,
// beyond a wall the velocity is 0.
__device__ inline double u_at(const double* __restrict__ u, const Geom& g, int comp, int x, int y,
                              int z, int axis, int s) {
  int p[3] = {x, y, z};
  const int n[3] = {g.nx, g.ny, g.nz};
  int v = p[axis] + s;
  if (v < 0 || v >= n[axis]) {
    if (g.wall[axis]) return 0.0;
    v = v < 0 ? v + n[axis] : v - n[axis];
  }
  p[axis] = v;
  return u[comp * g.cells + ((long long)p[2] * g.ny + p[1]) * g.nx + p[0]];
}

__device__ inline double ddx(const double* __restrict__ u, const Geom& g, int comp, int x, int y,
                             int z, int axis) {
  return 0.5 * (u_at(u, g, comp, x, y, z, axis, 1) - u_at(u, g, comp, x, y, z, axis, -1));
}

// omega = curl u by central differences, one thread per node.
__global__ __launch_bounds__(256) void k_curl(const double* __restrict__ u, Geom g,
                                              double* __restrict__ w) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.cells) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  const double wx = ddx(u, g, 2, x, y, z, 1) - ddx(u, g, 1, x, y, z, 2);
  const double wy = ddx(u, g, 0, x, y, z, 2) - ddx(u, g, 2, x, y, z, 0);
  const double wz = ddx(u, g, 1, x, y, z, 0) - ddx(u, g, 0, x, y, z, 1);
  w[c] = wx;
  w[g.cells + c] = wy;
  w[2 * g.cells + c] = wz;
}

// Cylindrical components (w.rho_hat, w.phi_hat, w.a) of a vector field
// about the axis through p along the unit vector a, one thread per node; the
// node's offset from p at the nearest periodic image; on the axis the
// radial and azimuthal components are 0.
struct Axis {
  double p[3], a[3];
};
__global__ __launch_bounds__(256) void k_cyl(const double* __restrict__ w, Geom g, Axis ax,
                                             double* __restrict__ out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.cells) return;
  const int node[3] = {(int)(c % g.nx), (int)((c / g.nx) % g.ny),
                       (int)(c / ((long long)g.nx * g.ny))};
  const int n[3] = {g.nx, g.ny, g.nz};
  double r[3];
  for (int k = 0; k < 3; ++k) {
    double x = (double)node[k] - ax.p[k];
    if (!g.wall[k]) {
      const double L = (double)n[k];
      if (x > 0.5 * L)
        x -= L;
      else if (x < -0.5 * L)
        x += L;
    }
    r[k] = x;
  }
  const double ra = r[0] * ax.a[0] + r[1] * ax.a[1] + r[2] * ax.a[2];
  double rp[3];
  for (int k = 0; k < 3; ++k) rp[k] = r[k] - ra * ax.a[k];
  const double nn = sqrt(rp[0] * rp[0] + rp[1] * rp[1] + rp[2] * rp[2]);
  double rh[3] = {0.0, 0.0, 0.0};
  if (nn > 0.0)
    for (int k = 0; k < 3; ++k) rh[k] = rp[k] / nn;
  const double ph[3] = {ax.a[1] * rh[2] - ax.a[2] * rh[1], ax.a[2] * rh[0] - ax.a[0] * rh[2],
                        ax.a[0] * rh[1] - ax.a[1] * rh[0]};
  const double wv[3] = {w[c], w[g.cells + c], w[2 * g.cells + c]};
  out[c] = wv[0] * rh[0] + wv[1] * rh[1] + wv[2] * rh[2];
  out[g.cells + c] = wv[0] * ph[0] + wv[1] * ph[1] + wv[2] * ph[2];
  out[2 * g.cells + c] = wv[0] * ax.a[0] + wv[1] * ax.a[1] + wv[2] * ax.a[2];
}

}  // namespace

hipError_t diag_cylindrical(Run& r, const double point[3], const double unit_dir[3],
                            const double* w, double* out) {
  Axis ax;
  for (int k = 0; k < 3; ++k) {
    ax.p[k] = point[k];
    ax.a[k] = unit_dir[k];
  }
  const int nb = (int)((r.cells + 255) / 256);
  hipLaunchKernelGGL(k_cyl, dim3(nb), dim3(256), 0, r.stream, w, r.geom, ax, out);
  return hipGetLastError();
}

hipError_t diag_line_length(Run& r, double* total, double* slabs) {
  const int nb = (int)((r.ncap + 255) / 256);
  hipLaunchKernelGGL(k_line_segs, dim3(nb), dim3(256), 0, r.stream, r.pos, r.nxt, r.cnt, r.ncap,
                     r.geom, r.seg);
  if (total)
    hipLaunchKernelGGL(k_line_total, dim3(1), dim3(1024), 0, r.stream, r.seg, r.cnt, r.ncap, total);
  if (slabs)
    hipLaunchKernelGGL(k_line_slabs, dim3(r.geom.nz, kSlabChunks), dim3(256), 0, r.stream, r.seg,
                       r.cnt, r.ncap, r.geom, slabs);
  return hipGetLastError();
}

hipError_t diag_curl(Run& r, const double* u, double* w) {
  const int nb = (int)((r.cells + 255) / 256);
  hipLaunchKernelGGL(k_curl, dim3(nb), dim3(256), 0, r.stream, u, r.geom, w);
  return hipGetLastError();
}

}  // namespace vlb
