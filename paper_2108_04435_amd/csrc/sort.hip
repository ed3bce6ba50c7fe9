// Stable LSD radix sort of (uint32 key, int32 value) pairs, 8-bit digits,
// used to bin filament points by lattice cell (force spreading) and by
// reconnection cell.  No atomics: inside a wave, the lanes that hold the
// same digit are found with 8 ballots (one per digit bit); their count and
// each lane's rank among them come from population counts.  Per pass:
//   1. per-tile digit counts (tiles of 1024 keys, 4 rounds of 256 threads),
//   2. exclusive scan of the counts in digit-major, tile-minor order,
//   3. stable scatter: tile offset + running count of the digit in the
//      tile + earlier waves of the round + rank inside the wave.
// Keys beyond the live points are padded by the caller with the largest
// key, so they sort to the end.  Nothing is allocated and no memset is
// issued, so the sort can be captured in a HIP graph.
#include "vlb_internal.h"

namespace vlb {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 4;
constexpr int kTileKeys = kThreads * kRounds;

// Lanes of this wave whose (valid) digit equals this lane's digit.
__device__ inline uint64_t peer_mask(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t x = __ballot(valid && bit);
    m &= bit ? x : ~x;
  }
  return m;
}

__global__ __launch_bounds__(kThreads) void k_rs_count(const uint32_t* __restrict__ keys, int n,
                                                       int shift, int ntiles,
                                                       int32_t* __restrict__ counts) {
  __shared__ int32_t cw[4][256];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int q = t; q < 4 * 256; q += kThreads) (&cw[0][0])[q] = 0;
  __syncthreads();
  const int base = blockIdx.x * kTileKeys;
  for (int q = 0; q < kRounds; ++q) {
    const int idx = base + q * kThreads + t;
    const bool valid = idx < n;
    const uint32_t d = valid ? (keys[idx] >> shift) & 255u : 0u;
    const uint64_t m = peer_mask(d, valid);
    if (valid && (int)(__ffsll((unsigned long long)m) - 1) == lane) cw[w][d] += __popcll(m);
  }
  __syncthreads();
  counts[t * ntiles + blockIdx.x] = cw[0][t] + cw[1][t] + cw[2][t] + cw[3][t];
}

__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                         const int32_t* __restrict__ vin,
                                                         uint32_t* __restrict__ kout,
                                                         int32_t* __restrict__ vout, int n,
                                                         int shift, int ntiles,
                                                         const int32_t* __restrict__ offs) {
  __shared__ int32_t run[256];
  __shared__ int32_t cw[4][256];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  run[t] = offs[t * ntiles + blockIdx.x];
  const int base = blockIdx.x * kTileKeys;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int q = 0; q < kRounds; ++q) {
    for (int e = lane; e < 256; e += 64) cw[w][e] = 0;
    const int idx = base + q * kThreads + t;
    const bool valid = idx < n;
    const uint32_t k = valid ? kin[idx] : 0u;
    const int32_t v = valid ? vin[idx] : 0;
    const uint32_t d = (k >> shift) & 255u;
    const uint64_t m = peer_mask(d, valid);
    const int rank = __popcll(m & lt);
    __syncthreads();
    if (valid && (int)(__ffsll((unsigned long long)m) - 1) == lane) cw[w][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      int dst = run[d] + rank;
      for (int u = 0; u < w; ++u) dst += cw[u][d];
      kout[dst] = k;
      vout[dst] = v;
    }
    __syncthreads();
    run[t] += cw[0][t] + cw[1][t] + cw[2][t] + cw[3][t];
    __syncthreads();
  }
}

}  // namespace

hipError_t scan_excl(Run& r, const int32_t* in, int32_t* out, const int32_t* np, int n,
                     int32_t* total);

size_t sort_tmp_bytes(long long n) {
  const long long ntiles = (n + kTileKeys - 1) / kTileKeys;
  return (size_t)(2 * 256 * ntiles + 16) * sizeof(int32_t);
}

// Sort ncap pairs (keys_a, vals_a) by the low `bits` bits of the key.
// Result pointers are returned (they alternate between the a and b
// buffers with the number of passes).
hipError_t sort_pairs(Run& r, int bits, uint32_t** kres, int32_t** vres) {
  const int n = (int)r.ncap;
  const int ntiles = (n + kTileKeys - 1) / kTileKeys;
  int32_t* counts = (int32_t*)r.sort_tmp;
  int32_t* offs = counts + 256 * ntiles;
  int32_t* total = offs + 256 * ntiles;
  uint32_t* kin = r.keys_a;
  uint32_t* kout = r.keys_b;
  int32_t* vin = r.vals_a;
  int32_t* vout = r.vals_b;
  const int passes = (bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_rs_count, dim3(ntiles), dim3(kThreads), 0, r.stream, kin, n, shift, ntiles, counts);
    hipError_t e = scan_excl(r, counts, offs, nullptr, 256 * ntiles, total);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kThreads), 0, r.stream, kin, vin, kout, vout, n,
                       shift, ntiles, offs);
    uint32_t* tk = kin;
    kin = kout;
    kout = tk;
    int32_t* tv = vin;
    vin = vout;
    vout = tv;
  }
  *kres = kin;
  *vres = vin;
  return hipGetLastError();
}

}  // namespace vlb
