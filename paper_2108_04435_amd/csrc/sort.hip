// Stable LSD radix sort of (uint32 key, int32 value) pairs, used to bin
// filament points by lattice cell for the force spreading.  Digits of up to
// 11 bits (2 passes for keys of up to 22 bits), one tile of 1024 keys per
// block of 1024 threads, one key per thread.  Inside a wave the lanes
// holding the same digit are found with one ballot per digit bit; their
// count and each lane's rank among them come from population counts.  Per
// pass three kernels:
//   1. per-tile digit counts (LDS histogram; the first pass can be fused
//      into the kernel that produces the keys);
//   2. digit offsets of every tile (keys of smaller digits anywhere plus
//      keys of the same digit in earlier tiles): a one-workgroup exclusive
//      scan of the digit-major count table;
//   3. stable scatter: the waves of a tile take turns in order; each key
//      goes to the running offset of its digit + its rank inside the wave,
//      and the lowest lane of each digit group advances that offset.
// Keys beyond the live points are padded by the caller with the largest
// key, so they sort to the end.  Nothing is allocated, no global atomics
// and no memset are issued, so the sort can be captured in a HIP graph.
#include "vlb_internal.h"

namespace vlb {

namespace {

__global__ __launch_bounds__(kSortThreads) void k_rs_count(const uint32_t* __restrict__ keys,
                                                           int n, int shift, int bits, int ntiles,
                                                           int32_t* __restrict__ counts) {
  __shared__ int32_t hist[kSortMaxBins];
  const int idx = blockIdx.x * kSortThreads + threadIdx.x;
  const bool valid = idx < n;
  const uint32_t k = valid ? keys[idx] : 0u;
  sort_tile_count(k, valid, shift, bits, ntiles, blockIdx.x, hist, counts);
}

// Digit offsets of every tile, once per pass (one workgroup): offs[d][b] =
// exclusive prefix of the digit-major count table read as one array.  Each
// thread takes kScanPer consecutive entries per round (vector loads where
// the round is full), so a table of up to 32768 entries is one round.
constexpr int kScanPer = 32;

__global__ __launch_bounds__(1024) void k_rs_offsets(const int32_t* __restrict__ counts, int M,
                                                     int32_t* __restrict__ offs) {
  __shared__ int32_t wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int carry = 0;
  for (int base = 0; base < M; base += kScanPer * 1024) {
    const int k0 = base + kScanPer * t;
    const bool full = k0 + kScanPer <= M;
    int v[kScanPer];
    if (full) {
      const int4* p = reinterpret_cast<const int4*>(counts + k0);
#pragma unroll
      for (int q = 0; q < kScanPer / 4; ++q) {
        const int4 x = p[q];
        v[4 * q] = x.x;
        v[4 * q + 1] = x.y;
        v[4 * q + 2] = x.z;
        v[4 * q + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < kScanPer; ++q) v[q] = (k0 + q < M) ? counts[k0 + q] : 0;
    }
    int mine = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) mine += v[q];
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
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      const int c = v[q];
      v[q] = run;
      run += c;
    }
    if (full) {
      int4* p = reinterpret_cast<int4*>(offs + k0);
#pragma unroll
      for (int q = 0; q < kScanPer / 4; ++q) p[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
      for (int q = 0; q < kScanPer; ++q)
        if (k0 + q < M) offs[k0 + q] = v[q];
    }
    carry += all;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                             const int32_t* __restrict__ vin,
                                                             uint32_t* __restrict__ kout,
                                                             int32_t* __restrict__ vout, int n,
                                                             int shift, int bits, int ntiles,
                                                             const int32_t* __restrict__ offs) {
  __shared__ int32_t run[kSortMaxBins];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int nbins = 1 << bits;
  for (int d = t; d < nbins; d += kSortThreads) run[d] = offs[(long long)d * ntiles + blockIdx.x];
  const int idx = blockIdx.x * kSortThreads + t;
  const bool valid = idx < n;
  const uint32_t k = valid ? kin[idx] : 0u;
  const int32_t v = valid ? vin[idx] : 0;
  const uint32_t d = (k >> shift) & (uint32_t)(nbins - 1);
  const uint64_t m = sort_peer_mask(d, valid, bits);
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  const int rank = __popcll(m & lt);
  const bool leader = valid && rank == 0;
  for (int turn = 0; turn < kSortThreads / 64; ++turn) {
    __syncthreads();
    if (turn == w && valid) {
      const int b = run[d];
      kout[b + rank] = k;
      vout[b + rank] = v;
      if (leader) run[d] = b + __popcll(m);
    }
  }
}

}  // namespace

size_t sort_tmp_bytes(long long n) {
  const long long ntiles = (n + kSortThreads - 1) / kSortThreads;
  return (size_t)(2 * (((long long)kSortMaxBins * ntiles + 63) & ~63LL) + 16) * sizeof(int32_t);
}

int sort_tiles(long long n) { return (int)((n + kSortThreads - 1) / kSortThreads); }

void sort_first_digit(int bits, int* dbits) {
  const int passes = (bits + kSortMaxBits - 1) / kSortMaxBits;
  const int db = (bits + passes - 1) / passes;
  *dbits = db < bits ? db : bits;
}

int32_t* sort_counts(Run& r) { return (int32_t*)r.sort_tmp; }

// Sort n pairs (ka, va) by the low `bits` bits of the key, with tmp of
// sort_tmp_bytes(n) bytes and the second buffers kb, vb.  first_counted: the
// tile counts of the first pass are already in the count table at tmp.
// Result pointers are returned (they alternate between the a and b buffers
// with the number of passes).
hipError_t sort_pairs_raw(long long nn, int bits, int first_counted, void* tmp, uint32_t* ka,
                          uint32_t* kb, int32_t* va, int32_t* vb, hipStream_t stream,
                          uint32_t** kres, int32_t** vres) {
  const int n = (int)nn;
  const int ntiles = sort_tiles(n);
  int32_t* counts = (int32_t*)tmp;
  int32_t* offs = counts + (((long long)kSortMaxBins * ntiles + 63) & ~63LL);
  uint32_t* kin = ka;
  uint32_t* kout = kb;
  int32_t* vin = va;
  int32_t* vout = vb;
  const int passes = (bits + kSortMaxBits - 1) / kSortMaxBits;
  const int dbits = (bits + passes - 1) / passes;
  for (int p = 0; p < passes; ++p) {
    const int shift = dbits * p;
    const int pb = (shift + dbits <= bits) ? dbits : bits - shift;
    if (p > 0 || !first_counted)
      hipLaunchKernelGGL(k_rs_count, dim3(ntiles), dim3(kSortThreads), 0, stream, kin, n, shift,
                         pb, ntiles, counts);
    hipLaunchKernelGGL(k_rs_offsets, dim3(1), dim3(1024), 0, stream, counts, ntiles << pb, offs);
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kSortThreads), 0, stream, kin, vin,
                       kout, vout, n, shift, pb, ntiles, offs);
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

// The run's ncap pairs (keys_a, vals_a).
hipError_t sort_pairs(Run& r, int bits, int first_counted, uint32_t** kres, int32_t** vres) {
  return sort_pairs_raw(r.ncap, bits, first_counted, r.sort_tmp, r.keys_a, r.keys_b, r.vals_a,
                        r.vals_b, r.stream, kres, vres);
}

}  // namespace vlb
