// Allocation-free variant of the stand-alone Biot-Savart sum
// (vlb_biot_savart_noalloc), for callers that cannot allocate device
// memory (code under graph capture, tight serving loops): the scratch of the
// sum lives in a file-scope device array of fixed size instead of a caller
// workspace.  Same kernels, chunking and summation order as vlb_biot_savart,
// so both give the same bits.
#include "vlb_internal.h"

#include <mutex>

using namespace vlb;

namespace {

// Largest call: kNoAllocMaxPoints points in FP64 (the larger layout) fits.
constexpr long long kNoAllocMaxPoints = 16384;
constexpr size_t kScratchBytes = 4608 * 1024;

// One copy per GPU, held until the process ends.  Host code never uses
// this name as an address: the device address of each GPU's copy comes
// from hipGetSymbolAddress (scratch_on).
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of the scratch array, looked up
// once per device with that device current.
int scratch_on(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_global(VLB_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail_global(VLB_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail_global(VLB_EDEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return VLB_OK;
}

}  // namespace

extern "C" int vlb_biot_savart_noalloc(const vlb_bs_desc* d, int64_t n_pts, const double* xyz_dev,
                                       const int32_t* next_dev, double* v_dev,
                                       void* hip_stream) {
  std::string msg;
  const int c = bs_check_desc(d, n_pts, msg);
  if (c != VLB_OK) return fail_global(c, msg);
  if (n_pts > kNoAllocMaxPoints)
    return fail_global(VLB_EINVAL, "n_pts above the allocation-free limit of 16384 points");
  if (n_pts == 0) return VLB_OK;
  if (!xyz_dev || !next_dev || !v_dev) return fail_global(VLB_EINVAL, "null device pointer");
  if (bs_solo_layout(d->precision, n_pts, nullptr, nullptr) > kScratchBytes)
    return fail_global(VLB_EINVAL, "scratch array too small for this call");
  void* base = nullptr;
  const int s = scratch_on(&base);
  if (s != VLB_OK) return s;
  BsSolo b;
  bs_solo_layout(d->precision, n_pts, (char*)base, &b);
  const int n[3] = {d->nx, d->ny, d->nz};
  const int wall[3] = {(int)(d->wall_axes & 1u), (int)((d->wall_axes >> 1) & 1u),
                       (int)((d->wall_axes >> 2) & 1u)};
  const hipError_t e = bs_solo(bs_make_axes(n, wall, false), d->precision, n_pts, xyz_dev, next_dev,
                               d->kappa, v_dev, b, (hipStream_t)hip_stream);
  if (e != hipSuccess)
    return fail_global(VLB_EDEVICE, std::string("vlb_biot_savart_noalloc: ") + hipGetErrorString(e));
  return VLB_OK;
}
