// hss_apply_noalloc: the compressed apply (Fig. 7 with m = L, plus D) for
// callers that cannot allocate device memory -- code under stream capture,
// serving loops, harnesses that forbid allocation.  Same kernels as
// hss_apply; their per-node expansions and row-chunk partials go to a
// fixed-size array in the library's own device memory instead of a per-call
// buffer.
#include <mutex>

#include "apply.h"
#include "handle.h"

using namespace hm;

namespace {

// Scratch of the apply kernels: each GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory; host code only uses the per-device address
// that hipGetSymbolAddress returns for it.
constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch, looked up on the first
// call on that device (with the device current) and kept.
void* device_scratch() {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    HM_THROW(HM_ERR_UNSUPPORTED, "apply_noalloc: device ordinal %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      HM_THROW(HM_ERR_HIP, "apply_noalloc: hipGetSymbolAddress(scratch) failed: %s",
               hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

template <class T>
void apply_static(const hm_hbs* h, int64_t nrhs, const T* x, int64_t ldx, T* y, int64_t ldy,
                  hipStream_t s) {
  void* work = device_scratch();
  // the workspace is linear in the column count: columns per pass such that
  // it fits the scratch array
  const size_t fixed = apply_work_bytes<T>(h->f, h->full, h->R, 0);
  const size_t per_col = apply_work_bytes<T>(h->f, h->full, h->R, 1) - fixed;
  if (fixed + per_col > kScratchBytes)
    HM_THROW(HM_ERR_UNSUPPORTED,
             "apply_noalloc: one column needs %zu bytes of scratch, the limit is %zu", fixed + per_col,
             kScratchBytes);
  const int64_t cpass = std::min<int64_t>(128, (int64_t)((kScratchBytes - fixed) / per_col));
  for (int64_t c0 = 0; c0 < nrhs; c0 += cpass) {
    const int c = (int)std::min<int64_t>(cpass, nrhs - c0);
    apply_forest<T>(h->d_nodes.as<Node>(), h->full, h->view<T>(), false, c, x + c0 * ldx, ldx,
                    y + c0 * ldy, ldy, T(1), T(0), work, h->f.nodes.size(), s);
  }
}

}  // namespace

extern "C" int hss_apply_noalloc(const hm_hbs* h, int64_t nrhs, const void* x, int64_t ldx,
                                 void* y, int64_t ldy, void* stream) {
  try {
    set_error("%s", "");
    if (!h || !x || !y || nrhs < 0) HM_THROW(HM_ERR_ARG, "apply_noalloc: bad arguments");
    const int64_t n = h->f.n_total;
    if (ldx < n || ldy < n) HM_THROW(HM_ERR_ARG, "apply_noalloc: ld < n");
    if (nrhs == 0) return HM_OK;
    hipStream_t s = (hipStream_t)stream;
    if (h->dtype == HM_F64)
      apply_static<double>(h, nrhs, static_cast<const double*>(x), ldx, static_cast<double*>(y),
                           ldy, s);
    else
      apply_static<float>(h, nrhs, static_cast<const float*>(x), ldx, static_cast<float*>(y), ldy,
                          s);
    return HM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    set_error("unexpected exception");
    return HM_ERR_HIP;
  }
}
