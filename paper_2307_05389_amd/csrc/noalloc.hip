// noalloc.hip -- ts_minmaxlttb_noalloc: MinMaxLTTB with the library's own
// device scratch instead of a caller workspace, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// The scratch is one file-scope device array per GPU (kScratchBytes, held
// until the process ends).  In host code the array's name is only a
// host-side stand-in, so its device address is looked up once per device
// with hipGetSymbolAddress (with that device current) and only that address
// is ever handed to kernels.  The call itself allocates nothing: it checks
// the size, looks up the address and runs the same launches as
// ts_minmaxlttb over the scratch.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace tsds {

// 64 MiB: MinMaxLTTB's workspace is about 4 bytes per KB of y (per-chunk
// partials) plus about 260 bytes per output point (bins, candidates, the LTTB
// map), so n_out of a few thousand fits series up to ~16 GB of y, and n_out
// up to ~200,000 fits series of a few GB.
constexpr size_t kScratchBytes = (size_t)64 << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`; looked up on the first call
// for that device, with the device made current for the lookup.
int scratch_on(int dev, void **ptr) {
  if (dev < 0 || dev >= kMaxDevices) return api_fail(TS_ERR_ARG, "device ordinal out of range for the static scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return api_fail(TS_ERR_HIP, "hipGetDevice failed");
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return api_fail(TS_ERR_HIP, "hipSetDevice failed");
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return api_fail(TS_ERR_HIP, "hipGetSymbolAddress of the static scratch failed");
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return TS_OK;
}
}  // namespace

}  // namespace tsds

using namespace tsds;

extern "C" {

size_t ts_noalloc_scratch_bytes(void) { return kScratchBytes; }

int ts_minmaxlttb_noalloc(const ts_series *s, int64_t n_out, int64_t minmax_ratio, int64_t *out_idx,
                          int64_t *out_count, void *stream) {
  // Size first, on the host only: nothing touches the GPU for a call the
  // scratch cannot hold.  need == 0 means invalid arguments or n <= n_out (no
  // workspace used); with missing outputs too, ts_minmaxlttb's own checks
  // report the error before any HIP call.  Its remaining checks (size
  // products) cannot fail for a series whose workspace fits the scratch.
  const size_t need = ts_workspace_bytes(TS_MINMAXLTTB, s, n_out, minmax_ratio);
  if (need > kScratchBytes)
    return api_fail(TS_ERR_WORKSPACE, "series needs more workspace than the 64 MiB static scratch "
                                      "(use ts_minmaxlttb with a caller workspace)");
  if (need == 0 || !out_idx || !out_count)
    return ts_minmaxlttb(s, n_out, minmax_ratio, out_idx, out_count, nullptr, 0, stream);
  int dev = -1;
  hipError_t e = stream ? hipStreamGetDevice((hipStream_t)stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return api_fail(TS_ERR_HIP, "cannot tell the stream's device");
  void *ws = nullptr;
  int rc = scratch_on(dev, &ws);
  if (rc) return rc;
  return ts_minmaxlttb(s, n_out, minmax_ratio, out_idx, out_count, ws, kScratchBytes, stream);
}

}  // extern "C"
