// gsm_match without device allocation: the same single-query path as
// gsm_match, with every buffer of the call laid out in one file-scope device
// array instead of the graph's growable workspace.
//
// The array is a device symbol: in host code its name is a host-side stand-in,
// not a device address.  Its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gsm_internal.h"

namespace {

constexpr size_t kScratchBytes = GSM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The scratch of every device the library runs on (each holds its own copy
// until the process ends).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
  std::mutex mu;          // serialises calls on this device
  void *ptr = nullptr;    // device address of scratch on this device
  bool looked_up = false;
};

DeviceScratch g_dev[kMaxDevices];

// Device address of the scratch on the current device (looked up on the
// first call there); the caller holds that device's mutex.
void *scratch_address(DeviceScratch &d) {
  if (!d.looked_up) {
    void *p = nullptr;
    GSM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw gsm::Error{GSM_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch"};
    d.ptr = p;
    d.looked_up = true;
  }
  return d.ptr;
}

}  // namespace

extern "C" gsm_status gsm_match_noalloc(gsm_graph_t g, gsm_query_t qh, const gsm_match_opts *opts,
                                        uint64_t *count, int32_t *rows, uint64_t rows_cap,
                                        uint64_t *rows_written) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    gsm::set_error("gsm_match_noalloc: no usable current device");
    return GSM_E_DEVICE;
  }
  DeviceScratch &d = g_dev[dev];
  std::lock_guard<std::mutex> lk(d.mu);
  try {
    void *base = scratch_address(d);
    gsm::Workspace ws(base, kScratchBytes);
    return gsm::match_call(g, qh, opts, count, rows, rows_cap, rows_written, &ws);
  } catch (const gsm::Error &e) {
    gsm::set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc &) {
    gsm::set_error("host allocation failed");
    return GSM_E_OOM;
  }
}
