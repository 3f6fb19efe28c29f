// rsd_apply_noalloc: the preconditioner application on a static device area, for
// callers that cannot allocate device memory (code being captured into a HIP graph,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The work memory of an application (permuted input and output, back-substitution
// right-hand side, leaf-boundary products, interleaved SpMV operand, symmetric-product
// partials, inner GMRES scratch) lives in one file-scope device array per GPU instead of
// the handle's grown-on-demand buffers.  Its device address is looked up once per device
// (at set-up, with the device current) and used wherever host code passes the area; the
// array's name itself is only a host-side stand-in.  Every kernel of the application
// writes the part of the area it later reads, so no call needs it cleared.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "engine.hpp"

namespace {

constexpr size_t kNoAllocBytes = size_t(256) << 20;   // 256 MiB per GPU, held until exit
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct DeviceArea {
  void* ptr = nullptr;              // device address of `scratch` on this GPU
  hipEvent_t last = nullptr;        // recorded at the end of every call on this GPU
  hipStream_t last_s = nullptr;
  bool has_last = false;
};

std::mutex g_mu;
std::map<int, DeviceArea> g_area;

// with `device` current: the device address of the array and the ordering event
hipError_t register_device(int device) {
  auto it = g_area.find(device);
  if (it != g_area.end() && it->second.ptr) return hipSuccess;
  DeviceArea& a = g_area[device];
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  e = hipEventCreateWithFlags(&a.last, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  a.ptr = p;
  return hipSuccess;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st == hipStreamCaptureStatusActive;
}

}  // namespace

namespace rsd {
// called by rsd_setup with the handle's device current; a failure is reported by the
// first rsd_apply_noalloc on that device (set-up does not depend on it)
void noalloc_register(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (register_device(device) != hipSuccess) (void)hipGetLastError();
}
}  // namespace rsd

extern "C" rsd_status rsd_apply_noalloc(rsd_handle h, int32_t nrhs, const double* r,
                                        int64_t ldr, double* z, int64_t ldz, void* stream) {
  if (!h) return RSD_ERR_INVALID_ARGUMENT;
  if (nrhs < 0) {
    h->err = "nrhs must be non-negative";
    return RSD_ERR_INVALID_ARGUMENT;
  }
  if (nrhs == 0) return RSD_OK;
  if (!r || !z || ldr < h->P.n || ldz < h->P.n) {
    h->err = "vector pointers must not be NULL and leading dimensions must be >= n";
    return RSD_ERR_INVALID_ARGUMENT;
  }
  if (static_cast<const void*>(r) == static_cast<const void*>(z)) {
    h->err = "input and output must not overlap";
    return RSD_ERR_INVALID_ARGUMENT;
  }
  try {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device) {
      h->err = "rsd_apply_noalloc: the handle's device must be the current device";
      return RSD_ERR_INVALID_ARGUMENT;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lock(g_mu);   // one caller at a time enqueues on the area
    const hipError_t e = register_device(dev);
    if (e != hipSuccess) {
      h->err = std::string("hipGetSymbolAddress of the static work area: ") + hipGetErrorString(e);
      return RSD_ERR_DEVICE;
    }
    DeviceArea& a = g_area.find(dev)->second;   // registered above
    const bool cap = stream_capturing(s);
    // the previous call on this GPU may still use the area on another stream
    if (!cap && a.has_last && a.last_s != s && hipStreamWaitEvent(s, a.last, 0) != hipSuccess) {
      h->err = "hipStreamWaitEvent failed";
      return RSD_ERR_DEVICE;
    }
    const rsd_status st = rsd::engine_apply_static(h, nrhs, r, ldr, z, ldz, a.ptr, kNoAllocBytes, s);
    if (st == RSD_OK && !cap) {
      if (hipEventRecord(a.last, s) != hipSuccess) {
        h->err = "hipEventRecord failed";
        return RSD_ERR_DEVICE;
      }
      a.last_s = s;
      a.has_last = true;
    }
    return st;
  } catch (...) {
    h->err = "unexpected exception in rsd_apply_noalloc";
    return RSD_ERR_DEVICE;
  }
}
