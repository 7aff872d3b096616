// Allocation-free matvec for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): the skeleton-vector arena and, for several right-hand sides,
// the two layout buffers live in one file-scope device array instead of the
// context's workspace.  Same launches and kernels as hbf_matvec.
#include <mutex>
#include <string>

#include "ctx.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

// Each device that runs this entry point holds its own copy until the
// process ends.  Host code must use the address hipGetSymbolAddress returns
// for the current device, never the array's name.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device's address of `scratch` (device current), looked up once per device.
hipError_t scratch_ptr(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

hbf_status fail(hbf_status st, const std::string& m) {
  hbf::set_error(m);
  return st;
}

}  // namespace

extern "C" hbf_status hbf_matvec_noalloc(hbf_ctx* c, const void* x, void* y, int32_t nrhs, hbf_dtype io,
                                         int32_t adjoint, void* stream) {
  if (!c || !x || !y) return fail(HBF_EINVAL, "hbf_matvec_noalloc: NULL argument");
  if (nrhs < 1 || nrhs > c->max_nrhs) return fail(HBF_EINVAL, "hbf_matvec_noalloc: nrhs out of range [1, max_nrhs]");
  if (io != HBF_C64 && io != HBF_C128) return fail(HBF_EINVAL, "hbf_matvec_noalloc: bad io dtype");
  if (c->dtype == HBF_C128 && io == HBF_C64)
    return fail(HBF_EINVAL, "hbf_matvec_noalloc: complex64 io on a complex128 context");
  const size_t R = static_cast<size_t>(nrhs);
  const size_t io_elt = io == HBF_C128 ? 16 : 8;
  const size_t arena = align256(static_cast<size_t>(std::max<int64_t>(c->P.arena_rows, 1)) * R * 16);
  const bool convert = nrhs > 1 || c->padded();
  const size_t vec = convert ? align256(static_cast<size_t>(c->n) * R * io_elt) : 0;
  if (arena + 2 * vec > kScratchBytes)
    return fail(HBF_EINVAL, "hbf_matvec_noalloc: needs " + std::to_string(arena + 2 * vec) +
                                " bytes of scratch, more than its fixed 64 MiB (use hbf_matvec)");
  if (hipSetDevice(c->device) != hipSuccess) return fail(HBF_EHIP, "hipSetDevice");
  void* base = nullptr;
  const hipError_t e = scratch_ptr(c->device, &base);
  if (e != hipSuccess) return fail(HBF_EHIP, std::string("hbf_matvec_noalloc: scratch address: ") + hipGetErrorString(e));
  char* p = static_cast<char*>(base);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool v128 = io == HBF_C128;
  if (!convert) return hbf::matvec_internal(c, const_cast<void*>(x), y, 1, v128, adjoint != 0, s, p);
  void* vin = p + arena;
  void* vout = p + arena + vec;
  if (hbf::launch_to_internal(x, v128, vin, v128, c->vmap, nrhs, s) != hipSuccess)
    return fail(HBF_EHIP, "hbf_matvec_noalloc: layout");
  const hbf_status st = hbf::matvec_internal(c, vin, vout, nrhs, v128, adjoint != 0, s, p);
  if (st != HBF_OK) return st;
  if (hbf::launch_to_external(vout, v128, y, v128, c->vmap, nrhs, s) != hipSuccess)
    return fail(HBF_EHIP, "hbf_matvec_noalloc: layout");
  return HBF_OK;
}
