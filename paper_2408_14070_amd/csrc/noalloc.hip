// rid_bias_force_noalloc: the bias path with its scratch in a fixed device
// array, for callers that cannot allocate device memory (code under graph
// capture, tight serving loops, harnesses that forbid allocation).
//
// The scratch (per-member free energies A [K][B], mean forces g [K][B][n]
// and, above the in-kernel gather's batch limit, the CV encoding x [B][2n])
// lives in `scratch`, a file-scope device array of kScratchFloats floats
// (32 MiB) that each GPU the library runs on holds until the process ends.
// Its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and kept; kernels receive that address, never the
// array's name.  Every kernel writes each scratch element it later reads
// (A and g for every walker row below B, x likewise), so nothing needs to
// start at zero.  All calls on one GPU share the array: calls that overlap
// on one GPU (different streams, or different host threads without ordering)
// race on it.
#include <mutex>

#include "rid_internal.h"

namespace rid {
namespace {

constexpr size_t kScratchFloats = (size_t)8 << 20;     // 32 MiB
constexpr int kMaxDevices = 64;

static __device__ __attribute__((aligned(256))) float scratch[kScratchFloats];

std::mutex g_mu;
float* g_ptr[kMaxDevices] = {};

// scratch's address on the current device (looked up on first use)
rid_status scratch_on_current_device(float** out) {
  int dev = -1;
  RID_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RID_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    }
    g_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_ptr[dev];
  return RID_OK;
}

// 256-byte aligned float offsets
inline size_t al64(size_t v) { return (v + 63) / 64 * 64; }

}  // namespace
}  // namespace rid

using namespace rid;

extern "C" {

size_t rid_noalloc_scratch_floats(void) { return kScratchFloats; }

rid_status rid_bias_force_noalloc(rid_system sys, rid_ensemble ens, const float* d_pos,
                                  int B, float eps0, float eps1, float* d_force,
                                  float* d_energy, float* d_eps, float* d_sigma,
                                  uint8_t* d_flags, rid_stream stream) {
  rid_status r = bias_force_check(sys, ens, d_pos, B, eps0, eps1, d_force);
  if (r != RID_OK) return r;
  rid_ensemble_impl& e = ens->impl;
  const size_t a_off = 0;
  const size_t g_off = al64(a_off + (size_t)e.K * B);
  const size_t x_off = al64(g_off + (size_t)e.K * B * e.n_cv);
  const size_t need = al64(x_off + (size_t)B * 2 * e.n_cv);
  if (need > kScratchFloats)
    return fail(RID_EINVAL, "batch too large for the no-allocation scratch: K*B*(n_cv+1) + "
                            "2*B*n_cv floats must fit 8388608 (32 MiB), with 256-byte padding");
  float* base = nullptr;
  if ((r = scratch_on_current_device(&base)) != RID_OK) return r;
  return bias_force_core(sys->impl, e, d_pos, B, eps0, eps1, base + a_off, base + g_off,
                         base + x_off, d_force, d_energy, d_eps, d_sigma, d_flags,
                         (hipStream_t)stream);
}

}  // extern "C"
