// Allocation-free single-call decode: ldpc_decode with its scratch memory taken from a fixed
// device array instead of the library's stream-ordered pool, for callers that cannot allocate.
//
// The array below is the library's only scratch of this kind.  Its name is a host-side stand-in
// in host code: the address each GPU's copy has is obtained once per device with
// hipGetSymbolAddress (with that device current) and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/ldpcci.h"
#include "kernels.hpp"

static __device__ __align__(256) unsigned char scratch[LDPC_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of that device's copy of scratch

// Address of the current device's scratch array, looked up on the first call on that device.
int current_scratch(void** out) {
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return ldpc::record_hip_failure(he);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return LDPC_OK;
  }
  void* ptr = nullptr;
  he = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (he != hipSuccess || ptr == nullptr) return ldpc::record_hip_failure(he != hipSuccess ? he : hipErrorInvalidSymbol);
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return LDPC_OK;
}

}  // namespace

extern "C" int ldpc_decode_noalloc(const ldpc_code* c, const ldpc_schedule* s, const float* llr_in, int32_t B,
                                   int64_t max_updates, const int32_t* replay, int64_t replay_len,
                                   const ldpc_outputs* out, void* stream) {
  if (!c || !s || !out || B < 0 || max_updates < 0) return LDPC_EINVAL;
  if (B == 0) return LDPC_OK;
  void* p = nullptr;
  if (int rc = current_scratch(&p)) return rc;
  return ldpc::decode_in_scratch(c, s, llr_in, B, max_updates, replay, replay_len, out, p,
                                 (size_t)LDPC_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
}
