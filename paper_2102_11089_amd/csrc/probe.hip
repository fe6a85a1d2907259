// LDS read-bandwidth probe: the denominator of an LDS roofline, measured instead of taken from the
// nominal per-CU figure.  Every lane reads aligned elements of 4, 8 or 16 bytes from a 16 KiB LDS
// buffer, consecutive lanes at consecutive addresses (no bank conflicts), and folds them into one
// word with one exclusive-or per 32-bit word read.
#include <hip/hip_runtime.h>

#include "../../include/ldpcci.h"
#include "kernels.hpp"

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeWords = 4096;  // 16 KiB of LDS per workgroup
constexpr int kProbeUnroll = 16;   // reads per lane per iteration, each at a distinct address

template <int W>
struct Elem;
template <>
struct Elem<1> {
  using type = uint32_t;
  __device__ static uint32_t fold(type v) { return v; }
};
template <>
struct Elem<2> {
  using type = uint2;
  __device__ static uint32_t fold(type v) { return v.x ^ v.y; }
};
template <>
struct Elem<4> {
  using type = uint4;
  __device__ static uint32_t fold(type v) { return v.x ^ v.y ^ v.z ^ v.w; }
};

// W 32-bit words per element.  Lane t reads element (t + k + u n / 16) mod n for u < 16 in
// iteration k, so the 16 reads of one iteration are distinct and every address changes between
// iterations; one xor per word read keeps them live.
template <int W>
__global__ __launch_bounds__(kProbeThreads) void k_lds_probe(long long iters, uint32_t* sink) {
  using T = typename Elem<W>::type;
  __shared__ uint4 raw[kProbeWords / 4];
  uint32_t* words = reinterpret_cast<uint32_t*>(raw);
  for (int i = threadIdx.x; i < kProbeWords; i += kProbeThreads) words[i] = (uint32_t)i * 2654435761u;
  __syncthreads();
  const T* b = reinterpret_cast<const T*>(raw);
  constexpr int n = kProbeWords / W;  // elements in the buffer (a power of two)
  constexpr int stride = n / kProbeUnroll;
  uint32_t acc[W] = {};
  int idx = threadIdx.x;
  for (long long it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      const T v = b[(idx + u * stride) & (n - 1)];
      if constexpr (W == 1) {
        acc[0] ^= v;
      } else if constexpr (W == 2) {
        acc[0] ^= v.x;
        acc[1] ^= v.y;
      } else {
        acc[0] ^= v.x;
        acc[1] ^= v.y;
        acc[2] ^= v.z;
        acc[3] ^= v.w;
      }
    }
    idx += 1;
  }
  uint32_t r = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) r ^= acc[w];
  if (threadIdx.x == 0) sink[blockIdx.x] = r;
}

}  // namespace

extern "C" int ldpc_probe_lds(int32_t width, int32_t blocks, int64_t iters, uint32_t* sink, void* stream,
                              double* bytes, float* ms) {
  if ((width != 4 && width != 8 && width != 16) || blocks < 1 || iters < 1 || iters > (1ll << 24) || !sink ||
      !bytes || !ms)
    return LDPC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he == hipSuccess) he = hipEventRecord(e0, st);
  if (he == hipSuccess) {
    if (width == 4) hipLaunchKernelGGL(k_lds_probe<1>, dim3(blocks), dim3(kProbeThreads), 0, st, iters, sink);
    else if (width == 8) hipLaunchKernelGGL(k_lds_probe<2>, dim3(blocks), dim3(kProbeThreads), 0, st, iters, sink);
    else hipLaunchKernelGGL(k_lds_probe<4>, dim3(blocks), dim3(kProbeThreads), 0, st, iters, sink);
    he = hipGetLastError();
  }
  if (he == hipSuccess) he = hipEventRecord(e1, st);
  if (he == hipSuccess) he = hipEventSynchronize(e1);
  float t = 0.f;
  if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (he != hipSuccess) return ldpc::record_hip_failure(he);
  *bytes = (double)blocks * kProbeThreads * (double)iters * kProbeUnroll * width;
  *ms = t;
  return LDPC_OK;
}
