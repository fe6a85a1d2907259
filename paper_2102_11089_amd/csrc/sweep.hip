// On-device channel frames and error counting for SNR sweeps (captured into one hipGraph by the
// host: per Eb/N0 point, generate -> decode -> count).
//
// Frames: frame f of point p carries codeword f mod P of a caller-supplied pool; bit n gets
// BPSK x = 1 - 2c plus Gaussian noise from one Box-Muller pair of Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) with counter (n, f, p, 0) and
// key (seed low word, seed high word):  u1 = (x0 + 1) 2^-32 in (0, 1],  u2 = x1 2^-32,
// z = sqrt(-2 ln u1) cos(2 pi u2),  llr = (2 / sigma^2)(x + sigma z)  (channel LLRs of Sec. II-A).
// Counting: per point, frames, frame errors (any decoded bit differs), bit errors and the sum of
// updates_used, accumulated with integer atomics (order-independent).
#include "common.hpp"
#include "kernels.hpp"

namespace ldpc {

namespace {

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                             uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
  const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
  const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
  c0 = n0;
  c1 = lo1;
  c2 = n2;
  c3 = lo0;
}

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1) {
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c0, c1, c2, c3, k0, k1);
    k0 += W0;
    k1 += W1;
  }
}

}  // namespace

__global__ void k_awgn_frames(const uint8_t* cw, int P, int N, int B, float sigma, float scale, const uint64_t* seed_dev,
                              uint64_t seed_val, int point, float* llr) {
  const uint64_t seed = seed_dev ? *seed_dev : seed_val;
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFull), k1 = (uint32_t)(seed >> 32);
  const long long total = (long long)B * N;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int f = (int)(i / N), n = (int)(i - (long long)f * N);
    uint32_t c0 = (uint32_t)n, c1 = (uint32_t)f, c2 = (uint32_t)point, c3 = 0u;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    const float u1 = ((float)c0 + 1.0f) * 2.3283064365386963e-10f;  // 2^-32
    const float u2 = (float)c1 * 2.3283064365386963e-10f;
    const float z = sqrtf(-2.0f * logf(u1)) * cosf(6.283185307179586f * u2);
    const float x = cw[(size_t)(f % P) * N + n] ? -1.0f : 1.0f;
    llr[i] = scale * (x + sigma * z);
  }
}

// one workgroup per frame
__global__ void k_count_errors(const uint8_t* bits, const uint8_t* cw, int P, int N, int B, const int64_t* upd,
                               unsigned long long* counters) {
  __shared__ int nerr;
  const int f = blockIdx.x;
  if (f >= B) return;
  if (threadIdx.x == 0) nerr = 0;
  __syncthreads();
  int local = 0;
  const uint8_t* b = bits + (size_t)f * N;
  const uint8_t* c = cw + (size_t)(f % P) * N;
  for (int n = threadIdx.x; n < N; n += blockDim.x) local += (b[n] != c[n]) ? 1 : 0;
  if (local) atomicAdd(&nerr, local);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&counters[0], 1ull);
    if (nerr) {
      atomicAdd(&counters[1], 1ull);
      atomicAdd(&counters[2], (unsigned long long)nerr);
    }
    atomicAdd(&counters[3], (unsigned long long)upd[f]);
  }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_awgn_frames(const uint8_t* cw, int P, int N, int B, float sigma2, const uint64_t* seed_dev,
                              uint64_t seed_val, int point, float* llr, hipStream_t st) {
  const long long total = (long long)B * N;
  if (total <= 0) return hipSuccess;
  const int grid = (int)std::min<long long>((total + 255) / 256, 65536);
  const float sigma = sqrtf(sigma2), scale = 2.0f / sigma2;
  hipLaunchKernelGGL(k_awgn_frames, dim3(grid), dim3(256), 0, st, cw, P, N, B, sigma, scale, seed_dev, seed_val, point,
                     llr);
  return hipGetLastError();
}

hipError_t launch_count_errors(const uint8_t* bits, const uint8_t* cw, int P, int N, int B, const int64_t* upd,
                               int64_t* counters, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_errors, dim3(B), dim3(256), 0, st, bits, cw, P, N, B, upd,
                     reinterpret_cast<unsigned long long*>(counters));
  return hipGetLastError();
}

hipError_t launch_fill_u64(int64_t* p, int n, uint64_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, st, reinterpret_cast<unsigned long long*>(p), n,
                     (unsigned long long)v);
  return hipGetLastError();
}

}  // namespace ldpc
