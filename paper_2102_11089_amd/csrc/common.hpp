// Device-side building blocks shared by the decoder kernels (gfx950, wave64).
//
// Arithmetic modes:
//   ArithF32 - sum-product in FP32.  The check rule of eq. (2) (Sec. II-A) is applied pairwise in
//              the Jacobian-logarithm form  a [+] b = s(a)s(b) (min(|a|,|b|) + g(|a|+|b|) - g(||a|-|b||)),
//              g(x) = log(1 + e^-x), which stays finite where the tanh product saturates in FP32.
//              CI (eq. (9), Sec. III-A): D = |p0(L) - p0(Lt)| = 0.5 |tanh(L/2) - tanh(Lt/2)|.
//   ArithFix - q-bit fixed-point min-sum (Sec. V): channel sat(round_half_away(llr 2^f)),
//              V2C = sat(L - c2v), C2V = sign product * min magnitude (sign of 0 is +), exact
//              integer L and Lt, CI from a p0 table (Sec. V-B): D = |T[L] - T[Lt]|.
//
// Selection keys: u64 (value bits << 32) | (0xFFFFFFFF - index).  Values are non-negative (CI,
// residual), so their FP32 bit patterns order like the values; a maximum over keys returns the
// largest value and, among equal values, the lowest index.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldpc {

constexpr int WAVE = 64;

// ------------------------------------------------------------------------------------------
// keys and wave reductions
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mkkey(uint32_t val, uint32_t idx) {
  return ((uint64_t)val << 32) | (uint64_t)(0xFFFFFFFFu - idx);
}
__device__ __forceinline__ uint32_t key_idx(uint64_t k) { return 0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull); }
__device__ __forceinline__ uint32_t key_val(uint64_t k) { return (uint32_t)(k >> 32); }

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// maximum over the 64 lanes, returned wave-uniform (scalar registers)
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t k) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) k = umax64(k, __shfl_xor(k, off));
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(k & 0xFFFFFFFFull));
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(k >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return __builtin_amdgcn_readfirstlane(v);
}

// exclusive prefix sum across the wave
__device__ __forceinline__ int wave_excl_scan(int v, int lane) {
  int x = v;
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x - v;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------------------------------------
// FP32 sum-product
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float softplus_neg(float x) {  // log(1 + e^-x), x >= 0
  return __logf(1.0f + __expf(-x));
}

struct ArithF32 {
  using msg_t = float;   // c2v / pre storage
  using llr_t = float;   // L / Lt storage
  using val_t = float;   // computation type
  static constexpr bool kFixed = false;

  float qmax;            // unused
  float scale;           // unused
  const int* lut;        // unused

  __device__ __forceinline__ val_t channel(float llr) const { return llr; }
  __device__ __forceinline__ val_t v2c(val_t L, val_t c2v) const { return L - c2v; }
  __device__ __forceinline__ val_t vin(val_t v) const { return v; }  // check input (no saturation)
  __device__ __forceinline__ val_t op(val_t a, val_t b) const {
    float aa = fabsf(a), ab = fabsf(b);
    float mag = fminf(aa, ab) + softplus_neg(aa + ab) - softplus_neg(fabsf(aa - ab));
    mag = fmaxf(mag, 0.0f);
    return ((a < 0.0f) != (b < 0.0f)) ? -mag : mag;  // sign of 0 counts as +
  }
  __device__ __forceinline__ static float half_tanh(float x) {  // tanh(x/2), odd-exact
    float t = __expf(-fabsf(x));
    float th = __fdividef(1.0f - t, 1.0f + t);
    return x < 0.0f ? -th : th;
  }
  __device__ __forceinline__ uint32_t ci(val_t L, val_t Lt) const {
    float d = 0.5f * fabsf(half_tanh(L) - half_tanh(Lt));
    return __float_as_uint(d);
  }
  __device__ __forceinline__ uint32_t res(val_t pre, val_t c2v) const { return __float_as_uint(fabsf(pre - c2v)); }
  __device__ __forceinline__ float out_llr(val_t L) const { return L; }
  __device__ __forceinline__ float as_float(val_t v) const { return v; }
  __device__ __forceinline__ float d_float(uint32_t d) const { return __uint_as_float(d); }
  __device__ __forceinline__ int bin(uint32_t d, int ng) const {
    int b = (int)floorf(__uint_as_float(d) * (float)ng);
    return b > ng - 1 ? ng - 1 : (b < 0 ? 0 : b);
  }
};

// ------------------------------------------------------------------------------------------
// fixed-point min-sum
// ------------------------------------------------------------------------------------------
struct ArithFix {
  using msg_t = int8_t;
  using llr_t = int;
  using val_t = int;
  static constexpr bool kFixed = true;

  int qmax;              // 2^(q-1) - 1
  float scale;           // 2^f
  const int* lut;        // p0 table in LDS, index x + 128

  __device__ __forceinline__ int sat(int x) const { return x > qmax ? qmax : (x < -qmax ? -qmax : x); }
  __device__ __forceinline__ val_t channel(float llr) const {
    float x = llr * scale;                         // exact: power-of-two scale
    float r = x < 0.0f ? -floorf(-x + 0.5f) : floorf(x + 0.5f);
    r = fminf(fmaxf(r, -(float)qmax), (float)qmax);
    return (int)r;
  }
  __device__ __forceinline__ val_t v2c(val_t L, val_t c2v) const { return sat(L - c2v); }
  __device__ __forceinline__ val_t vin(val_t v) const { return sat(v); }
  __device__ __forceinline__ val_t op(val_t a, val_t b) const {
    int m = min(abs(a), abs(b));
    return ((a < 0) != (b < 0)) ? -m : m;
  }
  __device__ __forceinline__ uint32_t ci(val_t L, val_t Lt) const {
    int a = L < -128 ? -128 : (L > 128 ? 128 : L);
    int b = Lt < -128 ? -128 : (Lt > 128 ? 128 : Lt);
    return (uint32_t)abs(lut[a + 128] - lut[b + 128]);
  }
  __device__ __forceinline__ uint32_t res(val_t pre, val_t c2v) const { return (uint32_t)abs(pre - c2v); }
  __device__ __forceinline__ float out_llr(val_t L) const { return (float)L / scale; }
  __device__ __forceinline__ float as_float(val_t v) const { return (float)v; }
  __device__ __forceinline__ float d_float(uint32_t d) const { return (float)d; }
  __device__ __forceinline__ int bin(uint32_t d, int ng) const {
    long long b = ((long long)d * ng) / 65535;
    return b > ng - 1 ? ng - 1 : (int)b;
  }
};

// ------------------------------------------------------------------------------------------
// code topology as seen by a kernel
// ------------------------------------------------------------------------------------------
struct DevCode {
  int M, N, E;
  int max_dc, max_dv, max_touch;  // max_touch = max over VNs of sum of degrees of its checks
  int n_layers;
  const int* row_ptr;    // [M+1]
  const int* col;        // [E]   VN of edge e (canonical row-major edge ids)
  const int* row_of;     // [E]   check of edge e
  const int* col_ptr;    // [N+1]
  const int* col_row;    // [E]   checks of VN n, ascending
  const int* col_eid;    // [E]   edge ids of VN n, ascending
  const int* layer_ptr;  // [n_layers+1]
};

// splitmix64 output function (Steele, Lea, Flood, 2014): golden-gamma increment + finaliser
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace ldpc
