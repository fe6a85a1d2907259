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
constexpr int NBR_PMAX = 8;  // two-hop neighbourhood of one VN: at most 8 passes of 64 lanes
// VNs met twice in one VN's two-hop table (4-cycles) are summed per group: groups 0..kGroups-1 in
// LDS, the rest (group kGroups) through atomics on Lt
constexpr int kGroups = 7;
constexpr int kGroupBytes = 4 * 4 * (kGroups + 1) + 16;  // sums, Lt, L, VN per group; the flag word

// ------------------------------------------------------------------------------------------
// keys and wave reductions
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mkkey(uint32_t val, uint32_t idx) {
  return ((uint64_t)val << 32) | (uint64_t)(0xFFFFFFFFu - idx);
}
__device__ __forceinline__ uint32_t key_idx(uint64_t k) { return 0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull); }
__device__ __forceinline__ uint32_t key_val(uint64_t k) { return (uint32_t)(k >> 32); }

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Cross-lane primitives built on DPP (data-parallel primitives: a VALU source operand taken from
// another lane of the same 16-lane row) and v_readlane for the four row results.  They must be
// called with all 64 lanes active.
//   quad_perm [1,0,3,2] / [2,3,0,1], row_half_mirror and row_mirror pair every lane of a row with a
//   distinct partner, so four steps leave the row's total in all 16 lanes;
//   row_shr:1,2,4,8 (identity fill) give an inclusive scan inside each row, row_bcast:15 and
//   row_bcast:31 carry the row totals forward.
#define LDPC_DPP_QXOR1 0xB1
#define LDPC_DPP_QXOR2 0x4E
#define LDPC_DPP_HALF_MIRROR 0x141
#define LDPC_DPP_MIRROR 0x140
#define LDPC_DPP_SHR(n) (0x110 + (n))
#define LDPC_DPP_BCAST15 0x142
#define LDPC_DPP_BCAST31 0x143

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
// the same exchange as a plain move: every pattern used here has a valid source lane for every
// lane, so no fill value is needed (the compiler then emits a single v_mov_b32_dpp)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, true);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  x = max(x, dpp_u32<LDPC_DPP_QXOR1>(x));
  x = max(x, dpp_u32<LDPC_DPP_QXOR2>(x));
  x = max(x, dpp_u32<LDPC_DPP_HALF_MIRROR>(x));
  x = max(x, dpp_u32<LDPC_DPP_MIRROR>(x));
  const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)x, 0);
  const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)x, 16);
  const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)x, 32);
  const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
  return max(max(a, b), max(c, d));
}

// maximum of u64 keys over the 64 lanes, returned wave-uniform: the high words first, then the
// low words of the lanes holding the maximal high word
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t k) {
  const uint32_t hi = (uint32_t)(k >> 32), lo = (uint32_t)(k & 0xFFFFFFFFull);
  const uint32_t mh = wave_max_u32(hi);
  const uint32_t ml = wave_max_u32(hi == mh ? lo : 0u);
  return ((uint64_t)mh << 32) | ml;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
  uint32_t x = (uint32_t)v;
  x += dpp_u32<LDPC_DPP_QXOR1>(x);
  x += dpp_u32<LDPC_DPP_QXOR2>(x);
  x += dpp_u32<LDPC_DPP_HALF_MIRROR>(x);
  x += dpp_u32<LDPC_DPP_MIRROR>(x);
  return __builtin_amdgcn_readlane((int)x, 0) + __builtin_amdgcn_readlane((int)x, 16) +
         __builtin_amdgcn_readlane((int)x, 32) + __builtin_amdgcn_readlane((int)x, 48);
}

// exclusive prefix sum across the wave (lane order)
__device__ __forceinline__ int wave_excl_scan(int v, int) {
  uint32_t x = (uint32_t)v;
  x += dpp_u32<LDPC_DPP_SHR(1)>(x);
  x += dpp_u32<LDPC_DPP_SHR(2)>(x);
  x += dpp_u32<LDPC_DPP_SHR(4)>(x);
  x += dpp_u32<LDPC_DPP_SHR(8)>(x);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, LDPC_DPP_BCAST15, 0xA, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, LDPC_DPP_BCAST31, 0xC, 0xF, false);
  return (int)x - v;
}

// Butterfly exchange inside aligned lane blocks of 2^L lanes: level 1..4 use DPP inside 16-lane
// rows (quad_perm xor 1, xor 2, row_half_mirror, row_mirror); level 5 pairs the two 16-lane rows
// of a 32-lane half with a ds_swizzle xor 16.  After level k every lane holds the result of its
// aligned 2^k group.
template <int LEVEL>
__device__ __forceinline__ uint32_t bfly(uint32_t x) {
  if constexpr (LEVEL == 1) return dpp_mov<LDPC_DPP_QXOR1>(x);
  else if constexpr (LEVEL == 2) return dpp_mov<LDPC_DPP_QXOR2>(x);
  else if constexpr (LEVEL == 3) return dpp_mov<LDPC_DPP_HALF_MIRROR>(x);
  else if constexpr (LEVEL == 4) return dpp_mov<LDPC_DPP_MIRROR>(x);
  else return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401F);
}
template <int LEVEL>
__device__ __forceinline__ float bflyf(float x) { return __uint_as_float(bfly<LEVEL>(__float_as_uint(x))); }

// Per-lane state of a whole-row reduction: sum of phi (S), the same sum without the row's
// smallest input (Sx), smallest magnitude (m1) with its edge id, second smallest (m2), sign
// parity (bit 31 of ap, the edge id in bits 0..30).  Merging two groups keeps the smaller
// minimum (lower edge id on ties); the merged Sx is the winner's Sx plus the other group's S.
struct RowRed {
  float S, Sx, m1, m2;
  uint32_t ap;  // edge id of m1 | parity << 31
};

template <int LEVEL, bool SUM>
__device__ __forceinline__ void rowred_step(RowRed& r, bool on) {
  const float pm1 = bflyf<LEVEL>(r.m1), pm2 = bflyf<LEVEL>(r.m2);
  const uint32_t pap = bfly<LEVEL>(r.ap);
  float pS = 0.0f, pSx = 0.0f;
  if constexpr (SUM) {
    pS = bflyf<LEVEL>(r.S);
    pSx = bflyf<LEVEL>(r.Sx);
  }
  // straight-line merge (selects, no branches): the partner's minimum wins if smaller, or equal
  // with a lower edge id
  const uint32_t par = (r.ap ^ pap) & 0x80000000u;
  const uint32_t a = r.ap & 0x7FFFFFFFu, pa = pap & 0x7FFFFFFFu;
  const bool take = pm1 < r.m1 || (pm1 == r.m1 && pa < a);
  const float m2 = take ? fminf(r.m1, pm2) : fminf(r.m2, pm1);
  const float m1 = take ? pm1 : r.m1;
  const uint32_t ap = (take ? pa : a) | par;
  if constexpr (SUM) {
    const float Sx = take ? pSx + r.S : r.Sx + pS;
    const float S = r.S + pS;
    r.Sx = on ? Sx : r.Sx;
    r.S = on ? S : r.S;
  }
  r.m2 = on ? m2 : r.m2;
  r.m1 = on ? m1 : r.m1;
  r.ap = on ? ap : r.ap;
}

// all butterfly levels up to the largest block of the pass (maxL2 is wave-uniform)
template <bool SUM>
__device__ __forceinline__ void rowred_all(RowRed& r, int L2, int maxL2) {
  if (maxL2 >= 1) rowred_step<1, SUM>(r, L2 >= 1);
  if (maxL2 >= 2) rowred_step<2, SUM>(r, L2 >= 2);
  if (maxL2 >= 3) rowred_step<3, SUM>(r, L2 >= 3);
  if (maxL2 >= 4) rowred_step<4, SUM>(r, L2 >= 4);
  if (maxL2 >= 5) rowred_step<5, SUM>(r, L2 >= 5);
}

// maximum of (hi, lo) pairs inside the block
template <int LEVEL>
__device__ __forceinline__ void keymax_step(uint32_t& hi, uint32_t& lo, bool on) {
  const uint32_t ph = bfly<LEVEL>(hi), pl = bfly<LEVEL>(lo);
  const bool take = on && ((((uint64_t)ph << 32) | pl) > (((uint64_t)hi << 32) | lo));
  hi = take ? ph : hi;
  lo = take ? pl : lo;
}
__device__ __forceinline__ uint64_t keymax_all(uint64_t k, int L2, int maxL2) {
  uint32_t hi = (uint32_t)(k >> 32), lo = (uint32_t)(k & 0xFFFFFFFFull);
  if (maxL2 >= 1) keymax_step<1>(hi, lo, L2 >= 1);
  if (maxL2 >= 2) keymax_step<2>(hi, lo, L2 >= 2);
  if (maxL2 >= 3) keymax_step<3>(hi, lo, L2 >= 3);
  if (maxL2 >= 4) keymax_step<4>(hi, lo, L2 >= 4);
  if (maxL2 >= 5) keymax_step<5>(hi, lo, L2 >= 5);
  return ((uint64_t)hi << 32) | lo;
}

// Ordering point for a workgroup that is exactly one wavefront: LDS operations of one wavefront
// execute in order, so only the compiler has to be kept from moving memory accesses across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// value of another lane (the lane index is wave-uniform)
template <class T>
__device__ __forceinline__ T lane_value(T x, int l) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
  else return (T)__builtin_amdgcn_readlane((int)x, l);
}

// the C2V message and the precomputed message of one edge, side by side: one load brings both
template <class msg_t>
struct alignas(2 * sizeof(msg_t)) MsgPair {
  msg_t c, p;
};

// ------------------------------------------------------------------------------------------
// FP32 sum-product
// ------------------------------------------------------------------------------------------
// reciprocal and natural logarithm from the hardware's approximate v_rcp_f32 and v_log_f32 (about
// 1 ulp; 1/0 = inf, log of inf = inf; no denormal arguments occur here): the sum-product terms
// need FP32-level relative accuracy, not correctly rounded results
__device__ __forceinline__ float rcp_approx(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float log_approx(float x) { return __builtin_amdgcn_logf(x) * 0.69314718056f; }

__device__ __forceinline__ float softplus_neg(float x) {  // log(1 + e^-x), x >= 0
  return log_approx(1.0f + __expf(-x));
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
    float th = (1.0f - t) * rcp_approx(1.0f + t);
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
// whole-row check update (eq. (2) for every edge of one check at once)
//
// Sum-product, FP32, Gallager's form of eq. (2):
//   |C2V_{m->j}| = phi( sum_{k != j} phi(|V2C_k|) ),  phi(x) = -log tanh(x/2) = phi^{-1}(x),
//   sign = product of the other signs (sign of 0 is +).
// Every lane of a row reads the row's (V2C, phi) pairs once; the sum leaving out the row's
// smallest input is accumulated separately so that no large term is ever subtracted from itself,
// and the result is clamped by the smallest other magnitude (|a [+] b| <= min(|a|, |b|)).
// Min-sum (fixed point): sign product times the smallest other magnitude, from (min1, argmin,
// min2, parity) of the row -- exactly the oracle's leave-one-out fold.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float phi_f32(float x) {  // -log(tanh(x/2)) = log((1 + t) / (1 - t)), t = e^-x
  const float t = __expf(-x);
  // 1 - e^-x: Taylor series below 0.25 (the subtraction would lose the low bits)
  const float ser = x * (1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f - x * (1.0f / 120.0f)))));
  const float y = x < 0.25f ? ser : 1.0f - t;
  const float ry = rcp_approx(y);
  const float lg = log_approx((1.0f + t) * ry);
  // above 4 the quotient is 1 + w, w = 2t/(1-t) < 0.04: log(1 + w) by its series
  const float w = (2.0f * t) * ry;
  const float lp = w * (1.0f - w * (0.5f - w * (1.0f / 3.0f - w * 0.25f)));
  return x > 4.0f ? lp : lg;
}

struct RowAccF32 {
  float S = 0.0f, Sx = 0.0f, min1 = __builtin_inff(), min2 = __builtin_inff();
  int arg = -1;
  uint32_t par = 0;
  __device__ __forceinline__ void add(int k, float v, float ph) {
    const float a = fabsf(v);
    par ^= v < 0.0f ? 1u : 0u;
    const float before = S;
    S += ph;
    if (a < min1) {
      Sx = before;
      min2 = min1;
      min1 = a;
      arg = k;
    } else {
      Sx += ph;
      if (a < min2) min2 = a;
    }
  }
  __device__ __forceinline__ float out(int j, float vj, float phj) const {
    const bool self = j == arg;
    const float mo = self ? min2 : min1;
    const float Sj = self ? Sx : (phj == __builtin_inff() ? __builtin_inff() : S - phj);
    const float mag = fminf(phi_f32(fmaxf(Sj, 0.0f)), mo);
    return ((par ^ (vj < 0.0f ? 1u : 0u)) & 1u) ? -mag : mag;
  }
};

struct RowAccFix {
  int min1 = 0x7fffffff, min2 = 0x7fffffff, arg = -1;
  uint32_t par = 0;
  __device__ __forceinline__ void add(int k, int v, float) {
    const int a = abs(v);
    par ^= v < 0 ? 1u : 0u;
    if (a < min1) {
      min2 = min1;
      min1 = a;
      arg = k;
    } else if (a < min2) {
      min2 = a;
    }
  }
  __device__ __forceinline__ int out(int j, int vj, float) const {
    const int mag = j == arg ? min2 : min1;
    return ((par ^ (vj < 0 ? 1u : 0u)) & 1u) ? -mag : mag;
  }
};

template <class A> struct RowAccOf;
template <> struct RowAccOf<ArithF32> { using type = RowAccF32; };
template <> struct RowAccOf<ArithFix> { using type = RowAccFix; };

// per-input auxiliary value stored next to each V2C (phi for sum-product, unused for min-sum)
__device__ __forceinline__ float row_aux(const ArithF32&, float v) { return phi_f32(fabsf(v)); }
__device__ __forceinline__ float row_aux(const ArithFix&, int) { return 0.0f; }

// Whole-row check update (eq. (2)) for the lane's edge, one row per aligned block of 2^L2 lanes:
// the lane holds input v of edge e (valid) or nothing; every lane of the wavefront must take part
// (maxL2 wave-uniform, the largest block of the wavefront).  Returns the lane's C2V output: the
// row's parity and smallest other magnitude (min-sum), or phi of the other inputs' phi-sum clamped
// by that magnitude (sum-product).
template <class A>
__device__ __forceinline__ typename A::val_t row_update_lane(const A& ar, bool valid, uint32_t e,
                                                             typename A::val_t v, int L2, int maxL2) {
  RowRed r;
  r.m1 = valid ? fabsf((float)v) : __builtin_inff();
  r.m2 = __builtin_inff();
  r.ap = (valid ? e : 0x7FFFFFFFu) | (valid && v < 0 ? 0x80000000u : 0u);
  if constexpr (A::kFixed) {
    rowred_all<false>(r, L2, maxL2);
    const bool me = e == (r.ap & 0x7FFFFFFFu);
    const int mag = (int)(me ? r.m2 : r.m1);
    return (((r.ap >> 31) ^ (v < 0 ? 1u : 0u)) & 1u) ? -mag : mag;
  } else {
    const float ph = valid ? row_aux(ar, v) : 0.0f;
    r.S = ph;
    r.Sx = 0.0f;
    rowred_all<true>(r, L2, maxL2);
    const bool me = e == (r.ap & 0x7FFFFFFFu);
    const float mo = me ? r.m2 : r.m1;
    const float Sj = me ? r.Sx : (ph == __builtin_inff() ? __builtin_inff() : r.S - ph);
    const float mag = fminf(phi_f32(fmaxf(Sj, 0.0f)), mo);
    return (((r.ap >> 31) ^ (v < 0.0f ? 1u : 0u)) & 1u) ? -mag : mag;
  }
}

// ------------------------------------------------------------------------------------------
// code topology as seen by a kernel
// ------------------------------------------------------------------------------------------
// Exact quotient n / d for 0 <= n < 2^31 and 1 <= d < 2^31 by a multiply and a shift: with
// l = ceil(log2 d), sh = 31 + l and mul = ceil(2^sh / d) (below 2^32), n mul / 2^sh exceeds n / d by
// less than n d / (d 2^sh) < 2^-l <= 1 / d, too little to carry the quotient past the next integer.
struct FastDiv {
  uint32_t mul, sh;
  __host__ __device__ static FastDiv of(uint32_t d) {
    uint32_t l = 0;
    while ((1u << l) < d) ++l;
    FastDiv f;
    f.sh = 31 + l;
    f.mul = (uint32_t)(((1ull << f.sh) + d - 1) / d);
    return f;
  }
  __host__ __device__ __forceinline__ int div(int n) const {
    return (int)(((uint64_t)(uint32_t)n * mul) >> sh);
  }
};

// Quasi-cyclic description (Sec. V codes are lifted base graphs): base row i has deg[i] blocks
// (j, shift) with ascending j; check m = i Z + r meets VN j Z + ((r + shift) mod Z).  Edge ids stay
// canonical: e = Z bptr[i] + r deg[i] + rank of j in row i.
struct DevQC {
  int Z, mb, nb, nblk;  // nblk = bptr[mb] = number of nonzero blocks
  const int* bdeg;      // [mb]
  const int* bptr;      // [mb+1]
  const int* brow;      // [nblk][2]  (j, shift) per row, ascending j
  const int* bcol_ptr;  // [nb+1]
  const int* bcol;      // [nblk][4]  (i, shift, rank in row i, 0) per column, ascending i
  const int* rowmap;    // [nblk]     base row of edge block e / Z
  const int* bdiv;      // [mb][2]    FastDiv (mul, sh) of deg[i]
  const int* border;    // [mb]       base rows by descending degree (ties: ascending index)
  int words;            // total ints of the tables (for copying into LDS)
  FastDiv zdiv;         // FastDiv of Z
};

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
  DevQC qc;              // valid when qc.Z > 0
  // two-hop neighbourhood table: for VN n, nbr[off(n) .. off(n) + cnt(n)) lists every edge of every
  // check of n, each check in an aligned block of 2^L lanes (largest blocks first, padding entries
  // have e = -1).  Entry = (edge id, VN | L << 24 | leader << 27 | twice << 28 | group << 29);
  // twice marks a VN other than n that lies on more than one check of n, group numbers such VNs.
  const int2* nbr;
  const int2* nbr_idx;   // [N] (off, cnt)
  const int2* nbr_col;   // quasi-cyclic codes: [nb] (off of VN j Z, cnt) -- off(n) = off + (n mod Z) cnt
  int nbr_max_cnt;
};

// Topology over CSR/CSC arrays (global memory or LDS copies)
struct TopoCSR {
  const int* row_ptr;
  const int* col;
  const int* row_of;
  const int* col_ptr;
  const int* col_row;
  const int* col_eid;
  __device__ __forceinline__ int vn_deg(int n) const { return col_ptr[n + 1] - col_ptr[n]; }
  __device__ __forceinline__ void vn_edge(int n, int k, int& m, int& e) const {
    const int x = col_ptr[n] + k;
    m = col_row[x];
    e = col_eid[x];
  }
  __device__ __forceinline__ int row_start(int m) const { return row_ptr[m]; }
  __device__ __forceinline__ int row_deg(int m) const { return row_ptr[m + 1] - row_ptr[m]; }
  __device__ __forceinline__ int row_vn(int m, int rs, int p) const { return col[rs + p]; }
  __device__ __forceinline__ int edge_vn(int e) const { return col[e]; }
  __device__ __forceinline__ int edge_row(int e) const { return row_of[e]; }
  const int2* nbr_idx;
  __device__ __forceinline__ int2 nbr(int n) const { return nbr_idx[n]; }
};

// Topology of a quasi-cyclic code from its base tables (in LDS): no per-edge index arrays; every
// division by Z or by a base-row degree is a FastDiv
struct TopoQC {
  int Z;
  FastDiv zdiv;
  const int* bdeg;
  const int* bptr;
  const int* brow;
  const int* bcol_ptr;
  const int* bcol;
  const int* rowmap;
  const int* bdiv;
  __device__ __forceinline__ int row_div(int i, int x) const {
    const FastDiv f{(uint32_t)bdiv[2 * i], (uint32_t)bdiv[2 * i + 1]};
    return f.div(x);
  }
  __device__ __forceinline__ int vn_deg(int n) const {
    const int j = zdiv.div(n);
    return bcol_ptr[j + 1] - bcol_ptr[j];
  }
  __device__ __forceinline__ void vn_edge(int n, int k, int& m, int& e) const {
    const int j = zdiv.div(n), c = n - j * Z;
    const int x = (bcol_ptr[j] + k) * 4;
    const int i = bcol[x], sh = bcol[x + 1], rank = bcol[x + 2];
    int r = c - sh;
    if (r < 0) r += Z;
    m = i * Z + r;
    e = Z * bptr[i] + r * bdeg[i] + rank;
  }
  __device__ __forceinline__ int row_start(int m) const {
    const int i = zdiv.div(m), r = m - i * Z;
    return Z * bptr[i] + r * bdeg[i];
  }
  __device__ __forceinline__ int row_deg(int m) const { return bdeg[zdiv.div(m)]; }
  __device__ __forceinline__ int row_vn(int m, int, int p) const {
    const int i = zdiv.div(m), r = m - i * Z;
    const int x = (bptr[i] + p) * 2;
    int c = r + brow[x + 1];
    if (c >= Z) c -= Z;
    return brow[x] * Z + c;
  }
  __device__ __forceinline__ int edge_row(int e) const {
    const int i = rowmap[zdiv.div(e)];
    const int r = row_div(i, e - Z * bptr[i]);
    return i * Z + r;
  }
  __device__ __forceinline__ int edge_vn(int e) const {
    const int i = rowmap[zdiv.div(e)];
    const int loc = e - Z * bptr[i];
    const int r = row_div(i, loc), p = loc - r * bdeg[i];
    const int x = (bptr[i] + p) * 2;
    int c = r + brow[x + 1];
    if (c >= Z) c -= Z;
    return brow[x] * Z + c;
  }
  const int* nbr_col;  // [nb][2] in LDS
  const int* border;   // [mb] base rows by descending degree, in LDS
  __device__ __forceinline__ int2 nbr(int n) const {
    const int j = zdiv.div(n), c = n - j * Z;
    const int cnt = nbr_col[2 * j + 1];
    return make_int2(nbr_col[2 * j] + c * cnt, cnt);
  }
};

// The process's abort flag (fine-grained host memory, written by ldpc_request_abort): a nonzero
// value stops decoders from starting further frames.  A system-scope load, so that a host write
// reaches kernels that are running.
__device__ __forceinline__ int abort_flag_value(const int* flag) {
  return flag ? __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0;
}

// Next frame of a work queue and the abort flag, read by lane 0 with both requests in flight
// together and made wave-uniform.
__device__ __forceinline__ int next_frame(int* queue, const int* flag, int lane, int& aborted) {
  int f = 0, a = 0;
  if (lane == 0) {
    f = atomicAdd(queue, 1);
    a = abort_flag_value(flag);
  }
  aborted = __builtin_amdgcn_readfirstlane(a);
  return __builtin_amdgcn_readfirstlane(f);
}

// splitmix64 output function (Steele, Lea, Flood, 2014): golden-gamma increment + finaliser
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace ldpc
