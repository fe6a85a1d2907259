// Single-edge dynamic schedules on gfx950: residual BP (RBP, Sec. II-A steps 1-4), CIRBP
// (Algorithm 1, Sec. III-B) and forced-order replay of a recorded schedule.
//
// One wavefront (64 lanes, one workgroup) decodes one codeword at a time; workgroups loop over
// frames.  The frame's state lives in LDS:
//   c2v[E], pre[E]      current and precomputed C2V messages (pre may live in a global scratch
//                        slot per workgroup when it does not fit),
//   L[N], Lt[N]         total and precomputed total LLRs,
//   D[N]                CI of every VN as key bits,
//   ckey[M]             per check: max over its edges of (residual, lowest edge id),
//   dblk[], cblk[]      max over blocks of 64 VNs / 64 checks (two-level max trees),
//   syn[M]              syndrome bits of the current hard decisions,
//   topology            CSR/CSC copies (small codes) or quasi-cyclic base tables.
// Per update (chain of dependent steps kept short; every row computed in registers):
//   selection      argmax over the block maxima (one wave reduction), or over the checks of n*,
//   propagation    c2v[e*] <- pre[e*], L_{n*} += delta, D_{n*} refresh, syndrome toggles,
//   touched checks the two-hop table of n* places every edge of every check of n* in an aligned
//                  block of lanes; one load brings V2C inputs, a butterfly inside each block gives
//                  the whole row's precomputed messages (eq. (2)) and its residual key,
//   CI             Lt_j += pre_new - pre_old, then D_j for the VNs of the touched checks,
//   max trees      block maxima raised with LDS atomic max; a block whose maximum leaf
//                  decreased is recomputed by one wave reduction.
#include "dyn_frame.hpp"

namespace ldpc {



template <class A, bool PRE_GLOBAL, int TOPO>
__global__ __launch_bounds__(WAVE) void k_dynamic(DevCode H, DynParams P) {
  using msg_t = typename A::msg_t;
  unsigned char* lds = dyn_lds();
  const int lane = threadIdx.x;
  msg_t* pre;
  if constexpr (PRE_GLOBAL) pre = reinterpret_cast<msg_t*>(P.pre_global) + (size_t)blockIdx.x * H.E;
  else pre = reinterpret_cast<msg_t*>(lds + P.off_pre);
  int* lut = reinterpret_cast<int*>(lds + P.off_lut);
  A ar;
  ar.qmax = P.qmax;
  ar.scale = P.scale;
  ar.lut = lut;
  if constexpr (A::kFixed) {
    for (int x = lane; x < 257; x += WAVE) lut[x] = P.lut_global[x];
  }
  const auto G = TopoSel<TOPO>::make(H, lds + P.off_topo, lane, WAVE);
  wave_sync();
  for (int f = blockIdx.x; f < P.B; f += gridDim.x) {
    FrameJob J;
    J.kind = P.kind;
    J.gamma_bits = P.gamma_bits;
    J.max_updates = P.max_updates;
    J.check_every = P.check_every;
    J.llr = P.llr + (size_t)f * H.N;
    J.replay = P.replay ? P.replay + (size_t)f * P.replay_len : nullptr;
    J.replay_len = P.replay_len;
    J.bits = P.out.bits + (size_t)f * H.N;
    J.llr_out = P.out.llr_out ? P.out.llr_out + (size_t)f * H.N : nullptr;
    J.updates_used = P.out.updates_used + f;
    J.steps_used = P.out.steps_used ? P.out.steps_used + f : nullptr;
    J.fallbacks = P.out.fallbacks ? P.out.fallbacks + f : nullptr;
    J.trace = P.out.trace ? P.out.trace + (size_t)f * P.max_updates : nullptr;
    J.dump_c2v = P.out.dump_c2v ? P.out.dump_c2v + (size_t)f * H.E : nullptr;
    J.dump_pre = P.out.dump_pre ? P.out.dump_pre + (size_t)f * H.E : nullptr;
    J.dump_L = P.out.dump_L ? P.out.dump_L + (size_t)f * H.N : nullptr;
    J.dump_Lt = P.out.dump_Lt ? P.out.dump_Lt + (size_t)f * H.N : nullptr;
    J.dump_D = P.out.dump_D ? P.out.dump_D + (size_t)f * H.N : nullptr;
    dyn_decode_frame<A, PRE_GLOBAL>(H, G, ar, P, pre, J);
  }
}

template <class A, bool PG, int TP>
static hipError_t launch_dyn(const DevCode& H, const DynParams& P, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_dynamic<A, PG, TP>), dim3(grid), dim3(WAVE), P.lds_bytes, st, H, P);
  return hipGetLastError();
}

template <class A, bool PG>
static hipError_t launch_dyn_t(const DevCode& H, const DynParams& P, int topo, int grid, hipStream_t st) {
  if (topo == TOPO_QC) return launch_dyn<A, PG, TOPO_QC>(H, P, grid, st);
  if (topo == TOPO_LDS) return launch_dyn<A, PG, TOPO_LDS>(H, P, grid, st);
  return launch_dyn<A, PG, TOPO_GLOBAL>(H, P, grid, st);
}

hipError_t launch_dynamic(const DevCode& H, const DynParams& P, bool fixed, bool pre_global, int topo, int grid,
                          hipStream_t st) {
  if (fixed)
    return pre_global ? launch_dyn_t<ArithFix, true>(H, P, topo, grid, st)
                      : launch_dyn_t<ArithFix, false>(H, P, topo, grid, st);
  return pre_global ? launch_dyn_t<ArithF32, true>(H, P, topo, grid, st)
                    : launch_dyn_t<ArithF32, false>(H, P, topo, grid, st);
}

template <class A, bool PG, int TP>
static hipError_t set_one(int bytes) {
  return hipFuncSetAttribute((const void*)k_dynamic<A, PG, TP>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t set_dynamic_lds_limit(int bytes) {
  hipError_t e = hipSuccess;
#define LDPC_SET(A, PG, TP) \
  if ((e = set_one<A, PG, TP>(bytes)) != hipSuccess) return e;
  LDPC_SET(ArithF32, false, TOPO_GLOBAL) LDPC_SET(ArithF32, false, TOPO_LDS) LDPC_SET(ArithF32, false, TOPO_QC)
  LDPC_SET(ArithF32, true, TOPO_GLOBAL) LDPC_SET(ArithF32, true, TOPO_LDS) LDPC_SET(ArithF32, true, TOPO_QC)
  LDPC_SET(ArithFix, false, TOPO_GLOBAL) LDPC_SET(ArithFix, false, TOPO_LDS) LDPC_SET(ArithFix, false, TOPO_QC)
  LDPC_SET(ArithFix, true, TOPO_GLOBAL) LDPC_SET(ArithFix, true, TOPO_LDS) LDPC_SET(ArithFix, true, TOPO_QC)
#undef LDPC_SET
  return e;
}

}  // namespace ldpc
