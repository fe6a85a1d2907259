// Single-edge dynamic schedules on gfx950: residual BP (RBP, Sec. II-A steps 1-4), CIRBP
// (Algorithm 1, Sec. III-B), forced-order replay of a recorded schedule, and the latest-message-
// driven LMDRBP, sLMDRBP and LMD-CIRBP (Algorithms 2 and 3, Sec. IV) as separate kernel variants.
//
// One wavefront (64 lanes) decodes one codeword at a time; a workgroup holds one or more such
// frames, which share the workgroup's copy of the topology (and p0 table) in LDS.  A persistent grid pulls
// frames from a device counter (frames differ widely in length, so fixed striding would leave a
// long tail); otherwise there is one workgroup per frame.  A frame's state is
//   c2v[E], pre[E]      current and precomputed C2V messages (separate arrays, or interleaved pairs),
//   L[N], Lt[N]         total and precomputed total LLRs (separate arrays, or one 8-byte (Lt, L)
//                        record per VN),
//   D[N]                CI of every VN as key bits (not stored with the records: evaluated from them),
//   ckey[M]             per check: max over its edges of (residual, lowest edge id),
//   dblk[], cblk[]      max over blocks of 64 VNs / 64 checks (two-level max trees),
//   syn[M]              syndrome bits of the current hard decisions,
//   topology            CSR/CSC copies (small codes) or quasi-cyclic base tables.
// The storage mode (Store) places it: everything in LDS for small codes, or, from the messages up
// to the whole frame and the check keys, in a global slot per frame, with the block maxima,
// masks, syndrome bits and topology left in LDS.  The planner picks the mode that keeps the most
// frames resident; the large codes (n of a few thousand) keep the whole frame in the slot.
// Per update (chain of dependent steps kept short; every row computed in registers):
//   selection      argmax over the block maxima (one wave reduction), or over the checks of n*,
//   propagation    c2v[e*] <- pre[e*], L_{n*} += delta, D_{n*} refresh, syndrome toggles,
//   touched checks the two-hop table of n* places every edge of every check of n* in an aligned
//                  block of lanes; one load brings V2C inputs, a butterfly inside each block gives
//                  the whole row's precomputed messages (eq. (2)) and its residual key,
//   CI             Lt_j += pre_new - pre_old, then D_j for the VNs of the touched checks,
//   max trees      block maxima raised with LDS atomic max; a block whose maximum leaf
//                  decreased is recomputed by one wave reduction.
#include <map>
#include <mutex>

#include "dyn_frame.hpp"

namespace ldpc {



// MF: several frames per workgroup (up to 16 wavefronts); otherwise one wavefront per workgroup,
// which lets the compiler keep the register count at the level of full occupancy.  LMD: the LMD
// schedules (their local choice keeps a few more values live across the update)
template <class A, int STORE, int TOPO, bool MF, bool LMD>
__global__ __launch_bounds__(MF ? 1024 : WAVE) void k_dynamic(DevCode H, DynParams P) {
  unsigned char* lds = dyn_lds();
  const int lane = threadIdx.x & (WAVE - 1);
  const auto ms = make_store<A, STORE, true>(P, (size_t)H.E);
  // shared by the workgroup's frames: the p0 table and the topology
  int* lut = reinterpret_cast<int*>(lds + P.off_lut);
  A ar;
  ar.qmax = P.qmax;
  ar.scale = P.scale;
  ar.lut = lut;
  if constexpr (A::kFixed) {
    for (int x = threadIdx.x; x < 257; x += blockDim.x) lut[x] = P.lut_global[x];
  }
  const auto G = TopoSel<TOPO>::make(H, lds + P.off_topo, threadIdx.x, blockDim.x);
  __syncthreads();  // the only workgroup barrier: the frames below run independently
  int f = (int)frame_slot(P), aborted = 0;
  if (P.queue) f = next_frame(P.queue, P.out.abort, lane, aborted);
  else aborted = uni(lane == 0 ? abort_flag_value(P.out.abort) : 0);
  while (f < P.B) {
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
    if (!aborted)
      dyn_decode_frame<A, STORE, decltype(G), LMD, true>(H, G, ar, P, ms, J);
    else if (lane == 0)
      *J.updates_used = -1;  // not started: the abort flag was set
    if (P.queue) {
      f = next_frame(P.queue, P.out.abort, lane, aborted);
    } else {
      f += gridDim.x * P.wpb;
      aborted = uni(lane == 0 ? abort_flag_value(P.out.abort) : 0);
    }
  }
}

template <class A, int ST, int TP, bool LMD>
static hipError_t launch_dyn_l(const DevCode& H, const DynParams& P, int grid, hipStream_t st) {
  if constexpr (TP != TOPO_GLOBAL) {
    if (P.wpb > 1) {
      hipLaunchKernelGGL((k_dynamic<A, ST, TP, true, LMD>), dim3(grid), dim3(WAVE * P.wpb), P.lds_bytes, st, H, P);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_dynamic<A, ST, TP, false, LMD>), dim3(grid), dim3(WAVE), P.lds_bytes, st, H, P);
  return hipGetLastError();
}

template <class A, int ST, int TP>
static hipError_t launch_dyn(const DevCode& H, const DynParams& P, int grid, hipStream_t st) {
  return is_lmd(P.kind) ? launch_dyn_l<A, ST, TP, true>(H, P, grid, st) : launch_dyn_l<A, ST, TP, false>(H, P, grid, st);
}

template <class A, int ST>
static hipError_t launch_dyn_t(const DevCode& H, const DynParams& P, int topo, int grid, hipStream_t st) {
  if (topo == TOPO_QC) return launch_dyn<A, ST, TOPO_QC>(H, P, grid, st);
  if (topo == TOPO_LDS) return launch_dyn<A, ST, TOPO_LDS>(H, P, grid, st);
  return launch_dyn<A, ST, TOPO_GLOBAL>(H, P, grid, st);
}

template <class A>
static hipError_t launch_dyn_s(const DevCode& H, const DynParams& P, int store, int topo, int grid, hipStream_t st) {
  if (store == STORE_FRAME_ALL) return launch_dyn_t<A, STORE_FRAME_ALL>(H, P, topo, grid, st);
  if (store == STORE_FRAME_REC) return launch_dyn_t<A, STORE_FRAME_REC>(H, P, topo, grid, st);
  if (store == STORE_FRAME_GLOBAL) return launch_dyn_t<A, STORE_FRAME_GLOBAL>(H, P, topo, grid, st);
  if (store == STORE_ALL_GLOBAL_LT) return launch_dyn_t<A, STORE_ALL_GLOBAL_LT>(H, P, topo, grid, st);
  if (store == STORE_ALL_GLOBAL) return launch_dyn_t<A, STORE_ALL_GLOBAL>(H, P, topo, grid, st);
  if (store == STORE_PRE_GLOBAL) return launch_dyn_t<A, STORE_PRE_GLOBAL>(H, P, topo, grid, st);
  return launch_dyn_t<A, STORE_LDS>(H, P, topo, grid, st);
}

hipError_t launch_dynamic(const DevCode& H, const DynParams& P, bool fixed, int store, int topo, int grid,
                          hipStream_t st) {
  return fixed ? launch_dyn_s<ArithFix>(H, P, store, topo, grid, st) : launch_dyn_s<ArithF32>(H, P, store, topo, grid, st);
}

template <class A, int ST, int TP, bool LMD>
static hipError_t set_one_l(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_dynamic<A, ST, TP, false, LMD>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if constexpr (TP != TOPO_GLOBAL) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_dynamic<A, ST, TP, true, LMD>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  }
  return e;
}

template <class A, int ST, int TP>
static hipError_t set_one(int bytes) {
  hipError_t e = set_one_l<A, ST, TP, false>(bytes);
  if (e == hipSuccess) e = set_one_l<A, ST, TP, true>(bytes);
  return e;
}

template <class A, int ST>
static hipError_t set_store(int bytes) {
  hipError_t e = set_one<A, ST, TOPO_GLOBAL>(bytes);
  if (e == hipSuccess) e = set_one<A, ST, TOPO_LDS>(bytes);
  if (e == hipSuccess) e = set_one<A, ST, TOPO_QC>(bytes);
  return e;
}

// VGPRs per lane of one kernel variant (0 if the runtime cannot tell), cached per variant
template <class A, int ST, bool LMD>
static const void* kernel_of(int topo, bool mf) {
  if (topo == TOPO_QC) return mf ? (const void*)k_dynamic<A, ST, TOPO_QC, true, LMD> : (const void*)k_dynamic<A, ST, TOPO_QC, false, LMD>;
  if (topo == TOPO_LDS) return mf ? (const void*)k_dynamic<A, ST, TOPO_LDS, true, LMD> : (const void*)k_dynamic<A, ST, TOPO_LDS, false, LMD>;
  return (const void*)k_dynamic<A, ST, TOPO_GLOBAL, false, LMD>;
}

template <class A, int ST>
static int vgprs_of(int topo, bool mf, bool lmd) {
  const void* f = lmd ? kernel_of<A, ST, true>(topo, mf) : kernel_of<A, ST, false>(topo, mf);
  hipFuncAttributes at{};
  if (hipFuncGetAttributes(&at, f) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return at.numRegs;
}

template <class A>
static int vgprs_s(int store, int topo, bool mf, bool lmd) {
  switch (store) {
    case STORE_LDS: return vgprs_of<A, STORE_LDS>(topo, mf, lmd);
    case STORE_PRE_GLOBAL: return vgprs_of<A, STORE_PRE_GLOBAL>(topo, mf, lmd);
    case STORE_ALL_GLOBAL: return vgprs_of<A, STORE_ALL_GLOBAL>(topo, mf, lmd);
    case STORE_ALL_GLOBAL_LT: return vgprs_of<A, STORE_ALL_GLOBAL_LT>(topo, mf, lmd);
    case STORE_FRAME_GLOBAL: return vgprs_of<A, STORE_FRAME_GLOBAL>(topo, mf, lmd);
    case STORE_FRAME_REC: return vgprs_of<A, STORE_FRAME_REC>(topo, mf, lmd);
    default: return vgprs_of<A, STORE_FRAME_ALL>(topo, mf, lmd);
  }
}

int dynamic_waves_per_simd(bool fixed, int store, int topo, bool mf, bool lmd) {
  static std::mutex mu;
  static std::map<int, int> cache;
  const int key = (((fixed ? 1 : 0) * kStores + store) * 8 + topo * 2 + (mf ? 1 : 0)) * 2 + (lmd ? 1 : 0);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const int regs = fixed ? vgprs_s<ArithFix>(store, topo, mf, lmd) : vgprs_s<ArithF32>(store, topo, mf, lmd);
  // 512 VGPRs per SIMD lane, allocated in granules of 8; at most 8 wavefronts per SIMD
  const int waves = regs > 0 ? std::max(1, std::min(8, 512 / ((regs + 7) / 8 * 8))) : 8;
  cache[key] = waves;
  return waves;
}

hipError_t set_dynamic_lds_limit(int bytes) {
  hipError_t e = hipSuccess;
  for (hipError_t r : {set_store<ArithF32, STORE_LDS>(bytes), set_store<ArithF32, STORE_PRE_GLOBAL>(bytes),
                       set_store<ArithF32, STORE_ALL_GLOBAL>(bytes), set_store<ArithF32, STORE_ALL_GLOBAL_LT>(bytes),
                       set_store<ArithF32, STORE_FRAME_GLOBAL>(bytes), set_store<ArithFix, STORE_LDS>(bytes),
                       set_store<ArithFix, STORE_PRE_GLOBAL>(bytes), set_store<ArithFix, STORE_ALL_GLOBAL>(bytes),
                       set_store<ArithFix, STORE_ALL_GLOBAL_LT>(bytes), set_store<ArithFix, STORE_FRAME_GLOBAL>(bytes),
                       set_store<ArithF32, STORE_FRAME_REC>(bytes), set_store<ArithFix, STORE_FRAME_REC>(bytes),
                       set_store<ArithF32, STORE_FRAME_ALL>(bytes), set_store<ArithFix, STORE_FRAME_ALL>(bytes)})
    if (r != hipSuccess && e == hipSuccess) e = r;
  return e;
}

}  // namespace ldpc
