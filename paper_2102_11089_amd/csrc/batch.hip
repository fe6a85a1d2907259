// Persistent batched decoding of uneven frames on gfx950: one launch, many codes (lengths, rates)
// and schedules (flooding, layered, RBP, CIRBP).
//
// Workers are single wavefronts.  Each pulls the next frame index from a device work queue
// (atomic counter), reads the frame's descriptor {code, schedule, gamma, cap, LLR offset, output
// offset}, loads the code's topology when it differs from the previous frame's, and decodes:
//   RBP / CIRBP     the single-edge per-frame body shared with the per-code kernel,
//   flooding        one lane per check: whole-row update from the previous V2C messages, then
//                   L_n = channel + sum of C2V (one lane per VN), syndrome from scratch,
//   layered         block rows in order, one lane per check of the layer (VN-disjoint rows).
// LDS is laid out for the largest code of the launch.  Descriptors are checked on the device:
// an unknown code or schedule or an offset outside the pools marks the frame with
// updates_used = -1 and skips it.
#include "dyn_frame.hpp"

namespace ldpc {

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// lanes of the wave exchange values through the frame's message store (LDS, or global memory)
template <int STORE>
__device__ __forceinline__ void store_sync() {
  if constexpr (STORE >= STORE_ALL_GLOBAL) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  wave_sync();
}

// flooding / layered for one wavefront: L and the C2V messages in the frame's store (LDS, the
// global slot, or the VN records)
template <class A, int STORE, class Topo>
__device__ __forceinline__ void wave_baseline_frame(const DevCode& H, const Topo& G, const A& ar, const DynParams& P,
                                                    const FrameStore<A, STORE>& ms, const FrameJob& J) {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  using val_t = typename A::val_t;
  using Acc = typename RowAccOf<A>::type;
  const int lane = threadIdx.x & (WAVE - 1);
  const int N = H.N, M = H.M, E = H.E;
  for (int n = lane; n < N; n += WAVE) ms.set_l(n, (llr_t)ar.channel(J.llr[n]));
  for (int e = lane; e < E; e += WAVE) ms.set_c(e, (msg_t)0);
  store_sync<STORE>();
  auto syndrome = [&]() {
    int u = 0;
    for (int m = lane; m < M; m += WAVE) {
      const int rs = G.row_start(m), dc = G.row_deg(m);
      int par = 0;
      for (int p = 0; p < dc; ++p) par ^= (val_t)ms.l(G.row_vn(m, rs, p)) < 0 ? 1 : 0;
      u += par;
    }
    return wave_sum_i32(u);
  };
  int unsat = syndrome();
  long long t = 0, it = 0;
  while (!(unsat == 0 && J.check_every > 0) && t + E <= J.max_updates) {
    if (J.kind == KIND_FLOODING) {
      for (int m = lane; m < M; m += WAVE) {
        const int rs = G.row_start(m), dc = G.row_deg(m);
        Acc acc;
        for (int p = 0; p < dc; ++p) {
          const val_t v = ar.vin(ar.v2c((val_t)ms.l(G.row_vn(m, rs, p)), (val_t)ms.c(rs + p)));
          acc.add(p, v, row_aux(ar, v));
        }
        for (int p = 0; p < dc; ++p) {
          const val_t v = ar.vin(ar.v2c((val_t)ms.l(G.row_vn(m, rs, p)), (val_t)ms.c(rs + p)));
          ms.set_c(rs + p, (msg_t)acc.out(p, v, row_aux(ar, v)));
        }
      }
      store_sync<STORE>();
      for (int n = lane; n < N; n += WAVE) {
        val_t l = ar.channel(J.llr[n]);
        const int dv = G.vn_deg(n);
        for (int k = 0; k < dv; ++k) {
          int m, e;
          G.vn_edge(n, k, m, e);
          l += (val_t)ms.c(e);
        }
        ms.set_l(n, (llr_t)l);
      }
      store_sync<STORE>();
    } else {
      for (int l = 0; l < H.n_layers; ++l) {
        const int r0 = H.layer_ptr[l], r1 = H.layer_ptr[l + 1];
        for (int m = r0 + lane; m < r1; m += WAVE) {
          const int rs = G.row_start(m), dc = G.row_deg(m);
          Acc acc;
          for (int p = 0; p < dc; ++p) {
            const int j = G.row_vn(m, rs, p);
            const val_t v = ar.vin((val_t)ms.l(j) - (val_t)ms.c(rs + p));
            acc.add(p, v, row_aux(ar, v));
          }
          for (int p = 0; p < dc; ++p) {
            const int j = G.row_vn(m, rs, p);
            const val_t vr = (val_t)ms.l(j) - (val_t)ms.c(rs + p);
            const val_t v = ar.vin(vr);
            const val_t o = acc.out(p, v, row_aux(ar, v));
            ms.set_c(rs + p, (msg_t)o);
            ms.set_l(j, (llr_t)(vr + o));
          }
        }
        store_sync<STORE>();
      }
    }
    t += E;
    it += 1;
    unsat = syndrome();
  }
  for (int n = lane; n < N; n += WAVE) {
    const val_t l = (val_t)ms.l(n);
    J.bits[n] = l < 0 ? 1 : 0;
    if (J.llr_out) J.llr_out[n] = ar.out_llr(l);
  }
  if (lane == 0) {
    *J.updates_used = t;
    if (J.steps_used) *J.steps_used = it;
    if (J.fallbacks) *J.fallbacks = 0;
  }
  store_sync<STORE>();
}

template <class A, int STORE, int TOPO>
__global__ __launch_bounds__(WAVE) void k_batch(BatchParams B) {
  const DynParams& P = B.P;
  unsigned char* lds = dyn_lds();
  const int lane = threadIdx.x;
  const auto ms = make_store<A, STORE>(P, (size_t)B.max_E);
  int* lut = reinterpret_cast<int*>(lds + P.off_lut);
  A ar;
  ar.qmax = P.qmax;
  ar.scale = P.scale;
  ar.lut = lut;
  if constexpr (A::kFixed) {
    for (int x = lane; x < 257; x += WAVE) lut[x] = P.lut_global[x];
  }
  int cur = -1;
  typename TopoSel<TOPO>::type G{};
  while (true) {
    int aborted = 0;
    const int f = next_frame(B.queue, B.abort, lane, aborted);
    if (f >= B.F) break;
    const BatchFrame d = B.frames[f];
    const bool kind_ok = d.kind == KIND_FLOODING || d.kind == KIND_LAYERED || d.kind == KIND_RBP || d.kind == KIND_CIRBP ||
                         is_lmd(d.kind);
    bool ok = d.code >= 0 && d.code < B.n_codes && kind_ok && d.max_updates >= 0 && d.llr_off >= 0 &&
              d.out_off >= 0 && d.gamma >= 0.0f;
    const DevCode& H = *B.codes[ok ? d.code : 0];
    ok = ok && d.llr_off + H.N <= B.llr_len && d.out_off + H.N <= B.out_len;
    if (!ok || aborted) {  // malformed, or not started because the abort flag was set
      if (lane == 0) {
        B.updates_used[f] = -1;
        if (B.steps_used) B.steps_used[f] = 0;
      }
      continue;
    }
    if (d.code != cur) {  // topology of a new code
      wave_sync();
      G = TopoSel<TOPO>::make(H, lds + P.off_topo, lane, WAVE);
      cur = d.code;
      wave_sync();
    }
    FrameJob J;
    J.kind = d.kind;
    if constexpr (A::kFixed) {
      // gamma_q = round_half_away(gamma * 65534) in double, as for the per-code launch (the
      // product of a float and 65534 is exact in double; gamma >= 0 here)
      const double g = floor((double)d.gamma * 65534.0 + 0.5);
      J.gamma_bits = g >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)g;
    } else {
      J.gamma_bits = __float_as_uint(d.gamma);
    }
    J.max_updates = d.max_updates;
    J.check_every = P.check_every;
    J.llr = B.llr_pool + d.llr_off;
    J.replay = nullptr;
    J.replay_len = 0;
    J.bits = B.bits_pool + d.out_off;
    J.llr_out = B.llr_out_pool ? B.llr_out_pool + d.out_off : nullptr;
    J.updates_used = B.updates_used + f;
    J.steps_used = B.steps_used ? B.steps_used + f : nullptr;
    J.fallbacks = B.fallbacks ? B.fallbacks + f : nullptr;
    J.trace = nullptr;
    J.dump_c2v = J.dump_pre = J.dump_L = J.dump_Lt = J.dump_D = nullptr;
    if (d.kind == KIND_FLOODING || d.kind == KIND_LAYERED) wave_baseline_frame<A, STORE>(H, G, ar, P, ms, J);
    else if (is_lmd(d.kind)) dyn_decode_frame<A, STORE, decltype(G), true>(H, G, ar, P, ms, J);
    else dyn_decode_frame<A, STORE>(H, G, ar, P, ms, J);
  }
}

template <class A, int ST, int TP>
static hipError_t launch_batch_k(const BatchParams& B, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, B.queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch<A, ST, TP>), dim3(grid), dim3(WAVE), B.P.lds_bytes, st, B);
  return hipGetLastError();
}

template <class A, int ST>
static hipError_t launch_batch_t(const BatchParams& B, int topo, int grid, hipStream_t st) {
  return topo == TOPO_QC ? launch_batch_k<A, ST, TOPO_QC>(B, grid, st) : launch_batch_k<A, ST, TOPO_GLOBAL>(B, grid, st);
}

template <class A>
static hipError_t launch_batch_s(const BatchParams& B, int store, int topo, int grid, hipStream_t st) {
  if (store == STORE_FRAME_REC) return launch_batch_t<A, STORE_FRAME_REC>(B, topo, grid, st);
  if (store == STORE_FRAME_GLOBAL) return launch_batch_t<A, STORE_FRAME_GLOBAL>(B, topo, grid, st);
  if (store == STORE_ALL_GLOBAL_LT) return launch_batch_t<A, STORE_ALL_GLOBAL_LT>(B, topo, grid, st);
  if (store == STORE_ALL_GLOBAL) return launch_batch_t<A, STORE_ALL_GLOBAL>(B, topo, grid, st);
  if (store == STORE_PRE_GLOBAL) return launch_batch_t<A, STORE_PRE_GLOBAL>(B, topo, grid, st);
  return launch_batch_t<A, STORE_LDS>(B, topo, grid, st);
}

hipError_t launch_batch(const BatchParams& B, bool fixed, int store, int topo, int grid, hipStream_t st) {
  return fixed ? launch_batch_s<ArithFix>(B, store, topo, grid, st) : launch_batch_s<ArithF32>(B, store, topo, grid, st);
}

template <class A, int ST, int TP>
static hipError_t set_batch_one(int bytes) {
  return hipFuncSetAttribute((const void*)k_batch<A, ST, TP>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <class A, int ST>
static hipError_t set_batch_store(int bytes) {
  hipError_t e = set_batch_one<A, ST, TOPO_GLOBAL>(bytes);
  if (e == hipSuccess) e = set_batch_one<A, ST, TOPO_QC>(bytes);
  return e;
}

hipError_t set_batch_lds_limit(int bytes) {
  hipError_t e = hipSuccess;
  for (hipError_t r : {set_batch_store<ArithF32, STORE_LDS>(bytes), set_batch_store<ArithF32, STORE_PRE_GLOBAL>(bytes),
                       set_batch_store<ArithF32, STORE_ALL_GLOBAL>(bytes),
                       set_batch_store<ArithF32, STORE_ALL_GLOBAL_LT>(bytes),
                       set_batch_store<ArithF32, STORE_FRAME_GLOBAL>(bytes), set_batch_store<ArithFix, STORE_LDS>(bytes),
                       set_batch_store<ArithFix, STORE_PRE_GLOBAL>(bytes),
                       set_batch_store<ArithFix, STORE_ALL_GLOBAL>(bytes),
                       set_batch_store<ArithFix, STORE_ALL_GLOBAL_LT>(bytes),
                       set_batch_store<ArithFix, STORE_FRAME_GLOBAL>(bytes),
                       set_batch_store<ArithF32, STORE_FRAME_REC>(bytes), set_batch_store<ArithFix, STORE_FRAME_REC>(bytes)})
    if (r != hipSuccess && e == hipSuccess) e = r;
  return e;
}

}  // namespace ldpc
