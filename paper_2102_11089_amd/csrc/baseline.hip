// Flooding and layered BP baselines (Sec. I) on gfx950.
//
// The check rule runs in its O(d_c) row form: a row's inputs are read once, and every output comes
// from row totals -- sum-product: Gallager's phi-sum, with the sum that leaves out the row's
// smallest input kept apart (RowAccF32); min-sum: sign parity and the two smallest magnitudes
// (RowAccFix, exactly the oracle's leave-one-out fold).  A row's inputs and their phi values stay in
// registers between the totals and the outputs (rows of up to kRegDc edges; the rest of a longer
// row is read and evaluated again).
//
// Edge slots.  C2V messages are stored in slot order: for a quasi-cyclic code the rows r = 0..Z-1
// of base row i are interleaved position by position (the p-th block of row (i, r) is slot
// Z bptr[i] + p Z + r), so that lanes working on consecutive rows of one base row, or on the
// consecutive VNs of one base column, touch consecutive words; for a CSR code the slot is the
// canonical edge id.
//
// flooding (k_flood): one workgroup decodes one frame at a time, with c2v, L and the channel
//   values in LDS.  An iteration: every row computes its new C2V messages from the V2C inputs
//   L - c2v of the previous iteration; then every VN sums L = channel + sum of C2V in ascending
//   check order, and a VN whose hard decision flipped toggles the syndrome bits of its checks.
//   Quasi-cyclic rows go to wavefronts by base row (lane = row of the base row), CSR rows in runs
//   of 64.
// layered (k_layered): one wavefront decodes one frame; the frames of a workgroup share its LDS
//   copy of the topology.  L is in LDS; c2v in LDS or, for large codes, in a global slot per frame.
//   Layers (the base rows of a quasi-cyclic code, else the code's layer partition) in order, one
//   lane per row: v = L - c2v (unsaturated), new C2V from the row's inputs sat(v), L = v + C2V.
// The syndrome is tested at t = 0 and after every iteration; an iteration counts E updates
// (Sec. II-A) and only whole iterations run.
#include "common.hpp"
#include "kernels.hpp"

namespace ldpc {

constexpr int kRegDc = 24;  // row inputs kept in registers

// A check row as the baseline kernels see it: its degree, the slot of its p-th edge and that edge's
// VN, for a quasi-cyclic base row (Topo = TopoQC) or a CSR row.
template <class Topo>
struct BaseRow;

template <>
struct BaseRow<TopoQC> {
  const TopoQC* G;
  int base, Z, r, dc, slot0;
  __device__ __forceinline__ BaseRow(const TopoQC& g, int i, int rr) : G(&g) {
    Z = g.Z;
    r = rr;
    base = g.bptr[i];
    dc = g.bdeg[i];
    slot0 = Z * base + r;
  }
  __device__ __forceinline__ int slot(int p) const { return slot0 + p * Z; }
  __device__ __forceinline__ int vn(int p) const {
    const int x = (base + p) * 2;
    int c = r + G->brow[x + 1];
    if (c >= Z) c -= Z;
    return G->brow[x] * Z + c;
  }
  // canonical edge id of the p-th edge (dumps)
  __device__ __forceinline__ int edge(int p) const { return Z * base + r * dc + p; }
};

template <>
struct BaseRow<TopoCSR> {
  const TopoCSR* G;
  int rs, dc;
  __device__ __forceinline__ BaseRow(const TopoCSR& g, int m) : G(&g) {
    rs = g.row_ptr[m];
    dc = g.row_ptr[m + 1] - rs;
  }
  __device__ __forceinline__ int slot(int p) const { return rs + p; }
  __device__ __forceinline__ int vn(int p) const { return G->col[rs + p]; }
  __device__ __forceinline__ int edge(int p) const { return rs + p; }
};

// slot of the k-th edge of VN n (ascending check order) and its check
__device__ __forceinline__ void vn_slot(const TopoQC& G, int n, int k, int& m, int& s) {
  const int j = G.zdiv.div(n), c = n - j * G.Z;
  const int x = (G.bcol_ptr[j] + k) * 4;
  const int i = G.bcol[x], sh = G.bcol[x + 1], rank = G.bcol[x + 2];
  int r = c - sh;
  if (r < 0) r += G.Z;
  m = i * G.Z + r;
  s = G.Z * (G.bptr[i] + rank) + r;
}
__device__ __forceinline__ void vn_slot(const TopoCSR& G, int n, int k, int& m, int& s) {
  const int x = G.col_ptr[n] + k;
  m = G.col_row[x];
  s = G.col_eid[x];
}

// New C2V messages of one row (eq. (2) for all its edges at once).  in(p) gives the row's p-th
// V2C value before the check input's saturation (vin); out(p, o, x) receives the p-th output o with
// that value x.
template <class A, class In, class Out>
__device__ __forceinline__ void row_outputs(const A& ar, int dc, In in, Out out) {
  using val_t = typename A::val_t;
  using Acc = typename RowAccOf<A>::type;
  Acc acc;
  val_t xx[kRegDc];
  float ph[kRegDc];
#pragma unroll
  for (int p = 0; p < kRegDc; ++p) {
    if (p < dc) {
      xx[p] = in(p);
      const val_t v = ar.vin(xx[p]);
      ph[p] = row_aux(ar, v);
      acc.add(p, v, ph[p]);
    }
  }
  for (int p = kRegDc; p < dc; ++p) {
    const val_t v = ar.vin(in(p));
    acc.add(p, v, row_aux(ar, v));
  }
#pragma unroll
  for (int p = 0; p < kRegDc; ++p)
    if (p < dc) out(p, acc.out(p, ar.vin(xx[p]), ph[p]), xx[p]);
  for (int p = kRegDc; p < dc; ++p) {
    const val_t x = in(p);
    const val_t v = ar.vin(x);
    out(p, acc.out(p, v, row_aux(ar, v)), x);
  }
}

// ------------------------------------------------------------------------------------------
// flooding: one frame per workgroup, state in LDS
// ------------------------------------------------------------------------------------------
template <class A, int TOPO>
__global__ __launch_bounds__(1024) void k_flood(DevCode H, BaseParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  using val_t = typename A::val_t;
  const int tid = threadIdx.x, BS = blockDim.x;
  const int lane = tid & (WAVE - 1), wid = tid >> 6, nw = BS >> 6;
  msg_t* c2v = reinterpret_cast<msg_t*>(lds + P.off_c2v);
  llr_t* L = reinterpret_cast<llr_t*>(lds + P.off_L);
  val_t* ch = reinterpret_cast<val_t*>(lds + P.off_ch);
  uint32_t* synw = reinterpret_cast<uint32_t*>(lds + P.off_syn);
  // [0] unsatisfied checks, [1] row counter, [2] the abort flag as read for the workgroup
  int* misc = reinterpret_cast<int*>(lds + P.off_misc);
  A ar;
  ar.qmax = P.qmax;
  ar.scale = P.scale;
  ar.lut = nullptr;
  const auto G = TopoSel<TOPO>::make(H, lds + P.off_topo, tid, BS);
  const int N = H.N, M = H.M, E = H.E;
  const int nsw = (M + 31) >> 5;
  constexpr bool kQC = TOPO == TOPO_QC;
  const int Z = kQC ? H.qc.Z : 1;
  const int mb = kQC ? H.qc.mb : 0;

  // rows of this thread: quasi-cyclic: base rows wid, wid + nw, ..., rows r = lane, lane + 64, ...;
  // CSR: runs of 64 rows
  auto for_rows = [&](auto fn) {
    if constexpr (kQC) {
      for (int i = wid; i < mb; i += nw)
        for (int r = lane; r < Z; r += WAVE) fn(BaseRow<TopoQC>(G, i, r), i * Z + r);
    } else {
      for (int m = tid; m < M; m += BS) fn(BaseRow<TopoCSR>(G, m), m);
    }
  };

  for (int f = blockIdx.x; f < P.B; f += gridDim.x) {
    const float* llr = P.llr + (size_t)f * N;
    __syncthreads();  // the previous frame's outputs are read
    if (tid == 0) misc[2] = abort_flag_value(P.out.abort);
    __syncthreads();
    if (misc[2] != 0) {  // not started: the abort flag was set
      if (tid == 0) P.out.updates_used[f] = -1;
      continue;
    }
    for (int n = tid; n < N; n += BS) {
      const val_t x = ar.channel(llr[n]);
      ch[n] = x;
      L[n] = (llr_t)x;
    }
    for (int e = tid; e < E; e += BS) c2v[e] = (msg_t)0;
    for (int w = tid; w < nsw; w += BS) synw[w] = 0u;
    if (tid == 0) {
      misc[0] = 0;  // unsatisfied checks
      misc[1] = 0;  // next base row of the row phase
    }
    __syncthreads();
    {  // syndrome of the channel hard decisions
      int u = 0;
      for_rows([&](const auto& row, int m) {
        int par = 0;
        for (int p = 0; p < row.dc; ++p) par ^= (val_t)L[row.vn(p)] < 0 ? 1 : 0;
        if (par) atomicOr(&synw[m >> 5], 1u << (m & 31));
        u += par;
      });
      u = wave_sum_i32(u);
      if (lane == 0 && u) atomicAdd(&misc[0], u);
    }
    __syncthreads();
    long long t = 0, it = 0;
    int unsat = misc[0];
    while (!(unsat == 0 && P.check_every > 0) && t + E <= P.max_updates) {
      // every row: new C2V from the previous iteration's V2C messages.  Quasi-cyclic base rows are
      // taken from a counter in descending degree order, so that wavefronts stay balanced
      auto row_update = [&](const auto& row) {
        row_outputs(
            ar, row.dc, [&](int p) { return ar.v2c((val_t)L[row.vn(p)], (val_t)c2v[row.slot(p)]); },
            [&](int p, val_t o, val_t) { c2v[row.slot(p)] = (msg_t)o; });
      };
      if constexpr (kQC) {
        while (true) {
          const int k = __builtin_amdgcn_readfirstlane(lane == 0 ? atomicAdd(&misc[1], 1) : 0);
          if (k >= mb) break;
          const int i = G.border[k];
          for (int r = lane; r < Z; r += WAVE) row_update(BaseRow<TopoQC>(G, i, r));
        }
      } else {
        for (int m = tid; m < M; m += BS) row_update(BaseRow<TopoCSR>(G, m));
      }
      __syncthreads();
      if (tid == 0) misc[1] = 0;  // read again only after the barrier that ends this iteration
      // every VN: L = channel + sum of C2V (ascending checks); flips toggle the syndrome
      int du = 0;
      for (int n = tid; n < N; n += BS) {
        val_t l = ch[n];
        const int dv = G.vn_deg(n);
        for (int k = 0; k < dv; ++k) {
          int m, s;
          vn_slot(G, n, k, m, s);
          l += (val_t)c2v[s];
        }
        const val_t old = (val_t)L[n];
        L[n] = (llr_t)l;
        if ((old < 0) != (l < 0)) {
          for (int k = 0; k < dv; ++k) {
            int m, s;
            vn_slot(G, n, k, m, s);
            const uint32_t bit = 1u << (m & 31);
            const uint32_t o = atomicXor(&synw[m >> 5], bit);
            du += (o & bit) ? -1 : 1;
          }
        }
      }
      du = wave_sum_i32(du);
      if (lane == 0 && du) atomicAdd(&misc[0], du);
      __syncthreads();
      t += E;
      it += 1;
      unsat = misc[0];
    }
    for (int n = tid; n < N; n += BS) {
      const val_t l = (val_t)L[n];
      P.out.bits[(size_t)f * N + n] = l < 0 ? 1 : 0;
      if (P.out.llr_out) P.out.llr_out[(size_t)f * N + n] = ar.out_llr(l);
      if (P.out.dump_L) P.out.dump_L[(size_t)f * N + n] = ar.as_float(l);
    }
    if (P.out.dump_c2v) {
      for_rows([&](const auto& row, int) {
        for (int p = 0; p < row.dc; ++p)
          P.out.dump_c2v[(size_t)f * E + row.edge(p)] = ar.as_float((val_t)c2v[row.slot(p)]);
      });
    }
    if (tid == 0) {
      P.out.updates_used[f] = t;
      if (P.out.steps_used) P.out.steps_used[f] = it;
      if (P.out.fallbacks) P.out.fallbacks[f] = 0;
    }
  }
}

// ------------------------------------------------------------------------------------------
// layered: one frame per wavefront
// ------------------------------------------------------------------------------------------
template <class A, int TOPO, bool C2V_GLOBAL>
__global__ __launch_bounds__(1024) void k_layered(DevCode H, BaseParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  using val_t = typename A::val_t;
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  A ar;
  ar.qmax = P.qmax;
  ar.scale = P.scale;
  ar.lut = nullptr;
  const auto G = TopoSel<TOPO>::make(H, lds + P.off_topo, threadIdx.x, blockDim.x);
  __syncthreads();  // the only workgroup barrier: the frames below run independently
  unsigned char* fl = lds + P.frame_base + w * P.frame_stride;
  llr_t* L = reinterpret_cast<llr_t*>(fl + P.off_L);
  uint32_t* synw = reinterpret_cast<uint32_t*>(fl + P.off_syn);
  const size_t wslot = (size_t)blockIdx.x * (size_t)P.wpb + (size_t)w;
  msg_t* c2v = C2V_GLOBAL ? reinterpret_cast<msg_t*>(P.c2v_global) + wslot * (size_t)P.slot_edges
                          : reinterpret_cast<msg_t*>(fl + P.off_c2v);
  const int N = H.N, M = H.M, E = H.E;
  const int nsw = (M + 31) >> 5;
  constexpr bool kQC = TOPO == TOPO_QC;
  const int Z = kQC ? H.qc.Z : 1;
  const int nl = kQC ? H.qc.mb : H.n_layers;

  int aborted = 0;
  int f = next_frame(P.queue, P.out.abort, lane, aborted);
  while (f < P.B) {
    if (aborted) {
      if (lane == 0) P.out.updates_used[f] = -1;  // not started: the abort flag was set
      f = next_frame(P.queue, P.out.abort, lane, aborted);
      continue;
    }
    const float* llr = P.llr + (size_t)f * N;
    for (int n = lane; n < N; n += WAVE) L[n] = (llr_t)ar.channel(llr[n]);
    for (int e = lane; e < E; e += WAVE) c2v[e] = (msg_t)0;
    for (int x = lane; x < nsw; x += WAVE) synw[x] = 0u;
    wave_sync();
    int unsat = 0;
    {
      int u = 0;
      for (int m = lane; m < M; m += WAVE) {
        int par = 0;
        if constexpr (kQC) {
          const int i = G.zdiv.div(m);
          const BaseRow<TopoQC> row(G, i, m - i * Z);
          for (int p = 0; p < row.dc; ++p) par ^= (val_t)L[row.vn(p)] < 0 ? 1 : 0;
        } else {
          const BaseRow<TopoCSR> row(G, m);
          for (int p = 0; p < row.dc; ++p) par ^= (val_t)L[row.vn(p)] < 0 ? 1 : 0;
        }
        if (par) atomicOr(&synw[m >> 5], 1u << (m & 31));
        u += par;
      }
      unsat = wave_sum_i32(u);
    }
    wave_sync();
    long long t = 0, it = 0;
    while (!(unsat == 0 && P.check_every > 0) && t + E <= P.max_updates) {
      int du = 0;
      for (int l = 0; l < nl; ++l) {
        auto one = [&](const auto& row) {
          uint64_t flipped = 0;  // positions p whose VN's hard decision flipped
          row_outputs(
              ar, row.dc, [&](int p) { return (val_t)L[row.vn(p)] - (val_t)c2v[row.slot(p)]; },
              [&](int p, val_t o, val_t vr) {  // vr = L - c2v, unsaturated
                const int j = row.vn(p);
                const val_t nl_ = vr + o;
                c2v[row.slot(p)] = (msg_t)o;
                if (((val_t)L[j] < 0) != (nl_ < 0)) {
                  if (p < 64) {
                    flipped |= 1ull << p;
                  } else {
                    const int dv = G.vn_deg(j);
                    for (int k = 0; k < dv; ++k) {
                      int m, s2;
                      vn_slot(G, j, k, m, s2);
                      const uint32_t bit = 1u << (m & 31);
                      const uint32_t old = atomicXor(&synw[m >> 5], bit);
                      du += (old & bit) ? -1 : 1;
                    }
                  }
                }
                L[j] = (llr_t)nl_;
              });
          while (flipped) {  // toggle the syndrome bits of the checks of every flipped VN
            const int p = __builtin_ctzll(flipped);
            flipped &= flipped - 1;
            const int j = row.vn(p), dv = G.vn_deg(j);
            for (int k = 0; k < dv; ++k) {
              int m, s2;
              vn_slot(G, j, k, m, s2);
              const uint32_t bit = 1u << (m & 31);
              const uint32_t old = atomicXor(&synw[m >> 5], bit);
              du += (old & bit) ? -1 : 1;
            }
          }
        };
        if constexpr (kQC) {
          for (int r = lane; r < Z; r += WAVE) one(BaseRow<TopoQC>(G, l, r));
        } else {
          const int r0 = H.layer_ptr[l], r1 = H.layer_ptr[l + 1];
          for (int m = r0 + lane; m < r1; m += WAVE) one(BaseRow<TopoCSR>(G, m));
        }
        wave_sync();
      }
      unsat += wave_sum_i32(du);
      t += E;
      it += 1;
    }
    for (int n = lane; n < N; n += WAVE) {
      const val_t l = (val_t)L[n];
      P.out.bits[(size_t)f * N + n] = l < 0 ? 1 : 0;
      if (P.out.llr_out) P.out.llr_out[(size_t)f * N + n] = ar.out_llr(l);
      if (P.out.dump_L) P.out.dump_L[(size_t)f * N + n] = ar.as_float(l);
    }
    if (P.out.dump_c2v) {
      for (int m = lane; m < M; m += WAVE) {
        if constexpr (kQC) {
          const int i = G.zdiv.div(m);
          const BaseRow<TopoQC> row(G, i, m - i * Z);
          for (int p = 0; p < row.dc; ++p) P.out.dump_c2v[(size_t)f * E + row.edge(p)] = ar.as_float((val_t)c2v[row.slot(p)]);
        } else {
          const BaseRow<TopoCSR> row(G, m);
          for (int p = 0; p < row.dc; ++p) P.out.dump_c2v[(size_t)f * E + row.edge(p)] = ar.as_float((val_t)c2v[row.slot(p)]);
        }
      }
    }
    if (lane == 0) {
      P.out.updates_used[f] = t;
      if (P.out.steps_used) P.out.steps_used[f] = it;
      if (P.out.fallbacks) P.out.fallbacks[f] = 0;
    }
    wave_sync();
    f = next_frame(P.queue, P.out.abort, lane, aborted);
  }
}

template <class A, int TP>
static hipError_t launch_base_t(const DevCode& H, const BaseParams& P, int grid, int block, hipStream_t st) {
  if (P.kind == KIND_FLOODING) {
    hipLaunchKernelGGL((k_flood<A, TP>), dim3(grid), dim3(block), P.lds_bytes, st, H, P);
  } else if (P.c2v_global) {
    hipLaunchKernelGGL((k_layered<A, TP, true>), dim3(grid), dim3(block), P.lds_bytes, st, H, P);
  } else {
    hipLaunchKernelGGL((k_layered<A, TP, false>), dim3(grid), dim3(block), P.lds_bytes, st, H, P);
  }
  return hipGetLastError();
}

template <class A>
static hipError_t launch_base_a(const DevCode& H, const BaseParams& P, int topo, int grid, int block,
                                hipStream_t st) {
  if (topo == TOPO_QC) return launch_base_t<A, TOPO_QC>(H, P, grid, block, st);
  if (topo == TOPO_LDS) return launch_base_t<A, TOPO_LDS>(H, P, grid, block, st);
  return launch_base_t<A, TOPO_GLOBAL>(H, P, grid, block, st);
}

hipError_t launch_baseline(const DevCode& H, const BaseParams& P, bool fixed, int topo, int grid, int block,
                           hipStream_t st) {
  return fixed ? launch_base_a<ArithFix>(H, P, topo, grid, block, st)
               : launch_base_a<ArithF32>(H, P, topo, grid, block, st);
}

template <class A, int TP>
static hipError_t set_base_t(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_flood<A, TP>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_layered<A, TP, true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_layered<A, TP, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

hipError_t set_baseline_lds_limit(int bytes) {
  hipError_t e = hipSuccess;
  for (hipError_t r : {set_base_t<ArithF32, TOPO_GLOBAL>(bytes), set_base_t<ArithF32, TOPO_LDS>(bytes),
                       set_base_t<ArithF32, TOPO_QC>(bytes), set_base_t<ArithFix, TOPO_GLOBAL>(bytes),
                       set_base_t<ArithFix, TOPO_LDS>(bytes), set_base_t<ArithFix, TOPO_QC>(bytes)})
    if (r != hipSuccess && e == hipSuccess) e = r;
  return e;
}

}  // namespace ldpc
