// Flooding and layered BP baselines (Sec. I) on gfx950.
//
// One workgroup decodes one codeword at a time with c2v[E] and L[N] in LDS.
//   flooding  per iteration: V2C of every edge into vbuf[E]; every check output from vbuf
//             (leave-one-out fold, one lane per edge) into c2v; L_n = channel + sum of c2v
//             (one lane per VN, gathering over the VN's edges in ascending check order).
//   layered   per layer (consecutive VN-disjoint rows; a quasi-cyclic block row), one lane per
//             edge of the layer: v = L - c2v (unsaturated), new outputs from sat(v), L = v + c2v.
// The syndrome is maintained by toggling check bits whenever a hard decision flips, and tested
// after every iteration.  An iteration counts E updates (Sec. II-A); only whole iterations run.
#include "common.hpp"
#include "kernels.hpp"

namespace ldpc {

template <class A>
__device__ __forceinline__ void flip_checks(const DevCode& H, int n, uint32_t* synw, int* unsat) {
  for (int k = H.col_ptr[n]; k < H.col_ptr[n + 1]; ++k) {
    int m = H.col_row[k];
    uint32_t bit = 1u << (m & 31);
    uint32_t old = atomicXor(&synw[m >> 5], bit);
    atomicAdd(unsat, (old & bit) ? -1 : 1);
  }
}

template <class A>
__global__ __launch_bounds__(1024) void k_baseline(DevCode H, BaseParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  using val_t = typename A::val_t;
  const int tid = threadIdx.x, BS = blockDim.x;
  msg_t* c2v = reinterpret_cast<msg_t*>(lds + P.off_c2v);
  llr_t* L = reinterpret_cast<llr_t*>(lds + P.off_L);
  val_t* vbuf = reinterpret_cast<val_t*>(lds + P.off_ch);
  uint32_t* synw = reinterpret_cast<uint32_t*>(lds + P.off_syn);
  int* misc = reinterpret_cast<int*>(lds + P.off_misc);  // [0] unsat
  A ar;
  ar.qmax = P.qmax;
  ar.scale = P.scale;
  ar.lut = nullptr;
  const int N = H.N, M = H.M, E = H.E;
  const int nsw = (M + 31) >> 5;

  for (int f = blockIdx.x; f < P.B; f += gridDim.x) {
    const float* llr = P.llr + (size_t)f * N;
    for (int n = tid; n < N; n += BS) L[n] = (llr_t)ar.channel(llr[n]);
    for (int e = tid; e < E; e += BS) c2v[e] = (msg_t)0;
    for (int w = tid; w < nsw; w += BS) synw[w] = 0u;
    if (tid == 0) misc[0] = 0;
    __syncthreads();
    for (int m = tid; m < M; m += BS) {
      int par = 0;
      for (int e = H.row_ptr[m]; e < H.row_ptr[m + 1]; ++e) par ^= ((val_t)L[H.col[e]] < 0) ? 1 : 0;
      if (par) {
        atomicOr(&synw[m >> 5], 1u << (m & 31));
        atomicAdd(&misc[0], 1);
      }
    }
    __syncthreads();
    long long t = 0, it = 0;
    int unsat = misc[0];
    while (!(unsat == 0 && P.check_every > 0) && t + E <= P.max_updates) {
      if (P.kind == KIND_FLOODING) {
        for (int e = tid; e < E; e += BS) vbuf[e] = ar.v2c((val_t)L[H.col[e]], (val_t)c2v[e]);
        __syncthreads();
        for (int e = tid; e < E; e += BS) {
          int m = H.row_of[e];
          int rs = H.row_ptr[m], re = H.row_ptr[m + 1];
          bool first = true;
          val_t acc = 0;
          for (int k = rs; k < re; ++k) {
            if (k == e) continue;
            val_t v = ar.vin(vbuf[k]);
            acc = first ? v : ar.op(acc, v);
            first = false;
          }
          c2v[e] = (msg_t)acc;
        }
        __syncthreads();
        for (int n = tid; n < N; n += BS) {
          val_t l = ar.channel(llr[n]);
          for (int k = H.col_ptr[n]; k < H.col_ptr[n + 1]; ++k) l += (val_t)c2v[H.col_eid[k]];
          val_t old = (val_t)L[n];
          L[n] = (llr_t)l;
          if ((old < 0) != (l < 0)) flip_checks<A>(H, n, synw, &misc[0]);
        }
        __syncthreads();
      } else {
        for (int l = 0; l < H.n_layers; ++l) {
          const int r0 = H.layer_ptr[l], r1 = H.layer_ptr[l + 1];
          const int e0 = H.row_ptr[r0], e1 = H.row_ptr[r1];
          for (int e = e0 + tid; e < e1; e += BS) vbuf[e - e0] = (val_t)L[H.col[e]] - (val_t)c2v[e];
          __syncthreads();
          for (int e = e0 + tid; e < e1; e += BS) {
            int m = H.row_of[e];
            int rs = H.row_ptr[m], re = H.row_ptr[m + 1];
            bool first = true;
            val_t acc = 0;
            for (int k = rs; k < re; ++k) {
              if (k == e) continue;
              val_t v = ar.vin(vbuf[k - e0]);
              acc = first ? v : ar.op(acc, v);
              first = false;
            }
            int n = H.col[e];
            val_t old = (val_t)L[n];
            val_t nl = vbuf[e - e0] + acc;
            c2v[e] = (msg_t)acc;
            L[n] = (llr_t)nl;
            if ((old < 0) != (nl < 0)) flip_checks<A>(H, n, synw, &misc[0]);
          }
          __syncthreads();
        }
      }
      t += E;
      it += 1;
      unsat = misc[0];
      __syncthreads();
    }
    for (int n = tid; n < N; n += BS) {
      val_t l = (val_t)L[n];
      P.out.bits[(size_t)f * N + n] = l < 0 ? 1 : 0;
      if (P.out.llr_out) P.out.llr_out[(size_t)f * N + n] = ar.out_llr(l);
      if (P.out.dump_L) P.out.dump_L[(size_t)f * N + n] = ar.as_float(l);
    }
    for (int e = tid; e < E; e += BS)
      if (P.out.dump_c2v) P.out.dump_c2v[(size_t)f * E + e] = ar.as_float((val_t)c2v[e]);
    if (tid == 0) {
      P.out.updates_used[f] = t;
      if (P.out.steps_used) P.out.steps_used[f] = it;
      if (P.out.fallbacks) P.out.fallbacks[f] = 0;
    }
    __syncthreads();
  }
}

hipError_t launch_baseline(const DevCode& H, const BaseParams& P, bool fixed, int grid, int block,
                           hipStream_t st) {
  if (fixed) hipLaunchKernelGGL(k_baseline<ArithFix>, dim3(grid), dim3(block), P.lds_bytes, st, H, P);
  else hipLaunchKernelGGL(k_baseline<ArithF32>, dim3(grid), dim3(block), P.lds_bytes, st, H, P);
  return hipGetLastError();
}

hipError_t set_baseline_lds_limit(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_baseline<ArithF32>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_baseline<ArithFix>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace ldpc
