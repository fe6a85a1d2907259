// Multi-edge CIRBP on gfx950: Algorithm 4 (VN selection by CI groups) and Algorithm 5 (the
// selected VNs updated together), Sec. VI.
//
// One workgroup decodes one frame at a time.  Per step, on a snapshot of the state:
//   1. the CI-group histogram hist[N_G] (kept up to date as D changes) gives the groups taken
//      whole (the largest k with |Q(k)| <= N_P) and the fill group with the number still needed;
//   2. the selected set P: every VN of the taken groups, plus the fill -- the lowest VN indices
//      (block prefix count) or the smallest keys splitmix64(splitmix64(splitmix64(seed ^ frame)
//      ^ step) ^ n) (a key threshold shrunk until at most CAND candidates remain, then ranked);
//   3. for each p in P (ascending): the incoming edge of largest residual (Algorithm 1 line 8);
//   4. all propagations c2v <- pre, L_p += delta, syndrome toggles;
//   5. every check of every p recomputed from the new state (one lane per check, each check once),
//      Lt updated by the precompute deltas; then D (and its group) of every VN of those checks.
// Messages c2v/pre stay in LDS when they fit, otherwise in a global scratch slot per workgroup.
#include "common.hpp"
#include "kernels.hpp"

namespace ldpc {

__device__ __forceinline__ uint64_t me_fill_key(uint64_t seed, uint64_t frame, uint64_t step, uint64_t n) {
  return splitmix64(splitmix64(splitmix64(seed ^ frame) ^ step) ^ n);
}

enum { MS_UNSAT = 0, MS_NROWS, MS_NSEL, MS_BSTAR, MS_FILL, MS_NEED, MS_CNT, MS_NCAND, MS_WAVESUM };

// exclusive prefix sum over the workgroup (lane order); wsum: one int per wave in LDS
__device__ __forceinline__ int block_excl_scan(int v, int* wsum) {
  const int tid = threadIdx.x, w = tid >> 6, nw = (blockDim.x + 63) >> 6;
  const int ex = wave_excl_scan(v, tid & 63);
  if ((tid & 63) == 63) wsum[w] = ex + v;
  __syncthreads();
  int base = 0;
  for (int k = 0; k < w; ++k) base += wsum[k];
  __syncthreads();
  (void)nw;
  return base + ex;
}

template <class A, bool MSG_GLOBAL, int TOPO>
__global__ __launch_bounds__(1024) void k_me(DevCode H, MeParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  using val_t = typename A::val_t;
  using Acc = typename RowAccOf<A>::type;
  const int tid = threadIdx.x, BS = blockDim.x;
  const int N = H.N, M = H.M, E = H.E;

  msg_t *c2v, *pre;
  if constexpr (MSG_GLOBAL) {
    c2v = reinterpret_cast<msg_t*>(P.msg_global) + (size_t)blockIdx.x * 2 * (size_t)E;
    pre = c2v + E;
  } else {
    c2v = reinterpret_cast<msg_t*>(lds + P.off_c2v);
    pre = reinterpret_cast<msg_t*>(lds + P.off_pre);
  }
  llr_t* L = reinterpret_cast<llr_t*>(lds + P.off_L);
  llr_t* Lt = reinterpret_cast<llr_t*>(lds + P.off_Lt);
  uint32_t* D = reinterpret_cast<uint32_t*>(lds + P.off_D);
  int* hist = reinterpret_cast<int*>(lds + P.off_hist);
  uint32_t* synw = reinterpret_cast<uint32_t*>(lds + P.off_synw);
  uint32_t* rowmark = reinterpret_cast<uint32_t*>(lds + P.off_rowmark);
  uint32_t* vnmark = reinterpret_cast<uint32_t*>(lds + P.off_vnmark);
  int* rows = reinterpret_cast<int*>(lds + P.off_rows);
  int* sel = reinterpret_cast<int*>(lds + P.off_sel);  // [64] unsorted, [64] sorted, [64] edges
  int* sel_s = sel + 64;
  int* sel_e = sel + 128;
  uint64_t* ckeys = reinterpret_cast<uint64_t*>(lds + P.off_cand);
  int* cidx = reinterpret_cast<int*>(ckeys + P.cand_cap);
  int* misc = reinterpret_cast<int*>(lds + P.off_misc);
  int* wsum = misc + 16;
  int* lut = reinterpret_cast<int*>(lds + P.off_lut);

  A ar;
  ar.qmax = P.qmax;
  ar.scale = P.scale;
  ar.lut = lut;
  if constexpr (A::kFixed) {
    for (int x = tid; x < 257; x += BS) lut[x] = P.lut_global[x];
  }
  const auto G = TopoSel<TOPO>::make(H, lds + P.off_topo, tid, BS);
  const int NG = P.n_g, NP = P.n_p;
  const int nsw = (M + 31) >> 5, nvw = (N + 31) >> 5;
  __syncthreads();

  for (int f = blockIdx.x; f < P.B; f += gridDim.x) {
    // ---------------- Algorithm 5 lines 1-3 --------------------------------------------
    const float* llr = P.llr + (size_t)f * N;
    for (int n = tid; n < N; n += BS) L[n] = (llr_t)ar.channel(llr[n]);
    for (int e = tid; e < E; e += BS) c2v[e] = (msg_t)0;
    for (int b = tid; b < NG; b += BS) hist[b] = 0;
    for (int w = tid; w < nsw; w += BS) synw[w] = 0u, rowmark[w] = 0u;
    for (int w = tid; w < nvw; w += BS) vnmark[w] = 0u;
    if (tid < 16) misc[tid] = 0;
    __syncthreads();
    for (int m = tid; m < M; m += BS) {
      const int rs = G.row_start(m), dc = G.row_deg(m);
      Acc acc;
      int par = 0;
      for (int p = 0; p < dc; ++p) {
        const val_t l = (val_t)L[G.row_vn(m, rs, p)];
        const val_t v = ar.vin(l);
        acc.add(p, v, row_aux(ar, v));
        par ^= l < 0 ? 1 : 0;
      }
      for (int p = 0; p < dc; ++p) {
        const val_t v = ar.vin((val_t)L[G.row_vn(m, rs, p)]);
        pre[rs + p] = (msg_t)acc.out(p, v, row_aux(ar, v));
      }
      if (par) {
        atomicOr(&synw[m >> 5], 1u << (m & 31));
        atomicAdd(&misc[MS_UNSAT], 1);
      }
    }
    if constexpr (MSG_GLOBAL) __threadfence_block();
    __syncthreads();
    for (int n = tid; n < N; n += BS) {
      val_t lt = (val_t)L[n];
      const int dv = G.vn_deg(n);
      for (int k = 0; k < dv; ++k) {
        int m, e;
        G.vn_edge(n, k, m, e);
        lt += (val_t)pre[e];
      }
      Lt[n] = (llr_t)lt;
      const uint32_t d = ar.ci((val_t)L[n], lt);
      D[n] = d;
      atomicAdd(&hist[ar.bin(d, NG)], 1);
    }
    __syncthreads();

    long long t = 0, steps = 0;
    const long long ce = P.check_every;
    bool done = ce > 0 && misc[MS_UNSAT] == 0;
    while (!done && t + NP <= P.max_updates) {
      const long long tprev = t;
      // ---- Algorithm 4 line 3: groups taken whole, fill group, number still needed ----
      if (tid == 0) {
        int c = 0, bstar = NG;
        for (int b = NG - 1; b >= 0; --b) {
          if (c + hist[b] > NP) break;
          c += hist[b];
          bstar = b;
        }
        const int fill = bstar > 0 ? bstar - 1 : -1;
        misc[MS_BSTAR] = bstar;
        misc[MS_FILL] = fill;
        misc[MS_NEED] = fill >= 0 ? NP - c : 0;
        misc[MS_NSEL] = 0;
        misc[MS_CNT] = 0;
        misc[MS_NCAND] = 0;
      }
      __syncthreads();
      const int bstar = misc[MS_BSTAR], fill = misc[MS_FILL], need = misc[MS_NEED];
      // ---- the selected set: groups taken whole ----
      const int chunk = (N + BS - 1) / BS;
      const int n0 = tid * chunk, n1 = min(N, n0 + chunk);
      int nfill = 0;
      for (int n = n0; n < n1; ++n) {
        const int b = ar.bin(D[n], NG);
        if (b >= bstar) sel[atomicAdd(&misc[MS_NSEL], 1)] = n;
        nfill += b == fill ? 1 : 0;
      }
      // ---- Algorithm 4 lines 4-6: the fill ----
      if (need > 0) {
        if (P.fill == 0) {  // lowest indices: rank of each fill member in index order
          int rank = block_excl_scan(nfill, wsum);
          for (int n = n0; n < n1 && rank < need; ++n) {
            if (ar.bin(D[n], NG) == fill) {
              sel[atomicAdd(&misc[MS_NSEL], 1)] = n;
              ++rank;
            }
          }
        } else {  // smallest keys: shrink a key threshold until few candidates remain, rank them
          const int members = hist[fill];
          uint64_t lo = 0, hi = ~0ull, T;
          {
            const double frac = fmin(1.0, (2.0 * need + 16.0) / (double)max(members, 1));
            T = frac >= 1.0 ? ~0ull : (uint64_t)(frac * 18446744073709551615.0);
          }
          for (int it = 0; it < 96; ++it) {
            int cnt = 0;
            for (int n = n0; n < n1; ++n)
              if (ar.bin(D[n], NG) == fill && me_fill_key(P.seed, (uint64_t)f, (uint64_t)steps, (uint64_t)n) < T) ++cnt;
            if (cnt) atomicAdd(&misc[MS_CNT], cnt);
            __syncthreads();
            const int total = misc[MS_CNT];
            __syncthreads();
            if (tid == 0) misc[MS_CNT] = 0;
            if (total >= need && total <= P.cand_cap) break;
            if (T == ~0ull) break;  // every member below the threshold
            if (total < need) lo = T;
            else hi = T;
            T = hi == ~0ull ? (lo > (~0ull >> 1) ? ~0ull : lo * 2 + 1) : lo + (hi - lo) / 2;
            if (T == lo) T = lo + 1;
            __syncthreads();
          }
          for (int n = n0; n < n1; ++n) {
            if (ar.bin(D[n], NG) != fill) continue;
            const uint64_t k = me_fill_key(P.seed, (uint64_t)f, (uint64_t)steps, (uint64_t)n);
            if (k < T || T == ~0ull) {
              const int i = atomicAdd(&misc[MS_NCAND], 1);
              if (i < P.cand_cap) {
                ckeys[i] = k;
                cidx[i] = n;
              }
            }
          }
          __syncthreads();
          const int nc = min(misc[MS_NCAND], P.cand_cap);
          for (int i = tid; i < nc; i += BS) {
            const uint64_t ki = ckeys[i];
            const int ni = cidx[i];
            int r = 0;
            for (int j = 0; j < nc; ++j) r += (ckeys[j] < ki || (ckeys[j] == ki && cidx[j] < ni)) ? 1 : 0;
            if (r < need) sel[atomicAdd(&misc[MS_NSEL], 1)] = ni;
          }
        }
      }
      __syncthreads();
      const int nsel = misc[MS_NSEL];
      // ascending order of P (distinct VN indices: rank = number of smaller ones)
      if (tid < nsel) {
        const int v = sel[tid];
        int r = 0;
        for (int j = 0; j < nsel; ++j) r += sel[j] < v ? 1 : 0;
        sel_s[r] = v;
      }
      __syncthreads();
      // ---- Algorithm 1 line 8 for every p: incoming edge of largest residual (snapshot) ----
      if (tid < nsel) {
        const int p = sel_s[tid];
        const int dv = G.vn_deg(p);
        uint64_t best = 0;
        for (int k = 0; k < dv; ++k) {
          int m, e;
          G.vn_edge(p, k, m, e);
          best = umax64(best, mkkey(ar.res((val_t)pre[e], (val_t)c2v[e]), (uint32_t)e));
        }
        const int e = (int)key_idx(best);
        sel_e[tid] = e;
        if (P.out.trace) P.out.trace[(size_t)f * P.max_updates + tprev + tid] = e;
      }
      __syncthreads();
      // ---- propagations (Algorithm 1 line 9 for every p) ----
      if (tid < nsel) {
        const int p = sel_s[tid], e = sel_e[tid];
        const val_t newv = (val_t)pre[e], oldv = (val_t)c2v[e];
        c2v[e] = (msg_t)newv;
        const val_t Lold = (val_t)L[p];
        const val_t Lnew = Lold + (newv - oldv);
        L[p] = (llr_t)Lnew;
        const bool flip = (Lold < 0) != (Lnew < 0);
        const int dv = G.vn_deg(p);
        for (int k = 0; k < dv; ++k) {
          int m, e2;
          G.vn_edge(p, k, m, e2);
          const uint32_t bit = 1u << (m & 31);
          if (flip) {
            const uint32_t old = atomicXor(&synw[m >> 5], bit);
            atomicAdd(&misc[MS_UNSAT], (old & bit) ? -1 : 1);
          }
          const uint32_t om = atomicOr(&rowmark[m >> 5], bit);
          if (!(om & bit)) rows[atomicAdd(&misc[MS_NROWS], 1)] = m;
        }
      }
      if constexpr (MSG_GLOBAL) __threadfence_block();
      __syncthreads();
      const int nrows = misc[MS_NROWS];
      // ---- every check of every p from the new state (Algorithm 1 lines 10-13) ----
      for (int r = tid; r < nrows; r += BS) {
        const int m = rows[r];
        const int rs = G.row_start(m), dc = G.row_deg(m);
        Acc acc;
        for (int p = 0; p < dc; ++p) {
          const val_t v = ar.vin(ar.v2c((val_t)L[G.row_vn(m, rs, p)], (val_t)c2v[rs + p]));
          acc.add(p, v, row_aux(ar, v));
        }
        for (int p = 0; p < dc; ++p) {
          const int j = G.row_vn(m, rs, p);
          const val_t v = ar.vin(ar.v2c((val_t)L[j], (val_t)c2v[rs + p]));
          const val_t o = acc.out(p, v, row_aux(ar, v));
          const val_t old = (val_t)pre[rs + p];
          pre[rs + p] = (msg_t)o;
          if (o != old) atomicAdd(&Lt[j], (llr_t)(o - old));
        }
      }
      if constexpr (MSG_GLOBAL) __threadfence_block();
      __syncthreads();
      // ---- CI and CI group of every VN of those checks ----
      for (int r = tid; r < nrows; r += BS) {
        const int m = rows[r];
        const int rs = G.row_start(m), dc = G.row_deg(m);
        for (int p = 0; p < dc; ++p) {
          const int j = G.row_vn(m, rs, p);
          const uint32_t bit = 1u << (j & 31);
          if (atomicOr(&vnmark[j >> 5], bit) & bit) continue;
          const uint32_t nd = ar.ci((val_t)L[j], (val_t)Lt[j]);
          const uint32_t od = D[j];
          D[j] = nd;
          const int ob = ar.bin(od, NG), nb = ar.bin(nd, NG);
          if (ob != nb) {
            atomicSub(&hist[ob], 1);
            atomicAdd(&hist[nb], 1);
          }
        }
      }
      __syncthreads();
      for (int w = tid; w < nsw; w += BS) rowmark[w] = 0u;
      for (int w = tid; w < nvw; w += BS) vnmark[w] = 0u;
      const int unsat = misc[MS_UNSAT];
      __syncthreads();
      if (tid == 0) misc[MS_NROWS] = 0;
      t += nsel;
      steps += 1;
      if (ce > 0 && (t / ce) != (tprev / ce) && unsat == 0) done = true;
      __syncthreads();
    }

    // ---------------- outputs -----------------------------------------------------------
    for (int n = tid; n < N; n += BS) {
      const val_t l = (val_t)L[n];
      P.out.bits[(size_t)f * N + n] = l < 0 ? 1 : 0;
      if (P.out.llr_out) P.out.llr_out[(size_t)f * N + n] = ar.out_llr(l);
      if (P.out.dump_L) P.out.dump_L[(size_t)f * N + n] = ar.as_float(l);
      if (P.out.dump_Lt) P.out.dump_Lt[(size_t)f * N + n] = ar.as_float((val_t)Lt[n]);
      if (P.out.dump_D) P.out.dump_D[(size_t)f * N + n] = ar.d_float(D[n]);
    }
    for (int e = tid; e < E; e += BS) {
      if (P.out.dump_c2v) P.out.dump_c2v[(size_t)f * E + e] = ar.as_float((val_t)c2v[e]);
      if (P.out.dump_pre) P.out.dump_pre[(size_t)f * E + e] = ar.as_float((val_t)pre[e]);
    }
    if (tid == 0) {
      P.out.updates_used[f] = t;
      if (P.out.steps_used) P.out.steps_used[f] = steps;
      if (P.out.fallbacks) P.out.fallbacks[f] = 0;
    }
    __syncthreads();
  }
}

template <class A, bool MG, int TP>
static hipError_t launch_me_k(const DevCode& H, const MeParams& P, int grid, int block, hipStream_t st) {
  hipLaunchKernelGGL((k_me<A, MG, TP>), dim3(grid), dim3(block), P.lds_bytes, st, H, P);
  return hipGetLastError();
}

template <class A, bool MG>
static hipError_t launch_me_t(const DevCode& H, const MeParams& P, int topo, int grid, int block, hipStream_t st) {
  if (topo == TOPO_QC) return launch_me_k<A, MG, TOPO_QC>(H, P, grid, block, st);
  if (topo == TOPO_LDS) return launch_me_k<A, MG, TOPO_LDS>(H, P, grid, block, st);
  return launch_me_k<A, MG, TOPO_GLOBAL>(H, P, grid, block, st);
}

hipError_t launch_me(const DevCode& H, const MeParams& P, bool fixed, bool msg_global, int topo, int grid, int block,
                     hipStream_t st) {
  if (fixed)
    return msg_global ? launch_me_t<ArithFix, true>(H, P, topo, grid, block, st)
                      : launch_me_t<ArithFix, false>(H, P, topo, grid, block, st);
  return msg_global ? launch_me_t<ArithF32, true>(H, P, topo, grid, block, st)
                    : launch_me_t<ArithF32, false>(H, P, topo, grid, block, st);
}

template <class A, bool MG, int TP>
static hipError_t set_me_one(int bytes) {
  return hipFuncSetAttribute((const void*)k_me<A, MG, TP>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t set_me_lds_limit(int bytes) {
  hipError_t e = hipSuccess;
#define LDPC_SET(A, MG, TP) \
  if ((e = set_me_one<A, MG, TP>(bytes)) != hipSuccess) return e;
  LDPC_SET(ArithF32, false, TOPO_GLOBAL) LDPC_SET(ArithF32, false, TOPO_LDS) LDPC_SET(ArithF32, false, TOPO_QC)
  LDPC_SET(ArithF32, true, TOPO_GLOBAL) LDPC_SET(ArithF32, true, TOPO_LDS) LDPC_SET(ArithF32, true, TOPO_QC)
  LDPC_SET(ArithFix, false, TOPO_GLOBAL) LDPC_SET(ArithFix, false, TOPO_LDS) LDPC_SET(ArithFix, false, TOPO_QC)
  LDPC_SET(ArithFix, true, TOPO_GLOBAL) LDPC_SET(ArithFix, true, TOPO_LDS) LDPC_SET(ArithFix, true, TOPO_QC)
#undef LDPC_SET
  return e;
}

}  // namespace ldpc
