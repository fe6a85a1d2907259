// Single-edge dynamic schedules on gfx950: residual BP (RBP, Sec. II-A steps 1-4), CIRBP
// (Algorithm 1, Sec. III-B) and forced-order replay of a recorded schedule.
//
// One wavefront (64 lanes, one workgroup) decodes one codeword at a time; workgroups loop over
// frames.  The frame's whole state lives in LDS:
//   c2v[E], pre[E]      current and precomputed C2V messages (pre may live in a global scratch
//                        slot per workgroup when it does not fit),
//   L[N], Lt[N]         total and precomputed total LLRs,
//   D[N]                CI of every VN as key bits,
//   ckey[M]             per check: max over its edges of (residual, lowest edge id),
//   dblk[], cblk[]      max over blocks of 64 VNs / 64 checks (two-level max trees),
//   syn[M]              syndrome bits of the current hard decisions.
// Per update only the touched part of the state is rewritten:
//   selection      argmax over the block maxima (one wave reduction), or over the checks of n*,
//   propagation    c2v[e*] <- pre[e*], L_{n*} += delta, syndrome toggles if the hard bit flips,
//   touched checks every i in M(n*) \ m*: new V2C from n*, new precomputed messages of its
//                  other edges (one lane per edge, leave-one-out fold), residual keys,
//   CI             Lt_j += pre_new - pre_old, D_j for the VNs of the touched checks and D_{n*},
//   max trees      block maxima raised with LDS atomic max; a block whose maximum leaf
//                  decreased is recomputed by one wave reduction.
#include "common.hpp"
#include "kernels.hpp"

namespace ldpc {

template <class A, bool PRE_GLOBAL>
__global__ __launch_bounds__(WAVE) void k_dynamic(DevCode H, DynParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  using val_t = typename A::val_t;
  const int lane = threadIdx.x;

  msg_t* c2v = reinterpret_cast<msg_t*>(lds + P.off_c2v);
  msg_t* pre;
  if constexpr (PRE_GLOBAL) pre = reinterpret_cast<msg_t*>(P.pre_global) + (size_t)blockIdx.x * H.E;
  else pre = reinterpret_cast<msg_t*>(lds + P.off_pre);
  llr_t* L = reinterpret_cast<llr_t*>(lds + P.off_L);
  llr_t* Lt = reinterpret_cast<llr_t*>(lds + P.off_Lt);
  uint32_t* D = reinterpret_cast<uint32_t*>(lds + P.off_D);
  uint64_t* ckey = reinterpret_cast<uint64_t*>(lds + P.off_ckey);
  uint64_t* dblk = reinterpret_cast<uint64_t*>(lds + P.off_dblk);
  uint64_t* cblk = reinterpret_cast<uint64_t*>(lds + P.off_cblk);
  uint32_t* dmask = reinterpret_cast<uint32_t*>(lds + P.off_dmask);
  uint32_t* cmask = reinterpret_cast<uint32_t*>(lds + P.off_cmask);
  uint8_t* syn = reinterpret_cast<uint8_t*>(lds + P.off_syn);
  val_t* vbuf = reinterpret_cast<val_t*>(lds + P.off_v);
  uint8_t* slot = reinterpret_cast<uint8_t*>(lds + P.off_slot);
  int* trow = reinterpret_cast<int*>(lds + P.off_trow);  // [3][WAVE]: row, row start, slot offset
  int* lut = reinterpret_cast<int*>(lds + P.off_lut);

  A ar;
  ar.qmax = P.qmax;
  ar.scale = P.scale;
  ar.lut = lut;
  if constexpr (A::kFixed) {
    for (int x = lane; x < 257; x += WAVE) lut[x] = P.lut_global[x];
  }
  const int N = H.N, M = H.M, E = H.E;
  const bool with_ci = P.kind != KIND_RBP;

  for (int f = blockIdx.x; f < P.B; f += gridDim.x) {
    // ---------------- Algorithm 1 lines 1-3: initial state --------------------------------
    const float* llr = P.llr + (size_t)f * N;
    for (int n = lane; n < N; n += WAVE) L[n] = (llr_t)ar.channel(llr[n]);
    for (int e = lane; e < E; e += WAVE) c2v[e] = (msg_t)0;
    for (int w = lane; w < P.nbd_words; w += WAVE) dmask[w] = 0u;
    for (int w = lane; w < P.nbc_words; w += WAVE) cmask[w] = 0u;
    __syncthreads();
    for (int e = lane; e < E; e += WAVE) {  // every precomputed C2V message from V2C = channel
      int m = H.row_of[e];
      int rs = H.row_ptr[m], re = H.row_ptr[m + 1];
      bool first = true;
      val_t acc = 0;
      for (int k = rs; k < re; ++k) {
        if (k == e) continue;
        val_t v = ar.vin((val_t)L[H.col[k]]);
        acc = first ? v : ar.op(acc, v);
        first = false;
      }
      pre[e] = (msg_t)acc;
    }
    __syncthreads();
    for (int n = lane; n < N; n += WAVE) {
      val_t lt = (val_t)L[n];
      for (int k = H.col_ptr[n]; k < H.col_ptr[n + 1]; ++k) lt += (val_t)pre[H.col_eid[k]];
      Lt[n] = (llr_t)lt;
      D[n] = with_ci ? ar.ci((val_t)L[n], lt) : 0u;
    }
    int unsat_local = 0;
    for (int m = lane; m < M; m += WAVE) {
      uint64_t k = 0;
      int par = 0;
      for (int e = H.row_ptr[m]; e < H.row_ptr[m + 1]; ++e) {
        k = umax64(k, mkkey(ar.res((val_t)pre[e], (val_t)c2v[e]), (uint32_t)e));
        par ^= ((val_t)L[H.col[e]] < 0) ? 1 : 0;
      }
      ckey[m] = k;
      syn[m] = (uint8_t)par;
      unsat_local += par;
    }
    int unsat = wave_sum_i32(unsat_local);
    __syncthreads();
    for (int b = 0; b < P.nbd; ++b) {
      int n = b * WAVE + lane;
      uint64_t k = n < N ? mkkey(D[n], (uint32_t)n) : 0ull;
      k = wave_max_u64(k);
      if (lane == 0) dblk[b] = k;
    }
    for (int b = 0; b < P.nbc; ++b) {
      int m = b * WAVE + lane;
      uint64_t k = m < M ? ckey[m] : 0ull;
      k = wave_max_u64(k);
      if (lane == 0) cblk[b] = k;
    }
    __syncthreads();

    // ---------------- update loop -------------------------------------------------------
    long long t = 0, nfall = 0;
    long long limit = P.max_updates;
    if (P.kind == KIND_REPLAY && P.replay_len < limit) limit = P.replay_len;
    const long long ce = P.kind == KIND_REPLAY ? 0 : P.check_every;
    bool done = ce > 0 && unsat == 0;
    while (!done && t < limit) {
      const long long tprev = t;
      // ---- selection (Algorithm 1 lines 4-8; RBP eq. (5)) ----
      int estar;
      if (P.kind == KIND_REPLAY) {
        estar = uni(P.replay[(size_t)f * P.replay_len + t]);
        if (estar < 0 || estar >= E) break;  // invalid edge id ends the frame's replay
      } else {
        bool global_res = P.kind == KIND_RBP;
        int nstar_sel = -1;
        if (!global_res) {
          uint64_t k = 0;
          for (int b = lane; b < P.nbd; b += WAVE) k = umax64(k, dblk[b]);
          k = wave_max_u64(k);
          nstar_sel = (int)key_idx(k);
          if (key_val(k) < P.gamma_bits) {  // D_{n*} < gamma: RBP fallback
            global_res = true;
            nfall += 1;
          }
        }
        if (global_res) {
          uint64_t k = 0;
          for (int b = lane; b < P.nbc; b += WAVE) k = umax64(k, cblk[b]);
          estar = (int)key_idx(wave_max_u64(k));
        } else {
          const int cb = H.col_ptr[nstar_sel], dv = H.col_ptr[nstar_sel + 1] - cb;
          uint64_t k = 0;
          for (int q = lane; q < dv; q += WAVE) {
            int e = H.col_eid[cb + q];
            k = umax64(k, mkkey(ar.res((val_t)pre[e], (val_t)c2v[e]), (uint32_t)e));
          }
          estar = (int)key_idx(wave_max_u64(k));
        }
      }
      const int mstar = uni(H.row_of[estar]);
      const int nstar = uni(H.col[estar]);
      const int cb = uni(H.col_ptr[nstar]);
      const int dv = uni(H.col_ptr[nstar + 1]) - cb;

      // ---- propagation (Algorithm 1 line 9) ----
      const val_t newv = (val_t)pre[estar];
      const val_t oldv = (val_t)c2v[estar];
      const val_t Lold = (val_t)L[nstar];
      const val_t Lnew = Lold + (newv - oldv);
      __syncthreads();
      if (lane == 0) {
        c2v[estar] = (msg_t)newv;
        L[nstar] = (llr_t)Lnew;
      }
      if ((Lold < 0) != (Lnew < 0)) {  // hard decision flipped: toggle the checks of n*
        int d = 0;
        for (int q = lane; q < dv; q += WAVE) {
          int m = H.col_row[cb + q];
          int s = syn[m];
          syn[m] = (uint8_t)(s ^ 1);
          d += s ? -1 : 1;
        }
        unsat += wave_sum_i32(d);
      }
      // ---- touched checks M(n*) \ m*: slot layout ----
      int my_row = -1, my_rs = 0, my_dc = 0;
      if (lane < dv) {
        my_row = H.col_row[cb + lane];
        my_rs = H.row_ptr[my_row];
        my_dc = my_row == mstar ? 0 : H.row_ptr[my_row + 1] - my_rs;
      }
      const int my_off = wave_excl_scan(my_dc, lane);
      const int T = wave_sum_i32(my_dc);
      if (lane < dv) {
        trow[lane] = my_row;
        trow[WAVE + lane] = my_rs;
        trow[2 * WAVE + lane] = my_off;
        for (int p = 0; p < my_dc; ++p) slot[my_off + p] = (uint8_t)lane;
      }
      __syncthreads();
      // new V2C messages of every edge of the touched checks (only n*'s changed)
      for (int s = lane; s < T; s += WAVE) {
        int q = slot[s];
        int e = trow[WAVE + q] + (s - trow[2 * WAVE + q]);
        vbuf[s] = ar.v2c((val_t)L[H.col[e]], (val_t)c2v[e]);
      }
      __syncthreads();
      // precomputed C2V messages (eq. (2) over the other inputs), residual keys, Lt deltas
      for (int s = lane; s < T; s += WAVE) {
        int q = slot[s];
        int off = trow[2 * WAVE + q];
        int rs = trow[WAVE + q];
        int dcq = H.row_ptr[trow[q] + 1] - rs;
        int e = rs + (s - off);
        int j = H.col[e];
        val_t pv;
        if (j == nstar) {
          pv = (val_t)pre[e];  // inputs unchanged: same value as before
        } else {
          bool first = true;
          val_t acc = 0;
          for (int k = 0; k < dcq; ++k) {
            if (k == s - off) continue;
            val_t v = ar.vin(vbuf[off + k]);
            acc = first ? v : ar.op(acc, v);
            first = false;
          }
          pv = acc;
          val_t old = (val_t)pre[e];
          pre[e] = (msg_t)pv;
          if (with_ci) {
            if constexpr (A::kFixed) atomicAdd(&Lt[j], pv - old);
            else atomicAdd(&Lt[j], pv - old);
          }
        }
        // residual key of this edge, kept in vbuf's companion region
        reinterpret_cast<uint64_t*>(lds + P.off_kbuf)[s] = mkkey(ar.res(pv, (val_t)c2v[e]), (uint32_t)e);
      }
      __syncthreads();
      // ---- check keys of the touched checks and of m* ----
      {
        // lanes q < dv: serial max over the row's slot keys (touched checks)
        uint64_t* kbuf = reinterpret_cast<uint64_t*>(lds + P.off_kbuf);
        uint64_t newk = 0, oldk = 0;
        int myc = -1;
        if (lane < dv && my_dc > 0) {
          for (int p = 0; p < my_dc; ++p) newk = umax64(newk, kbuf[my_off + p]);
          myc = my_row;
        }
        // m*: its residual at e* is now zero, others unchanged
        const int rs_m = uni(H.row_ptr[mstar]);
        const int dc_m = uni(H.row_ptr[mstar + 1]) - rs_m;
        uint64_t km = 0;
        for (int p = lane; p < dc_m; p += WAVE) {
          int e = rs_m + p;
          km = umax64(km, mkkey(ar.res((val_t)pre[e], (val_t)c2v[e]), (uint32_t)e));
        }
        km = wave_max_u64(km);
        if (lane == dv) {  // one spare lane handles m* (dv < WAVE)
          myc = mstar;
          newk = km;
        }
        if (myc >= 0) {
          oldk = ckey[myc];
          ckey[myc] = newk;
          int b = myc >> 6;
          if (newk > oldk) {
            atomicMax(reinterpret_cast<unsigned long long*>(&cblk[b]), (unsigned long long)newk);
          }
        }
        __syncthreads();
        if (myc >= 0 && newk < oldk && cblk[myc >> 6] == oldk) atomicOr(&cmask[(myc >> 6) >> 5], 1u << ((myc >> 6) & 31));
        __syncthreads();
        for (int w = 0; w < P.nbc_words; ++w) {
          uint32_t bits = (uint32_t)uni((int)cmask[w]);
          while (bits) {
            int b = w * 32 + __builtin_ctz(bits);
            bits &= bits - 1;
            int m = b * WAVE + lane;
            uint64_t k = m < M ? ckey[m] : 0ull;
            k = wave_max_u64(k);
            if (lane == 0) cblk[b] = k;
          }
          if (lane == 0) cmask[w] = 0u;
        }
      }
      // ---- CI of the VNs of the touched checks and of n* (Algorithm 1 line 12) ----
      if (with_ci) {
        uint32_t newd = 0, oldd = 0;
        int myj = -1;
        // slots first, then n* on an extra pass lane
        for (int s0 = 0; s0 < T + 1; s0 += WAVE) {
          int s = s0 + lane;
          myj = -1;
          if (s < T) {
            int q = slot[s];
            int e = trow[WAVE + q] + (s - trow[2 * WAVE + q]);
            int j = H.col[e];
            if (j != nstar) myj = j;
          } else if (s == T) {
            myj = nstar;
          }
          if (myj >= 0) {
            newd = ar.ci((val_t)L[myj], (val_t)Lt[myj]);
            oldd = D[myj];
          }
          __syncthreads();
          if (myj >= 0) {
            D[myj] = newd;
            uint64_t nk = mkkey(newd, (uint32_t)myj), ok = mkkey(oldd, (uint32_t)myj);
            if (nk > ok) atomicMax(reinterpret_cast<unsigned long long*>(&dblk[myj >> 6]), (unsigned long long)nk);
          }
          __syncthreads();
          if (myj >= 0) {
            uint64_t nk = mkkey(newd, (uint32_t)myj), ok = mkkey(oldd, (uint32_t)myj);
            if (nk < ok && dblk[myj >> 6] == ok) atomicOr(&dmask[(myj >> 6) >> 5], 1u << ((myj >> 6) & 31));
          }
        }
        __syncthreads();
        for (int w = 0; w < P.nbd_words; ++w) {
          uint32_t bits = (uint32_t)uni((int)dmask[w]);
          while (bits) {
            int b = w * 32 + __builtin_ctz(bits);
            bits &= bits - 1;
            int n = b * WAVE + lane;
            uint64_t k = n < N ? mkkey(D[n], (uint32_t)n) : 0ull;
            k = wave_max_u64(k);
            if (lane == 0) dblk[b] = k;
          }
          if (lane == 0) dmask[w] = 0u;
        }
      }
      __syncthreads();
      if (P.out.trace && lane == 0) P.out.trace[(size_t)f * P.max_updates + t] = estar;
      t += 1;
      if (ce > 0 && (t / ce) != (tprev / ce) && unsat == 0) done = true;
    }

    // ---------------- outputs (a8) -----------------------------------------------------
    for (int n = lane; n < N; n += WAVE) {
      val_t l = (val_t)L[n];
      P.out.bits[(size_t)f * N + n] = l < 0 ? 1 : 0;
      if (P.out.llr_out) P.out.llr_out[(size_t)f * N + n] = ar.out_llr(l);
      if (P.out.dump_L) P.out.dump_L[(size_t)f * N + n] = ar.as_float(l);
      if (P.out.dump_Lt) P.out.dump_Lt[(size_t)f * N + n] = ar.as_float((val_t)Lt[n]);
      if (P.out.dump_D) P.out.dump_D[(size_t)f * N + n] = ar.d_float(D[n]);
    }
    for (int e = lane; e < E; e += WAVE) {
      if (P.out.dump_c2v) P.out.dump_c2v[(size_t)f * E + e] = ar.as_float((val_t)c2v[e]);
      if (P.out.dump_pre) P.out.dump_pre[(size_t)f * E + e] = ar.as_float((val_t)pre[e]);
    }
    if (lane == 0) {
      P.out.updates_used[f] = t;
      if (P.out.steps_used) P.out.steps_used[f] = t;
      if (P.out.fallbacks) P.out.fallbacks[f] = nfall;
    }
    __syncthreads();
  }
}

template <class A, bool PG>
static hipError_t launch_dyn(const DevCode& H, const DynParams& P, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_dynamic<A, PG>), dim3(grid), dim3(WAVE), P.lds_bytes, st, H, P);
  return hipGetLastError();
}

hipError_t launch_dynamic(const DevCode& H, const DynParams& P, bool fixed, bool pre_global, int grid,
                          hipStream_t st) {
  if (fixed) return pre_global ? launch_dyn<ArithFix, true>(H, P, grid, st) : launch_dyn<ArithFix, false>(H, P, grid, st);
  return pre_global ? launch_dyn<ArithF32, true>(H, P, grid, st) : launch_dyn<ArithF32, false>(H, P, grid, st);
}

hipError_t set_dynamic_lds_limit(int bytes) {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)k_dynamic<ArithF32, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_dynamic<ArithF32, true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_dynamic<ArithFix, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_dynamic<ArithFix, true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace ldpc
