// Multi-edge CIRBP on gfx950: Algorithm 4 (VN selection by CI groups) and Algorithm 5 (the
// selected VNs updated together), Sec. VI; and multi-edge LMD-CIRBP (Algorithm 6), whose next set
// starts from the VNs the updated ones propose.
//
// One workgroup decodes one frame at a time.  Per step, on a snapshot of the state:
//   1. the CI-group histogram hist[N_G] (kept up to date as D changes) gives the groups taken
//      whole (the largest k with |Q(k)| <= N_P) and the fill group with the number still needed;
//   2. the selected set P: every VN of the taken groups, plus the fill -- the lowest VN indices
//      (block prefix count) or the smallest keys splitmix64(splitmix64(splitmix64(seed ^ frame)
//      ^ step) ^ n) (a key threshold shrunk until at most CAND candidates remain, then ranked);
//   3. for each p in P (ascending): the incoming edge of largest residual (Algorithm 1);
//   4. all propagations c2v <- pre, L_p += delta, syndrome toggles;
//   5. every check of every p recomputed from the new state (one lane per check, each check once),
//      Lt updated by the precompute deltas (FP32: kept per edge and summed per VN in ascending
//      check order, so that reruns round alike); then D (and its group) of every VN of those checks;
//   6. ME-LMD-CIRBP only: each p proposes the VN of largest CI among U(m*_p, p) (N(m*_p) \ p when p
//      has degree 1); the distinct proposals P' start the next set, whose remaining N_P - |P'| VNs
//      come from steps 1-2 run on the VNs outside P' (their histogram counts taken out, their
//      membership marked in vnmark for the selection).
// Messages c2v/pre stay in LDS when they fit, otherwise in a global scratch slot per workgroup.
#include "common.hpp"
#include "kernels.hpp"

namespace ldpc {

#ifdef LDPC_PROFILE
// phase timing for development builds only: thread 0's clock64() deltas per phase, summed over steps
#define ME_PROF_DECL long long mp_acc[8] = {0, 0, 0, 0, 0, 0, 0, 0}; long long mp_t = clock64();
#define ME_PROF_MARK(i) { if (tid == 0) { long long now_ = clock64(); mp_acc[i] += now_ - mp_t; mp_t = now_; } }
#define ME_PROF_FLUSH { if (tid == 0 && P.prof) for (int i_ = 0; i_ < 8; ++i_) atomicAdd((unsigned long long*)&P.prof[i_], (unsigned long long)mp_acc[i_]); }
#else
#define ME_PROF_DECL
#define ME_PROF_MARK(i)
#define ME_PROF_FLUSH
#endif


enum { MS_UNSAT = 0, MS_NROWS, MS_NSEL, MS_BSTAR, MS_FILL, MS_NEED, MS_CNT, MS_NCAND, MS_WAVESUM, MS_RBIN, MS_RBELOW,
       MS_L2,                 // MS_L2 + c - 1: touched checks with blocks of 2^c lanes, c = 1..5
       MS_NSUCC = MS_L2 + 5,  // ME-LMD-CIRBP: |P'|
       MS_ABORT,              // the abort flag as read for the workgroup at a frame's start
       MS_NMULTI,             // FP32: VNs that several checks of the step changed
       kMiscWords = 32 };     // misc[0, kMiscWords): the counters above; then one word per wavefront

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

  // (c2v, pre) pairs of the frame: one load brings both values of an edge
  MsgPair<msg_t>* mp = MSG_GLOBAL ? reinterpret_cast<MsgPair<msg_t>*>(P.msg_global) + (size_t)blockIdx.x * (size_t)E
                                  : reinterpret_cast<MsgPair<msg_t>*>(lds + P.off_c2v);
  llr_t* L = reinterpret_cast<llr_t*>(lds + P.off_L);
  llr_t* Lt = reinterpret_cast<llr_t*>(lds + P.off_Lt);
  uint32_t* D = reinterpret_cast<uint32_t*>(lds + P.off_D);
  int* hist = reinterpret_cast<int*>(lds + P.off_hist);
  uint32_t* synw = reinterpret_cast<uint32_t*>(lds + P.off_synw);
  uint32_t* rowmark = reinterpret_cast<uint32_t*>(lds + P.off_rowmark);
  uint32_t* vnmark = reinterpret_cast<uint32_t*>(lds + P.off_vnmark);
  // FP32: VNs whose precomputed total two or more checks of the step change, and the step's
  // changes of the precomputed messages (global, one float per edge of this workgroup's frame)
  uint32_t* vnmulti = reinterpret_cast<uint32_t*>(lds + P.off_vnmulti);
  int* mpref = reinterpret_cast<int*>(lds + P.off_mpref);
  long long* macc = reinterpret_cast<long long*>(lds + P.off_macc);
  float* dbuf = A::kFixed ? nullptr : P.dbuf + (size_t)blockIdx.x * (size_t)E;
  int* rows = reinterpret_cast<int*>(lds + P.off_rows);
  int* rows2 = reinterpret_cast<int*>(lds + P.off_rows2);
  int* sel = reinterpret_cast<int*>(lds + P.off_sel);  // [64] unsorted, [64] sorted
  int* sel_s = sel + 64;
  int* succ = sel + 192;  // ME-LMD-CIRBP: the proposals P' [64]
  int* selm = sel + 256;  // the check whose message sel_s[i] received [64]
  uint64_t* ckeys = reinterpret_cast<uint64_t*>(lds + P.off_cand);
  int* cidx = reinterpret_cast<int*>(ckeys + P.cand_cap);
  int* misc = reinterpret_cast<int*>(lds + P.off_misc);
  int* wsum = misc + kMiscWords;
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
  const bool lmd = P.lmd != 0;
  const int nsw = (M + 31) >> 5, nvw = (N + 31) >> 5;
  __syncthreads();

  for (int f = blockIdx.x; f < P.B; f += gridDim.x) {
    __syncthreads();  // the previous frame is done with the workgroup's LDS
    if (tid == 0) misc[MS_ABORT] = abort_flag_value(P.out.abort);
    __syncthreads();
    if (misc[MS_ABORT] != 0) {  // not started: the abort flag was set
      if (tid == 0) P.out.updates_used[f] = -1;
      continue;
    }
    // ---------------- Algorithm 5, initialisation ---------------------------------------
    const float* llr = P.llr + (size_t)f * N;
    for (int n = tid; n < N; n += BS) L[n] = (llr_t)ar.channel(llr[n]);
    for (int e = tid; e < E; e += BS) mp[e].c = (msg_t)0;
    for (int b = tid; b < NG; b += BS) hist[b] = 0;
    for (int w = tid; w < nsw; w += BS) synw[w] = 0u, rowmark[w] = 0u;
    for (int w = tid; w < nvw; w += BS) vnmark[w] = 0u, vnmulti[w] = 0u;
    if (tid < kMiscWords) misc[tid] = 0;
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
        mp[rs + p].p = (msg_t)acc.out(p, v, row_aux(ar, v));
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
        lt += (val_t)mp[e].p;
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
    ME_PROF_DECL
    while (!done && t + NP <= P.max_updates) {
      ME_PROF_MARK(7)
      const long long tprev = t;
      // ---- ME-LMD-CIRBP: P' goes into the set first and is taken out of Algorithm 4's view ----
      const int nsucc = lmd ? misc[MS_NSUCC] : 0;
      if (nsucc > 0) {
        if (tid < nsucc) {
          const int v = succ[tid];
          sel[tid] = v;
          atomicOr(&vnmark[v >> 5], 1u << (v & 31));
          atomicSub(&hist[ar.bin(D[v], NG)], 1);
        }
        __syncthreads();
      }
      const int np_eff = NP - nsucc;
      // excluded from this step's Algorithm 4: the members of P'
      auto excluded = [&](int n) -> bool { return nsucc > 0 && ((vnmark[n >> 5] >> (n & 31)) & 1u); };
      // ---- Algorithm 4, group selection: groups taken whole, fill group, number still needed ----
      if (tid == 0) {
        int c = 0, bstar = NG;
        for (int b = NG - 1; b >= 0; --b) {
          if (c + hist[b] > np_eff) break;
          c += hist[b];
          bstar = b;
        }
        const int fill = bstar > 0 ? bstar - 1 : -1;
        misc[MS_BSTAR] = bstar;
        misc[MS_FILL] = fill;
        misc[MS_NEED] = fill >= 0 ? np_eff - c : 0;
        misc[MS_NSEL] = nsucc;
        misc[MS_NSUCC] = 0;
        misc[MS_CNT] = 0;
        misc[MS_NCAND] = 0;
        for (int c = 0; c < 5; ++c) {
          misc[MS_L2 + c] = 0;
          sel[128 + c] = 0;
        }
      }
      __syncthreads();
      const int bstar = misc[MS_BSTAR], fill = misc[MS_FILL], need = misc[MS_NEED];
      // keyed fill: the per-step part of the key is uniform, a VN's key is one more splitmix64
      const bool keyed = P.fill != 0 && need > 0;
      const uint64_t s2 = splitmix64(splitmix64(P.seed ^ (uint64_t)f) ^ (uint64_t)steps);
      int* h256 = cidx;  // key-byte histogram of the fill group (radix selection only)
      // keyed fill, first try: the keys are uniform, so a threshold below which about
      // min(3 need, 56) of the fill group's members fall (its size is the histogram's count)
      // gives, whenever between `need` and 64 keys lie below it, a candidate list that holds the
      // `need` smallest keys and is ranked inside one wavefront
      uint64_t thr = 0ull;
      if (keyed) {
        const int mf = hist[fill], want = min(3 * need, 56);
        thr = want >= mf ? ~0ull : (uint64_t)((double)want / (double)mf * 18446744073709551616.0);
      }
      auto offer = [&](int n, uint64_t k) {  // a fill member whose key is below the threshold
        if (thr == ~0ull || k < thr) {
          const int c = atomicAdd(&misc[MS_NCAND], 1);
          if (c < P.cand_cap) {
            ckeys[c] = k;
            cidx[c] = n;
          }
        }
      };
      // ---- the selected set: groups taken whole; the fill group counted, and for the keyed
      //      fill its members below the threshold listed in the same pass.  A thread's VNs are
      //      n0..n1; up to kKeep of them keep their fill membership and key in registers for the
      //      passes below (larger codes recompute them) ----
      constexpr int kKeep = 12;
      const int chunk = (N + BS - 1) / BS;
      const int n0 = tid * chunk, n1 = min(N, n0 + chunk);
      const bool keep = chunk <= kKeep;
      uint64_t kk[kKeep];
      uint32_t kmask = 0u;  // bit i: VN n0 + i is in the fill group
      int nfill = 0;
      if (keep) {
#pragma unroll
        for (int i = 0; i < kKeep; ++i) {
          kk[i] = 0ull;
          const int n = n0 + i;
          if (n < n1 && !excluded(n)) {
            const int b = ar.bin(D[n], NG);
            if (b >= bstar) sel[atomicAdd(&misc[MS_NSEL], 1)] = n;
            if (b == fill) {
              nfill += 1;
              kmask |= 1u << i;
              if (keyed) {
                kk[i] = splitmix64(s2 ^ (uint64_t)n);
                offer(n, kk[i]);
              }
            }
          }
        }
      } else {
        for (int n = n0; n < n1; ++n) {
          if (excluded(n)) continue;
          const int b = ar.bin(D[n], NG);
          if (b >= bstar) sel[atomicAdd(&misc[MS_NSEL], 1)] = n;
          if (b == fill) {
            nfill += 1;
            if (keyed) offer(n, splitmix64(s2 ^ (uint64_t)n));
          }
        }
      }
      // every fill member of this thread with its key: f(n, key)
      auto for_members = [&](auto&& fn) {
        if (keep) {
#pragma unroll
          for (int i = 0; i < kKeep; ++i)
            if ((kmask >> i) & 1u) fn(n0 + i, kk[i]);
        } else {
          for (int n = n0; n < n1; ++n)
            if (ar.bin(D[n], NG) == fill && !excluded(n)) fn(n, splitmix64(s2 ^ (uint64_t)n));
        }
      };
      ME_PROF_MARK(0)
      // ---- Algorithm 4: the fill ----
      if (need > 0) {
        if (P.fill == 0) {  // lowest indices: rank of each fill member in index order
          int rank = block_excl_scan(nfill, wsum);
          for (int n = n0; n < n1 && rank < need; ++n) {
            if (ar.bin(D[n], NG) == fill && !excluded(n)) {
              sel[atomicAdd(&misc[MS_NSEL], 1)] = n;
              ++rank;
            }
          }
        } else {
          // the `need` smallest keys (ties: lower index) among the nc listed candidates: `take` of
          // them by rank
          auto take_smallest = [&](int nc, int take) {
            if (nc <= WAVE) {  // one wavefront: candidate per lane, ranks from register reads
              if (tid < WAVE) {
                const uint64_t ki = tid < nc ? ckeys[tid] : ~0ull;
                const int ni = tid < nc ? cidx[tid] : 0x7FFFFFFF;
                const uint32_t khi = (uint32_t)(ki >> 32), klo = (uint32_t)ki;
                int r = 0;
                for (int j = 0; j < nc; ++j) {
                  const uint64_t kj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)khi, j) << 32) |
                                      (uint32_t)__builtin_amdgcn_readlane((int)klo, j);
                  const int nj = __builtin_amdgcn_readlane(ni, j);
                  r += (kj < ki || (kj == ki && nj < ni)) ? 1 : 0;
                }
                if (tid < nc && r < take) sel[atomicAdd(&misc[MS_NSEL], 1)] = ni;
              }
            } else {  // chunks of 64: a wavefront ranks its chunk against each chunk in turn, one LDS
                      // load per lane per chunk and then register reads
              const int nchunk = (nc + WAVE - 1) / WAVE, lw = tid & (WAVE - 1);
              for (int c0 = tid >> 6; c0 < nchunk; c0 += BS >> 6) {
                const int i = c0 * WAVE + lw;
                const uint64_t ki = i < nc ? ckeys[i] : ~0ull;
                const int ni = i < nc ? cidx[i] : 0x7FFFFFFF;
                int r = 0;
                for (int c1 = 0; c1 < nchunk; ++c1) {
                  const int x = c1 * WAVE + lw;
                  const uint64_t kx = x < nc ? ckeys[x] : ~0ull;
                  const int nx = x < nc ? cidx[x] : 0x7FFFFFFF;
                  const uint32_t xhi = (uint32_t)(kx >> 32), xlo = (uint32_t)kx;
                  const int cnt = min(WAVE, nc - c1 * WAVE);
                  for (int j = 0; j < cnt; ++j) {
                    const uint64_t kj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)xhi, j) << 32) |
                                        (uint32_t)__builtin_amdgcn_readlane((int)xlo, j);
                    const int nj = __builtin_amdgcn_readlane(nx, j);
                    r += (kj < ki || (kj == ki && nj < ni)) ? 1 : 0;
                  }
                }
                if (i < nc && r < take) sel[atomicAdd(&misc[MS_NSEL], 1)] = ni;
              }
            }
          };
          __syncthreads();  // the threshold's candidates are listed
          const int ncand = misc[MS_NCAND];
          if (ncand >= need && ncand <= WAVE) {
            take_smallest(ncand, need);
          } else {
            // fewer keys below the threshold than needed (sets that need many fill members), or
            // more than one wavefront ranks.
            // Radix selection over every member: find the key bucket (a run of leading bytes)
            // that holds the need-th smallest, narrowing it a byte at a time until it has at most
            // cand_cap members; keys below it are taken, keys inside it ranked
            __syncthreads();  // every thread has read the count
            if (tid == 0) misc[MS_NCAND] = 0;
            for (int x = tid; x < 256; x += BS) h256[x] = 0;
            __syncthreads();
            for_members([&](int, uint64_t k) { atomicAdd(&h256[k >> 56], 1); });
            uint64_t lo = 0;
            int shift = 56, below = 0;
            while (true) {
              __syncthreads();  // histogram complete
              if (tid < WAVE) {
                const int c0 = h256[4 * tid], c1 = h256[4 * tid + 1], c2 = h256[4 * tid + 2], c3 = h256[4 * tid + 3];
                const int ex = below + wave_excl_scan(c0 + c1 + c2 + c3, tid);
                const int cs[4] = {c0, c1, c2, c3};
                int before = ex;
                for (int u = 0; u < 4; ++u) {
                  if (cs[u] > 0 && before < need && need <= before + cs[u]) {
                    misc[MS_RBIN] = 4 * tid + u;
                    misc[MS_RBELOW] = before;
                    misc[MS_CNT] = cs[u];
                  }
                  before += cs[u];
                }
              }
              __syncthreads();
              lo |= (uint64_t)misc[MS_RBIN] << shift;
              below = misc[MS_RBELOW];
              const int cnt = misc[MS_CNT];
              if (cnt <= P.cand_cap || shift == 0) break;
              shift -= 8;
              for (int x = tid; x < 256; x += BS) h256[x] = 0;
              __syncthreads();
              const uint64_t upper = ~0ull << (shift + 8);  // the bytes fixed so far
              for_members([&](int, uint64_t k) {
                if ((k & upper) == lo) atomicAdd(&h256[(k >> shift) & 255], 1);
              });
            }
            __syncthreads();  // the histogram's last reader is done before candidates overwrite it
            const uint64_t hi = lo + ((shift == 0) ? 0ull : ((1ull << shift) - 1ull));
            for_members([&](int n, uint64_t k) {
              if (k < lo) {
                sel[atomicAdd(&misc[MS_NSEL], 1)] = n;
              } else if (k <= hi) {
                const int i = atomicAdd(&misc[MS_NCAND], 1);
                if (i < P.cand_cap) {
                  ckeys[i] = k;
                  cidx[i] = n;
                }
              }
            });
            __syncthreads();
            take_smallest(min(misc[MS_NCAND], P.cand_cap), need - below);
          }
        }
      }
      __syncthreads();
      ME_PROF_MARK(1)
      const int nsel = misc[MS_NSEL];
      if (nsucc > 0 && tid < nsucc) {  // P' back into Algorithm 4's view (D has not changed)
        const int v = succ[tid];
        atomicAnd(&vnmark[v >> 5], ~(1u << (v & 31)));
        atomicAdd(&hist[ar.bin(D[v], NG)], 1);
      }
      // ascending order of P (distinct VN indices: rank = number of smaller ones; at most 64,
      // one wavefront, ranks from register reads)
      if (tid < WAVE) {
        const int v = tid < nsel ? sel[tid] : 0x7FFFFFFF;
        int r = 0;
        for (int j = 0; j < nsel; ++j) r += __builtin_amdgcn_readlane(v, j) < v ? 1 : 0;
        if (tid < nsel) sel_s[r] = v;
      }
      __syncthreads();
      const int nwv = BS >> 6, wv = tid >> 6, ln = tid & 63;
      // ---- Algorithm 1 edge choice and propagation for every p: the incoming edge of largest residual, then its
      //      propagation.  A VN's choice reads only its own edges and a propagation writes only
      //      its own edge and L, so choosing and propagating VN by VN equals choosing all on the
      //      snapshot first.  One wavefront per selected VN, one lane per edge (and per check, for
      //      the syndrome toggles and the list of touched checks); a wavefront requests the edges
      //      of up to four VNs at once. ----
      constexpr int kVB = 4;
      for (int i0 = 0; i0 < nsel; i0 += kVB * nwv) {
        int pv_[kVB], dv_[kVB], m_[kVB], e_[kVB];
        MsgPair<msg_t> x_[kVB];
#pragma unroll
        for (int u = 0; u < kVB; ++u) {
          const int i = i0 + u * nwv + wv;
          pv_[u] = -1;
          dv_[u] = 0;
          m_[u] = -1;
          e_[u] = -1;
          x_[u] = MsgPair<msg_t>{(msg_t)0, (msg_t)0};
          if (i < nsel) {
            pv_[u] = sel_s[i];
            dv_[u] = G.vn_deg(pv_[u]);
            if (ln < dv_[u]) {
              G.vn_edge(pv_[u], ln, m_[u], e_[u]);
              x_[u] = mp[e_[u]];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kVB; ++u) {
          const int i = i0 + u * nwv + wv;
          if (i >= nsel) break;  // whole wavefronts
          const int p = pv_[u], dv = dv_[u];
          const uint64_t k = ln < dv ? mkkey(ar.res((val_t)x_[u].p, (val_t)x_[u].c), (uint32_t)e_[u]) : 0ull;
          const uint64_t kmax = wave_max_u64(k);
          const int e = (int)key_idx(kmax);
          const int wl = (int)__builtin_ctzll(__ballot(ln < dv && k == kmax));
          const val_t newv = (val_t)lane_value(x_[u].p, wl), oldv = (val_t)lane_value(x_[u].c, wl);
          const val_t Lold = (val_t)L[p];
          const val_t Lnew = Lold + (newv - oldv);
          const bool flip = (Lold < 0) != (Lnew < 0);
          if (ln < dv) {
            const int m = m_[u];
            const uint32_t bit = 1u << (m & 31);
            if (flip) {
              const uint32_t old = atomicXor(&synw[m >> 5], bit);
              atomicAdd(&misc[MS_UNSAT], (old & bit) ? -1 : 1);
            }
            const uint32_t om = atomicOr(&rowmark[m >> 5], bit);
            if (!(om & bit)) {
              rows[atomicAdd(&misc[MS_NROWS], 1)] = m;
              atomicAdd(&misc[MS_L2 + 31 - __clz(G.row_deg(m) - 1)], 1);
            }
          }
          const int mwin = __builtin_amdgcn_readlane(m_[u], wl);
          wave_sync();
          if (ln == 0) {
            if (P.out.trace) P.out.trace[(size_t)f * P.max_updates + tprev + i] = e;
            mp[e].c = (msg_t)newv;
            L[p] = (llr_t)Lnew;
            selm[i] = mwin;
          }
        }
      }
      ME_PROF_MARK(2)
      if constexpr (MSG_GLOBAL) __threadfence_block();
      __syncthreads();
      const int nrows = misc[MS_NROWS];
      // touched checks by block size (2^c lanes for c = ceil(log2 dc)), largest first, so that
      // every block starts at a multiple of its size: counting sort into rows2
      int rb[6], lo[6];  // per class c: first row in rows2, first lane
      rb[5] = 0;
      lo[5] = 0;
      for (int c = 5; c > 1; --c) {
        const int nc_ = misc[MS_L2 + c - 1];
        rb[c - 1] = rb[c] + nc_;
        lo[c - 1] = lo[c] + (nc_ << c);
      }
      const int total = lo[1] + (misc[MS_L2] << 1);
      int* placed = sel + 128;  // rows placed so far per class
      for (int r = tid; r < nrows; r += BS) {
        const int m = rows[r];
        const int c = 32 - __clz(G.row_deg(m) - 1);
        rows2[rb[c] + atomicAdd(&placed[c - 1], 1)] = m;
      }
      __syncthreads();
      ME_PROF_MARK(3)
      // packed lane gi -> (check, position in its row, log2 block); false beyond the last block
      auto lane_row = [&](int gi, int& m, int& pos, int& l2) -> bool {
        if (gi >= total) return false;
        int c = 5;
        while (c > 1 && gi >= lo[c - 1]) --c;
        const int rel = gi - lo[c];
        m = rows2[rb[c] + (rel >> c)];
        pos = rel & ((1 << c) - 1);
        l2 = c;
        return true;
      };
      // ---- every check of every p from the new state (Algorithm 1, the loop over M(n*) \ m*): the whole-row
      //      update by butterflies inside each check's block; the next pass's message pairs are
      //      requested before this pass computes ----
      struct RowIn {
        int e, j, l2;
        MsgPair<msg_t> x;
      };
      auto row_in = [&](int base) -> RowIn {
        RowIn q{-1, 0, 0, MsgPair<msg_t>{(msg_t)0, (msg_t)0}};
        int m, pos, l2;
        if (lane_row(base + tid, m, pos, l2)) {
          q.l2 = l2;
          const int rs = G.row_start(m), dc = G.row_deg(m);
          if (pos < dc) {
            q.e = rs + pos;
            q.j = G.row_vn(m, rs, pos);
            q.x = mp[q.e];
          }
        }
        return q;
      };
      RowIn cur = row_in(0);
      for (int base = 0; base < total; base += BS) {
        const RowIn nxt = base + BS < total ? row_in(base + BS) : RowIn{-1, 0, 0, MsgPair<msg_t>{(msg_t)0, (msg_t)0}};
        const bool valid = cur.e >= 0;
        const val_t po = (val_t)cur.x.p;
        const val_t v = valid ? ar.vin(ar.v2c((val_t)L[cur.j], (val_t)cur.x.c)) : (val_t)0;
        const val_t o = row_update_lane(ar, valid, (uint32_t)cur.e, v, cur.l2, 5);
        if (valid) {
          mp[cur.e].p = (msg_t)o;
          if constexpr (A::kFixed) {
            if (o != po) atomicAdd(&Lt[cur.j], (llr_t)(o - po));  // integer sums: any order is exact
          } else {
            // FP32: the change is kept per edge and added to Lt after the pass (a VN that several
            // checks of the step change, marked in vnmulti, takes its changes in ascending check
            // order), so that a rerun rounds the same way
            dbuf[cur.e] = o - po;
            const uint32_t bit = 1u << (cur.j & 31);
            if (atomicOr(&vnmark[cur.j >> 5], bit) & bit) atomicOr(&vnmulti[cur.j >> 5], bit);
          }
        }
        cur = nxt;
      }
      if constexpr (MSG_GLOBAL || !A::kFixed) __threadfence_block();  // pairs and step changes in global memory
      __syncthreads();
      ME_PROF_MARK(4)
      // ---- FP32: the changes of a VN that several checks of the step changed are summed exactly,
      //      each rounded to a multiple of 2^-32 and added as a 64-bit integer into the VN's LDS
      //      slot (its rank among those VNs), so that no order of the adds matters.  With more
      //      such VNs than slots, the CI pass sums their changes in ascending check order. ----
      bool use_acc = false;
      if constexpr (!A::kFixed) {
        if (tid < WAVE) {  // exclusive prefix of the per-word counts of multiply-changed VNs
          int run = 0;
          for (int w0 = 0; w0 < nvw; w0 += WAVE) {
            const int w = w0 + tid;
            const int c = w < nvw ? __popc(vnmulti[w]) : 0;
            const int ex = run + wave_excl_scan(c, tid);
            if (w < nvw) mpref[w] = ex;
            run = __builtin_amdgcn_readlane(ex + c, WAVE - 1);
          }
          if (tid == 0) misc[MS_NMULTI] = run;
        }
        __syncthreads();
        const int nmulti = misc[MS_NMULTI];
        use_acc = nmulti <= kMeAccSlots;
        if (use_acc && nmulti > 0) {
          for (int x = tid; x < nmulti; x += BS) macc[x] = 0;
          __syncthreads();
          for (int base = 0; base < total; base += BS) {
            int m, pos, l2;
            if (lane_row(base + tid, m, pos, l2)) {
              const int rs = G.row_start(m), dc = G.row_deg(m);
              if (pos < dc) {
                const int j = G.row_vn(m, rs, pos);
                const uint32_t w = vnmulti[j >> 5], bit = 1u << (j & 31);
                if (w & bit) {
                  const long long q = __float2ll_rn(dbuf[rs + pos] * 4294967296.0f);
                  atomicAdd(reinterpret_cast<unsigned long long*>(&macc[mpref[j >> 5] + __popc(w & (bit - 1))]),
                            (unsigned long long)q);
                }
              }
            }
          }
          __syncthreads();
        }
      }
      // ---- CI and CI group of every VN of those checks (each VN once) ----
      for (int base = 0; base < total; base += BS) {
        int m, pos, l2;
        if (lane_row(base + tid, m, pos, l2)) {
          const int rs = G.row_start(m), dc = G.row_deg(m);
          if (pos < dc) {
            const int j = G.row_vn(m, rs, pos);
            const uint32_t bit = 1u << (j & 31);
            // each VN once: fixed point marks it here; FP32 clears the mark the row pass set
            bool owner;
            if constexpr (A::kFixed) owner = !(atomicOr(&vnmark[j >> 5], bit) & bit);
            else owner = (atomicAnd(&vnmark[j >> 5], ~bit) & bit) != 0;
            if (owner) {
              if constexpr (!A::kFixed) {
                const uint32_t mw = vnmulti[j >> 5];
                if ((mw & bit) && use_acc) {  // the exact sum of the step's changes
                  const long long q = macc[mpref[j >> 5] + __popc(mw & (bit - 1))];
                  Lt[j] = (llr_t)((double)Lt[j] + (double)q * 0x1p-32);
                } else if (mw & bit) {  // the changes of every check of the step, ascending
                  val_t lt = (val_t)Lt[j];
                  const int dvj = G.vn_deg(j);
                  for (int k0 = 0; k0 < dvj; k0 += 16) {  // 16 loads in flight, then the sums in order
                    float dd[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                      dd[u] = 0.0f;
                      if (k0 + u < dvj) {
                        int mi, ei;
                        G.vn_edge(j, k0 + u, mi, ei);
                        if (rowmark[mi >> 5] & (1u << (mi & 31))) dd[u] = dbuf[ei];
                      }
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                      if (dd[u] != 0.0f) lt += dd[u];
                  }
                  Lt[j] = (llr_t)lt;
                } else {  // this lane's check is the only one
                  const float d = dbuf[rs + pos];
                  if (d != 0.0f) Lt[j] = (llr_t)((val_t)Lt[j] + d);
                }
              }
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
        }
      }
      __syncthreads();
      ME_PROF_MARK(5)
      for (int w = tid; w < nsw; w += BS) rowmark[w] = 0u;
      for (int w = tid; w < nvw; w += BS) vnmark[w] = 0u, vnmulti[w] = 0u;
      const int unsat = misc[MS_UNSAT];
      __syncthreads();
      if (lmd) {
        // ---- Algorithm 6: each p proposes the VN of largest CI among U(m*_p, p) (lowest index on
        //      ties), from the state after the step; distinct proposals are kept (marked in vnmark,
        //      which the next step's selection reads).  One wavefront per p ----
        for (int i = wv; i < nsel; i += nwv) {
          const int p = sel_s[i], ms = selm[i];
          const int rs = G.row_start(ms), dc = G.row_deg(ms);
          uint64_t best = 0;
          if (G.vn_deg(p) == 1) {  // Sec. V: the other VNs of m*_p
            for (int pos = ln; pos < dc; pos += WAVE) {
              const int j = G.row_vn(ms, rs, pos);
              if (j != p) best = umax64(best, mkkey(D[j], (uint32_t)j));
            }
          } else {  // the VNs other than p of p's checks other than m*_p (two-hop table)
            const int2 nb = G.nbr(p);
            for (int idx = ln; idx < nb.y; idx += WAVE) {
              const int2 ent = H.nbr[nb.x + idx];
              const int j = ent.y & 0xFFFFFF;
              if (ent.x >= 0 && j != p && (ent.x < rs || ent.x >= rs + dc)) best = umax64(best, mkkey(D[j], (uint32_t)j));
            }
          }
          best = wave_max_u64(best);
          if (ln == 0 && best != 0ull) {
            const int q = (int)key_idx(best);
            const uint32_t bit = 1u << (q & 31);
            if (!(atomicOr(&vnmark[q >> 5], bit) & bit)) succ[atomicAdd(&misc[MS_NSUCC], 1)] = q;
          }
        }
        __syncthreads();
      }
      if (tid == 0) misc[MS_NROWS] = 0;
      t += nsel;
      steps += 1;
      if (ce > 0 && (t / ce) != (tprev / ce) && unsat == 0) done = true;
      __syncthreads();
      ME_PROF_MARK(6)
    }
    ME_PROF_FLUSH

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
      if (P.out.dump_c2v) P.out.dump_c2v[(size_t)f * E + e] = ar.as_float((val_t)mp[e].c);
      if (P.out.dump_pre) P.out.dump_pre[(size_t)f * E + e] = ar.as_float((val_t)mp[e].p);
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
