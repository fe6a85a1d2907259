// Per-frame body of the single-edge dynamic decoder (RBP, CIRBP, replay, and the latest-message-
// driven LMDRBP, sLMDRBP and LMD-CIRBP) for one wavefront; used by the per-code kernel and by the
// persistent batched kernel.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace ldpc {

#ifdef LDPC_PROFILE
// phase timing for development builds only: per-phase clock64() deltas summed over updates
#define PROF_DECL long long prof_acc[8] = {0, 0, 0, 0, 0, 0, 0, 0}; long long prof_t = clock64();
#define PROF_MARK(i) { long long now_ = clock64(); prof_acc[i] += now_ - prof_t; prof_t = now_; }
#define PROF_FLUSH { if (lane == 0 && P.prof) for (int i_ = 0; i_ < 8; ++i_) atomicAdd((unsigned long long*)&P.prof[i_], (unsigned long long)prof_acc[i_]); }
#else
#define PROF_DECL
#define PROF_MARK(i)
#define PROF_FLUSH
#endif

__device__ __forceinline__ unsigned char* dyn_lds() {
  extern __shared__ __align__(16) unsigned char lds_dyn[];
  return lds_dyn;
}

// A workgroup holds P.wpb frames, one per wavefront: the LDS region of this wavefront's frame, and
// the index of its frame slot in global scratch
// (the wavefront index is made scalar so that frame addresses stay wave-uniform)
__device__ __forceinline__ int wave_in_group() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }
__device__ __forceinline__ unsigned char* frame_lds(const DynParams& P) {
  return dyn_lds() + P.frame_base + wave_in_group() * P.frame_stride;
}
__device__ __forceinline__ size_t frame_slot(const DynParams& P) {
  return (size_t)blockIdx.x * (size_t)P.wpb + (size_t)wave_in_group();
}

// Where a frame's state lives.  C2V messages (c2v), precomputed messages (pre), precomputed totals
// (Lt), totals (L) and CIs (D): all in LDS; pre in a global scratch slot; c2v and pre as
// interleaved (c2v, pre) pairs (one load brings the two values of an edge) in a global slot; those
// pairs followed by Lt in the slot; the whole frame in the slot (Lt, L and D as arrays, or as one
// 8-byte (Lt, L) record per VN with D evaluated from it).  A frame is read and written by its own
// wavefront only, so lanes
// exchange values through global memory under the wavefront's program order (wave_sync).
template <class A, int STORE, bool PAIRS = (STORE >= STORE_ALL_GLOBAL), bool STREAM = false>
struct MsgStore {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  static constexpr bool kDerivedD = false;
  msg_t* c2v;  // LDS
  msg_t* pre;  // LDS (STORE_LDS) or global (STORE_PRE_GLOBAL)
  llr_t* Lt;   // LDS
  llr_t* Lp;   // LDS
  uint32_t* Dp;
  __device__ __forceinline__ msg_t c(int e) const { return c2v[e]; }
  __device__ __forceinline__ msg_t p(int e) const { return pre[e]; }
  __device__ __forceinline__ void set_c(int e, msg_t v) const { c2v[e] = v; }
  __device__ __forceinline__ void set_p(int e, msg_t v) const { pre[e] = v; }
  __device__ __forceinline__ void cp(int e, msg_t& cv, msg_t& pv) const {
    cv = c2v[e];
    pv = pre[e];
  }
  __device__ __forceinline__ llr_t lt(int n) const { return Lt[n]; }
  __device__ __forceinline__ void set_lt(int n, llr_t v) const { Lt[n] = v; }
  __device__ __forceinline__ void add_lt(int n, llr_t d) const { atomicAdd(&Lt[n], d); }
  __device__ __forceinline__ llr_t l(int n) const { return Lp[n]; }
  __device__ __forceinline__ void set_l(int n, llr_t v) const { Lp[n] = v; }
  __device__ __forceinline__ uint32_t d(int n) const { return Dp[n]; }
  __device__ __forceinline__ void set_d(int n, uint32_t v) const { Dp[n] = v; }
  __device__ __forceinline__ void lt_l(int n, llr_t& ltv, llr_t& lv) const {
    ltv = Lt[n];
    lv = Lp[n];
  }
  __device__ __forceinline__ void set_lt_d(int n, llr_t ltv, uint32_t dv) const {
    Lt[n] = ltv;
    Dp[n] = dv;
  }
};

// per-VN record of the record layouts: Lt and L in one aligned 8-byte word.  D is not stored: it
// is the function ci(L, Lt) of the record and is evaluated where it is needed (kDerivedD).
template <class llr_t>
struct alignas(8) VnRec {
  llr_t lt;
  llr_t l;
};

template <class A, int STORE, bool STREAM>
struct MsgStore<A, STORE, true, STREAM> {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  static constexpr bool kRec = STORE == STORE_FRAME_REC || STORE == STORE_FRAME_ALL;
  static constexpr bool kDerivedD = kRec;
  MsgPair<msg_t>* m;  // global, [E]
  llr_t* Lt;          // LDS (STORE_ALL_GLOBAL) or global, [N]
  llr_t* Lp;          // LDS, or global (STORE_FRAME_GLOBAL), [N]
  uint32_t* Dp;
  VnRec<llr_t>* r;    // STORE_FRAME_REC, [N]
  __device__ __forceinline__ msg_t c(int e) const { return m[e].c; }
  __device__ __forceinline__ msg_t p(int e) const { return m[e].p; }
  // STREAM: the per-code kernel's frames whose whole state lives in global memory exceed the L2
  // and MALL by far; their message pairs are read and written with the non-temporal hint, which
  // leaves the caches to the VN records and the code's tables (c1: 3.6% more frames/s; the same
  // hint on the records cost 12%).  The batched kernel's mix of small codes keeps part of its
  // pairs in the caches and goes without it (the hint cost it 11-18%).
  static constexpr bool kStream = STREAM && STORE >= STORE_FRAME_GLOBAL;
  using pair_bits_t = typename std::conditional<sizeof(MsgPair<msg_t>) == 8, unsigned long long, unsigned short>::type;
  __device__ __forceinline__ void set_c(int e, msg_t v) const {
    if constexpr (kStream) __builtin_nontemporal_store(v, &m[e].c);
    else m[e].c = v;
  }
  __device__ __forceinline__ void set_p(int e, msg_t v) const {
    if constexpr (kStream) __builtin_nontemporal_store(v, &m[e].p);
    else m[e].p = v;
  }
  __device__ __forceinline__ void cp(int e, msg_t& cv, msg_t& pv) const {
    MsgPair<msg_t> x;
    if constexpr (kStream) x = __builtin_bit_cast(MsgPair<msg_t>, __builtin_nontemporal_load(reinterpret_cast<const pair_bits_t*>(m + e)));
    else x = m[e];
    cv = x.c;
    pv = x.p;
  }
  __device__ __forceinline__ llr_t lt(int n) const {
    if constexpr (kRec) return r[n].lt;
    else return Lt[n];
  }
  __device__ __forceinline__ void set_lt(int n, llr_t v) const {
    if constexpr (kRec) r[n].lt = v;
    else Lt[n] = v;
  }
  __device__ __forceinline__ void add_lt(int n, llr_t d) const {
    if constexpr (kRec) atomicAdd(&r[n].lt, d);
    else atomicAdd(&Lt[n], d);
  }
  __device__ __forceinline__ llr_t l(int n) const {
    if constexpr (kRec) return r[n].l;
    else return Lp[n];
  }
  __device__ __forceinline__ void set_l(int n, llr_t v) const {
    if constexpr (kRec) r[n].l = v;
    else Lp[n] = v;
  }
  __device__ __forceinline__ uint32_t d(int n) const {  // stored CI (not for the record layouts)
    static_assert(!kRec, "the record layouts derive D from the record");
    return Dp[n];
  }
  __device__ __forceinline__ void set_d(int n, uint32_t v) const {
    if constexpr (!kRec) Dp[n] = v;
  }
  __device__ __forceinline__ void lt_l(int n, llr_t& ltv, llr_t& lv) const {
    if constexpr (kRec) {
      const VnRec<llr_t> x = r[n];  // one 8-byte load
      ltv = x.lt;
      lv = x.l;
    } else {
      ltv = Lt[n];
      lv = Lp[n];
    }
  }
  __device__ __forceinline__ void set_lt_d(int n, llr_t ltv, uint32_t dv) const {
    if constexpr (kRec) {
      r[n].lt = ltv;  // D follows from the record
    } else {
      Lt[n] = ltv;
      Dp[n] = dv;
    }
  }
};

// message store of the workgroup's frame slot (slot_edges = edges reserved per workgroup when
// only pre is global; the pair-slot layout comes from P.slot_bytes and the slot offsets)
template <class A, int STORE, bool STREAM = false>
using FrameStore = MsgStore<A, STORE, (STORE >= STORE_ALL_GLOBAL), STREAM>;

template <class A, int STORE, bool STREAM = false>
__device__ __forceinline__ FrameStore<A, STORE, STREAM> make_store(const DynParams& P, size_t slot_edges) {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  unsigned char* lds = frame_lds(P);
  FrameStore<A, STORE, STREAM> ms;
  ms.Lp = reinterpret_cast<llr_t*>(lds + P.off_L);
  ms.Dp = reinterpret_cast<uint32_t*>(lds + P.off_D);
  ms.Lt = reinterpret_cast<llr_t*>(lds + P.off_Lt);
  if constexpr (STORE >= STORE_ALL_GLOBAL) {
    unsigned char* base = reinterpret_cast<unsigned char*>(P.pre_global) + frame_slot(P) * (size_t)P.slot_bytes;
    ms.m = reinterpret_cast<MsgPair<msg_t>*>(base);
    ms.r = nullptr;
    if constexpr (STORE == STORE_ALL_GLOBAL_LT || STORE == STORE_FRAME_GLOBAL)
      ms.Lt = reinterpret_cast<llr_t*>(base + P.slot_lt_off);
    if constexpr (STORE == STORE_FRAME_GLOBAL) {
      ms.Lp = reinterpret_cast<llr_t*>(base + P.slot_l_off);
      ms.Dp = reinterpret_cast<uint32_t*>(base + P.slot_d_off);
    }
    if constexpr (STORE == STORE_FRAME_REC || STORE == STORE_FRAME_ALL)
      ms.r = reinterpret_cast<VnRec<llr_t>*>(base + P.slot_lt_off);
  } else {
    ms.c2v = reinterpret_cast<msg_t*>(lds + P.off_c2v);
    if constexpr (STORE == STORE_PRE_GLOBAL) ms.pre = reinterpret_cast<msg_t*>(P.pre_global) + frame_slot(P) * slot_edges;
    else ms.pre = reinterpret_cast<msg_t*>(lds + P.off_pre);
  }
  return ms;
}

// Block-maximum maintenance after the leaf key of index i in block b moved from its old value to
// nk: a larger key raises the block maximum; a smaller one marks the block for recomputation if
// i held the maximum (a maximum key carries its index, so the old value is not needed).  Lanes
// racing on one block in one instruction stay correct in either order: a raise by another lane
// only makes the old maximum irrelevant, and a marked block is recomputed from the leaves.
__device__ __forceinline__ void leaf_moved(uint64_t* blk, uint32_t* mask, int b, uint32_t i, uint64_t nk) {
  const uint64_t cur = blk[b];
  if (nk > cur) atomicMax(reinterpret_cast<unsigned long long*>(&blk[b]), (unsigned long long)nk);
  else if (nk < cur && key_idx(cur) == i) atomicOr(&mask[b >> 5], 1u << (b & 31));
}

// LMD: the variant for the LMD schedules (a separate instantiation, so that the others keep their
// register budget); J.kind must then be one of them
template <class A, int STORE, class Topo, bool LMD = false, bool STREAM = false>
__device__ __forceinline__ void dyn_decode_frame(const DevCode& H, const Topo& G, const A& ar, const DynParams& P,
                                                 const FrameStore<A, STORE, STREAM>& ms, const FrameJob& J) {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  using val_t = typename A::val_t;
  using Acc = typename RowAccOf<A>::type;
  const int lane = threadIdx.x & (WAVE - 1);
  unsigned char* lds = frame_lds(P);
  // per check: the largest residual of its edges (value bits); block keys pair it with the check
  // index, and the edge is found again inside the check's row when the check is selected (edge ids
  // are row-major, so (value, lowest check), then (value, lowest edge) in the row is the global
  // (value, lowest edge))
  constexpr bool kKeysG = STORE == STORE_FRAME_ALL;  // check keys in the slot
  constexpr bool kStageG = STORE >= STORE_ALL_GLOBAL;  // late-CI staging in the slot
  unsigned char* slot = kStageG ? reinterpret_cast<unsigned char*>(P.pre_global) + frame_slot(P) * (size_t)P.slot_bytes
                                : nullptr;
  uint32_t* ckey = kKeysG ? reinterpret_cast<uint32_t*>(slot + P.slot_ckey_off) : reinterpret_cast<uint32_t*>(lds + P.off_ckey);
  uint64_t* dblk = reinterpret_cast<uint64_t*>(lds + P.off_dblk);
  uint64_t* cblk = reinterpret_cast<uint64_t*>(lds + P.off_cblk);
  uint32_t* dmask = reinterpret_cast<uint32_t*>(lds + P.off_dmask);
  uint32_t* cmask = reinterpret_cast<uint32_t*>(lds + P.off_cmask);
  uint32_t* synw = reinterpret_cast<uint32_t*>(lds + P.off_syn);  // syndrome bits
  int* tj = kStageG ? reinterpret_cast<int*>(slot + P.slot_tj_off)
                    : reinterpret_cast<int*>(lds + P.off_v);  // VN of a table lane whose CI is refreshed late
  // VNs met twice in the two-hop table: per group, the sum of this update's Lt changes, the VN's
  // Lt and L before the update, the VN; a flag word of the groups changed
  llr_t* gacc = reinterpret_cast<llr_t*>(lds + P.off_grp);
  llr_t* glt = gacc + (kGroups + 1);
  llr_t* gl = glt + (kGroups + 1);
  int* gj = reinterpret_cast<int*>(gl + (kGroups + 1));
  uint32_t* gflag = reinterpret_cast<uint32_t*>(gj + (kGroups + 1));
  const int N = H.N, M = H.M, E = H.E;
  const int nbd = (N + WAVE - 1) / WAVE, nbc = (M + WAVE - 1) / WAVE;
  const int nbd_words = (nbd + 31) / 32, nbc_words = (nbc + 31) / 32;
  // LMD schedules (Sec. IV): after the first update the next one is chosen among the messages the
  // update just precomputed, so the global selection keys are used once and then left stale
  constexpr bool lmd = LMD;
  const bool lmd_ci = LMD && J.kind == KIND_LMD_CIRBP;
  const bool with_ci = J.kind == KIND_CIRBP || J.kind == KIND_REPLAY || lmd_ci;
  // CI of VN n: stored, or evaluated from the VN's record (record layouts); RBP and the residual
  // LMD schedules keep none
  auto d_of = [&](int n) -> uint32_t {
    if constexpr (FrameStore<A, STORE, STREAM>::kDerivedD) {
      llr_t ltv, lv;
      ms.lt_l(n, ltv, lv);
      return with_ci ? ar.ci((val_t)lv, (val_t)ltv) : 0u;
    } else {
      return ms.d(n);
    }
  };
  // ---------------- Algorithm 1, initialisation: initial state ---------------------------
  const float* llr = J.llr;
  for (int n = lane; n < N; n += WAVE) ms.set_l(n, (llr_t)ar.channel(llr[n]));
  for (int e = lane; e < E; e += WAVE) ms.set_c(e, (msg_t)0);
  for (int w = lane; w < nbd_words; w += WAVE) dmask[w] = 0u;
  for (int w = lane; w < nbc_words; w += WAVE) cmask[w] = 0u;
  for (int w = lane; w < (M + 31) / 32; w += WAVE) synw[w] = 0u;
  if (lane <= kGroups) gacc[lane] = (llr_t)0;
  if (lane == 0) *gflag = 0u;
  wave_sync();
  // every precomputed C2V message from V2C = channel value: one lane per check row
  int unsat_local = 0;
  for (int m = lane; m < M; m += WAVE) {
    const int rs = G.row_start(m), dc = G.row_deg(m);
    Acc acc;
    int par = 0;
    for (int p = 0; p < dc; ++p) {
      const val_t l = (val_t)ms.l(G.row_vn(m, rs, p));
      const val_t v = ar.vin(l);
      acc.add(p, v, row_aux(ar, v));
      par ^= l < 0 ? 1 : 0;
    }
    uint64_t k = 0;
    for (int p = 0; p < dc; ++p) {
      const val_t v = ar.vin((val_t)ms.l(G.row_vn(m, rs, p)));
      const val_t o = acc.out(p, v, row_aux(ar, v));
      ms.set_p(rs + p, (msg_t)o);
      k = umax64(k, mkkey(ar.res(o, (val_t)0), (uint32_t)(rs + p)));
    }
    ckey[m] = key_val(k);
    if (par) atomicOr(&synw[m >> 5], 1u << (m & 31));
    unsat_local += par;
  }
  int unsat = wave_sum_i32(unsat_local);
  wave_sync();
  for (int n = lane; n < N; n += WAVE) {
    const val_t l = (val_t)ms.l(n);
    val_t lt = l;
    const int dv = G.vn_deg(n);
    for (int k = 0; k < dv; ++k) {
      int m, e;
      G.vn_edge(n, k, m, e);
      lt += (val_t)ms.p(e);
    }
    ms.set_lt_d(n, (llr_t)lt, with_ci ? ar.ci(l, lt) : 0u);
  }
  wave_sync();
  for (int b = 0; b < nbd; ++b) {
    const int n = b * WAVE + lane;
    uint64_t k = n < N ? mkkey(d_of(n), (uint32_t)n) : 0ull;
    k = wave_max_u64(k);
    if (lane == 0) dblk[b] = k;
  }
  for (int b = 0; b < nbc; ++b) {
    const int m = b * WAVE + lane;
    uint64_t k = m < M ? mkkey(ckey[m], (uint32_t)m) : 0ull;
    k = wave_max_u64(k);
    if (lane == 0) cblk[b] = k;
  }
  wave_sync();

  // ---------------- update loop -------------------------------------------------------
  long long t = 0, nfall = 0;
  // LMD: the choice the last update made (an edge for sLMDRBP, the VN n' otherwise); -1 before the
  // first update, whose choice is global
  int lmd_next = -1;
  long long limit = J.max_updates;
  if (J.kind == KIND_REPLAY && J.replay_len < limit) limit = J.replay_len;
  const long long ce = J.kind == KIND_REPLAY ? 0 : J.check_every;
  long long until_check = ce;  // updates left until the next syndrome test
  bool done = ce > 0 && unsat == 0;
  PROF_DECL
  while (!done && t < limit) {
    PROF_MARK(7)
    // ---- selection (Algorithm 1: CI maximum, threshold test, incoming edge; RBP eq. (5)) ----
    int estar, mstar = -1, nstar = -1;
    msg_t c_star = (msg_t)0, p_star = (msg_t)0;  // messages of e*, taken from the selection's loads
    bool have_star = false;
    bool have_row = false;                        // lane p holds the pairs of edge row_start(m*) + p
    msg_t row_cm = (msg_t)0, row_pm = (msg_t)0;
    // n*'s record and two-hop table entries are requested as soon as n* is known (on the CI path
    // before the selection's own loads), so that their round trips overlap
    int dv = 0, ncnt = 0, npass = 0, noff = 0, rs_m = 0, re_m = 0, dc_m = 0;
    bool row_only = false;  // n* on no check but m*: nothing is precomputed again
    llr_t lt_n = (llr_t)0, l_n = (llr_t)0;
    int2 ent0 = make_int2(-1, 0), ent_next = make_int2(-1, 0);
    auto load_ent = [&](int ps) -> int2 {
      const int idx = ps * WAVE + lane;
      return idx < ncnt ? H.nbr[noff + idx] : make_int2(-1, 0);
    };
    auto start_nstar = [&](int n) {
      if (with_ci) ms.lt_l(n, lt_n, l_n);
      else l_n = ms.l(n);
      dv = uni(G.vn_deg(n));
      row_only = dv == 1;
      if (!row_only) {
        const int2 nb = G.nbr(n);
        noff = uni(nb.x);
        ncnt = uni(nb.y);
        npass = (ncnt + WAVE - 1) / WAVE;
        ent0 = load_ent(0);
        if (npass > 1) ent_next = load_ent(1);
      }
    };
    if (J.kind == KIND_REPLAY) {
      estar = uni(J.replay[t]);
      if (estar < 0 || estar >= E) break;  // invalid edge id ends the frame's replay
      mstar = uni(G.edge_row(estar));
      nstar = uni(G.edge_vn(estar));
      start_nstar(nstar);
    } else if (lmd && J.kind == KIND_SLMDRBP && lmd_next >= 0) {  // sLMDRBP: the edge chosen last time
      estar = lmd_next;
      mstar = uni(G.edge_row(estar));
      nstar = uni(G.edge_vn(estar));
      start_nstar(nstar);
    } else {
      // RBP, and the first update of LMDRBP / sLMDRBP: the global residual maximum
      bool global_res = J.kind == KIND_RBP || (lmd && J.kind != KIND_LMD_CIRBP && lmd_next < 0);
      int nsel = -1;
      if (lmd && !global_res && lmd_next >= 0) {
        nsel = lmd_next;  // LMDRBP, LMD-CIRBP: n' receives its incoming edge of largest residual
      } else if (!global_res) {
        uint64_t k = 0;
        for (int b = lane; b < nbd; b += WAVE) k = umax64(k, dblk[b]);
        k = wave_max_u64(k);
        nsel = (int)key_idx(k);
        if (J.kind == KIND_CIRBP && key_val(k) < J.gamma_bits) {  // D_{n*} < gamma: RBP fallback
          global_res = true;
          nfall += 1;
        }
      }
      if (global_res) {
        uint64_t k = 0;
        for (int b = lane; b < nbc; b += WAVE) k = umax64(k, cblk[b]);
        const int mrow = (int)key_idx(wave_max_u64(k));
        const int rs = uni(G.row_start(mrow)), dc = uni(G.row_deg(mrow));
        uint64_t ke = 0;
        msg_t cm = (msg_t)0, pm = (msg_t)0;
        if (lane < dc) {  // the largest residual of the check's row, lowest edge on ties
          ms.cp(rs + lane, cm, pm);
          ke = mkkey(ar.res((val_t)pm, (val_t)cm), (uint32_t)(rs + lane));
        }
        estar = (int)key_idx(wave_max_u64(ke));
        mstar = mrow;
        nstar = uni(G.row_vn(mrow, rs, estar - rs));
        start_nstar(nstar);
        c_star = lane_value(cm, estar - rs);
        p_star = lane_value(pm, estar - rs);
        have_star = true;
        have_row = true;
        row_cm = cm;
        row_pm = pm;
      } else {
        nstar = nsel;
        start_nstar(nstar);
        uint64_t k = 0;
        int mk = -1;
        msg_t cm = (msg_t)0, pm = (msg_t)0;
        if (lane < dv) {
          int e;
          G.vn_edge(nsel, lane, mk, e);
          ms.cp(e, cm, pm);
          k = mkkey(ar.res((val_t)pm, (val_t)cm), (uint32_t)e);
        }
        const uint64_t kmax = wave_max_u64(k);
        estar = (int)key_idx(kmax);
        const unsigned long long win = __ballot(lane < dv && k == kmax);
        const int wl = (int)__builtin_ctzll(win);
        mstar = __builtin_amdgcn_readlane(mk, wl);
        c_star = lane_value(cm, wl);
        p_star = lane_value(pm, wl);
        have_star = true;
      }
    }
    PROF_MARK(0)
    int my_m = -1;
    if (lane < dv) {
      int e;
      G.vn_edge(nstar, lane, my_m, e);
    }
    rs_m = uni(G.row_start(mstar));
    dc_m = uni(G.row_deg(mstar));
    re_m = rs_m + dc_m;
    // Inputs of the touched-check passes are loaded ahead of use: table entries two passes ahead,
    // message pairs, L and Lt one pass ahead.  Nothing a pass writes is read by a later pass
    // except Lt of a VN listed twice in the two-hop table (such VNs take the summed paths below and
    // do not use the early value), and propagation changes only c2v[e*] and L[n*] (both
    // overridden where used), so the early loads see the values the passes need.  Lanes of m*'s
    // row and of n* itself update nothing and load no VN record.
    struct PassIn {
      int2 ent;
      msg_t cm, pm;
      llr_t lj, ltj;
    };
    auto load_in = [&](int2 ent) -> PassIn {
      PassIn q;
      q.ent = ent;
      q.cm = (msg_t)0;
      q.pm = (msg_t)0;
      q.lj = (llr_t)0;
      q.ltj = (llr_t)0;
      if (ent.x >= 0) {
        ms.cp(ent.x, q.cm, q.pm);
        const int j = ent.y & 0xFFFFFF;
        if (j != nstar && (ent.x < rs_m || ent.x >= re_m)) {
          if (with_ci) ms.lt_l(j, q.ltj, q.lj);
          else q.lj = ms.l(j);
        }
      }
      return q;
    };

    // ---- propagation (Algorithm 1) and D_{n*} ----
    if (!have_star) ms.cp(estar, c_star, p_star);
    PassIn in_cur{make_int2(-1, 0), (msg_t)0, (msg_t)0, (llr_t)0, (llr_t)0};
    if (!row_only) in_cur = load_in(ent0);
    else if (!have_row && lane < dc_m) ms.cp(rs_m + lane, row_cm, row_pm);
    const val_t newv = (val_t)p_star;
    const val_t oldv = (val_t)c_star;
    const val_t Lold = (val_t)l_n;
    const val_t Lnew = Lold + (newv - oldv);
    const uint32_t dn_new = with_ci ? ar.ci(Lnew, (val_t)lt_n) : 0u;
    wave_sync();
    if (lane == 0) {
      ms.set_c(estar, (msg_t)newv);
      ms.set_l(nstar, (llr_t)Lnew);
      if (with_ci) {
        ms.set_d(nstar, dn_new);
        if (!lmd) leaf_moved(dblk, dmask, nstar >> 6, (uint32_t)nstar, mkkey(dn_new, (uint32_t)nstar));
      }
    }
    if ((Lold < 0) != (Lnew < 0)) {  // hard decision flipped: toggle the checks of n*
      int d = 0;
      if (lane < dv) {
        const uint32_t bit = 1u << (my_m & 31);
        const uint32_t old = atomicXor(&synw[my_m >> 5], bit);
        d = (old & bit) ? -1 : 1;
      }
      unsat += wave_sum_i32(d);
    }
    wave_sync();
    PROF_MARK(1)

    // LMD candidates of this lane: the largest key (residual and edge, or CI and VN) and its VN
    uint64_t lk = 0;
    int lkj = -1;
    auto lmd_offer = [&](uint64_t k, int j) {
      if (k > lk) {
        lk = k;
        lkj = j;
      }
    };
    if (row_only && lmd) {  // n* has degree 1: the candidates are the other edges / VNs of m* (Sec. V)
      if (lane < dc_m) {
        const int e = rs_m + lane;
        const int j = G.row_vn(mstar, rs_m, lane);
        if (j != nstar) {
          if (lmd_ci) lmd_offer(mkkey(d_of(j), (uint32_t)j), j);
          else lmd_offer(mkkey(ar.res((val_t)row_pm, (val_t)row_cm), (uint32_t)e), j);
        }
      }
    } else if (row_only) {  // m*'s new residual key: its row with c2v[e*] = pre[e*]
      uint64_t k = 0;
      if (lane < dc_m) {
        const int e = rs_m + lane;
        const val_t cv = e == estar ? newv : (val_t)row_cm;
        k = mkkey(ar.res((val_t)row_pm, cv), (uint32_t)e);
      }
      const uint32_t kv = key_val(wave_max_u64(k));
      if (lane == 0) {
        ckey[mstar] = kv;
        leaf_moved(cblk, cmask, mstar >> 6, (uint32_t)mstar, mkkey(kv, (uint32_t)mstar));
      }
    }

    // ---- touched checks: V2C inputs, whole-row update, residual keys, and the CI of every VN
    //      listed once in the table (Algorithm 1, the loop over M(n*) \ m*; one pass per 64 lanes) ----
    bool late_ci = false;  // a VN of the overflow group was updated: its CI is refreshed after the passes
    uint32_t late_passes = 0u;  // passes that staged such VNs (only those write and read the staging)
    for (int ps = 0; ps < npass; ++ps) {
      PassIn in_next{make_int2(-1, 0), (msg_t)0, (msg_t)0, (llr_t)0, (llr_t)0};
      int2 ent_after = make_int2(-1, 0);
      if (ps + 1 < npass) in_next = load_in(ent_next);
      if (ps + 2 < npass) ent_after = load_ent(ps + 2);
      const int2 ent = in_cur.ent;
      const int e = ent.x;
      const bool valid = e >= 0;
      const int j = ent.y & 0xFFFFFF;
      const int L2 = (ent.y >> 24) & 7;
      const bool leader = valid && ((ent.y >> 27) & 1);
      const bool twice = (ent.y >> 28) & 1;
      const int grp = (ent.y >> 29) & 7;
      const bool in_m = valid && e >= rs_m && e < re_m;
      const bool self = valid && j == nstar;
      val_t cv = 0, po = 0, lv = 0;
      if (valid) {
        cv = e == estar ? newv : (val_t)in_cur.cm;  // this update's propagation
        po = (val_t)in_cur.pm;
        lv = self ? Lnew : (val_t)in_cur.lj;
      }
      const bool upd = valid && !in_m && !self;
      val_t pv = po;
      const int maxL2 = uni(L2);  // lane 0 starts the pass's largest block
      if (__ballot(upd) != 0ull) {  // some row of the pass is precomputed again
        const val_t v = ar.vin(ar.v2c(lv, cv));
        const val_t o = row_update_lane(ar, valid, (uint32_t)e, v, L2, maxL2);
        if (upd) pv = o;
      }
      if (upd) {
        // a value that did not change is not written again: the frame state of the large codes
        // lives in global memory, where every scattered write costs the memory system a request
        if (pv != po) ms.set_p(e, (msg_t)pv);
        if (with_ci) {
          const val_t dlt = pv - po;
          if (!twice) {  // the only change of Lt_j in this update: new Lt_j and D_j right here
            const val_t ltn = (val_t)in_cur.ltj + dlt;
            const uint32_t nd = ar.ci(lv, ltn);
            if (ltn != (val_t)in_cur.ltj) ms.set_lt_d(j, (llr_t)ltn, nd);  // else Lt_j and D_j stand
            if (lmd) lmd_offer(mkkey(nd, (uint32_t)j), j);
            else leaf_moved(dblk, dmask, j >> 6, (uint32_t)j, mkkey(nd, (uint32_t)j));
          } else if (grp < kGroups) {  // summed in LDS; Lt_j itself is untouched until the passes end
            atomicAdd(&gacc[grp], (llr_t)dlt);
            gj[grp] = j;
            glt[grp] = in_cur.ltj;
            gl[grp] = (llr_t)lv;
            atomicOr(gflag, 1u << grp);
          } else {
            ms.add_lt(j, (llr_t)dlt);
          }
        }
      }
      const bool late = with_ci && upd && twice && grp == kGroups;
      if (__ballot(late) != 0ull) {  // rare: staging lives in the global slot for the large codes
        tj[ps * WAVE + lane] = late ? j : -1;
        late_passes |= 1u << ps;
        late_ci = true;
      }
      if (lmd) {
        if (upd && !lmd_ci) lmd_offer(mkkey(ar.res(pv, cv), (uint32_t)e), j);
      } else {
        const uint64_t rk = keymax_all(valid ? mkkey(ar.res(pv, cv), (uint32_t)e) : 0ull, L2, maxL2);
        if (leader) {  // one lane per check: new residual key, block maximum
          const int m = G.edge_row(e);
          ckey[m] = key_val(rk);
          leaf_moved(cblk, cmask, m >> 6, (uint32_t)m, mkkey(key_val(rk), (uint32_t)m));
        }
      }
      in_cur = in_next;
      ent_next = ent_after;
    }
    wave_sync();
    PROF_MARK(3)
    // ---- VNs listed twice: Lt_j plus the summed changes, then D_j ----
    const uint32_t gf = (uint32_t)uni((int)*gflag);
    if (gf) {
      if (lane < kGroups && ((gf >> lane) & 1u)) {
        const val_t ltn = (val_t)glt[lane] + (val_t)gacc[lane];
        const int jg = gj[lane];
        const uint32_t nd = ar.ci((val_t)gl[lane], ltn);
        ms.set_lt_d(jg, (llr_t)ltn, nd);
        if (lmd) lmd_offer(mkkey(nd, (uint32_t)jg), jg);
        else leaf_moved(dblk, dmask, jg >> 6, (uint32_t)jg, mkkey(nd, (uint32_t)jg));
        gacc[lane] = (llr_t)0;
      }
      wave_sync();
      if (lane == 0) *gflag = 0u;
      wave_sync();
    }
    // ---- CI of the VNs of the overflow group (their Lt took several atomic additions) ----
    if (late_ci) {
      for (int ps = 0; ps < npass; ++ps) {
        if (!((late_passes >> ps) & 1u)) continue;  // nothing staged in this pass
        const int j = tj[ps * WAVE + lane];
        uint32_t nd = 0;
        if (j >= 0) {
          llr_t ltv, lv;
          ms.lt_l(j, ltv, lv);
          nd = ar.ci((val_t)lv, (val_t)ltv);
        }
        wave_sync();
        if (j >= 0) {
          ms.set_d(j, nd);
          if (lmd) lmd_offer(mkkey(nd, (uint32_t)j), j);
          else leaf_moved(dblk, dmask, j >> 6, (uint32_t)j, mkkey(nd, (uint32_t)j));
        }
        wave_sync();
      }
    }
    PROF_MARK(5)
    // ---- LMD: the next choice, the largest candidate key (lowest edge / VN on ties).  The set is
    //      never empty: every check has degree 2 or more, so m* or a check of M(n*) \ m* has a VN
    //      other than n* ----
    if constexpr (LMD) {
      const uint64_t kmax = wave_max_u64(lk);
      const unsigned long long win = __ballot(lk == kmax && lk != 0ull);
      if (J.kind == KIND_SLMDRBP) lmd_next = kmax ? (int)key_idx(kmax) : -1;
      else lmd_next = win ? __builtin_amdgcn_readlane(lkj, (int)__builtin_ctzll(win)) : -1;
    }
    // ---- blocks whose maximum leaf decreased: one check block and one VN block per round, so
    //      that their leaf loads share a round trip (nothing to do for the LMD schedules) ----
    if (!lmd) {
      int cw = 0, dw = 0;
      uint32_t cbits = nbc_words > 0 ? (uint32_t)uni((int)cmask[0]) : 0u;
      uint32_t dbits = (with_ci && nbd_words > 0) ? (uint32_t)uni((int)dmask[0]) : 0u;
      while (true) {
        while (cbits == 0u && cw + 1 < nbc_words) {
          if (lane == 0) cmask[cw] = 0u;
          cw += 1;
          cbits = (uint32_t)uni((int)cmask[cw]);
        }
        while (with_ci && dbits == 0u && dw + 1 < nbd_words) {
          if (lane == 0) dmask[dw] = 0u;
          dw += 1;
          dbits = (uint32_t)uni((int)dmask[dw]);
        }
        if (cbits == 0u && dbits == 0u) break;
        int bc = -1, bd = -1;
        if (cbits) {
          bc = cw * 32 + __builtin_ctz(cbits);
          cbits &= cbits - 1;
        }
        if (dbits) {
          bd = dw * 32 + __builtin_ctz(dbits);
          dbits &= dbits - 1;
        }
        const int m = bc * WAVE + lane, n = bd * WAVE + lane;
        const uint32_t kc = (bc >= 0 && m < M) ? ckey[m] : 0u;
        const uint32_t kd = (bd >= 0 && n < N) ? d_of(n) : 0u;
        if (bc >= 0) {
          const uint64_t k = wave_max_u64(m < M ? mkkey(kc, (uint32_t)m) : 0ull);
          if (lane == 0) cblk[bc] = k;
        }
        if (bd >= 0) {
          const uint64_t k = wave_max_u64(n < N ? mkkey(kd, (uint32_t)n) : 0ull);
          if (lane == 0) dblk[bd] = k;
        }
      }
      if (lane == 0) {
        if (nbc_words > 0) cmask[cw] = 0u;
        if (with_ci && nbd_words > 0) dmask[dw] = 0u;
      }
    }
    wave_sync();
    PROF_MARK(6)
#ifdef LDPC_SELFCHECK
    // ---- self-checking builds: the state of the touched neighbourhood against its definition.
    //      For every VN of the two-hop table, of m*'s row and n* itself: L = channel + sum of
    //      C2V, Lt = channel + sum of the precomputed messages, a stored D = ci(L, Lt) (exact in
    //      fixed point; FP32 within 1e-3 of the larger magnitude, the incremental sums having
    //      rounded in another order); for every check of n*, its key = the largest residual of its
    //      row; the VN block of n* and the check block of m* = the largest of their leaves (keys
    //      and blocks not for the LMD schedules, which leave them stale by design).  Mismatches
    //      are counted per kind; nothing stops the decode. ----
    if (P.selfcheck) {
      auto close = [&](val_t a, val_t b) -> bool {
        if constexpr (A::kFixed) {
          return a == b;
        } else {
          const float x = ar.as_float(a), y = ar.as_float(b);
          return fabsf(x - y) <= 1e-3f * fmaxf(1.0f, fmaxf(fabsf(x), fabsf(y)));
        }
      };
      auto check_vn = [&](int j) -> int {
        const val_t ch = ar.channel(J.llr[j]);
        val_t sl = ch, slt = ch;
        const int dvj = G.vn_deg(j);
        for (int k = 0; k < dvj; ++k) {
          int mm, ee;
          G.vn_edge(j, k, mm, ee);
          sl += (val_t)ms.c(ee);
          slt += (val_t)ms.p(ee);
        }
        int bad = close((val_t)ms.l(j), sl) ? 0 : 1;
        if (with_ci) {
          if (!close((val_t)ms.lt(j), slt)) bad |= 2;
          if constexpr (!FrameStore<A, STORE, STREAM>::kDerivedD) {
            if (ms.d(j) != ar.ci((val_t)ms.l(j), (val_t)ms.lt(j))) bad |= 4;
          }
        }
        return bad;
      };
      int bad = 0;
      for (int ps = 0; ps < npass; ++ps) {
        const int2 ent = load_ent(ps);
        if (ent.x >= 0) bad |= check_vn(ent.y & 0xFFFFFF);
      }
      if (lane < dc_m) bad |= check_vn(G.row_vn(mstar, rs_m, lane));
      if (lane == 0) bad |= check_vn(nstar);
      if (!lmd) {
        if (lane < dv) {  // the key of every check of n*
          const int rs = G.row_start(my_m), dc = G.row_deg(my_m);
          uint32_t kv = 0;
          for (int p = 0; p < dc; ++p) {
            msg_t cm, pm;
            ms.cp(rs + p, cm, pm);
            kv = max(kv, ar.res((val_t)pm, (val_t)cm));
          }
          if (kv != ckey[my_m]) bad |= 8;
        }
        const int nb = (nstar >> 6) * WAVE + lane, mb = (mstar >> 6) * WAVE + lane;
        const uint64_t kd = wave_max_u64((with_ci && nb < N) ? mkkey(d_of(nb), (uint32_t)nb) : 0ull);
        const uint64_t kc = wave_max_u64(mb < M ? mkkey(ckey[mb], (uint32_t)mb) : 0ull);
        if (lane == 0 && with_ci && kd != dblk[nstar >> 6]) bad |= 16;
        if (lane == 0 && kc != cblk[mstar >> 6]) bad |= 32;
      }
      for (int kind = 0; kind < 6; ++kind) {
        const int cnt = wave_sum_i32((bad >> kind) & 1);
        if (lane == 0 && cnt) atomicAdd(&P.selfcheck[kind], (unsigned long long)cnt);
      }
      if (lane == 0) atomicAdd(&P.selfcheck[7], 1ull);
      wave_sync();
    }
#endif
    if (J.trace && lane == 0) J.trace[t] = estar;
    t += 1;
    if (ce > 0) {
      until_check -= 1;
      if (until_check == 0) {
        until_check = ce;
        if (unsat == 0) done = true;
      }
    }
  }
  PROF_FLUSH

  // ---------------- outputs -----------------------------------------------------------
  for (int n = lane; n < N; n += WAVE) {
    const val_t l = (val_t)ms.l(n);
    J.bits[n] = l < 0 ? 1 : 0;
    if (J.llr_out) J.llr_out[n] = ar.out_llr(l);
    if (J.dump_L) J.dump_L[n] = ar.as_float(l);
    if (J.dump_Lt) J.dump_Lt[n] = ar.as_float((val_t)ms.lt(n));
    if (J.dump_D) J.dump_D[n] = ar.d_float(d_of(n));
  }
  for (int e = lane; e < E; e += WAVE) {
    if (J.dump_c2v) J.dump_c2v[e] = ar.as_float((val_t)ms.c(e));
    if (J.dump_pre) J.dump_pre[e] = ar.as_float((val_t)ms.p(e));
  }
  if (lane == 0) {
    *J.updates_used = t;
    if (J.steps_used) *J.steps_used = t;
    if (J.fallbacks) *J.fallbacks = nfall;
  }
  wave_sync();
}

}  // namespace ldpc
