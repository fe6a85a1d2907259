// Per-frame body of the single-edge dynamic decoder (RBP, CIRBP, replay) for one wavefront;
// used by the per-code kernel and by the persistent batched kernel.
#pragma once
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

// Where a frame's C2V messages (c2v), precomputed messages (pre) and precomputed totals (Lt)
// live: all in LDS; pre in a global scratch slot; c2v and pre as interleaved (c2v, pre) pairs (one
// load brings the two values of an edge) in a global slot per workgroup; or those pairs followed
// by Lt in the slot.
template <class A, int STORE, bool PAIRS = (STORE >= STORE_ALL_GLOBAL)>
struct MsgStore {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  msg_t* c2v;  // LDS
  msg_t* pre;  // LDS (STORE_LDS) or global (STORE_PRE_GLOBAL)
  llr_t* Lt;   // LDS
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
};

template <class msg_t>
struct alignas(2 * sizeof(msg_t)) MsgPair {
  msg_t c, p;
};

template <class A, int STORE>
struct MsgStore<A, STORE, true> {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  MsgPair<msg_t>* m;  // global, [E]
  llr_t* Lt;          // LDS (STORE_ALL_GLOBAL) or global, [N]
  llr_t* Lg;          // STORE_FRAME_GLOBAL: L and D in the slot, [N]
  uint32_t* Dg;
  __device__ __forceinline__ msg_t c(int e) const { return m[e].c; }
  __device__ __forceinline__ msg_t p(int e) const { return m[e].p; }
  __device__ __forceinline__ void set_c(int e, msg_t v) const { m[e].c = v; }
  __device__ __forceinline__ void set_p(int e, msg_t v) const { m[e].p = v; }
  __device__ __forceinline__ void cp(int e, msg_t& cv, msg_t& pv) const {
    const MsgPair<msg_t> x = m[e];
    cv = x.c;
    pv = x.p;
  }
  __device__ __forceinline__ llr_t lt(int n) const { return Lt[n]; }
  __device__ __forceinline__ void set_lt(int n, llr_t v) const { Lt[n] = v; }
  __device__ __forceinline__ void add_lt(int n, llr_t d) const { atomicAdd(&Lt[n], d); }
};

// message store of the workgroup's frame slot (slot_edges = edges reserved per workgroup when
// only pre is global; the pair-slot layout comes from P.slot_bytes and the slot offsets)
template <class A, int STORE>
__device__ __forceinline__ MsgStore<A, STORE> make_store(const DynParams& P, size_t slot_edges) {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  unsigned char* lds = frame_lds(P);
  MsgStore<A, STORE> ms;
  if constexpr (STORE >= STORE_ALL_GLOBAL) {
    unsigned char* base = reinterpret_cast<unsigned char*>(P.pre_global) + frame_slot(P) * (size_t)P.slot_bytes;
    ms.m = reinterpret_cast<MsgPair<msg_t>*>(base);
    if constexpr (STORE >= STORE_ALL_GLOBAL_LT) ms.Lt = reinterpret_cast<llr_t*>(base + P.slot_lt_off);
    else ms.Lt = reinterpret_cast<llr_t*>(lds + P.off_Lt);
    if constexpr (STORE == STORE_FRAME_GLOBAL) {
      ms.Lg = reinterpret_cast<llr_t*>(base + P.slot_l_off);
      ms.Dg = reinterpret_cast<uint32_t*>(base + P.slot_d_off);
    }
  } else {
    ms.c2v = reinterpret_cast<msg_t*>(lds + P.off_c2v);
    ms.Lt = reinterpret_cast<llr_t*>(lds + P.off_Lt);
    if constexpr (STORE == STORE_PRE_GLOBAL) ms.pre = reinterpret_cast<msg_t*>(P.pre_global) + frame_slot(P) * slot_edges;
    else ms.pre = reinterpret_cast<msg_t*>(lds + P.off_pre);
  }
  return ms;
}

// total LLRs L and CIs D of the frame: in LDS, or in the global slot (STORE_FRAME_GLOBAL)
template <class A, int STORE>
__device__ __forceinline__ typename A::llr_t* frame_L(const MsgStore<A, STORE>& ms, const DynParams& P) {
  if constexpr (STORE == STORE_FRAME_GLOBAL) return ms.Lg;
  else return reinterpret_cast<typename A::llr_t*>(frame_lds(P) + P.off_L);
}
template <class A, int STORE>
__device__ __forceinline__ uint32_t* frame_D(const MsgStore<A, STORE>& ms, const DynParams& P) {
  if constexpr (STORE == STORE_FRAME_GLOBAL) return ms.Dg;
  else return reinterpret_cast<uint32_t*>(frame_lds(P) + P.off_D);
}
// ordering point for values exchanged between lanes through the frame store: a workgroup-scope
// fence (wait for global stores) when the exchanged array lives in global memory
template <bool GLOBAL>
__device__ __forceinline__ void frame_sync() {
  if constexpr (GLOBAL) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  wave_sync();
}

// value of another lane (the lane index is wave-uniform)
template <class T>
__device__ __forceinline__ T lane_value(T x, int l) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
  else return (T)__builtin_amdgcn_readlane((int)x, l);
}

template <class A, int STORE, class Topo>
__device__ __forceinline__ void dyn_decode_frame(const DevCode& H, const Topo& G, const A& ar, const DynParams& P,
                                                 const MsgStore<A, STORE>& ms, const FrameJob& J) {
  using msg_t = typename A::msg_t;
  using llr_t = typename A::llr_t;
  using val_t = typename A::val_t;
  using Acc = typename RowAccOf<A>::type;
  const int lane = threadIdx.x & (WAVE - 1);
  unsigned char* lds = frame_lds(P);
  llr_t* L = frame_L(ms, P);
  uint32_t* D = frame_D(ms, P);
  constexpr bool kLDG = STORE == STORE_FRAME_GLOBAL;  // L and D in global memory
  // per check: the largest residual of its edges (value bits); block keys pair it with the check
  // index, and the edge is found again inside the check's row when the check is selected (edge ids
  // are row-major, so (value, lowest check), then (value, lowest edge) in the row is the global
  // (value, lowest edge))
  uint32_t* ckey = reinterpret_cast<uint32_t*>(lds + P.off_ckey);
  uint64_t* dblk = reinterpret_cast<uint64_t*>(lds + P.off_dblk);
  uint64_t* cblk = reinterpret_cast<uint64_t*>(lds + P.off_cblk);
  uint32_t* dmask = reinterpret_cast<uint32_t*>(lds + P.off_dmask);
  uint32_t* cmask = reinterpret_cast<uint32_t*>(lds + P.off_cmask);
  uint32_t* synw = reinterpret_cast<uint32_t*>(lds + P.off_syn);  // syndrome bits
  int* tj = reinterpret_cast<int*>(lds + P.off_v);  // touched VN of each table lane, per pass
  const int N = H.N, M = H.M, E = H.E;
  const int nbd = (N + WAVE - 1) / WAVE, nbc = (M + WAVE - 1) / WAVE;
  const int nbd_words = (nbd + 31) / 32, nbc_words = (nbc + 31) / 32;
  const bool with_ci = J.kind != KIND_RBP;
  // ---------------- Algorithm 1 lines 1-3: initial state --------------------------------
  const float* llr = J.llr;
  for (int n = lane; n < N; n += WAVE) L[n] = (llr_t)ar.channel(llr[n]);
  for (int e = lane; e < E; e += WAVE) ms.set_c(e, (msg_t)0);
  for (int w = lane; w < nbd_words; w += WAVE) dmask[w] = 0u;
  for (int w = lane; w < nbc_words; w += WAVE) cmask[w] = 0u;
  for (int w = lane; w < (M + 31) / 32; w += WAVE) synw[w] = 0u;
  frame_sync<kLDG>();
  // every precomputed C2V message from V2C = channel value: one lane per check row
  int unsat_local = 0;
  for (int m = lane; m < M; m += WAVE) {
    const int rs = G.row_start(m), dc = G.row_deg(m);
    Acc acc;
    int par = 0;
    for (int p = 0; p < dc; ++p) {
      const val_t l = (val_t)L[G.row_vn(m, rs, p)];
      const val_t v = ar.vin(l);
      acc.add(p, v, row_aux(ar, v));
      par ^= l < 0 ? 1 : 0;
    }
    uint64_t k = 0;
    for (int p = 0; p < dc; ++p) {
      const val_t v = ar.vin((val_t)L[G.row_vn(m, rs, p)]);
      const val_t o = acc.out(p, v, row_aux(ar, v));
      ms.set_p(rs + p, (msg_t)o);
      k = umax64(k, mkkey(ar.res(o, (val_t)0), (uint32_t)(rs + p)));
    }
    ckey[m] = key_val(k);
    if (par) atomicOr(&synw[m >> 5], 1u << (m & 31));
    unsat_local += par;
  }
  int unsat = wave_sum_i32(unsat_local);
  if constexpr (STORE != STORE_LDS) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // message stores done
  wave_sync();
  for (int n = lane; n < N; n += WAVE) {
    val_t lt = (val_t)L[n];
    const int dv = G.vn_deg(n);
    for (int k = 0; k < dv; ++k) {
      int m, e;
      G.vn_edge(n, k, m, e);
      lt += (val_t)ms.p(e);
    }
    ms.set_lt(n, (llr_t)lt);
    D[n] = with_ci ? ar.ci((val_t)L[n], lt) : 0u;
  }
  frame_sync<kLDG>();
  for (int b = 0; b < nbd; ++b) {
    const int n = b * WAVE + lane;
    uint64_t k = n < N ? mkkey(D[n], (uint32_t)n) : 0ull;
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
  long long limit = J.max_updates;
  if (J.kind == KIND_REPLAY && J.replay_len < limit) limit = J.replay_len;
  const long long ce = J.kind == KIND_REPLAY ? 0 : J.check_every;
  long long until_check = ce;  // updates left until the next syndrome test
  bool done = ce > 0 && unsat == 0;
  PROF_DECL
  while (!done && t < limit) {
    PROF_MARK(7)
    // ---- selection (Algorithm 1 lines 4-8; RBP eq. (5)) ----
    int estar, mstar = -1, nstar = -1;
    msg_t c_star = (msg_t)0, p_star = (msg_t)0;  // messages of e*, taken from the selection's loads
    bool have_star = false;
    if (J.kind == KIND_REPLAY) {
      estar = uni(J.replay[t]);
      if (estar < 0 || estar >= E) break;  // invalid edge id ends the frame's replay
    } else {
      bool global_res = J.kind == KIND_RBP;
      int nsel = -1;
      if (!global_res) {
        uint64_t k = 0;
        for (int b = lane; b < nbd; b += WAVE) k = umax64(k, dblk[b]);
        k = wave_max_u64(k);
        nsel = (int)key_idx(k);
        if (key_val(k) < J.gamma_bits) {  // D_{n*} < gamma: RBP fallback
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
        c_star = lane_value(cm, estar - rs);
        p_star = lane_value(pm, estar - rs);
        have_star = true;
      } else {
        const int dvs = uni(G.vn_deg(nsel));
        uint64_t k = 0;
        int mk = -1;
        msg_t cm = (msg_t)0, pm = (msg_t)0;
        if (lane < dvs) {
          int e;
          G.vn_edge(nsel, lane, mk, e);
          ms.cp(e, cm, pm);
          k = mkkey(ar.res((val_t)pm, (val_t)cm), (uint32_t)e);
        }
        const uint64_t kmax = wave_max_u64(k);
        estar = (int)key_idx(kmax);
        const unsigned long long win = __ballot(lane < dvs && k == kmax);
        const int wl = (int)__builtin_ctzll(win);
        mstar = __builtin_amdgcn_readlane(mk, wl);
        nstar = nsel;
        c_star = lane_value(cm, wl);
        p_star = lane_value(pm, wl);
        have_star = true;
      }
    }
    if (mstar < 0) {
      mstar = uni(G.edge_row(estar));
      nstar = uni(G.edge_vn(estar));
    }
    PROF_MARK(0)
    const int dv = uni(G.vn_deg(nstar));
    int my_m = -1;
    if (lane < dv) {
      int e;
      G.vn_edge(nstar, lane, my_m, e);
    }
    const int2 nb = G.nbr(nstar);
    const int noff = uni(nb.x), ncnt = uni(nb.y);
    const int npass = (ncnt + WAVE - 1) / WAVE;
    const int rs_m = uni(G.row_start(mstar));
    const int re_m = rs_m + uni(G.row_deg(mstar));
    // Inputs of the touched-check passes are loaded ahead of use: table entries two passes ahead,
    // message pairs and L one pass ahead.  Nothing a pass writes (its own checks' pre, Lt, keys)
    // is read by a later pass, propagation changes only c2v[e*] and L[n*] (both overridden where
    // used), so the early loads see the values the passes need.
    auto load_ent = [&](int ps) -> int2 {
      const int idx = ps * WAVE + lane;
      return idx < ncnt ? H.nbr[noff + idx] : make_int2(-1, 0);
    };
    struct PassIn {
      int2 ent;
      msg_t cm, pm;
      llr_t lj;
    };
    auto load_in = [&](int2 ent) -> PassIn {
      PassIn q;
      q.ent = ent;
      q.cm = (msg_t)0;
      q.pm = (msg_t)0;
      q.lj = (llr_t)0;
      if (ent.x >= 0) {
        ms.cp(ent.x, q.cm, q.pm);
        q.lj = L[ent.y & 0xFFFFFF];
      }
      return q;
    };
    const int2 ent0 = load_ent(0);
    int2 ent_next = npass > 1 ? load_ent(1) : make_int2(-1, 0);

    // ---- propagation (Algorithm 1 line 9) and D_{n*} ----
    if (!have_star) ms.cp(estar, c_star, p_star);
    PassIn in_cur = load_in(ent0);
    const val_t newv = (val_t)p_star;
    const val_t oldv = (val_t)c_star;
    const val_t Lold = (val_t)L[nstar];
    const val_t Lnew = Lold + (newv - oldv);
    const uint32_t dn_old = D[nstar];
    const uint32_t dn_new = with_ci ? ar.ci(Lnew, (val_t)ms.lt(nstar)) : 0u;
    wave_sync();
    if (lane == 0) {
      ms.set_c(estar, (msg_t)newv);
      L[nstar] = (llr_t)Lnew;
      if (with_ci) {
        D[nstar] = dn_new;
        const uint64_t nk = mkkey(dn_new, (uint32_t)nstar), ok = mkkey(dn_old, (uint32_t)nstar);
        if (nk > ok) atomicMax(reinterpret_cast<unsigned long long*>(&dblk[nstar >> 6]), (unsigned long long)nk);
        else if (nk < ok && dblk[nstar >> 6] == ok) atomicOr(&dmask[(nstar >> 6) >> 5], 1u << ((nstar >> 6) & 31));
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

    // ---- touched checks: V2C inputs, whole-row update, residual keys (one pass per 64 lanes) ----
    for (int ps = 0; ps < npass; ++ps) {
      PassIn in_next{make_int2(-1, 0), (msg_t)0, (msg_t)0, (llr_t)0};
      int2 ent_after = make_int2(-1, 0);
      if (ps + 1 < npass) in_next = load_in(ent_next);
      if (ps + 2 < npass) ent_after = load_ent(ps + 2);
      const int2 ent = in_cur.ent;
      const int e = ent.x;
      const bool valid = e >= 0;
      const int j = ent.y & 0xFFFFFF;
      const int L2 = (ent.y >> 24) & 7;
      const bool leader = valid && ((ent.y >> 27) & 1);
      const bool in_m = valid && e >= rs_m && e < re_m;
      const bool self = valid && j == nstar;
      val_t cv = 0, po = 0, lv = 0;
      if (valid) {
        cv = e == estar ? newv : (val_t)in_cur.cm;  // this update's propagation
        po = (val_t)in_cur.pm;
        lv = self ? Lnew : (val_t)in_cur.lj;
      }
      const val_t v = ar.vin(ar.v2c(lv, cv));
      const int maxL2 = uni(L2);  // lane 0 starts the pass's largest block
      RowRed r;
      r.m1 = valid ? fabsf((float)v) : __builtin_inff();
      r.m2 = __builtin_inff();
      r.ap = (valid ? (uint32_t)e : 0x7FFFFFFFu) | (valid && v < 0 ? 0x80000000u : 0u);
      const bool upd = valid && !in_m && !self;
      val_t pv = po;
      if constexpr (A::kFixed) {
        rowred_all<false>(r, L2, maxL2);
        const bool me = (uint32_t)e == (r.ap & 0x7FFFFFFFu);
        const int mag = (int)(me ? r.m2 : r.m1);
        const int o = (((r.ap >> 31) ^ (v < 0 ? 1u : 0u)) & 1u) ? -mag : mag;
        if (upd) pv = o;
      } else {
        const float ph = valid ? row_aux(ar, v) : 0.0f;
        r.S = ph;
        r.Sx = 0.0f;
        rowred_all<true>(r, L2, maxL2);
        const bool me = (uint32_t)e == (r.ap & 0x7FFFFFFFu);
        const float mo = me ? r.m2 : r.m1;
        const float Sj = me ? r.Sx : (ph == __builtin_inff() ? __builtin_inff() : r.S - ph);
        const float mag = fminf(phi_f32(fmaxf(Sj, 0.0f)), mo);
        const float o = (((r.ap >> 31) ^ (v < 0.0f ? 1u : 0u)) & 1u) ? -mag : mag;
        if (upd) pv = o;
      }
      if (upd) {
        ms.set_p(e, (msg_t)pv);
        if (with_ci) ms.add_lt(j, (llr_t)(pv - po));
      }
      tj[ps * WAVE + lane] = upd ? j : -1;
      const uint64_t rk = keymax_all(valid ? mkkey(ar.res(pv, cv), (uint32_t)e) : 0ull, L2, maxL2);
      if (leader) {  // one lane per check: new residual key, block maximum
        const int m = G.edge_row(e);
        const uint32_t ov = ckey[m];
        ckey[m] = key_val(rk);
        const uint64_t nk = mkkey(key_val(rk), (uint32_t)m), ok = mkkey(ov, (uint32_t)m);
        if (nk > ok) atomicMax(reinterpret_cast<unsigned long long*>(&cblk[m >> 6]), (unsigned long long)nk);
        else if (nk < ok && cblk[m >> 6] == ok) atomicOr(&cmask[(m >> 6) >> 5], 1u << ((m >> 6) & 31));
      }
      in_cur = in_next;
      ent_next = ent_after;
    }
    if constexpr (STORE != STORE_LDS) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // message stores done
    wave_sync();
    PROF_MARK(3)
    // ---- CI of the VNs of the touched checks (Algorithm 1 line 12) ----
    if (with_ci) {
      for (int ps = 0; ps < npass; ++ps) {
        const int j = tj[ps * WAVE + lane];
        uint32_t nd = 0, od = 0;
        if (j >= 0) {
          nd = ar.ci((val_t)L[j], (val_t)ms.lt(j));
          od = D[j];
        }
        wave_sync();
        if (j >= 0) {
          D[j] = nd;
          const uint64_t nk = mkkey(nd, (uint32_t)j), ok = mkkey(od, (uint32_t)j);
          if (nk > ok) atomicMax(reinterpret_cast<unsigned long long*>(&dblk[j >> 6]), (unsigned long long)nk);
          else if (nk < ok && dblk[j >> 6] == ok) atomicOr(&dmask[(j >> 6) >> 5], 1u << ((j >> 6) & 31));
        }
        wave_sync();
      }
    }
    if constexpr (kLDG) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // D stores done
    PROF_MARK(5)
    // ---- blocks whose maximum leaf decreased ----
    for (int w = 0; w < nbc_words; ++w) {
      uint32_t bits = (uint32_t)uni((int)cmask[w]);
      while (bits) {
        const int b = w * 32 + __builtin_ctz(bits);
        bits &= bits - 1;
        const int m = b * WAVE + lane;
        uint64_t k = m < M ? mkkey(ckey[m], (uint32_t)m) : 0ull;
        k = wave_max_u64(k);
        if (lane == 0) cblk[b] = k;
      }
      if (lane == 0) cmask[w] = 0u;
    }
    if (with_ci) {
      for (int w = 0; w < nbd_words; ++w) {
        uint32_t bits = (uint32_t)uni((int)dmask[w]);
        while (bits) {
          const int b = w * 32 + __builtin_ctz(bits);
          bits &= bits - 1;
          const int n = b * WAVE + lane;
          uint64_t k = n < N ? mkkey(D[n], (uint32_t)n) : 0ull;
          k = wave_max_u64(k);
          if (lane == 0) dblk[b] = k;
        }
        if (lane == 0) dmask[w] = 0u;
      }
    }
    wave_sync();
    PROF_MARK(6)
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
    const val_t l = (val_t)L[n];
    J.bits[n] = l < 0 ? 1 : 0;
    if (J.llr_out) J.llr_out[n] = ar.out_llr(l);
    if (J.dump_L) J.dump_L[n] = ar.as_float(l);
    if (J.dump_Lt) J.dump_Lt[n] = ar.as_float((val_t)ms.lt(n));
    if (J.dump_D) J.dump_D[n] = ar.d_float(D[n]);
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
