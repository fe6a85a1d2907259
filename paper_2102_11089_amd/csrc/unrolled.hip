// Differentiable unrolled decoder on gfx950: damped replay of a recorded single-edge schedule
// (forward, with checkpoints) and its hand-written adjoint.
//
// The schedule (one edge id per step, recorded by a CIRBP/RBP decode and held fixed) is replayed
// with a weight per edge: step t on edge e (check m, VN n) moves
//     c2v_e += w_e (pre_e - c2v_e),   L_n += the same amount,
// where pre_e is the C2V rule of eq. (2) (Sec. II-A) over V2C_{k->m} = L_k - c2v_{m->k}, k != n.
// With w = 1 this is the propagation step of the single-edge schedules (Sec. II-A, steps 3-4).
//
// One wavefront per frame; c2v[E] and L[N] of the frame live in LDS.  Per step the row of m is
// read by lanes 0..dc-1 and pre_e is evaluated in the phi domain,
//     |pre_e| = min( phi( sum_{k != n} phi(|v_k|) ), min_{k != n} |v_k| ),  phi(x) = -log tanh(x/2),
// with one DPP butterfly for the sum, the minimum and the sign parity (|a [+] b| <= min(|a|,|b|)
// holds exactly, so the clamp only removes FP32 underflow of phi for very large inputs).  Step
// descriptors (edge, row start, degree, position, VN, weight) are fetched by 64 lanes at once for 64
// steps and broadcast with readlane, so no topology lookup sits on the per-step dependency chain.
//
// Adjoint.  Checkpoints of (c2v, L) are written every K steps.  The backward kernel walks the
// segments in reverse: it reloads a checkpoint, recomputes the segment forward into an LDS tape
// (row inputs v_k, their VNs, pre_e, c2v_e before the step), then runs the steps backwards with
// adjoints ch (of c2v) and Lh (of L):
//     s = ch_e + Lh_n;   dw_e += s (pre_e - c2v_e);   ch_e -= w_e s;
//     for k != n:  g = d pre_e / d v_k = sinh(pre_e) / sinh(v_k);
//                  Lh_{VN of k} += w_e s g;   ch_{m->k} -= w_e s g.
// sinh(a [+] b)/sinh(a) is the exact partial derivative of the pairwise rule (it follows from
// phi being an involution with phi'(x) = -1/sinh(x)); a zero input takes the limit tanh(q/2), q the
// rule over the remaining inputs.  A step's weight gradient goes into the tape during the reverse
// sweep; after each segment the contributions to each edge are summed in descending step order and
// added to the frame's scratch row in global memory (one read-modify-write per distinct edge, so
// the row leaves LDS for more resident frames).  The rows are summed over frames in a fixed order
// (frames in fixed chunks, then chunks), so grad_w is deterministic.
#include "common.hpp"
#include "kernels.hpp"

namespace ldpc {

namespace {

__device__ __forceinline__ unsigned char* un_lds() {
  extern __shared__ __align__(16) unsigned char lds_un[];
  return lds_un;
}

// step descriptors of steps t0 + lane (lane < cnt); false if any edge id is invalid
struct StepBlk {
  int e, rs, dcx, n;  // dcx = degree | position << 8
  float w;
};

__device__ __forceinline__ bool load_steps(const DevCode& H, const int* tr, const float* w, int t0, int cnt,
                                           StepBlk& s) {
  const int lane = threadIdx.x & (WAVE - 1);
  bool bad = false;
  s.e = 0; s.rs = 0; s.dcx = 0; s.n = 0; s.w = 0.0f;
  if (lane < cnt) {
    const int e = tr[t0 + lane];
    if ((unsigned)e < (unsigned)H.E) {
      const int m = H.row_of[e], rs = H.row_ptr[m];
      s.e = e;
      s.rs = rs;
      s.dcx = (H.row_ptr[m + 1] - rs) | ((e - rs) << 8);
      s.n = H.col[e];
      s.w = w[e];
    } else {
      bad = true;
    }
  }
  return __builtin_amdgcn_ballot_w64(bad) == 0;
}

struct Step {
  int e, rs, dc, x, n;
  float w;
};

__device__ __forceinline__ Step step_of(const StepBlk& b, int i) {
  Step s;
  s.e = __builtin_amdgcn_readlane(b.e, i);
  s.rs = __builtin_amdgcn_readlane(b.rs, i);
  const int dcx = __builtin_amdgcn_readlane(b.dcx, i);
  s.dc = dcx & 0xFF;
  s.x = dcx >> 8;
  s.n = __builtin_amdgcn_readlane(b.n, i);
  s.w = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.w), i));
  return s;
}

// pre_e over the row inputs held by lanes 0..dc-1 (lane x excluded); every lane of 0..31 returns it
__device__ __forceinline__ float row_pre(float v, bool on) {
  float S = on ? phi_f32(fabsf(v)) : 0.0f;
  float mn = on ? fabsf(v) : __builtin_inff();
  uint32_t neg = (on && v < 0.0f) ? 1u : 0u;
  S += bflyf<1>(S); mn = fminf(mn, bflyf<1>(mn)); neg ^= bfly<1>(neg);
  S += bflyf<2>(S); mn = fminf(mn, bflyf<2>(mn)); neg ^= bfly<2>(neg);
  S += bflyf<3>(S); mn = fminf(mn, bflyf<3>(mn)); neg ^= bfly<3>(neg);
  S += bflyf<4>(S); mn = fminf(mn, bflyf<4>(mn)); neg ^= bfly<4>(neg);
  S += bflyf<5>(S); mn = fminf(mn, bflyf<5>(mn)); neg ^= bfly<5>(neg);
  const float mag = fminf(phi_f32(S), mn);
  return neg ? -mag : mag;
}

// VN of the lane's position in the step's row (0 beyond the row): the one topology read of a step,
// which depends on the schedule only, so callers request it a step ahead
__device__ __forceinline__ int row_vn_of(const DevCode& H, const Step& s) {
  const int lane = threadIdx.x & (WAVE - 1);
  return lane < s.dc ? H.col[s.rs + lane] : 0;
}

// one forward step, j = row_vn_of(H, s); returns (for the tape) the lane's row input v, its VN j,
// and pre_e / c2v_e
__device__ __forceinline__ void fwd_step(float* c2v, float* L, const Step& s, int j, float& v_out, int& j_out,
                                         float& p_out, float& c_out) {
  const int lane = threadIdx.x & (WAVE - 1);
  float v = 0.0f, c = 0.0f, lj = 0.0f;
  if (lane < s.dc) {
    c = c2v[s.rs + lane];
    lj = L[j];
    v = __fsub_rn(lj, c);
  }
  const bool on = lane < s.dc && lane != s.x;
  const float p = row_pre(v, on);
  const float cx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c), s.x));
  const float delta = __fmul_rn(s.w, __fsub_rn(p, cx));
  if (lane == s.x) {
    c2v[s.e] = __fadd_rn(c, delta);
    L[s.n] = __fadd_rn(lj, delta);
  }
  wave_sync();
  v_out = v;
  j_out = j;
  p_out = p;
  c_out = cx;
}

__device__ __forceinline__ void copy_out(const float* src, float* dst, int n) {
  const int lane = threadIdx.x & (WAVE - 1);
  for (int i = lane; i < n; i += WAVE) dst[i] = src[i];
}

__device__ __forceinline__ void fill_row(float* dst, int n, float x) {
  const int lane = threadIdx.x & (WAVE - 1);
  for (int i = lane; i < n; i += WAVE) dst[i] = x;
}

}  // namespace

__global__ __launch_bounds__(WAVE) void k_unroll_fwd(DevCode H, UnrollParams U) {
  unsigned char* lds = un_lds();
  float* c2v = reinterpret_cast<float*>(lds + U.off_c2v);
  float* L = reinterpret_cast<float*>(lds + U.off_L);
  const int lane = threadIdx.x;
  const int E = H.E, N = H.N, T = U.T, K = U.ckpt_every;
  for (int f = blockIdx.x; f < U.B; f += gridDim.x) {
    const float* llr = U.llr + (size_t)f * N;
    const int* tr = U.trace + (size_t)f * T;
    for (int i = lane; i < E; i += WAVE) c2v[i] = 0.0f;
    for (int i = lane; i < N; i += WAVE) L[i] = llr[i];
    wave_sync();
    bool ok = true;
    for (int t0 = 0; t0 < T && ok; t0 += WAVE) {
      const int cnt = min(WAVE, T - t0);
      StepBlk blk;
      ok = load_steps(H, tr, U.w, t0, cnt, blk);
      if (!ok) break;
      Step s = step_of(blk, 0);
      int jn = row_vn_of(H, s);
      for (int i = 0; i < cnt; ++i) {
        const int t = t0 + i;
        if (U.ckpt && t % K == 0) {
          float* ck = U.ckpt + ((size_t)f * U.n_ckpt + t / K) * (size_t)(E + N);
          copy_out(c2v, ck, E);
          copy_out(L, ck + E, N);
        }
        const Step cur = s;
        const int jc = jn;
        if (i + 1 < cnt) {  // the next step's row VNs are requested before this step computes
          s = step_of(blk, i + 1);
          jn = row_vn_of(H, s);
        }
        float v, p, c;
        int j;
        fwd_step(c2v, L, cur, jc, v, j, p, c);
      }
    }
    float* out = U.soft_out + (size_t)f * N;
    if (ok) {
      copy_out(L, out, N);
      if (U.c2v_out) copy_out(c2v, U.c2v_out + (size_t)f * E, E);
    } else {
      fill_row(out, N, __builtin_nanf(""));
      if (U.c2v_out) fill_row(U.c2v_out + (size_t)f * E, E, __builtin_nanf(""));
    }
    wave_sync();
  }
}

__global__ __launch_bounds__(WAVE) void k_unroll_bwd(DevCode H, UnrollParams U) {
  unsigned char* lds = un_lds();
  float* c2v = reinterpret_cast<float*>(lds + U.off_c2v);
  float* L = reinterpret_cast<float*>(lds + U.off_L);
  float* ch = reinterpret_cast<float*>(lds + U.off_ch);
  float* Lh = reinterpret_cast<float*>(lds + U.off_Lh);
  const int TS = U.tstride;  // largest row degree
  float* tv = reinterpret_cast<float*>(lds + U.off_tape);          // [K][TS] row inputs
  int* tj = reinterpret_cast<int*>(lds + U.off_tape) + U.ckpt_every * TS;  // [K][TS] their VNs
  float4* th = reinterpret_cast<float4*>(lds + U.off_tape_hdr);      // [K] (p, c_old, dw, -)
  const int lane = threadIdx.x;
  const int E = H.E, N = H.N, T = U.T, K = U.ckpt_every;
  const int nseg = (T + K - 1) / K;
  for (int f = blockIdx.x; f < U.B; f += gridDim.x) {
    const int* tr = U.trace + (size_t)f * T;
    const float* gs = U.grad_soft + (size_t)f * N;
    float* gp = U.gw_part + (size_t)f * E;
    for (int i = lane; i < N; i += WAVE) Lh[i] = gs[i];
    for (int i = lane; i < E; i += WAVE) {
      ch[i] = 0.0f;
      gp[i] = 0.0f;
    }
    wave_sync();
    bool ok = true;
    for (int sg = nseg - 1; sg >= 0 && ok; --sg) {
      const int t0 = sg * K, t1 = min(T, t0 + K);
      const float* ck = U.ckpt + ((size_t)f * U.n_ckpt + sg) * (size_t)(E + N);
      for (int i = lane; i < E; i += WAVE) c2v[i] = ck[i];
      for (int i = lane; i < N; i += WAVE) L[i] = ck[E + i];
      wave_sync();
      // the segment's step descriptors stay in registers for both sweeps: steps t0 + lane and
      // t0 + 64 + lane (a segment has at most 128 steps)
      const int len = t1 - t0;
      StepBlk blka{}, blkb{};
      ok = load_steps(H, tr, U.w, t0, min(WAVE, len), blka);
      if (ok && len > WAVE) ok = load_steps(H, tr, U.w, t0 + WAVE, len - WAVE, blkb);
      if (!ok) break;
      auto seg_step = [&](int r) -> Step { return r < WAVE ? step_of(blka, r) : step_of(blkb, r - WAVE); };
      // recompute the segment, recording the tape (each step's row VNs requested a step ahead)
      int jn = row_vn_of(H, seg_step(0));
      for (int r = 0; r < len; ++r) {
        const Step s = seg_step(r);
        const int jc = jn;
        if (r + 1 < len) jn = row_vn_of(H, seg_step(r + 1));
        float v, p, c;
        int j;
        fwd_step(c2v, L, s, jc, v, j, p, c);
        if (lane < TS) {
          tv[r * TS + lane] = v;
          tj[r * TS + lane] = j;
        }
        if (lane == 0) th[r] = make_float4(p, c, 0.0f, 0.0f);
      }
      wave_sync();
      // reverse sweep over the segment
      for (int r = len - 1; r >= 0; --r) {
        const float4 hd = th[r];
        const Step si = seg_step(r);
        const int e = si.e, dc = si.dc, x = si.x, n = si.n;
        const float p = hd.x, cold = hd.y, w = si.w;
        const float sadj = __fadd_rn(ch[e], Lh[n]);
        const float ws = __fmul_rn(w, sadj);
        float v = 0.0f;
        int j = 0;
        if (lane < dc) {
          v = tv[r * TS + lane];
          j = tj[r * TS + lane];
        }
        const bool on = lane < dc && lane != x;
        float g = 0.0f;
        if (on && v != 0.0f) {
          const float ap = fabsf(p), av = fabsf(v);
          g = expf(ap - av) * (expm1f(-2.0f * ap) / expm1f(-2.0f * av));
          if ((p < 0.0f) != (v < 0.0f)) g = -g;
        }
        const uint64_t zmask = __builtin_amdgcn_ballot_w64(on && v == 0.0f);
        if (zmask) {  // an input of exactly zero: d pre / d v_k = tanh(q/2) for that input
          const bool fin = on && v != 0.0f;
          float S = fin ? phi_f32(fabsf(v)) : 0.0f;
          float mn = fin ? fabsf(v) : __builtin_inff();
          uint32_t neg = (on && v < 0.0f) ? 1u : 0u;
          S += bflyf<1>(S); mn = fminf(mn, bflyf<1>(mn)); neg ^= bfly<1>(neg);
          S += bflyf<2>(S); mn = fminf(mn, bflyf<2>(mn)); neg ^= bfly<2>(neg);
          S += bflyf<3>(S); mn = fminf(mn, bflyf<3>(mn)); neg ^= bfly<3>(neg);
          S += bflyf<4>(S); mn = fminf(mn, bflyf<4>(mn)); neg ^= bfly<4>(neg);
          S += bflyf<5>(S); mn = fminf(mn, bflyf<5>(mn)); neg ^= bfly<5>(neg);
          if (on && v == 0.0f) {
            const float q = fminf(phi_f32(S), mn);
            g = __popcll(zmask) == 1 ? tanhf(0.5f * q) : 0.0f;
            if (neg) g = -g;
          }
        }
        if (on) {
          const float a = __fmul_rn(ws, g);
          Lh[j] = __fadd_rn(Lh[j], a);
          ch[si.rs + lane] = __fsub_rn(ch[si.rs + lane], a);
        }
        if (lane == x) {
          th[r].z = __fmul_rn(sadj, __fsub_rn(p, cold));  // this step's d loss / d w_e
          ch[e] = __fsub_rn(ch[e], ws);
        }
        wave_sync();
      }
      // the segment's weight gradients into the frame's row: each lane takes the steps lane and
      // lane + 64; a step whose edge occurs at no later step of the segment owns that edge and sums
      // its contributions in descending step order
      {
        const int ra = lane, rb = lane + WAVE;
        const int ea = ra < len ? blka.e : -1, eb = rb < len ? blkb.e : -1;
        float sa = 0.0f, sb = 0.0f;
        bool oa = ea >= 0, ob = eb >= 0;
        for (int q = len - 1; q >= 0; --q) {
          const int eq = seg_step(q).e;
          const float vq = th[q].z;
          if (eq == ea) {
            if (q > ra) oa = false;
            else sa = __fadd_rn(sa, vq);
          }
          if (eq == eb) {
            if (q > rb) ob = false;
            else sb = __fadd_rn(sb, vq);
          }
        }
        if (oa) gp[ea] = __fadd_rn(gp[ea], sa);
        if (ob) gp[eb] = __fadd_rn(gp[eb], sb);
        wave_sync();
      }
    }
    float* gl = U.grad_llr + (size_t)f * N;
    if (ok) {
      copy_out(Lh, gl, N);
    } else {
      fill_row(gl, N, __builtin_nanf(""));
      fill_row(gp, E, __builtin_nanf(""));
    }
    wave_sync();
  }
}

// fixed-order sum over frames: chunk c sums its frames in ascending order
__global__ void k_gw_chunks(const float* part, int B, int E, int chunk, float* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (e >= E) return;
  const int f0 = c * chunk, f1 = min(B, f0 + chunk);
  float acc = 0.0f;
  for (int f = f0; f < f1; ++f) acc = __fadd_rn(acc, part[(size_t)f * E + e]);
  out[(size_t)c * E + e] = acc;
}

__global__ void k_gw_final(const float* chunks, int nch, int E, float* grad_w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  float acc = 0.0f;
  for (int c = 0; c < nch; ++c) acc = __fadd_rn(acc, chunks[(size_t)c * E + e]);
  grad_w[e] = acc;
}

hipError_t launch_unroll_fwd(const DevCode& H, const UnrollParams& U, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_unroll_fwd, dim3(grid), dim3(WAVE), U.lds_fwd, st, H, U);
  return hipGetLastError();
}

hipError_t launch_unroll_bwd(const DevCode& H, const UnrollParams& U, int grid, float* chunks, int nch,
                             int chunk, float* grad_w, hipStream_t st) {
  if (U.B > 0) {
    hipLaunchKernelGGL(k_unroll_bwd, dim3(grid), dim3(WAVE), U.lds_bwd, st, H, U);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gw_chunks, dim3((H.E + 255) / 256, nch), dim3(256), 0, st, U.gw_part, U.B, H.E, chunk,
                       chunks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gw_final, dim3((H.E + 255) / 256), dim3(256), 0, st, chunks, U.B > 0 ? nch : 0, H.E, grad_w);
  return hipGetLastError();
}

hipError_t set_unroll_lds_limit(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_unroll_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_unroll_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace ldpc
