// Kernel parameter blocks and launchers (host <-> device contract inside the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ldpcci.h"
#include "common.hpp"

namespace ldpc {

enum Kind {
  KIND_FLOODING = 0,
  KIND_LAYERED = 1,
  KIND_RBP = 2,
  KIND_CIRBP = 3,
  KIND_ME_CIRBP = 4,
  KIND_REPLAY = 5,
  KIND_LMDRBP = 6,
  KIND_SLMDRBP = 7,
  KIND_LMD_CIRBP = 8,
  KIND_ME_LMD_CIRBP = 9
};
__host__ __device__ constexpr bool is_lmd(int k) { return k == KIND_LMDRBP || k == KIND_SLMDRBP || k == KIND_LMD_CIRBP; }
enum Topo { TOPO_GLOBAL = 0, TOPO_LDS = 1, TOPO_QC = 2 };
// single-edge frame storage: c2v and pre in LDS; pre in a global slot; both in a global slot; both
// and the precomputed totals Lt in a global slot; the whole frame (messages, Lt, L, D) in a global
// slot, leaving only check keys, block maxima, syndrome bits and staging in LDS; the same with the
// per-VN values in one 8-byte (Lt, L) record, D evaluated from it (one cache line per touched VN
// instead of three);
// and that with the check keys and the late-CI staging in the slot as well (LDS keeps only block
// maxima, dirty masks, syndrome bits and the repeated-VN groups: the most frames per CU)
enum Store {
  STORE_LDS = 0,
  STORE_PRE_GLOBAL = 1,
  STORE_ALL_GLOBAL = 2,
  STORE_ALL_GLOBAL_LT = 3,
  STORE_FRAME_GLOBAL = 4,
  STORE_FRAME_REC = 5,
  STORE_FRAME_ALL = 6
};
constexpr int kStores = 7;

struct DecOut {
  uint8_t* bits;            // [B][N]
  float* llr_out;           // [B][N] or null
  int64_t* updates_used;    // [B]
  int64_t* steps_used;      // [B] or null
  int64_t* fallbacks;       // [B] or null
  int32_t* trace;           // [B][max_updates] or null
  float* dump_c2v;          // [B][E] or null
  float* dump_pre;          // [B][E] or null
  float* dump_L;            // [B][N] or null
  float* dump_Lt;           // [B][N] or null
  float* dump_D;            // [B][N] or null
  const int* abort;         // the device's abort flag (nonzero: frames not yet started are skipped)
};

struct DynParams {
  int kind;
  int B;
  long long max_updates, check_every;
  uint32_t gamma_bits;      // FP32: bit pattern of gamma; fixed point: gamma_q
  const float* llr;         // [B][N]
  const int32_t* replay;    // [B][replay_len]
  long long replay_len;
  DecOut out;
  int qmax;
  float scale;
  const int* lut_global;    // 257 entries (fixed point)
  void* pre_global;         // per-workgroup message slots when messages are not in LDS
  int frame_base;           // LDS: the shared region (p0 table, topology) comes first; frame w of a
  int frame_stride;         // workgroup starts at frame_base + w * frame_stride (frame offsets below
  int wpb;                  // are relative to it); wpb = frames (wavefronts) per workgroup
  long long slot_bytes;     // STORE_ALL_GLOBAL and up: bytes per slot ((c2v, pre) pairs, Lt, L, D)
  int slot_lt_off;          // STORE_ALL_GLOBAL_LT and up: byte offset of Lt (STORE_FRAME_REC: of the
                            // VN records) in a slot
  int slot_l_off;           // STORE_FRAME_GLOBAL: byte offsets of L and D in a slot
  int slot_d_off;
  int slot_ckey_off;        // STORE_FRAME_ALL: byte offsets of the check keys and the late-CI
  int slot_tj_off;          // staging in a slot
  int* queue;               // persistent launch: next-frame counter (zeroed before launch); null:
                            // workgroup b decodes frames b, b + grid, ...
  // ME-CIRBP
  int n_p, n_g, fill;
  unsigned long long seed;
  // LDS layout (byte offsets)
  int off_c2v, off_pre, off_L, off_Lt, off_D, off_ckey, off_dblk, off_cblk, off_dmask, off_cmask;
  int off_syn, off_v, off_grp, off_lut, off_topo;
  int lds_bytes;
  int nbd, nbc, nbd_words, nbc_words;
  long long* prof;          // development builds only: per-phase cycle sums (null otherwise)
  // self-checking builds only: mismatches per kind (L, Lt, D, check key, VN block, check block;
  // [7] updates checked), null otherwise
  unsigned long long* selfcheck;
};

// one frame of a dynamic-schedule decode: limits and frame-local input/output pointers
struct FrameJob {
  int kind;
  uint32_t gamma_bits;
  long long max_updates, check_every;
  const float* llr;         // N channel LLRs
  const int32_t* replay;    // replay row (KIND_REPLAY)
  long long replay_len;
  uint8_t* bits;
  float* llr_out;
  int64_t* updates_used;
  int64_t* steps_used;
  int64_t* fallbacks;
  int32_t* trace;           // trace row (max_updates entries)
  float *dump_c2v, *dump_pre, *dump_L, *dump_Lt, *dump_D;
};

struct BaseParams {
  int kind;                 // KIND_FLOODING or KIND_LAYERED
  int B;
  long long max_updates, check_every;
  const float* llr;
  DecOut out;
  int qmax;
  float scale;
  // LDS layout (byte offsets).  Flooding: one frame per workgroup (c2v, L, channel, syndrome
  // words, counter, topology copy).  Layered: the topology copy at off_topo, then wpb frames of
  // frame_stride bytes from frame_base, each with L, syndrome words and (unless c2v_global) c2v.
  int off_c2v, off_L, off_ch, off_syn, off_misc, off_topo;
  int frame_base, frame_stride, wpb;
  void* c2v_global;         // layered, large codes: per-wavefront c2v slots of slot_edges messages
  long long slot_edges;
  int* queue;               // layered: next-frame counter of the persistent grid (zeroed before launch)
  int lds_bytes;
};

// Copy the topology into LDS when requested and return the accessor.
template <int TOPO>
struct TopoSel;
template <>
struct TopoSel<TOPO_GLOBAL> {
  using type = TopoCSR;
  __device__ static type make(const DevCode& H, unsigned char*, int, int) {
    TopoCSR t{H.row_ptr, H.col, H.row_of, H.col_ptr, H.col_row, H.col_eid};
    t.nbr_idx = H.nbr_idx;
    return t;
  }
};
template <>
struct TopoSel<TOPO_LDS> {
  using type = TopoCSR;
  __device__ static type make(const DevCode& H, unsigned char* base, int tid, int nthr) {
    int* p = reinterpret_cast<int*>(base);
    const int M = H.M, N = H.N, E = H.E;
    int* row_ptr = p;
    int* col = row_ptr + (M + 1);
    int* row_of = col + E;
    int* col_ptr = row_of + E;
    int* col_row = col_ptr + (N + 1);
    int* col_eid = col_row + E;
    int2* nidx = reinterpret_cast<int2*>(col_eid + E + (((M + 1) + (N + 1)) & 1));
    for (int x = tid; x <= M; x += nthr) row_ptr[x] = H.row_ptr[x];
    for (int x = tid; x <= N; x += nthr) col_ptr[x] = H.col_ptr[x];
    for (int x = tid; x < E; x += nthr) {
      col[x] = H.col[x];
      row_of[x] = H.row_of[x];
      col_row[x] = H.col_row[x];
      col_eid[x] = H.col_eid[x];
    }
    for (int x = tid; x < N; x += nthr) nidx[x] = H.nbr_idx[x];
    TopoCSR t{row_ptr, col, row_of, col_ptr, col_row, col_eid};
    t.nbr_idx = nidx;
    return t;
  }
};
template <>
struct TopoSel<TOPO_QC> {
  using type = TopoQC;
  __device__ static type make(const DevCode& H, unsigned char* base, int tid, int nthr) {
    int* p = reinterpret_cast<int*>(base);
    const DevQC& q = H.qc;
    for (int x = tid; x < q.words; x += nthr) p[x] = q.bdeg[x];  // tables are contiguous from bdeg
    const int o_bptr = (int)(q.bptr - q.bdeg), o_brow = (int)(q.brow - q.bdeg);
    const int o_bcp = (int)(q.bcol_ptr - q.bdeg), o_bcol = (int)(q.bcol - q.bdeg), o_rm = (int)(q.rowmap - q.bdeg);
    const int o_bdiv = (int)(q.bdiv - q.bdeg);
    TopoQC t{q.Z, q.zdiv, p, p + o_bptr, p + o_brow, p + o_bcp, p + o_bcol, p + o_rm, p + o_bdiv};
    t.nbr_col = p + (int)(reinterpret_cast<const int*>(H.nbr_col) - q.bdeg);
    t.border = p + (int)(q.border - q.bdeg);
    return t;
  }
};

hipError_t launch_dynamic(const DevCode& H, const DynParams& P, bool fixed, int store, int topo, int grid,
                          hipStream_t st);
// address of the current device's abort flag (set by ldpc_request_abort), null if it cannot be had
const int* abort_flag_address();
hipError_t set_dynamic_lds_limit(int bytes);
// wavefronts of one single-edge kernel variant a SIMD can hold by its register count (1..8)
int dynamic_waves_per_simd(bool fixed, int store, int topo, bool mf, bool lmd);
hipError_t launch_baseline(const DevCode& H, const BaseParams& P, bool fixed, int topo, int grid, int block,
                           hipStream_t st);
hipError_t set_baseline_lds_limit(int bytes);
struct MeParams {
  int B;
  long long max_updates, check_every;
  const float* llr;
  DecOut out;
  int qmax;
  float scale;
  const int* lut_global;
  int n_p, n_g, fill;
  int lmd;                  // ME-LMD-CIRBP (Algorithm 6): the next set starts from the proposals
  unsigned long long seed;
  void* msg_global;         // grid x 2E messages (c2v then pre) when they are not in LDS
  float* dbuf;              // FP32: grid x E changes of the precomputed messages of one step
  int off_c2v, off_pre, off_L, off_Lt, off_D, off_hist, off_synw, off_rowmark, off_vnmark, off_rows, off_sel;
  int off_cand, off_misc, off_lut, off_topo, off_rows2, off_vnmulti;
  int off_mpref, off_macc;  // FP32: prefix counts of vnmulti words, 64-bit sums of multiply-changed VNs
  int lds_bytes;
  int rows_cap, cand_cap;
  long long* prof;          // development builds only: per-phase cycle sums (null otherwise)
};

// FP32 multi-edge: LDS slots for the exact sums of the VNs that several checks of one step change
// (a step with more such VNs sums them in check order instead)
constexpr int kMeAccSlots = 2048;

// batched launch: one descriptor per frame (layout of ldpc_frame_desc)
struct BatchFrame {
  int32_t code, kind;
  float gamma;
  int32_t reserved;
  int64_t max_updates, llr_off, out_off;
};

struct BatchParams {
  DynParams P;              // arithmetic, LDS layout for the largest code, pre scratch
  const DevCode* codes[64]; // device copies of the code descriptors
  int n_codes;
  const BatchFrame* frames; // [F] in device memory
  int F;
  const float* llr_pool;
  long long llr_len;
  uint8_t* bits_pool;
  float* llr_out_pool;
  long long out_len;
  int64_t* updates_used;
  int64_t* steps_used;
  int64_t* fallbacks;
  int* queue;               // work-queue counter
  int max_E;
  const int* abort;         // the device's abort flag
};

// damped replay of a fixed schedule (forward with checkpoints) and its adjoint
struct UnrollParams {
  int B, T, ckpt_every, n_ckpt, tstride;
  const float* llr;        // [B][N]
  const float* w;          // [E]
  const int* trace;        // [B][T]
  float* ckpt;             // [B][n_ckpt][E + N] (c2v then L at t = 0, K, 2K, ...)
  float* soft_out;         // [B][N]
  float* c2v_out;          // [B][E] or null
  const float* grad_soft;  // [B][N]
  float* grad_llr;         // [B][N]
  float* gw_part;          // [B][E] per-frame weight gradients (scratch, accumulated in place)
  int off_c2v, off_L, off_ch, off_Lh, off_tape, off_tape_hdr;
  int lds_fwd, lds_bwd;
};
hipError_t launch_unroll_fwd(const DevCode& H, const UnrollParams& U, int grid, hipStream_t st);
hipError_t launch_unroll_bwd(const DevCode& H, const UnrollParams& U, int grid, float* chunks, int nch, int chunk,
                             float* grad_w, hipStream_t st);
hipError_t set_unroll_lds_limit(int bytes);

// channel frames and error counters of SNR sweeps
hipError_t launch_awgn_frames(const uint8_t* cw, int P, int N, int B, float sigma2, const uint64_t* seed_dev,
                              uint64_t seed_val, int point, float* llr, hipStream_t st);
hipError_t launch_count_errors(const uint8_t* bits, const uint8_t* cw, int P, int N, int B, const int64_t* upd,
                               int64_t* counters, hipStream_t st);
hipError_t launch_fill_u64(int64_t* p, int n, uint64_t v, hipStream_t st);

hipError_t launch_batch(const BatchParams& B, bool fixed, int store, int topo, int grid, hipStream_t st);
hipError_t set_batch_lds_limit(int bytes);

hipError_t launch_me(const DevCode& H, const MeParams& P, bool fixed, bool msg_global, int topo, int grid,
                     int block, hipStream_t st);
hipError_t set_me_lds_limit(int bytes);

// host.cpp: ldpc_decode with the caller's scratch buffer (cap bytes at scratch) in place of an
// allocation; a persistent grid is lowered until its frame slots fit.  LDPC_ECAPACITY when not
// even one workgroup's slots fit.  Allocates no device memory.
int decode_in_scratch(const ldpc_code* c, const ldpc_schedule* s, const float* llr_in, int32_t B,
                      int64_t max_updates, const int32_t* replay, int64_t replay_len, const ldpc_outputs* out,
                      void* scratch, size_t cap, hipStream_t st);
// host.cpp: record a failed HIP call for ldpc_last_hip_error and return LDPC_EHIP
int record_hip_failure(hipError_t e);

}  // namespace ldpc
