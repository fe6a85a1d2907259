// Kernel parameter blocks and launchers (host <-> device contract inside the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace ldpc {

enum Kind { KIND_FLOODING = 0, KIND_LAYERED = 1, KIND_RBP = 2, KIND_CIRBP = 3, KIND_ME_CIRBP = 4, KIND_REPLAY = 5 };
enum Topo { TOPO_GLOBAL = 0, TOPO_LDS = 1, TOPO_QC = 2 };

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
  void* pre_global;         // grid x E messages when pre[] is not in LDS
  // ME-CIRBP
  int n_p, n_g, fill;
  unsigned long long seed;
  // LDS layout (byte offsets)
  int off_c2v, off_pre, off_L, off_Lt, off_D, off_ckey, off_dblk, off_cblk, off_dmask, off_cmask;
  int off_syn, off_v, off_pbuf, off_jbuf, off_kbuf, off_slot, off_trow, off_lut, off_topo, off_extra;
  int lds_bytes;
  int nbd, nbc, nbd_words, nbc_words;
  long long* prof;          // development builds only: per-phase cycle sums (null otherwise)
};

struct BaseParams {
  int kind;                 // KIND_FLOODING or KIND_LAYERED
  int B;
  long long max_updates, check_every;
  const float* llr;
  DecOut out;
  int qmax;
  float scale;
  int off_c2v, off_L, off_ch, off_syn, off_misc;
  int lds_bytes;
};

hipError_t launch_dynamic(const DevCode& H, const DynParams& P, bool fixed, bool pre_global, int topo, int grid,
                          hipStream_t st);
hipError_t set_dynamic_lds_limit(int bytes);
hipError_t launch_baseline(const DevCode& H, const BaseParams& P, bool fixed, int grid, int block,
                           hipStream_t st);
hipError_t set_baseline_lds_limit(int bytes);
hipError_t launch_me(const DevCode& H, const DynParams& P, bool fixed, bool pre_global, int topo, int grid,
                     int block, hipStream_t st);
hipError_t set_me_lds_limit(int bytes);

}  // namespace ldpc
