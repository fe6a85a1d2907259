/*
 * ldpcci.h -- C ABI of the MI355X (gfx950) dynamic-schedule LDPC belief-propagation decoder.
 *
 * The decoder computes, for each frame of channel LLRs, the message-passing schedules of
 * Chang, Wang, Weng, Lee, Su, "Belief-Propagation Decoding of LDPC Codes with Variable
 * Node-Centric Dynamic Schedules" (arXiv 2102.11089):
 *   - residual BP (RBP): Sec. II-A, steps 1)-4), argmax of eq. (5) over all edges;
 *   - conditional-innovation RBP (CIRBP): Algorithm 1 (Sec. III-B) with the CI metric eq. (9);
 *   - multi-edge CIRBP (ME-CIRBP): Algorithm 5 with the VN selection of Algorithm 4 (Sec. VI);
 *   - latest-message-driven schedules (Sec. IV): LMDRBP and its simplified form sLMDRBP
 *     (Algorithm 2), LMD-CIRBP (Algorithm 3), with the degree-1 rule of Sec. V, and multi-edge
 *     LMD-CIRBP (ME-LMD-CIRBP, Algorithm 6);
 *   - flooding and layered BP baselines (Sec. I);
 *   - replay of a recorded edge order (the schedule held fixed).
 * Messages follow eqs. (1)-(3) (Sec. II-A): V2C, C2V by the tanh rule (sum-product), total LLR
 * and hard decision bsgn(L) (bit 0 iff L >= 0).  An iteration is E C2V propagations (Sec. II-A),
 * and `max_updates` always counts C2V propagations.
 *
 * Conventions
 *   - Every function returns 0 on success or a negative LDPC_E* code; nothing is thrown across
 *     the ABI and nothing is enqueued when an error is returned.  ldpc_strerror() names a code.
 *   - Device buffers are allocated and owned by the caller (e.g. PyTorch); the library reads
 *     inputs and writes outputs on the caller's HIP stream (`stream` is a hipStream_t, NULL =
 *     the default stream).  Calls are enqueue-only: outputs are valid once the stream is
 *     synchronised.
 *   - The library owns only ldpc_code handles.  A handle is immutable after creation and may be
 *     shared by concurrent calls on different streams; decode calls are reentrant.  Scratch
 *     memory needed by a call is allocated and freed by the library inside the call, stream-
 *     ordered, from a memory pool of the library's own per device that keeps up to 2 GiB of
 *     freed memory for later calls until the process ends.
 *   - Layouts are row-major and frame-contiguous: [B][N] for per-VN arrays, [B][E] for per-edge
 *     arrays, [B] for per-frame scalars.  Edge ids are canonical: the position of the nonzero
 *     (m, n) in the row-major (check-major, VN-ascending) enumeration of H.
 */
#ifndef LDPCCI_H
#define LDPCCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define LDPC_OK 0
#define LDPC_EINVAL (-1)       /* malformed argument (shape, range, null pointer)            */
#define LDPC_ENOMEM (-2)       /* host or device allocation failed                            */
#define LDPC_EHIP (-3)         /* a HIP runtime call failed; see ldpc_last_hip_error()        */
#define LDPC_ECAPACITY (-4)    /* the frame state does not fit the device's on-chip memory    */
#define LDPC_EUNSUPPORTED (-5) /* schedule/arithmetic combination or code shape not supported */

/* Testing hook for the error paths: with the environment variable LDPCCI_FAULT=alloc every
   scratch allocation of a decode fails (LDPC_ENOMEM); with LDPCCI_FAULT=launch every decode
   launch fails (LDPC_EHIP, ldpc_last_hip_error() = hipErrorLaunchFailure).  Nothing reaches the
   device in either case.  Read at each call. */

/* schedules */
#define LDPC_FLOODING 0
#define LDPC_LAYERED 1
#define LDPC_RBP 2
#define LDPC_CIRBP 3
#define LDPC_ME_CIRBP 4
#define LDPC_REPLAY 5
/* LMD schedules: the first update is chosen globally (LMDRBP, sLMDRBP: the edge of largest
   residual; LMD-CIRBP: the VN of largest CI, then its incoming edge of largest residual).  After an
   update of (m*, n*) the next one is chosen among the checks of M(n*) \ m*, which have just
   received n*'s new V2C messages (among m* itself when n* has degree 1, Sec. V):
     LMDRBP     the edge (i, j), j != n*, of largest residual; then VN j receives its incoming edge
                of largest residual (Algorithm 2);
     sLMDRBP    that edge (i, j) itself (Sec. IV-A);
     LMD-CIRBP  the VN j != n* of largest CI; then its incoming edge of largest residual
                (Algorithm 3, which leaves that edge choice implicit after the first update).
   Ties go to the lowest edge id / VN index; there is no gamma threshold. */
#define LDPC_LMDRBP 6
#define LDPC_SLMDRBP 7
#define LDPC_LMD_CIRBP 8
/* multi-edge LMD-CIRBP (Algorithm 6, Sec. VI): the first step's set comes from Algorithm 4 (n_p,
   n_g, fill as for LDPC_ME_CIRBP).  After a step, every updated VN p proposes the VN of largest CI
   among U(m*_p, p), where m*_p is the check whose message p received (N(m*_p) \ p when p has degree
   1); the distinct proposals P' start the next set, and Algorithm 4 run on the VNs outside P' adds
   the remaining n_p - |P'| (Algorithm 6 names |P| there; this is the count that keeps the set at
   n_p).  Sets are sent in ascending VN order, as for LDPC_ME_CIRBP. */
#define LDPC_ME_LMD_CIRBP 9
/* Reproducibility: every schedule gives a frame the same outputs on every run and in every launch
   shape (tested bit for bit), in both arithmetics.  In the multi-edge schedules several checks
   updated in one step can change the precomputed total LLR of the same VN; in LDPC_SPA_F32 those
   changes are summed exactly per VN (each rounded to a multiple of 2^-32, added as 64-bit
   integers), or, in a step that changes more than 2048 such VNs, in ascending check order. */

/* arithmetic */
#define LDPC_SPA_F32 0  /* sum-product, FP32 messages                                          */
#define LDPC_MS_FIX 1   /* fixed-point min-sum (Sec. V), q_bits <= 8, frac_bits fractional bits */

/* Algorithm 4 fill of the partially selected CI group */
#define LDPC_FILL_LOWEST 0 /* lowest VN indices                                                */
#define LDPC_FILL_HASH 1   /* smallest keys splitmix64(splitmix64(splitmix64(seed^frame)^step)^n) */

typedef struct ldpc_code ldpc_code; /* opaque, library-owned */

typedef struct {
  int32_t kind;        /* LDPC_FLOODING .. LDPC_ME_LMD_CIRBP                                    */
  int32_t arith;       /* LDPC_SPA_F32 or LDPC_MS_FIX                                            */
  int32_t q_bits;      /* LDPC_MS_FIX: message width, 2..8 (saturation at +-(2^(q-1)-1))         */
  int32_t frac_bits;   /* LDPC_MS_FIX: channel quantisation llr * 2^frac_bits, 0..6              */
  float gamma;         /* CIRBP threshold: fall back to the global residual search if D_{n*} < gamma
                          (Algorithm 1 threshold test); MS_FIX compares D_q with round(gamma * 65534)    */
  int32_t n_p;         /* ME schedules: VNs updated per step (N_P, Sec. VI), 1..64               */
  int32_t n_g;         /* ME schedules: CI groups (N_G, Algorithm 4), 1..65535                   */
  int32_t fill;        /* ME schedules: LDPC_FILL_LOWEST or LDPC_FILL_HASH                       */
  uint64_t seed;       /* ME schedules: key of the hashed fill                                   */
  int64_t check_every; /* syndrome test at t = 0 and whenever t passes a multiple of check_every
                          (1 = after every update; E = end of each iteration as in Sec. II-A;
                          0 = never stop early).  Flooding/layered test after every iteration. */
} ldpc_schedule;

typedef struct {
  uint8_t* bits;         /* device [B][N], required: hard decisions bsgn(L_n)                    */
  float* llr_out;        /* device [B][N], nullable: total LLRs L_n (MS_FIX: L_q / 2^frac_bits)  */
  int64_t* updates_used; /* device [B], required: C2V propagations performed                     */
  int64_t* steps_used;   /* device [B], nullable: update steps (ME: VN sets; flooding/layered:
                            iterations; single-edge: = updates)                                  */
  int64_t* fallbacks;    /* device [B], nullable: CIRBP updates that used the RBP fallback       */
  int32_t* trace;        /* device [B][max_updates], nullable: edge id of every propagation     */
  float* dump_c2v;       /* device [B][E], nullable: final C2V messages                          */
  float* dump_pre;       /* device [B][E], nullable: final precomputed C2V messages (dynamic)    */
  float* dump_L;         /* device [B][N], nullable: final L (MS_FIX: integer units)             */
  float* dump_Lt;        /* device [B][N], nullable: final precomputed total LLRs (dynamic)      */
  float* dump_D;         /* device [B][N], nullable: final CI values (MS_FIX: D_q in [0,65534])  */
} ldpc_outputs;

typedef struct {
  int32_t M, N, E;
  int32_t max_dv, max_dc, n_layers;
  int32_t max_touch;         /* max over VNs of the summed degrees of its checks               */
  int64_t lds_bytes_f32;     /* LDS bytes per frame of the single-edge decoder, FP32 mode       */
  int64_t lds_bytes_fix;     /* same, fixed-point mode                                          */
  float mean_dv, mean_dc;    /* E / N and E / M                                                 */
  int32_t gf2_rank;          /* rank of H over GF(2) once ldpc_code_rank has computed it, else -1 */
  int32_t reserved;
} ldpc_code_stats;

/* Create a code handle from H in CSR form (host pointers; Sec. II-A: M x N parity-check matrix,
   N(m) = row m).  Column indices must be strictly ascending inside each row, every row must have
   at least 2 entries and every column at least 1.  layer_ptr (nullable) lists n_layers + 1 row
   offsets of consecutive layers whose rows share no VN (layered baseline); NULL = one row per
   layer.  The library copies the arrays; the caller keeps ownership of its buffers.
   Errors: LDPC_EINVAL on a malformed matrix or layer partition, LDPC_EUNSUPPORTED (a check of
   degree > 32, or N >= 2^24), LDPC_ENOMEM, LDPC_EHIP. */
int ldpc_code_from_csr(int32_t M, int32_t N, const int32_t* row_ptr, const int32_t* col_idx,
                       const int32_t* layer_ptr, int32_t n_layers, ldpc_code** out);

/* Create a code handle from a quasi-cyclic base matrix (host pointer shift[mb][nb], row-major;
   -1 = zero block, s in [0, Z) = circulant): check i Z + r meets VN j Z + ((r + s) mod Z) (the
   lifting used by the paper's Sec. V codes).  The expanded H uses canonical edge ids; the block
   rows form the layers.  Kernels use the base tables instead of per-edge index arrays.
   Errors: LDPC_EINVAL (shift out of range, a base row with < 2 blocks, an empty base column, more
   than 2^26 VNs or checks), LDPC_EUNSUPPORTED (a base row of more than 32 blocks, N >= 2^24),
   LDPC_ENOMEM, LDPC_EHIP. */
int ldpc_code_from_qc(int32_t mb, int32_t nb, int32_t Z, const int32_t* shift, ldpc_code** out);

/* Fill *out with the sizes and per-frame on-chip memory needs of a code. */
int ldpc_code_info(const ldpc_code* code, ldpc_code_stats* out);

/* Rank of H over GF(2) (the code has 2^(N - rank) codewords; the design rate of Sec. V's codes
   is 1 - M / N only when H has full rank).  Gaussian elimination on bit-packed rows on the host:
   O(M^2 N / 64) word operations and M N / 8 bytes, done once per handle (thread-safe) and kept;
   ldpc_code_info reports it afterwards.  Errors: LDPC_EINVAL (null pointer), LDPC_ENOMEM. */
int ldpc_code_rank(const ldpc_code* code, int32_t* rank);

/* Release a handle (and its device copy).  NULL is ignored. */
void ldpc_code_free(ldpc_code* code);

/* Decode B frames of channel LLRs llr_in (device [B][N], FP32: 2 y_n / sigma^2, Sec. II-A).
   replay (device [B][replay_len] edge ids, nullable) is used by LDPC_REPLAY only: update t
   propagates edge replay[f][t], with no selection and no early stop, for min(max_updates,
   replay_len) updates; an id outside [0, E) ends that frame early (updates_used tells where).
   Outputs as described in ldpc_outputs.
   Errors: LDPC_EINVAL (null required pointer, B < 0, max_updates < 0, bad schedule field),
   LDPC_EUNSUPPORTED (combination not implemented, a VN of degree > 63), LDPC_ECAPACITY (frame
   state exceeds on-chip memory), LDPC_EHIP (launch failure). */
int ldpc_decode(const ldpc_code* code, const ldpc_schedule* schedule, const float* llr_in, int32_t B,
                int64_t max_updates, const int32_t* replay, int64_t replay_len,
                const ldpc_outputs* out, void* stream);

/* Allocation-free ldpc_decode, for callers that cannot allocate device memory during the call
   (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Arguments,
   outputs, tuning and errors are those of ldpc_decode; the outputs a frame gets are identical.
   Scratch memory (the work-queue counter and the frame slots of the state that does not stay on
   chip) comes from one device array of LDPC_NOALLOC_SCRATCH_BYTES that the library holds on each
   GPU it runs on until the process ends, instead of the memory pool: the call allocates nothing.
   A decode whose slots would exceed the array runs on fewer persistent workgroups (same outputs,
   lower throughput); LDPC_ECAPACITY when not even one workgroup's slots fit.  Calls on one GPU share
   its array: calls that overlap on that GPU (on different streams, or from different threads
   without ordering) race and corrupt each other's frames.  The queue counter is cleared by a small
   kernel on the caller's stream at the start of each call.  Errors: as ldpc_decode, and LDPC_EHIP
   if the array's device address cannot be obtained. */
#define LDPC_NOALLOC_SCRATCH_BYTES (128ll << 20)
int ldpc_decode_noalloc(const ldpc_code* code, const ldpc_schedule* schedule, const float* llr_in, int32_t B,
                        int64_t max_updates, const int32_t* replay, int64_t replay_len,
                        const ldpc_outputs* out, void* stream);

/* One frame of a batched launch (device memory, 40 bytes). */
typedef struct {
  int32_t code;        /* index into the codes array of ldpc_decode_batch                         */
  int32_t kind;        /* LDPC_FLOODING, LDPC_LAYERED, LDPC_RBP, LDPC_CIRBP or an LMD schedule    */
                       /* (LDPC_LMDRBP, LDPC_SLMDRBP, LDPC_LMD_CIRBP)                            */
  float gamma;         /* CIRBP threshold (>= 0)                                                   */
  int32_t reserved;
  int64_t max_updates; /* cap in C2V propagations                                                  */
  int64_t llr_off;     /* element offset of the frame's N channel LLRs in llr_pool                 */
  int64_t out_off;     /* element offset of the frame's N outputs in bits_pool and llr_out_pool    */
} ldpc_frame_desc;

/* Decode F frames of uneven codes and schedules in one persistent launch (the batched form of
   ldpc_decode; the schedules are those of Sec. I, II-A, Algorithm 1 and Algorithms 2-3).  codes: host array of
   n_codes handles (1..64, all created on the current device).  s supplies the arithmetic (arith,
   q_bits, frac_bits) and check_every for every frame; frames (device [F]) the rest.  Workers pull
   frames from a device work queue in descriptor order (put the longest decodes first for the
   best balance).  llr_pool (device, llr_len floats), bits_pool (device, out_len bytes),
   llr_out_pool (device, out_len floats, nullable), updates_used / steps_used / fallbacks (device
   [F], the latter two nullable).  A descriptor with an unknown code or schedule, a negative gamma
   or cap, or an offset that does not leave room for N values in its pool is not decoded and gets
   updates_used = -1.  The launch shape follows ldpc_set_batch_tuning when a tuning is set.
   Errors: LDPC_EINVAL, LDPC_EUNSUPPORTED (a code with VN degree > 63 or a check of degree > 32),
   LDPC_ECAPACITY, LDPC_ENOMEM, LDPC_EHIP. */
int ldpc_decode_batch(const ldpc_code* const* codes, int32_t n_codes, const ldpc_schedule* s,
                      const ldpc_frame_desc* frames, int32_t F, const float* llr_pool, int64_t llr_len,
                      uint8_t* bits_pool, float* llr_out_pool, int64_t out_len, int64_t* updates_used,
                      int64_t* steps_used, int64_t* fallbacks, void* stream);

/* ---- differentiable unrolled decoder ------------------------------------------------------
   A schedule recorded by a single-edge decode (ldpc_outputs.trace of LDPC_RBP, LDPC_CIRBP or an
   LMD schedule with check_every = 0, so that every frame runs exactly T updates) is replayed with
   a weight w_e per edge.  From c2v = 0 and L = llr, step t on edge e = trace[f][t] (check m, VN n) does
       c2v_e += w_e (pre_e - c2v_e),   L_n += the same amount,
   where pre_e is the C2V rule of eq. (2) over the V2C messages L_k - c2v_{m->k}, k != n (the
   propagation step of Sec. II-A, steps 3-4, which it equals for w_e = 1).  FP32 sum-product.
   The schedule is held fixed: gradients do not flow through the selection. */

#define LDPC_UNROLL_MAX_CKPT_EVERY 128

/* Floats of checkpoint storage per frame: ceil(T / ckpt_every) * (E + N); negative on bad
   arguments. */
int64_t ldpc_unrolled_ckpt_floats(const ldpc_code* code, int32_t T, int32_t ckpt_every);

/* Forward pass of B frames.  llr (device [B][N]), w (device [E]), trace (device [B][T] edge ids),
   soft_out (device [B][N]): the final L; c2v_out (device [B][E], nullable): the final messages;
   ckpt (device, B * ldpc_unrolled_ckpt_floats(code, T, ckpt_every) floats, nullable): the state
   (c2v then L) at t = 0, ckpt_every, 2 ckpt_every, ... for ldpc_unrolled_backward.
   ckpt_every in 1..LDPC_UNROLL_MAX_CKPT_EVERY.  A frame whose trace holds an id outside [0, E)
   gets NaN outputs.  Enqueue-only on stream; the caller owns every buffer.
   Errors: LDPC_EINVAL, LDPC_EUNSUPPORTED (a check of degree < 2 or > 32), LDPC_ECAPACITY,
   LDPC_EHIP. */
int ldpc_unrolled_forward(const ldpc_code* code, const float* llr, const float* w, const int32_t* trace,
                          int32_t B, int32_t T, int32_t ckpt_every, float* ckpt, float* soft_out,
                          float* c2v_out, void* stream);

/* Adjoint of ldpc_unrolled_forward: given grad_soft = d loss / d soft_out (device [B][N]) and the
   checkpoints the forward wrote with the same trace, w, T and ckpt_every, writes
   grad_llr = d loss / d llr (device [B][N]) and grad_w = d loss / d w (device [E], the sum over
   frames in a fixed order: bitwise reproducible).  Each segment of ckpt_every steps is recomputed
   from its checkpoint.  A frame with an invalid trace id gets NaN in grad_llr and contributes NaN
   to grad_w.  Allocates B * E + 64 * E floats of stream-ordered scratch.  Errors as above, plus
   LDPC_ENOMEM. */
int ldpc_unrolled_backward(const ldpc_code* code, const float* w, const int32_t* trace, int32_t B, int32_t T,
                           int32_t ckpt_every, const float* ckpt, const float* grad_soft, float* grad_llr,
                           float* grad_w, void* stream);

/* ---- launch tuning --------------------------------------------------------------------------
   The arithmetic of a decode does not depend on these knobs (outputs are identical for every
   setting); they only choose where state lives and how the launch is shaped.  Zero = default. */
#define LDPC_STORE_AUTO 0        /* messages in LDS when they fit, else the next mode that fits   */
#define LDPC_STORE_LDS 1         /* C2V and precomputed messages in LDS                           */
#define LDPC_STORE_GLOBAL 2      /* precomputed messages in a global scratch slot (ME: all)       */
#define LDPC_STORE_GLOBAL_ALL 3  /* C2V and precomputed messages as interleaved pairs in a global
                                    slot                                                          */
#define LDPC_STORE_GLOBAL_LT 4   /* those pairs and the precomputed total LLRs in a global slot   */
#define LDPC_STORE_GLOBAL_FRAME 5 /* the whole frame (messages, precomputed and total LLRs, CIs)
                                     in a global slot; only keys and trees stay in LDS: the most
                                     frames per CU                                                */
#define LDPC_STORE_GLOBAL_REC 6   /* as GLOBAL_FRAME, with the precomputed total and the total of
                                     a VN in one 8-byte record (the CI is evaluated from it;
                                     single-edge schedules only)                                  */
#define LDPC_STORE_GLOBAL_STATE 7 /* as GLOBAL_REC, with the check keys in the slot too: LDS holds
                                     only block maxima and small bookkeeping (single-edge only)   */
#define LDPC_TOPO_AUTO 0    /* quasi-cyclic tables, else LDS copies, else global arrays       */
#define LDPC_TOPO_GLOBAL 1
#define LDPC_TOPO_LDS 2
#define LDPC_TOPO_QC 3

typedef struct {
  int32_t block;         /* threads per workgroup (64..1024, step 64): per frame for flooding,
                            layered and ME-CIRBP; for RBP / CIRBP / replay 64 x the frames that
                            share a workgroup (and its LDS copy of the topology)                   */
  int32_t frames_per_cu; /* single-edge and ME: resident frames per CU of a persistent grid (1..32) */
  int32_t storage;       /* LDPC_STORE_*: where the messages of a frame live                        */
  int32_t topology;      /* LDPC_TOPO_*: where the kernels read H from                              */
} ldpc_tuning;

/* Set (t non-null) or clear (t null) the tuning that ldpc_decode uses for this code (any handle
   with the same H), schedule kind and arithmetic.  Process-wide, thread-safe.  A knob that does
   not fit a later call (e.g. LDS storage that does not fit) makes that call fail with
   LDPC_ECAPACITY / LDPC_EUNSUPPORTED.  Errors: LDPC_EINVAL (bad kind, arith or knob value). */
int ldpc_set_tuning(const ldpc_code* code, int32_t kind, int32_t arith, const ldpc_tuning* t);

/* The stored tuning (all zero if none): returns 1 if an entry exists, 0 if not, <0 on error. */
int ldpc_get_tuning(const ldpc_code* code, int32_t kind, int32_t arith, ldpc_tuning* out);

/* The launch ldpc_decode would make for B frames of this code and schedule (with the tuning stored
   for it, if any), without decoding: for reports and for sizing.  The device must be current, as
   for ldpc_decode.  Errors: LDPC_EINVAL (null pointer, B < 1, bad schedule), LDPC_ECAPACITY,
   LDPC_EUNSUPPORTED (as ldpc_decode would return them), LDPC_EHIP. */
typedef struct {
  int32_t kernel;               /* 0 flooding / layered, 1 single-edge (RBP, CIRBP, replay), 2 ME-CIRBP,
                                   3 batched (ldpc_describe_batch_plan)                                  */
  int32_t storage;              /* LDPC_STORE_* chosen (never AUTO); flooding / layered: LDS           */
  int32_t topology;             /* LDPC_TOPO_* chosen (never AUTO); flooding / layered: GLOBAL         */
  int32_t block;                /* threads per workgroup                                               */
  int32_t grid;                 /* workgroups launched                                                 */
  int32_t frames_per_workgroup; /* frames one workgroup decodes at once (single-edge: its wavefronts) */
  int32_t workgroups_per_cu;    /* workgroups a CU can hold by LDS and by wavefront slots at the
                                   kernel's register count                                          */
  int32_t persistent;           /* 1: fewer workgroups than frames, each takes frames in turn (single-
                                   edge: from a device work queue)                                     */
  int32_t lds_bytes;            /* dynamic LDS per workgroup                                           */
  int32_t reserved;
  int64_t scratch_bytes;        /* stream-ordered device scratch the decode allocates                 */
} ldpc_plan_info;

int ldpc_describe_plan(const ldpc_code* code, const ldpc_schedule* s, int32_t B, ldpc_plan_info* info);

/* The launch ldpc_decode_batch would make for F frames over these codes with this schedule's
   arithmetic (and the tuning of ldpc_set_batch_tuning, if set), without decoding: kernel = 3
   (batched; one frame per workgroup of one wavefront), the storage mode and topology source chosen
   for the largest code, the frames per CU the LDS layout allows (workgroups_per_cu), grid, LDS and
   scratch bytes.  Errors: LDPC_EINVAL, LDPC_EUNSUPPORTED, LDPC_ECAPACITY, LDPC_EHIP. */
int ldpc_describe_batch_plan(const ldpc_code* const* codes, int32_t n_codes, const ldpc_schedule* s, int32_t F,
                             ldpc_plan_info* info);

/* Project autotuner: times every distinct launch plan the knobs give for this schedule on the
   caller's frames (llr_in: device [B][N]; best of reps timed runs after one warm-up, HIP events on
   stream), stores the fastest with ldpc_set_tuning and returns it (best, best_ms nullable).
   Tune on a batch of the size that will be decoded: a small batch cannot use the frame
   residency that large batches gain from, and favours low-latency plans.
   Blocking: synchronizes stream.  Candidates: block in {64..1024} for flooding / layered;
   storage (LDS, pre global, all messages global, messages and Lt global, whole frame global as
   arrays or as VN records, whole frame and check keys global) x
   topology x frames per workgroup in {auto, 4, 8} x
   frames_per_cu in {auto, 1, 2, 4, 8, 16}
   (and block in {64, 256, 1024} for ME-CIRBP) for the dynamic schedules.  A candidate whose
   scratch memory cannot be allocated is skipped.  Errors: LDPC_EINVAL, LDPC_EUNSUPPORTED (replay),
   LDPC_ECAPACITY (no candidate fits), LDPC_EHIP. */
int ldpc_autotune(const ldpc_code* code, const ldpc_schedule* s, const float* llr_in, int32_t B,
                  int64_t max_updates, int32_t reps, ldpc_tuning* best, float* best_ms, void* stream);

/* Launch tuning of ldpc_decode_batch, process-wide (one frame per workgroup there, so block and
   topology must be 0): storage (LDPC_STORE_AUTO .. LDPC_STORE_GLOBAL_REC; LDPC_STORE_GLOBAL_STATE
   has no batched form: LDPC_EUNSUPPORTED) and a cap on resident frames per CU (0 = as many as
   LDS allows, at most 32).  NULL restores the default policy.  ldpc_get_batch_tuning returns 1
   and fills *out if a tuning is set, else 0.  Errors: LDPC_EINVAL. */
int ldpc_set_batch_tuning(const ldpc_tuning* t);
int ldpc_get_batch_tuning(ldpc_tuning* out);

/* Project autotuner of the batched launch: decodes the caller's batch (arguments as for
   ldpc_decode_batch; outputs go to scratch buffers and are discarded) under every storage x
   frames-per-CU cap in {auto, 4, 8, 12, 16, 24}, takes the best of reps timed launches after one
   warm-up (HIP events on stream), stores the fastest with ldpc_set_batch_tuning and returns it
   (best, best_ms nullable).  Candidates whose state does not fit are skipped.  Blocking:
   synchronizes stream.  Errors: LDPC_EINVAL, LDPC_ECAPACITY (no candidate fits), LDPC_ENOMEM,
   LDPC_EHIP. */
int ldpc_autotune_batch(const ldpc_code* const* codes, int32_t n_codes, const ldpc_schedule* s,
                        const ldpc_frame_desc* frames, int32_t F, const float* llr_pool, int64_t llr_len,
                        int64_t out_len, int32_t reps, ldpc_tuning* best, float* best_ms, void* stream);

/* Write every stored tuning (per code, and the batched launch's) to a JSON file, tagged with the
   current device's architecture and CU count; ldpc_tuning_load reads such a file back (entries of
   another device are ignored) and returns the number loaded.  Errors: LDPC_EINVAL (path),
   LDPC_EHIP. */
int ldpc_tuning_save(const char* path);
int ldpc_tuning_load(const char* path);

/* ---- SNR sweeps -----------------------------------------------------------------------------
   Channel frames on the device: frame f of sweep point p carries codeword f mod P of a pool
   (device [P][N] bytes 0/1); bit n gets x = 1 - 2c plus noise sigma z, z one Box-Muller normal
   from Philox4x32-10 (Salmon et al., SC 2011) with counter (n, f, p, 0) and key (seed mod 2^32,
   seed >> 32): u1 = (x0 + 1) 2^-32, u2 = x1 2^-32, z = sqrt(-2 ln u1) cos(2 pi u2).  The LLR is
   (2 / sigma^2)(x + sigma z), the channel LLR of Sec. II-A. */

/* Write B frames of point `point` to llr_out (device [B][N]).  Errors: LDPC_EINVAL, LDPC_EHIP. */
int ldpc_awgn_frames(const uint8_t* codewords, int32_t P, int32_t N, int32_t B, float sigma2, uint64_t seed,
                     int32_t point, float* llr_out, void* stream);

typedef struct ldpc_sweep ldpc_sweep;

/* Capture an SNR sweep into one hipGraph: for each of the S points (Eb/N0 in dB, host array,
   sigma^2 = 1 / (2 rate 10^(EbN0/10))) generate B frames from the codeword pool, decode them with
   schedule s (cap max_updates, the tuning stored for this code if any), and count per point
   {frames, frame errors, bit errors, sum of updates_used}.  The library allocates the frame
   buffers and decode scratch once; the pool (device [P][N]) must stay valid for the sweep's life.
   Errors: LDPC_EINVAL, LDPC_EUNSUPPORTED (replay), LDPC_ECAPACITY, LDPC_ENOMEM, LDPC_EHIP. */
int ldpc_sweep_create(const ldpc_code* code, const ldpc_schedule* s, int64_t max_updates, const uint8_t* codewords,
                      int32_t P, const float* ebn0_db, int32_t S, float rate, int32_t B, ldpc_sweep** out);

/* Launch the captured sweep with a seed on stream and copy its counters to `counters` (device
   [S][4] int64).  Enqueue-only.  Runs of one sweep object must not overlap (they share buffers).
   Errors: LDPC_EINVAL, LDPC_EHIP. */
int ldpc_sweep_run(ldpc_sweep* sweep, uint64_t seed, int64_t* counters, void* stream);

/* Destroy a sweep (waits for the device first).  NULL is ignored. */
void ldpc_sweep_free(ldpc_sweep* sweep);

/* ---- stopping decodes ------------------------------------------------------------------------
   Process-wide abort flag, for serving loops that must stop work in flight.  While it is set
   (on != 0), every decode running or launched later on any device starts no further frame: each
   frame it has not started gets updates_used = -1, its other outputs left as they were (and the
   counters of an SNR sweep run meanwhile are not meaningful).  Frames already started finish
   normally.  Clear it (on = 0) before decoding again.  The flag lives in pinned host memory that
   the kernels read before each frame, so it takes effect without waiting for the decode's stream.
   Errors: LDPC_EHIP (the flag could not be created). */
int ldpc_request_abort(int32_t on);

/* ---- measurement ----------------------------------------------------------------------------
   The denominator of an LDS roofline, measured: `blocks` workgroups of 256 lanes each fill a
   16 KiB LDS buffer, then every lane makes iters x 16 aligned reads of `width` bytes (4, 8 or 16:
   one ds_read_b32 / b64 / b128 each), consecutive lanes at consecutive addresses, folding them
   into one word that lane 0 writes to sink[workgroup] (device [blocks] uint32, caller-owned).
   *bytes receives the bytes read, *ms the time between two events recorded on stream around the
   launch; the call waits for the second event.  Errors: LDPC_EINVAL (width, blocks < 1, iters
   outside 1..2^24, null pointer), LDPC_EHIP. */
int ldpc_probe_lds(int32_t width, int32_t blocks, int64_t iters, uint32_t* sink, void* stream, double* bytes,
                   float* ms);

/* Human-readable name of an error code (static string). */
const char* ldpc_strerror(int code);

/* The last hipError_t recorded by a failing call on this thread (0 if none). */
int ldpc_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LDPCCI_H */
