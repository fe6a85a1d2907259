/*
 * ldpc_oracle.c -- plain, slow CPU oracle for LDPC belief-propagation decoding with
 * flooding, layered, residual (RBP), conditional-innovation RBP (CIRBP, Algorithm 1),
 * multi-edge CIRBP (Algorithms 4 and 5), latest-message-driven (LMDRBP and sLMDRBP,
 * Algorithm 2; LMD-CIRBP, Algorithm 3) and multi-edge LMD-CIRBP (Algorithm 6) schedules.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  It shares no code, header, table or constant generator with the
 * GPU library.
 *
 * Everything is kept in the plainest form: per-edge arrays, linear-scan argmax with strict '>'
 * (so the lowest index wins ties), from-scratch sums for the total and precomputed LLRs.
 *
 * Arithmetic modes
 *   ARITH_SPA   : sum-product in double.  The C2V rule of eq. (2) (Sec. II-A) is evaluated
 *                 pairwise with the exact identity
 *                   a [+] b = 2 atanh(tanh(a/2) tanh(b/2))
 *                       = s(a)s(b) min(|a|,|b|) + log1p(e^-(|a|+|b|)) - log1p(e^-||a|-|b||),
 *                 folded over the other inputs of the check in ascending VN order.
 *                 CI (eq. (9), Sec. III-A): D = |p0(L) - p0(Lt)|, p0(x) = e^x / (1 + e^x),
 *                 evaluated as 0.5 |tanh(L/2) - tanh(Lt/2)| (p0(x) = (1 + tanh(x/2)) / 2).
 *   ARITH_MSFIX : fixed-point min-sum (Sec. V names min-sum as the cheaper C2V rule).  All values
 *                 are integers (held exactly in doubles): channel ch = sat(round_half_away(llr*2^f)),
 *                 sat(x) = clamp(x, -(2^(q-1)-1), 2^(q-1)-1), V2C = sat(L - c2v),
 *                 C2V = (product of signs, sign(0) = +) * min |V2C| over the other inputs,
 *                 L and Lt exact (unsaturated).  CI uses a p0 look-up table (Sec. V-B mentions
 *                 a table look-up of p0): T[x] = round_half_away(32767 tanh(x 2^-f / 2)),
 *                 x in [-128, 128] (index clamped), D = |T[L] - T[Lt]| in [0, 65534];
 *                 the threshold is gamma_q = round(gamma * 65534).
 *
 * Readings of points the paper leaves open (the same readings are used by the GPU path):
 *   - bsgn(0) = 0 (Sec. II-A), and the min-sum sign of a zero V2C is '+'.
 *   - D of the updated VN n* is refreshed after L_{n*} changes (Algorithm 1 only lists the
 *     neighbours of the touched checks; without the refresh n* would stay the global maximum).
 *   - ties: lowest VN index, lowest check index, lowest canonical (row-major) edge id.
 *   - stop rule: syndrome tested at t = 0 and every `check_every` updates (0 = never); the
 *     decoder also stops when t reaches max_updates.  Flooding and layered test after each
 *     iteration (E updates) and only run whole iterations.
 *   - ME-CIRBP: VN set chosen on the current snapshot (Algorithm 4), each selected VN picks its
 *     incoming edge on the snapshot, all propagations are applied, then every check adjacent to
 *     a selected VN is recomputed from the new state.  The random fill of Algorithm 4 takes
 *     either the lowest VN indices of the fill group, or the VNs with the smallest keys
 *     splitmix64(splitmix64(splitmix64(seed ^ frame) ^ step) ^ n) (ties: lower n), a uniform
 *     random subset that is reproducible from (seed, frame, step).
 *   - LMD schedules (Sec. IV): the first update is chosen globally (Algorithm 2: largest residual;
 *     Algorithm 3: largest CI, then the incoming edge of largest residual).  After an update of
 *     e* = (m*, n*) the next one is chosen among the messages just precomputed: LMDRBP takes the
 *     edge (i, j) of largest residual over i in M(n*) \ m*, j in N(i) \ n*, then n' = j receives
 *     its incoming edge of largest residual; sLMDRBP sends the edge (i, j) itself; LMD-CIRBP takes
 *     the VN n' of largest CI over the same VNs, U(m*, n*), and n' then receives its incoming edge
 *     of largest residual (Algorithm 3 keeps m* implicit after the first update; this reading
 *     chooses it as for the first one).  When n* has degree 1 the candidates come from m* itself:
 *     edges (m*, j), VNs j of N(m*) \ n* (Sec. V).  Ties go to the lowest edge id / VN index.  An
 *     empty candidate set (only with checks of degree 1) sends the next update to the global
 *     choice again.
 *   - ME-LMD-CIRBP (Algorithm 6): the first step's set P comes from Algorithm 4.  After a step
 *     (the ME-CIRBP step above), every p in P proposes p', the VN of largest CI among U(m*_p, p)
 *     on the state after the step (m*_p the check whose message p received; N(m*_p) \ p when p has
 *     degree 1).  The distinct proposals form P'; if |P'| < N_P, Algorithm 4 adds N_P - |P'| VNs
 *     chosen among the VNs outside P' (its groups counted without P'), and the union is the next
 *     step's P.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
  OC_FLOODING = 0,
  OC_LAYERED = 1,
  OC_RBP = 2,
  OC_CIRBP = 3,
  OC_MECIRBP = 4,
  OC_REPLAY = 5,
  OC_LMDRBP = 6,
  OC_SLMDRBP = 7,
  OC_LMDCIRBP = 8,
  OC_MELMDCIRBP = 9
};
enum { ARITH_SPA = 0, ARITH_MSFIX = 1 };
enum {
  CNT_PROP = 0,   /* C2V propagations (= updates)                                   */
  CNT_V2C,        /* V2C messages regenerated                                       */
  CNT_PRE,        /* C2V pre-updates (precomputed messages + residuals)             */
  CNT_CI,         /* CI updates at neighbours of touched checks (pairs (i, j))      */
  CNT_CI_SELF,    /* CI refreshes of the updated VN itself                          */
  CNT_FALLBACK,   /* CIRBP updates with D_{n*} < gamma (global residual search)     */
  CNT_CMP,        /* real-number comparisons in the selection scans                 */
  CNT_STEPS,      /* update steps (single-edge: = updates; ME: number of VN sets)   */
  OC_NCOUNT
};
enum { OC_OK = 0, OC_EINVAL = -1, OC_ENOMEM = -2, OC_ESELFCHECK = -7 };

typedef struct {
  int32_t M, N, E;
  const int32_t *row_ptr, *col;                  /* CSR; edge id = CSR position          */
  const int32_t *col_ptr, *col_row, *col_eid;    /* CSC; checks ascending per column      */
  int32_t n_layers;
  const int32_t *layer_ptr;                      /* consecutive row ranges, may be NULL   */
} oc_code;

typedef struct {
  int32_t kind, arith, q_bits, frac_bits;
  double gamma;
  int32_t n_p, n_g;
  int64_t check_every;
  int32_t selfcheck;
  int32_t fill;      /* Algorithm 4 fill: 0 = lowest VN indices, 1 = keyed random subset */
  uint64_t seed;     /* key of the random fill                                          */
} oc_sched;

/* ------------------------------------------------------------------------------------------ */
/* scalar rules                                                                                */
/* ------------------------------------------------------------------------------------------ */
static double sgn_pos(double x) { return x < 0.0 ? -1.0 : 1.0; }

/* pairwise check rule of eq. (2) in the exact Jacobian-logarithm form (sum-product) */
double oc_boxplus(double a, double b) {
  double aa = fabs(a), ab = fabs(b);
  double mag = fmin(aa, ab) + log1p(exp(-(aa + ab))) - log1p(exp(-fabs(aa - ab)));
  return sgn_pos(a) * sgn_pos(b) * mag;
}

/* eq. (2) in its literal tanh-product form (only used by tests as a cross-check) */
double oc_c2v_tanh(const double *v, int n) {
  double p = 1.0;
  for (int i = 0; i < n; ++i) p *= tanh(0.5 * v[i]);
  return 2.0 * atanh(p);
}

static double round_half_away(double x) { return x < 0 ? -floor(-x + 0.5) : floor(x + 0.5); }

typedef struct {
  const oc_code *H;
  const oc_sched *s;
  int arith;
  double qmax;       /* saturation bound for ARITH_MSFIX                       */
  double lut[257];   /* p0 table (ARITH_MSFIX), index x + 128                  */
  double gamma_eff;  /* gamma in the metric's own units                        */
  /* per-frame state */
  double *ch, *c2v, *pre, *L, *Lt, *D, *tmp;
  uint8_t *syn;
  int64_t unsat;
  int32_t *row_of;
} st_t;

static double sat(const st_t *S, double x) {
  if (S->arith == ARITH_SPA) return x;
  if (x > S->qmax) return S->qmax;
  if (x < -S->qmax) return -S->qmax;
  return x;
}

static double check_rule(const st_t *S, double a, double b) {
  if (S->arith == ARITH_SPA) return oc_boxplus(a, b);
  /* min-sum: sign product times minimum magnitude */
  return sgn_pos(a) * sgn_pos(b) * fmin(fabs(a), fabs(b));
}

double oc_ci_spa(double L, double Lt) { return 0.5 * fabs(tanh(0.5 * L) - tanh(0.5 * Lt)); }

static double ci(const st_t *S, double L, double Lt) {
  if (S->arith == ARITH_SPA) return oc_ci_spa(L, Lt);
  int a = (int)(L < -128 ? -128 : (L > 128 ? 128 : L));
  int b = (int)(Lt < -128 ? -128 : (Lt > 128 ? 128 : Lt));
  return fabs(S->lut[a + 128] - S->lut[b + 128]);
}

static int bsgn(double L) { return L >= 0.0 ? 0 : 1; }

/* ------------------------------------------------------------------------------------------ */
/* derived quantities, each from its definition                                                */
/* ------------------------------------------------------------------------------------------ */
static double v2c(const st_t *S, int32_t e) {
  return sat(S, S->L[S->H->col[e]] - S->c2v[e]);     /* eq. (1): L_n minus own C2V */
}

/* precomputed C2V messages of every edge of check m (eq. (2) over N(m) \ n) */
static void recompute_row(st_t *S, int32_t m) {
  const oc_code *H = S->H;
  int32_t b = H->row_ptr[m], e_end = H->row_ptr[m + 1];
  for (int32_t e = b; e < e_end; ++e) S->tmp[e - b] = v2c(S, e);
  for (int32_t e = b; e < e_end; ++e) {
    int first = 1;
    double acc = 0.0;
    for (int32_t k = b; k < e_end; ++k) {
      if (k == e) continue;
      acc = first ? S->tmp[k - b] : check_rule(S, acc, S->tmp[k - b]);
      first = 0;
    }
    S->pre[e] = acc;
  }
}

static double residual(const st_t *S, int32_t e) { return fabs(S->pre[e] - S->c2v[e]); } /* eq. (4) */

static double total_llr(const st_t *S, int32_t n) { /* eq. (3) */
  const oc_code *H = S->H;
  double acc = S->ch[n];
  for (int32_t k = H->col_ptr[n]; k < H->col_ptr[n + 1]; ++k) acc += S->c2v[H->col_eid[k]];
  return acc;
}

static double pre_llr(const st_t *S, int32_t n) { /* precomputed total LLR (Sec. II-B) */
  const oc_code *H = S->H;
  double acc = S->ch[n];
  for (int32_t k = H->col_ptr[n]; k < H->col_ptr[n + 1]; ++k) acc += S->pre[H->col_eid[k]];
  return acc;
}

static void recompute_syndrome(st_t *S) {
  const oc_code *H = S->H;
  S->unsat = 0;
  for (int32_t m = 0; m < H->M; ++m) {
    int x = 0;
    for (int32_t e = H->row_ptr[m]; e < H->row_ptr[m + 1]; ++e) x ^= bsgn(S->L[H->col[e]]);
    S->syn[m] = (uint8_t)x;
    S->unsat += x;
  }
}

static void syndrome_rows_of_vn(st_t *S, int32_t n) {
  const oc_code *H = S->H;
  for (int32_t k = H->col_ptr[n]; k < H->col_ptr[n + 1]; ++k) {
    int32_t m = H->col_row[k];
    int x = 0;
    for (int32_t e = H->row_ptr[m]; e < H->row_ptr[m + 1]; ++e) x ^= bsgn(S->L[H->col[e]]);
    S->unsat += x - S->syn[m];
    S->syn[m] = (uint8_t)x;
  }
}

/* Algorithm 1, initialisation: c2v = 0, L = channel, all precomputed messages, Lt and D */
static void init_dynamic(st_t *S) {
  const oc_code *H = S->H;
  for (int32_t e = 0; e < H->E; ++e) S->c2v[e] = 0.0;
  for (int32_t n = 0; n < H->N; ++n) S->L[n] = S->ch[n];
  for (int32_t m = 0; m < H->M; ++m) recompute_row(S, m);
  for (int32_t n = 0; n < H->N; ++n) {
    S->Lt[n] = pre_llr(S, n);
    S->D[n] = ci(S, S->L[n], S->Lt[n]);
  }
  recompute_syndrome(S);
}

/* invariant check: every derived quantity equals its from-scratch definition */
static int selfcheck(st_t *S) {
  const oc_code *H = S->H;
  double tol = S->arith == ARITH_SPA ? 1e-9 : 0.0;
  double *save = (double *)malloc(sizeof(double) * (size_t)H->E);
  if (!save) return OC_ENOMEM;
  memcpy(save, S->pre, sizeof(double) * (size_t)H->E);
  for (int32_t m = 0; m < H->M; ++m) recompute_row(S, m);
  int bad = 0;
  for (int32_t e = 0; e < H->E && !bad; ++e)
    if (fabs(save[e] - S->pre[e]) > tol * fmax(1.0, fabs(S->pre[e]))) bad = 1;
  memcpy(S->pre, save, sizeof(double) * (size_t)H->E);
  free(save);
  for (int32_t n = 0; n < H->N && !bad; ++n) {
    if (fabs(total_llr(S, n) - S->L[n]) > tol * fmax(1.0, fabs(S->L[n]))) bad = 2;
    if (fabs(pre_llr(S, n) - S->Lt[n]) > tol * fmax(1.0, fabs(S->Lt[n]))) bad = 3;
    if (fabs(ci(S, S->L[n], S->Lt[n]) - S->D[n]) > tol) bad = 4;
    if (S->D[n] < 0.0 || (S->arith == ARITH_SPA && S->D[n] >= 1.0)) bad = 5;
  }
  int64_t u = S->unsat;
  recompute_syndrome(S);
  if (u != S->unsat) bad = 6;
  return bad ? OC_ESELFCHECK : OC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* single-edge update (Algorithm 1 propagation and precompute loop / RBP steps 3-4)             */
/* ------------------------------------------------------------------------------------------ */
static void apply_edge(st_t *S, int32_t estar, int64_t *cnt) {
  const oc_code *H = S->H;
  int32_t mstar = S->row_of[estar], nstar = H->col[estar];
  int old_bit = bsgn(S->L[nstar]);
  S->c2v[estar] = S->pre[estar];               /* propagate; its residual becomes 0 */
  S->L[nstar] = total_llr(S, nstar);
  if (bsgn(S->L[nstar]) != old_bit) syndrome_rows_of_vn(S, nstar);
  cnt[CNT_PROP] += 1;
  /* new V2C from n* to every other check, then precompute that check again */
  for (int32_t k = H->col_ptr[nstar]; k < H->col_ptr[nstar + 1]; ++k) {
    int32_t i = H->col_row[k];
    if (i == mstar) continue;
    recompute_row(S, i);
    cnt[CNT_V2C] += 1;
    int32_t dci = H->row_ptr[i + 1] - H->row_ptr[i];
    cnt[CNT_PRE] += dci - 1;
    cnt[CNT_CI] += dci - 1;
  }
  /* precomputed total LLR and CI of the neighbours of the touched checks */
  for (int32_t k = H->col_ptr[nstar]; k < H->col_ptr[nstar + 1]; ++k) {
    int32_t i = H->col_row[k];
    if (i == mstar) continue;
    for (int32_t e = H->row_ptr[i]; e < H->row_ptr[i + 1]; ++e) {
      int32_t j = H->col[e];
      if (j == nstar) continue;
      S->Lt[j] = pre_llr(S, j);
      S->D[j] = ci(S, S->L[j], S->Lt[j]);
    }
  }
  S->D[nstar] = ci(S, S->L[nstar], S->Lt[nstar]);
  cnt[CNT_CI_SELF] += 1;
}

/* global residual argmax over all edges (eq. (5)); lowest edge id on ties */
static int32_t argmax_residual(const st_t *S, int64_t *cnt) {
  int32_t best = 0;
  double bv = residual(S, 0);
  for (int32_t e = 1; e < S->H->E; ++e) {
    double r = residual(S, e);
    cnt[CNT_CMP] += 1;
    if (r > bv) { bv = r; best = e; }
  }
  return best;
}

static int32_t argmax_ci(const st_t *S, int64_t *cnt) {
  int32_t best = 0;
  for (int32_t n = 1; n < S->H->N; ++n) {
    cnt[CNT_CMP] += 1;
    if (S->D[n] > S->D[best]) best = n;
  }
  return best;
}

/* edge into VN n with the largest residual (Algorithm 1 edge choice); lowest check on ties */
static int32_t argmax_into(const st_t *S, int32_t n, int64_t *cnt) {
  const oc_code *H = S->H;
  int32_t best = H->col_eid[H->col_ptr[n]];
  for (int32_t k = H->col_ptr[n] + 1; k < H->col_ptr[n + 1]; ++k) {
    int32_t e = H->col_eid[k];
    cnt[CNT_CMP] += 1;
    if (residual(S, e) > residual(S, best)) best = e;
  }
  return best;
}

/* Algorithm 2, local edge choice: after the update of e*, the edge (i, j) of largest residual
   with i a check of n* other than m* (m* itself when n* has degree 1, Sec. V) and j != n*; lowest
   edge id on ties; -1 when there is no candidate */
static int32_t lmd_edge(const st_t *S, int32_t estar, int64_t *cnt) {
  const oc_code *H = S->H;
  int32_t mstar = S->row_of[estar], nstar = H->col[estar];
  int deg1 = H->col_ptr[nstar + 1] - H->col_ptr[nstar] == 1;
  int32_t best = -1;
  double bv = 0.0;
  for (int32_t k = H->col_ptr[nstar]; k < H->col_ptr[nstar + 1]; ++k) {
    int32_t i = H->col_row[k];
    if (i == mstar && !deg1) continue;
    for (int32_t e = H->row_ptr[i]; e < H->row_ptr[i + 1]; ++e) {
      if (H->col[e] == nstar) continue;
      double r = residual(S, e);
      if (best < 0) {
        best = e;
        bv = r;
        continue;
      }
      cnt[CNT_CMP] += 1;
      if (r > bv || (r == bv && e < best)) {
        best = e;
        bv = r;
      }
    }
  }
  return best;
}

/* Algorithm 3, local VN choice: after the update of e*, the VN of largest CI among U(m*, n*), the
   VNs other than n* of the checks of n* other than m* (of m* itself when n* has degree 1, Sec. V);
   lowest VN index on ties; -1 when there is no candidate */
static int32_t lmd_vn(const st_t *S, int32_t estar, int64_t *cnt) {
  const oc_code *H = S->H;
  int32_t mstar = S->row_of[estar], nstar = H->col[estar];
  int deg1 = H->col_ptr[nstar + 1] - H->col_ptr[nstar] == 1;
  int32_t best = -1;
  for (int32_t k = H->col_ptr[nstar]; k < H->col_ptr[nstar + 1]; ++k) {
    int32_t i = H->col_row[k];
    if (i == mstar && !deg1) continue;
    for (int32_t e = H->row_ptr[i]; e < H->row_ptr[i + 1]; ++e) {
      int32_t j = H->col[e];
      if (j == nstar) continue;
      if (best < 0) {
        best = j;
        continue;
      }
      cnt[CNT_CMP] += 1;
      if (S->D[j] > S->D[best] || (S->D[j] == S->D[best] && j < best)) best = j;
    }
  }
  return best;
}

static int32_t select_cirbp(st_t *S, int64_t *cnt) {
  int32_t nstar = argmax_ci(S, cnt);
  cnt[CNT_CMP] += 1; /* the threshold test */
  if (S->D[nstar] < S->gamma_eff) {
    cnt[CNT_FALLBACK] += 1;
    return argmax_residual(S, cnt);
  }
  return argmax_into(S, nstar, cnt);
}

/* ------------------------------------------------------------------------------------------ */
/* Algorithm 4 (VN selection) and one ME-CIRBP step (Algorithm 5)                              */
/* ------------------------------------------------------------------------------------------ */
static int32_t bin_of(const st_t *S, double D, int32_t ng) {
  int64_t b;
  if (S->arith == ARITH_SPA) b = (int64_t)floor(D * ng);
  else b = ((int64_t)D * ng) / 65535;
  if (b > ng - 1) b = ng - 1;
  if (b < 0) b = 0;
  return (int32_t)b;
}

/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014): one increment of the golden
   gamma followed by the variant-13 finaliser */
uint64_t oc_splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

uint64_t oc_fill_key(uint64_t seed, uint64_t frame, uint64_t step, uint64_t n) {
  return oc_splitmix64(oc_splitmix64(oc_splitmix64(seed ^ frame) ^ step) ^ n);
}

/* Algorithm 4 over the VNs n with excl[n] == 0 (excl == NULL: all VNs).  keys == NULL: fill with
   the lowest indices; otherwise with the smallest keys.  Fills sel[] in ascending VN order and
   returns |P|. */
int32_t oc_alg4_select_excl(int32_t N, const int32_t *bins, int32_t ng, int32_t np, const uint64_t *keys,
                            const uint8_t *excl, int32_t *sel) {
  if (N <= 0 || ng <= 0) return 0;
  int32_t *count = (int32_t *)calloc((size_t)ng, sizeof(int32_t));
  for (int32_t n = 0; n < N; ++n)
    if (!excl || !excl[n]) count[bins[n]] += 1;
  int32_t kstar = 0, q = 0;
  for (int32_t k = 1; k <= ng; ++k) {
    if (q + count[ng - k] > np) break;
    q += count[ng - k];
    kstar = k;
  }
  int32_t fill_bin = ng - kstar - 1;
  int32_t need = np - q;
  uint8_t *take = (uint8_t *)calloc((size_t)N, 1);
  for (int32_t n = 0; n < N; ++n)
    if (bins[n] >= ng - kstar && (!excl || !excl[n])) take[n] = 1;
  /* repeatedly take the fill-group member with the smallest (key, index) not yet taken */
  for (int32_t r = 0; r < need && fill_bin >= 0; ++r) {
    int32_t best = -1;
    for (int32_t n = 0; n < N; ++n) {
      if (bins[n] != fill_bin || take[n] || (excl && excl[n])) continue;
      if (best < 0) { best = n; continue; }
      if (keys && keys[n] < keys[best]) best = n;
    }
    if (best < 0) break;
    take[best] = 1;
  }
  int32_t out = 0;
  for (int32_t n = 0; n < N; ++n)
    if (take[n]) sel[out++] = n;
  free(take);
  free(count);
  return out;
}

int32_t oc_alg4_select_keyed(int32_t N, const int32_t *bins, int32_t ng, int32_t np,
                             const uint64_t *keys, int32_t *sel) {
  return oc_alg4_select_excl(N, bins, ng, np, keys, NULL, sel);
}

/* fills sel[] (ascending VN order) and returns |P| (lowest-index fill) */
int32_t oc_alg4_select(int32_t N, const int32_t *bins, int32_t ng, int32_t np, int32_t *sel) {
  return oc_alg4_select_keyed(N, bins, ng, np, NULL, sel);
}

/* One multi-edge step (Algorithm 5; Algorithm 6 when succ != NULL).  succ[0..*nsucc) holds the
   previous step's proposals P' on entry (empty at the first step) and this step's on return. */
static void me_step(st_t *S, int64_t *cnt, int32_t *trace_out, int64_t *t, int32_t frame, int32_t *succ,
                    int32_t *nsucc) {
  const oc_code *H = S->H;
  int32_t N = H->N, ng = S->s->n_g, np = S->s->n_p;
  int32_t *bins = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  int32_t *sel = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  int32_t *edge = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  uint8_t *touched = (uint8_t *)calloc((size_t)H->M, 1);
  uint8_t *vtouch = (uint8_t *)calloc((size_t)N, 1);
  uint64_t *keys = NULL;
  for (int32_t n = 0; n < N; ++n) bins[n] = bin_of(S, S->D[n], ng);
  if (S->s->fill == 1) {
    keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    for (int32_t n = 0; n < N; ++n)
      keys[n] = oc_fill_key(S->s->seed, (uint64_t)frame, (uint64_t)cnt[CNT_STEPS], (uint64_t)n);
  }
  int32_t P;
  if (!succ) {
    P = oc_alg4_select_keyed(N, bins, ng, np, keys, sel);
  } else {
    /* P' first, then Algorithm 4 for the rest among the VNs outside P'; ascending VN order */
    uint8_t *excl = (uint8_t *)calloc((size_t)N, 1);
    for (int32_t k = 0; k < *nsucc; ++k) excl[succ[k]] = 1;
    int32_t need = np - *nsucc;
    int32_t extra = need > 0 ? oc_alg4_select_excl(N, bins, ng, need, keys, excl, sel) : 0;
    for (int32_t k = 0; k < extra; ++k) excl[sel[k]] = 1;
    P = 0;
    for (int32_t n = 0; n < N; ++n)
      if (excl[n]) sel[P++] = n;
    free(excl);
  }
  free(keys);
  /* edge choice for every selected VN on the snapshot */
  for (int32_t p = 0; p < P; ++p) edge[p] = argmax_into(S, sel[p], cnt);
  /* apply all propagations (precomputed values of the snapshot) */
  for (int32_t p = 0; p < P; ++p) S->c2v[edge[p]] = S->pre[edge[p]];
  for (int32_t p = 0; p < P; ++p) S->L[sel[p]] = total_llr(S, sel[p]);
  for (int32_t p = 0; p < P; ++p) {
    int32_t n = sel[p];
    for (int32_t k = H->col_ptr[n]; k < H->col_ptr[n + 1]; ++k) touched[H->col_row[k]] = 1;
    trace_out[p] = edge[p];
  }
  /* recompute every touched check from the new state */
  for (int32_t m = 0; m < H->M; ++m) {
    if (!touched[m]) continue;
    recompute_row(S, m);
    for (int32_t e = H->row_ptr[m]; e < H->row_ptr[m + 1]; ++e) vtouch[H->col[e]] = 1;
  }
  for (int32_t p = 0; p < P; ++p) vtouch[sel[p]] = 1;
  for (int32_t n = 0; n < N; ++n) {
    if (!vtouch[n]) continue;
    S->Lt[n] = pre_llr(S, n);
    S->D[n] = ci(S, S->L[n], S->Lt[n]);
  }
  recompute_syndrome(S);
  if (succ) { /* Algorithm 6: each p proposes the VN of largest CI among U(m*_p, p); distinct ones */
    int32_t ns = 0;
    for (int32_t p = 0; p < P; ++p) {
      int32_t q = lmd_vn(S, edge[p], cnt);
      if (q < 0) continue;
      int dup = 0;
      for (int32_t k = 0; k < ns; ++k) dup |= succ[k] == q;
      if (!dup) succ[ns++] = q;
    }
    *nsucc = ns;
  }
  cnt[CNT_PROP] += P;
  cnt[CNT_STEPS] += 1;
  *t += P;
  free(bins); free(sel); free(edge); free(touched); free(vtouch);
}

/* ------------------------------------------------------------------------------------------ */
/* flooding and layered baselines                                                              */
/* ------------------------------------------------------------------------------------------ */
static void flooding_iteration(st_t *S) {
  const oc_code *H = S->H;
  /* all check outputs from the V2C messages of the previous iteration */
  for (int32_t m = 0; m < H->M; ++m) recompute_row(S, m);
  for (int32_t e = 0; e < H->E; ++e) S->c2v[e] = S->pre[e];
  for (int32_t n = 0; n < H->N; ++n) S->L[n] = total_llr(S, n);
}

static void layered_iteration(st_t *S) {
  const oc_code *H = S->H;
  /* rows in ascending order; a layer is a set of VN-disjoint consecutive rows, so the
     sequential order equals the layer-parallel one */
  for (int32_t m = 0; m < H->M; ++m) {
    int32_t b = H->row_ptr[m], en = H->row_ptr[m + 1];
    for (int32_t e = b; e < en; ++e) S->tmp[e - b] = S->L[H->col[e]] - S->c2v[e]; /* unsaturated */
    for (int32_t e = b; e < en; ++e) {
      int first = 1;
      double acc = 0.0;
      for (int32_t k = b; k < en; ++k) {
        if (k == e) continue;
        double v = sat(S, S->tmp[k - b]);
        acc = first ? v : check_rule(S, acc, v);
        first = 0;
      }
      S->pre[e] = acc;
    }
    for (int32_t e = b; e < en; ++e) {
      S->c2v[e] = S->pre[e];
      S->L[H->col[e]] = S->tmp[e - b] + S->c2v[e];
    }
  }
}

/* ------------------------------------------------------------------------------------------ */
/* one frame                                                                                   */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  const oc_code *H;
  const oc_sched *s;
  int32_t B;
  const double *llr;
  int64_t max_updates;
  const int32_t *replay;
  int64_t replay_len;
  uint8_t *bits;
  double *llr_out;
  int64_t *updates_used, *steps_used;
  int32_t *trace;
  int64_t *counters;
  double *dump_c2v, *dump_pre, *dump_L, *dump_Lt, *dump_D;
  int32_t nthreads, tid;
  int rc;
} job_t;

static int stop_now(const st_t *S, int64_t t, int64_t check_every) {
  if (check_every <= 0) return 0;
  if (t % check_every != 0) return 0;
  return S->unsat == 0;
}

static int decode_frame(job_t *J, st_t *S, int32_t f) {
  const oc_code *H = J->H;
  const oc_sched *s = J->s;
  int64_t cnt[OC_NCOUNT];
  memset(cnt, 0, sizeof(cnt));
  const double *llr = J->llr + (size_t)f * H->N;
  double scale = ldexp(1.0, s->frac_bits);
  for (int32_t n = 0; n < H->N; ++n)
    S->ch[n] = S->arith == ARITH_SPA ? llr[n] : sat(S, round_half_away(llr[n] * scale));
  int32_t *tr = J->trace ? J->trace + (size_t)f * (size_t)J->max_updates : NULL;
  int64_t t = 0;
  int kind = s->kind;
  int rc = OC_OK;
  int32_t *succ = NULL; /* ME-LMD-CIRBP: the proposals P' of the last step */
  if (kind == OC_FLOODING || kind == OC_LAYERED) {
    for (int32_t e = 0; e < H->E; ++e) S->c2v[e] = 0.0;
    for (int32_t n = 0; n < H->N; ++n) S->L[n] = S->ch[n];
    recompute_syndrome(S);
    while (!(S->unsat == 0 && s->check_every > 0) && t + H->E <= J->max_updates) {
      if (kind == OC_FLOODING) flooding_iteration(S);
      else layered_iteration(S);
      recompute_syndrome(S);
      t += H->E;
      cnt[CNT_PROP] += H->E;
      cnt[CNT_STEPS] += 1;
    }
  } else {
    init_dynamic(S);
    if (s->selfcheck && (rc = selfcheck(S)) != OC_OK) goto done;
    int64_t limit = J->max_updates;
    if (kind == OC_REPLAY && J->replay_len < limit) limit = J->replay_len;
    int64_t ce = kind == OC_REPLAY ? 0 : s->check_every;
    int lmd = kind == OC_LMDRBP || kind == OC_SLMDRBP || kind == OC_LMDCIRBP;
    int32_t next_e = -1; /* LMD schedules: the edge chosen by the last update */
    int32_t nsucc = 0;
    if (kind == OC_MELMDCIRBP) succ = (int32_t *)malloc(sizeof(int32_t) * (size_t)s->n_p);
    if (!stop_now(S, 0, ce)) {
      while (t < limit) {
        int64_t tprev = t;
        if (kind == OC_MECIRBP || kind == OC_MELMDCIRBP) {
          /* whole steps only: a step may propagate up to n_p messages */
          if (t + s->n_p > limit) break;
          int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)H->N);
          me_step(S, cnt, buf, &t, f, kind == OC_MELMDCIRBP ? succ : NULL, &nsucc);
          for (int64_t k = tprev; k < t; ++k)
            if (tr) tr[k] = buf[k - tprev];
          free(buf);
          if (t == tprev) break; /* an empty set (not reachable with N >= 1) would never end */
        } else {
          int32_t estar;
          if (kind == OC_RBP) estar = argmax_residual(S, cnt);
          else if (kind == OC_CIRBP) estar = select_cirbp(S, cnt);
          else if (lmd && next_e >= 0) estar = next_e;
          else if (kind == OC_LMDRBP || kind == OC_SLMDRBP) estar = argmax_residual(S, cnt);
          else if (kind == OC_LMDCIRBP) estar = argmax_into(S, argmax_ci(S, cnt), cnt);
          else {
            /* replay: an edge id outside [0, E) ends the frame's recorded order */
            estar = J->replay[(size_t)f * (size_t)J->replay_len + (size_t)t];
            if (estar < 0 || estar >= H->E) break;
          }
          apply_edge(S, estar, cnt);
          if (kind == OC_SLMDRBP) {
            next_e = lmd_edge(S, estar, cnt);
          } else if (kind == OC_LMDRBP) {
            int32_t e2 = lmd_edge(S, estar, cnt);
            next_e = e2 < 0 ? -1 : argmax_into(S, H->col[e2], cnt);
          } else if (kind == OC_LMDCIRBP) {
            int32_t n2 = lmd_vn(S, estar, cnt);
            next_e = n2 < 0 ? -1 : argmax_into(S, n2, cnt);
          }
          cnt[CNT_STEPS] += 1;
          if (tr) tr[t] = estar;
          t += 1;
        }
        if (s->selfcheck && (rc = selfcheck(S)) != OC_OK) goto done;
        /* syndrome test whenever t passes a multiple of check_every */
        if (ce > 0 && t / ce != tprev / ce && S->unsat == 0) break;
      }
    }
  }
done:
  free(succ);
  for (int32_t n = 0; n < H->N; ++n) {
    J->bits[(size_t)f * H->N + n] = (uint8_t)bsgn(S->L[n]);
    if (J->llr_out) J->llr_out[(size_t)f * H->N + n] = S->arith == ARITH_SPA ? S->L[n] : S->L[n] / scale;
  }
  J->updates_used[f] = t;
  if (J->steps_used) J->steps_used[f] = cnt[CNT_STEPS];
  if (J->counters) memcpy(J->counters + (size_t)f * OC_NCOUNT, cnt, sizeof(cnt));
  if (J->dump_c2v) memcpy(J->dump_c2v + (size_t)f * H->E, S->c2v, sizeof(double) * (size_t)H->E);
  if (J->dump_pre) memcpy(J->dump_pre + (size_t)f * H->E, S->pre, sizeof(double) * (size_t)H->E);
  if (J->dump_L) memcpy(J->dump_L + (size_t)f * H->N, S->L, sizeof(double) * (size_t)H->N);
  if (J->dump_Lt) memcpy(J->dump_Lt + (size_t)f * H->N, S->Lt, sizeof(double) * (size_t)H->N);
  if (J->dump_D) memcpy(J->dump_D + (size_t)f * H->N, S->D, sizeof(double) * (size_t)H->N);
  return rc;
}

static void *worker(void *arg) {
  job_t *J = (job_t *)arg;
  const oc_code *H = J->H;
  st_t S;
  memset(&S, 0, sizeof(S));
  S.H = H;
  S.s = J->s;
  S.arith = J->s->arith;
  S.qmax = ldexp(1.0, J->s->q_bits - 1) - 1.0;
  for (int x = -128; x <= 128; ++x)
    S.lut[x + 128] = round_half_away(32767.0 * tanh(0.5 * ldexp((double)x, -J->s->frac_bits)));
  S.gamma_eff = S.arith == ARITH_SPA ? J->s->gamma : round_half_away(J->s->gamma * 65534.0);
  int32_t maxdc = 1;
  for (int32_t m = 0; m < H->M; ++m)
    if (H->row_ptr[m + 1] - H->row_ptr[m] > maxdc) maxdc = H->row_ptr[m + 1] - H->row_ptr[m];
  S.ch = (double *)malloc(sizeof(double) * (size_t)H->N);
  S.L = (double *)malloc(sizeof(double) * (size_t)H->N);
  S.Lt = (double *)calloc((size_t)H->N, sizeof(double));
  S.D = (double *)calloc((size_t)H->N, sizeof(double));
  S.c2v = (double *)malloc(sizeof(double) * (size_t)H->E);
  S.pre = (double *)calloc((size_t)H->E, sizeof(double));
  S.tmp = (double *)malloc(sizeof(double) * (size_t)maxdc);
  S.syn = (uint8_t *)malloc((size_t)H->M);
  S.row_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)H->E);
  if (!S.ch || !S.L || !S.Lt || !S.D || !S.c2v || !S.pre || !S.tmp || !S.syn || !S.row_of) {
    J->rc = OC_ENOMEM;
  } else {
    for (int32_t m = 0; m < H->M; ++m)
      for (int32_t e = H->row_ptr[m]; e < H->row_ptr[m + 1]; ++e) S.row_of[e] = m;
    for (int32_t f = J->tid; f < J->B; f += J->nthreads) {
      int rc = decode_frame(J, &S, f);
      if (rc != OC_OK) J->rc = rc;
    }
  }
  free(S.ch); free(S.L); free(S.Lt); free(S.D); free(S.c2v); free(S.pre); free(S.tmp);
  free(S.syn); free(S.row_of);
  return NULL;
}

/* Decode B frames.  llr is B x N (channel LLRs 2y/sigma^2), outputs are B x N / B.
   trace (nullable) is B x max_updates; replay (kind == OC_REPLAY) is B x replay_len;
   counters (nullable) is B x OC_NCOUNT; dumps (nullable) are B x E or B x N. */
int oc_decode(const oc_code *H, const oc_sched *s, int32_t B, const double *llr, int64_t max_updates,
              const int32_t *replay, int64_t replay_len, uint8_t *bits, double *llr_out,
              int64_t *updates_used, int64_t *steps_used, int32_t *trace, int64_t *counters,
              double *dump_c2v, double *dump_pre, double *dump_L, double *dump_Lt, double *dump_D,
              int32_t nthreads) {
  if (!H || !s || B < 0 || !llr || !bits || !updates_used || max_updates < 0) return OC_EINVAL;
  if (s->kind < 0 || s->kind > OC_MELMDCIRBP || (s->arith != ARITH_SPA && s->arith != ARITH_MSFIX))
    return OC_EINVAL;
  if (s->kind == OC_REPLAY && (!replay || replay_len < 0)) return OC_EINVAL;
  if ((s->kind == OC_MECIRBP || s->kind == OC_MELMDCIRBP) && (s->n_p < 1 || s->n_g < 1)) return OC_EINVAL;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > B && B > 0) nthreads = B;
  job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return OC_ENOMEM; }
  for (int32_t i = 0; i < nthreads; ++i) {
    job_t J = {H, s, B, llr, max_updates, replay, replay_len, bits, llr_out, updates_used, steps_used,
               trace, counters, dump_c2v, dump_pre, dump_L, dump_Lt, dump_D, nthreads, i, OC_OK};
    jobs[i] = J;
  }
  for (int32_t i = 1; i < nthreads; ++i) pthread_create(&th[i], NULL, worker, &jobs[i]);
  worker(&jobs[0]);
  int rc = jobs[0].rc;
  for (int32_t i = 1; i < nthreads; ++i) {
    pthread_join(th[i], NULL);
    if (jobs[i].rc != OC_OK) rc = jobs[i].rc;
  }
  free(jobs);
  free(th);
  return rc;
}
