/*
 * unrolled_oracle.c -- plain FP64 oracle for the damped replay of a recorded single-edge schedule
 * and its exact gradient (reverse mode).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  It shares no code, header, table or constant generator with the
 * GPU library.
 *
 * The paper has no damping and no learning; this is the differentiable form of its single-edge
 * update (Sec. II-A, steps 3-4, which Algorithm 1 repeats with its own selection).  A schedule is
 * a recorded list of edges, held fixed.  State: c2v[E] and L[N], starting from c2v = 0 and
 * L = channel LLRs.  Step t applies edge e = trace[t] (check m, VN n):
 *
 *     p      = pre_e, the C2V rule of eq. (2) over V2C_{k->m} = L_k - c2v_{m->k}, k in N(m)\{n}
 *     delta  = w_e (p - c2v_e)
 *     c2v_e += delta,   L_n += delta
 *
 * With w_e = 1 this is the propagation c2v_e <- pre_e with L_n moved by the same difference, so
 * the replayed totals equal those of the undamped decoder.  pre_e is evaluated from its definition
 * at every step (the undamped decoder keeps it up to date incrementally; both give the same value).
 * The pairwise rule is the Jacobian-logarithm form of a [+] b, folded over N(m)\{n} in ascending
 * VN order, as in the main oracle.
 *
 * Gradient.  For a loss whose gradient with respect to the final L is gL, reverse mode walks the
 * steps backwards with adjoints Lh (for L) and ch (for c2v), starting from Lh = gL, ch = 0:
 *     s      = ch_e + Lh_n                (adjoint of delta)
 *     gw_e  += s (p - c2v_e)              (c2v_e taken before the step)
 *     ch_e  -= w_e s                      (c2v_e enters delta with weight -w_e)
 *     for k in N(m)\{n}:  g = dp/dv_k;  Lh_k += w_e s g;  ch_{m->k} -= w_e s g
 * and finally d loss / d llr = Lh.  The partial derivative of the pairwise rule is
 *     d(a [+] b)/da = (1 - tanh^2(a/2)) tanh(b/2) / (1 - tanh^2((a [+] b)/2)),
 * applied with a = v_k and b = the rule over the remaining inputs N(m)\{n, k} (b = +inf, i.e.
 * tanh(b/2) = 1, when that set is empty), in a form that avoids the 1 - tanh^2 cancellation.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t M, N, E;
  const int32_t *row_ptr, *col;
  const int32_t *col_ptr, *col_row, *col_eid;
  int32_t n_layers;
  const int32_t *layer_ptr;
} ou_code;

enum { OU_OK = 0, OU_EINVAL = -1, OU_ENOMEM = -2 };

static double sgn_pos(double x) { return x < 0.0 ? -1.0 : 1.0; }

/* a [+] b, Jacobian-logarithm form of eq. (2) for two inputs */
static double boxplus(double a, double b) {
  double aa = fabs(a), ab = fabs(b);
  double mag = fmin(aa, ab) + log1p(exp(-(aa + ab))) - log1p(exp(-fabs(aa - ab)));
  return sgn_pos(a) * sgn_pos(b) * mag;
}

/* d(a [+] b)/da with b = +inf allowed (then the rule is the identity and the derivative 1).
   1 - tanh^2(x/2) = 4 e^-|x| / (1 + e^-|x|)^2, so the ratio of the two such factors is
   e^-(|a| - |p|) ((1 + e^-|p|) / (1 + e^-|a|))^2, with |p| <= |a|. */
double ou_boxplus_grad(double a, double b) {
  if (isinf(b)) return 1.0;
  double p = boxplus(a, b);
  double aa = fabs(a), ap = fabs(p);
  double r = (1.0 + exp(-ap)) / (1.0 + exp(-aa));
  return tanh(0.5 * b) * exp(-(aa - ap)) * r * r;
}

/* rule over the inputs v[0..d) leaving out positions x1 and x2 (pass -1 to keep all);
   returns +inf for an empty set */
static double fold_except(const double *v, int d, int x1, int x2) {
  int first = 1;
  double acc = INFINITY;
  for (int k = 0; k < d; ++k) {
    if (k == x1 || k == x2) continue;
    acc = first ? v[k] : boxplus(acc, v[k]);
    first = 0;
  }
  return acc;
}

typedef struct {
  const ou_code *H;
  int32_t B, T;
  const double *llr, *w;
  const int32_t *trace;
  const double *gL;           /* backward only */
  double *L_out, *c2v_out;    /* forward */
  double *g_llr, *g_w;        /* backward: g_w is B x E (per frame) */
  int32_t nthreads, tid, rc;
} ou_job;

static int32_t *row_of_edges(const ou_code *H) {
  int32_t *r = (int32_t *)malloc(sizeof(int32_t) * (size_t)(H->E > 0 ? H->E : 1));
  if (!r) return NULL;
  for (int32_t m = 0; m < H->M; ++m)
    for (int32_t e = H->row_ptr[m]; e < H->row_ptr[m + 1]; ++e) r[e] = m;
  return r;
}

static int32_t max_row_degree(const ou_code *H) {
  int32_t d = 1;
  for (int32_t m = 0; m < H->M; ++m) {
    int32_t x = H->row_ptr[m + 1] - H->row_ptr[m];
    if (x > d) d = x;
  }
  return d;
}

/* one frame forward; if tape is non-NULL it receives, per step, the inputs v_k of the row
   (dc entries, position of n holds 0), p and c2v_e before the step */
static void frame_forward(const ou_code *H, const int32_t *row_of, const double *llr, const double *w,
                          const int32_t *tr, int32_t T, double *c2v, double *L, double *v, int32_t dmax,
                          double *tape_v, double *tape_p, double *tape_c) {
  for (int32_t e = 0; e < H->E; ++e) c2v[e] = 0.0;
  for (int32_t n = 0; n < H->N; ++n) L[n] = llr[n];
  for (int32_t t = 0; t < T; ++t) {
    const int32_t e = tr[t], m = row_of[e], n = H->col[e];
    const int32_t rs = H->row_ptr[m], d = H->row_ptr[m + 1] - rs;
    for (int32_t k = 0; k < d; ++k) v[k] = (rs + k == e) ? 0.0 : L[H->col[rs + k]] - c2v[rs + k];
    const double p = fold_except(v, d, e - rs, -1);
    if (tape_v) {
      memcpy(tape_v + (size_t)t * dmax, v, sizeof(double) * (size_t)d);
      tape_p[t] = p;
      tape_c[t] = c2v[e];
    }
    const double delta = w[e] * (p - c2v[e]);
    c2v[e] += delta;
    L[n] += delta;
  }
}

static int valid_trace(const ou_code *H, const int32_t *tr, int64_t len) {
  for (int64_t t = 0; t < len; ++t)
    if (tr[t] < 0 || tr[t] >= H->E) return 0;
  return 1;
}

static void *fwd_worker(void *arg) {
  ou_job *J = (ou_job *)arg;
  const ou_code *H = J->H;
  int32_t dmax = max_row_degree(H);
  int32_t *row_of = row_of_edges(H);
  double *c2v = (double *)malloc(sizeof(double) * (size_t)(H->E + 1));
  double *L = (double *)malloc(sizeof(double) * (size_t)(H->N + 1));
  double *v = (double *)malloc(sizeof(double) * (size_t)dmax);
  if (!row_of || !c2v || !L || !v) {
    J->rc = OU_ENOMEM;
  } else {
    for (int32_t f = J->tid; f < J->B; f += J->nthreads) {
      frame_forward(H, row_of, J->llr + (size_t)f * H->N, J->w, J->trace + (size_t)f * J->T, J->T, c2v, L, v,
                    dmax, NULL, NULL, NULL);
      memcpy(J->L_out + (size_t)f * H->N, L, sizeof(double) * (size_t)H->N);
      if (J->c2v_out) memcpy(J->c2v_out + (size_t)f * H->E, c2v, sizeof(double) * (size_t)H->E);
    }
  }
  free(row_of); free(c2v); free(L); free(v);
  return NULL;
}

static void *bwd_worker(void *arg) {
  ou_job *J = (ou_job *)arg;
  const ou_code *H = J->H;
  const int32_t T = J->T;
  int32_t dmax = max_row_degree(H);
  int32_t *row_of = row_of_edges(H);
  double *c2v = (double *)malloc(sizeof(double) * (size_t)(H->E + 1));
  double *L = (double *)malloc(sizeof(double) * (size_t)(H->N + 1));
  double *v = (double *)malloc(sizeof(double) * (size_t)dmax);
  double *tv = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * (size_t)dmax);
  double *tp = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
  double *tc = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
  double *Lh = (double *)malloc(sizeof(double) * (size_t)(H->N + 1));
  double *ch = (double *)malloc(sizeof(double) * (size_t)(H->E + 1));
  if (!row_of || !c2v || !L || !v || !tv || !tp || !tc || !Lh || !ch) {
    J->rc = OU_ENOMEM;
  } else {
    for (int32_t f = J->tid; f < J->B; f += J->nthreads) {
      const int32_t *tr = J->trace + (size_t)f * T;
      const double *w = J->w;
      double *gw = J->g_w + (size_t)f * H->E;
      frame_forward(H, row_of, J->llr + (size_t)f * H->N, w, tr, T, c2v, L, v, dmax, tv, tp, tc);
      memcpy(Lh, J->gL + (size_t)f * H->N, sizeof(double) * (size_t)H->N);
      for (int32_t e = 0; e < H->E; ++e) { ch[e] = 0.0; gw[e] = 0.0; }
      for (int32_t t = T - 1; t >= 0; --t) {
        const int32_t e = tr[t], m = row_of[e], n = H->col[e];
        const int32_t rs = H->row_ptr[m], d = H->row_ptr[m + 1] - rs, x = e - rs;
        const double *vt = tv + (size_t)t * dmax;
        const double s = ch[e] + Lh[n];
        gw[e] += s * (tp[t] - tc[t]);
        ch[e] -= w[e] * s;
        const double ps = w[e] * s;
        for (int32_t k = 0; k < d; ++k) {
          if (k == x) continue;
          const double g = ou_boxplus_grad(vt[k], fold_except(vt, d, x, k));
          Lh[H->col[rs + k]] += ps * g;
          ch[rs + k] -= ps * g;
        }
      }
      memcpy(J->g_llr + (size_t)f * H->N, Lh, sizeof(double) * (size_t)H->N);
    }
  }
  free(row_of); free(c2v); free(L); free(v); free(tv); free(tp); free(tc); free(Lh); free(ch);
  return NULL;
}

static int run_jobs(ou_job *proto, int32_t nthreads, void *(*fn)(void *)) {
  if (nthreads < 1) nthreads = 1;
  if (proto->B > 0 && nthreads > proto->B) nthreads = proto->B;
  ou_job *jobs = (ou_job *)calloc((size_t)nthreads, sizeof(ou_job));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return OU_ENOMEM; }
  for (int32_t i = 0; i < nthreads; ++i) {
    jobs[i] = *proto;
    jobs[i].nthreads = nthreads;
    jobs[i].tid = i;
    jobs[i].rc = OU_OK;
  }
  for (int32_t i = 1; i < nthreads; ++i) pthread_create(&th[i], NULL, fn, &jobs[i]);
  fn(&jobs[0]);
  int rc = jobs[0].rc;
  for (int32_t i = 1; i < nthreads; ++i) {
    pthread_join(th[i], NULL);
    if (jobs[i].rc != OU_OK) rc = jobs[i].rc;
  }
  free(jobs);
  free(th);
  return rc;
}

/* Damped replay forward of B frames: llr B x N, w [E], trace B x T (edge ids).
   Outputs L_out B x N and (nullable) c2v_out B x E. */
int ou_forward(const ou_code *H, int32_t B, const double *llr, const double *w, const int32_t *trace, int32_t T,
               double *L_out, double *c2v_out, int32_t nthreads) {
  if (!H || B < 0 || T < 0 || !llr || !w || (T > 0 && !trace) || !L_out) return OU_EINVAL;
  if (!valid_trace(H, trace, (int64_t)B * T)) return OU_EINVAL;
  ou_job J;
  memset(&J, 0, sizeof(J));
  J.H = H; J.B = B; J.T = T; J.llr = llr; J.w = w; J.trace = trace; J.L_out = L_out; J.c2v_out = c2v_out;
  return run_jobs(&J, nthreads, fwd_worker);
}

/* Gradient of a loss with d loss / d L_final = gL (B x N): g_llr B x N and the per-frame
   weight gradients g_w B x E (the total is their sum over frames). */
int ou_backward(const ou_code *H, int32_t B, const double *llr, const double *w, const int32_t *trace, int32_t T,
                const double *gL, double *g_llr, double *g_w, int32_t nthreads) {
  if (!H || B < 0 || T < 0 || !llr || !w || (T > 0 && !trace) || !gL || !g_llr || !g_w) return OU_EINVAL;
  if (!valid_trace(H, trace, (int64_t)B * T)) return OU_EINVAL;
  ou_job J;
  memset(&J, 0, sizeof(J));
  J.H = H; J.B = B; J.T = T; J.llr = llr; J.w = w; J.trace = trace; J.gL = gL; J.g_llr = g_llr; J.g_w = g_w;
  return run_jobs(&J, nthreads, bwd_worker);
}
