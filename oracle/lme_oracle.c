/*
 * lme_oracle.c -- plain, slow, obviously correct FP64 oracle for the Lindblad
 * master equation.  TEST INFRASTRUCTURE ONLY (see lme_oracle.h): the GPU
 * library never links, loads or calls this file.
 *
 * Everything is written as the textbook definition with sparse-times-dense
 * products in fixed loop order.  Deliberately no folding of the Hamiltonian and
 * the anticommutator into one non-Hermitian operator, no Hermitian shortcuts,
 * no blocking, no fusion.
 *
 * Paper references (arXiv:1110.0573):
 *   Sec. 3.1, Eq. (master_equation): the right-hand side
 *       drho/dt = -i[H(t), rho] + sum_n ( C_n rho C_n^+ - 1/2 rho C_n^+ C_n
 *                                                    - 1/2 C_n^+ C_n rho ).
 *   Sec. 4.4 (Landau-Zener): a time-dependent Hamiltonian given as constant
 *       operators times scalar functions of time; here H0 + sum_j u_j(t) H_j
 *       with u_j piecewise constant.
 *   Sec. 4 (odesolve): expectation values Tr(E rho) at each output time,
 *       the first output time being the initial time.
 * The paper names no integrator; classic RK4 (fixed step) and the
 * Dormand-Prince 5(4) pair (adaptive) are used, with the error norm, step
 * controller and starting-step rule written out below.
 */
#include "lme_oracle.h"

#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* Sparse (CSR) x dense primitives on n x n row-major matrices.               */
/* Every routine accumulates: out += alpha * (product).                       */
/* ------------------------------------------------------------------------- */

static const cplx *cval(const orc_csr *m) { return (const cplx *)m->val; }

/* out += alpha * M Y,  (M Y)_ij = sum_l M_il Y_lj */
static void mul_csr_dense(int n, const orc_csr *M, const cplx *Y, cplx alpha,
                          cplx *out) {
  const cplx *mv = cval(M);
  for (int i = 0; i < n; ++i)
    for (int p = M->row_ptr[i]; p < M->row_ptr[i + 1]; ++p) {
      const int l = M->col[p];
      const cplx a = alpha * mv[p];
      for (int j = 0; j < n; ++j) out[(size_t)i * n + j] += a * Y[(size_t)l * n + j];
    }
}

/* out += alpha * M^+ Y,  (M^+ Y)_ij = sum_l conj(M_li) Y_lj */
static void mul_csrdag_dense(int n, const orc_csr *M, const cplx *Y, cplx alpha,
                             cplx *out) {
  const cplx *mv = cval(M);
  for (int l = 0; l < n; ++l)
    for (int p = M->row_ptr[l]; p < M->row_ptr[l + 1]; ++p) {
      const int i = M->col[p];
      const cplx a = alpha * conj(mv[p]);
      for (int j = 0; j < n; ++j) out[(size_t)i * n + j] += a * Y[(size_t)l * n + j];
    }
}

/* out += alpha * Y M,  (Y M)_ij = sum_l Y_il M_lj */
static void mul_dense_csr(int n, const cplx *Y, const orc_csr *M, cplx alpha,
                          cplx *out) {
  const cplx *mv = cval(M);
  for (int l = 0; l < n; ++l)
    for (int p = M->row_ptr[l]; p < M->row_ptr[l + 1]; ++p) {
      const int j = M->col[p];
      const cplx a = alpha * mv[p];
      for (int i = 0; i < n; ++i) out[(size_t)i * n + j] += a * Y[(size_t)i * n + l];
    }
}

/* out += alpha * Y M^+,  (Y M^+)_ij = sum_l Y_il conj(M_jl) */
static void mul_dense_csrdag(int n, const cplx *Y, const orc_csr *M, cplx alpha,
                             cplx *out) {
  const cplx *mv = cval(M);
  for (int j = 0; j < n; ++j)
    for (int p = M->row_ptr[j]; p < M->row_ptr[j + 1]; ++p) {
      const int l = M->col[p];
      const cplx a = alpha * conj(mv[p]);
      for (int i = 0; i < n; ++i) out[(size_t)i * n + j] += a * Y[(size_t)i * n + l];
    }
}

/* ------------------------------------------------------------------------- */
/* Validation                                                                 */
/* ------------------------------------------------------------------------- */

static int check_csr(const orc_csr *m, int n) {
  if (m->n != n || m->nnz < 0 || !m->row_ptr) return ORC_EINVAL;
  if (m->nnz > 0 && (!m->col || !m->val)) return ORC_EINVAL;
  if (m->row_ptr[0] != 0 || m->row_ptr[n] != m->nnz) return ORC_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (m->row_ptr[i + 1] < m->row_ptr[i]) return ORC_EINVAL;
    for (int p = m->row_ptr[i]; p < m->row_ptr[i + 1]; ++p)
      if (m->col[p] < 0 || m->col[p] >= n) return ORC_EINVAL;
  }
  return ORC_OK;
}

static int check_system(const orc_system *s) {
  if (!s || s->n < 1) return ORC_EINVAL;
  int rc = check_csr(&s->H0, s->n);
  if (rc) return rc;
  if (s->n_ctrl < 0 || s->n_c < 0 || s->n_e < 0 || s->n_seg < 0) return ORC_EINVAL;
  for (int j = 0; j < s->n_ctrl; ++j)
    if ((rc = check_csr(&s->Hc[j], s->n))) return rc;
  for (int k = 0; k < s->n_c; ++k)
    if ((rc = check_csr(&s->C[k], s->n))) return rc;
  for (int m = 0; m < s->n_e; ++m)
    if ((rc = check_csr(&s->E[m], s->n))) return rc;
  if (s->fn) {
    if (s->n_ctrl < 1) return ORC_EINVAL;
    for (int i = 0; i < 7 * s->n_ctrl; ++i)
      if (!isfinite(s->fn[i])) return ORC_EINVAL;
  } else if (s->n_seg > 0) {
    if (!s->edges || (s->n_ctrl > 0 && !s->u)) return ORC_EINVAL;
    for (int q = 0; q < s->n_seg; ++q)
      if (!(s->edges[q + 1] > s->edges[q])) return ORC_EINVAL;
  }
  return ORC_OK;
}

/* Amplitudes of the control Hamiltonians at time t: the value of the segment
 * [edges[q], edges[q+1]) containing t, zero outside all segments.  Returns q,
 * or -1 when t lies outside. */
static int controls_at(const orc_system *s, double t, double *uval) {
  if (s->fn) {
    /* closed-form amplitudes: c0 + c1 t + c2 t^2 + c3 t^3 + a cos(w t + phi) */
    for (int j = 0; j < s->n_ctrl; ++j) {
      const double *c = s->fn + 7 * (size_t)j;
      uval[j] = c[0] + c[1] * t + c[2] * t * t + c[3] * t * t * t + c[4] * cos(c[5] * t + c[6]);
    }
    return 0;
  }
  int q = -1;
  if (s->n_seg > 0 && t >= s->edges[0] && t < s->edges[s->n_seg])
    for (q = 0; q < s->n_seg - 1; ++q)
      if (t < s->edges[q + 1]) break;
  for (int j = 0; j < s->n_ctrl; ++j)
    uval[j] = (q >= 0) ? s->u[(size_t)j * s->n_seg + q] : 0.0;
  return q;
}

/* ------------------------------------------------------------------------- */
/* The Lindblad right-hand side and its Hilbert-Schmidt adjoint               */
/* ------------------------------------------------------------------------- */

typedef struct {
  cplx *Z, *W; /* n*n scratch */
} work_t;

static int work_init(work_t *w, int n) {
  const size_t n2 = (size_t)n * n;
  w->Z = (cplx *)malloc(n2 * sizeof(cplx));
  w->W = (cplx *)malloc(n2 * sizeof(cplx));
  if (!w->Z || !w->W) {
    free(w->Z);
    free(w->W);
    return ORC_ENOMEM;
  }
  return ORC_OK;
}
static void work_free(work_t *w) {
  free(w->Z);
  free(w->W);
}

/* out = -i[H, y] + sum_k ( C_k y C_k^+ - 1/2 C_k^+ C_k y - 1/2 y C_k^+ C_k ),
 * H = H0 + sum_j uval[j] H_j.   (Eq. (master_equation), hbar = 1.) */
static void lindblad(const orc_system *s, const double *uval, const cplx *y,
                     cplx *out, work_t *w) {
  const int n = s->n;
  const size_t n2 = (size_t)n * n;
  memset(out, 0, n2 * sizeof(cplx));
  /* -i H y + i y H */
  mul_csr_dense(n, &s->H0, y, -I, out);
  mul_dense_csr(n, y, &s->H0, I, out);
  for (int j = 0; j < s->n_ctrl; ++j) {
    if (uval[j] == 0.0) continue;
    mul_csr_dense(n, &s->Hc[j], y, -I * uval[j], out);
    mul_dense_csr(n, y, &s->Hc[j], I * uval[j], out);
  }
  for (int k = 0; k < s->n_c; ++k) {
    const orc_csr *C = &s->C[k];
    /* Z = C y;  out += Z C^+  (= C y C^+);  out -= 1/2 C^+ Z  (= C^+ C y) */
    memset(w->Z, 0, n2 * sizeof(cplx));
    mul_csr_dense(n, C, y, 1.0, w->Z);
    mul_dense_csrdag(n, w->Z, C, 1.0, out);
    mul_csrdag_dense(n, C, w->Z, -0.5, out);
    /* W = y C^+;  out -= 1/2 W C  (= y C^+ C) */
    memset(w->W, 0, n2 * sizeof(cplx));
    mul_dense_csrdag(n, y, C, 1.0, w->W);
    mul_dense_csr(n, w->W, C, -0.5, out);
  }
}

/* out = i[H, x] + sum_k ( C_k^+ x C_k - 1/2 C_k^+ C_k x - 1/2 x C_k^+ C_k ):
 * the adjoint of lindblad() under <X, Y> = Tr(X^+ Y). */
static void lindblad_dag(const orc_system *s, const double *uval, const cplx *x,
                         cplx *out, work_t *w) {
  const int n = s->n;
  const size_t n2 = (size_t)n * n;
  memset(out, 0, n2 * sizeof(cplx));
  mul_csr_dense(n, &s->H0, x, I, out);
  mul_dense_csr(n, x, &s->H0, -I, out);
  for (int j = 0; j < s->n_ctrl; ++j) {
    if (uval[j] == 0.0) continue;
    mul_csr_dense(n, &s->Hc[j], x, I * uval[j], out);
    mul_dense_csr(n, x, &s->Hc[j], -I * uval[j], out);
  }
  for (int k = 0; k < s->n_c; ++k) {
    const orc_csr *C = &s->C[k];
    /* Z = C^+ x;  out += Z C  (= C^+ x C) */
    memset(w->Z, 0, n2 * sizeof(cplx));
    mul_csrdag_dense(n, C, x, 1.0, w->Z);
    mul_dense_csr(n, w->Z, C, 1.0, out);
    /* W = C x;  out -= 1/2 C^+ W  (= C^+ C x) */
    memset(w->W, 0, n2 * sizeof(cplx));
    mul_csr_dense(n, C, x, 1.0, w->W);
    mul_csrdag_dense(n, C, w->W, -0.5, out);
    /* W = x C^+;  out -= 1/2 W C  (= x C^+ C) */
    memset(w->W, 0, n2 * sizeof(cplx));
    mul_dense_csrdag(n, x, C, 1.0, w->W);
    mul_dense_csr(n, w->W, C, -0.5, out);
  }
}

/* Tr(E rho) = sum_i sum_l E_il rho_li */
static cplx trace_prod(int n, const orc_csr *E, const cplx *rho) {
  const cplx *ev = cval(E);
  cplx acc = 0.0;
  for (int i = 0; i < n; ++i)
    for (int p = E->row_ptr[i]; p < E->row_ptr[i + 1]; ++p)
      acc += ev[p] * rho[(size_t)E->col[p] * n + i];
  return acc;
}

static int all_finite(const cplx *a, size_t len) {
  for (size_t i = 0; i < len; ++i)
    if (!isfinite(creal(a[i])) || !isfinite(cimag(a[i]))) return 0;
  return 1;
}

/* Write the expectation values (and optionally the state) for output k. */
static void record(const orc_system *s, const cplx *rho, int32_t n_t, int32_t k,
                   double *expect, double *states) {
  const size_t n2 = (size_t)s->n * s->n;
  for (int m = 0; m < s->n_e; ++m) {
    const cplx e = trace_prod(s->n, &s->E[m], rho);
    expect[2 * ((size_t)m * n_t + k)] = creal(e);
    expect[2 * ((size_t)m * n_t + k) + 1] = cimag(e);
  }
  if (states) memcpy(states + 2 * n2 * (size_t)k, rho, n2 * sizeof(cplx));
}

/* ------------------------------------------------------------------------- */
/* Public single-application entry points                                     */
/* ------------------------------------------------------------------------- */

int orc_apply_L(const orc_system *s, double t, const double *y, double *out) {
  int rc = check_system(s);
  if (rc) return rc;
  double *uval = (double *)calloc((size_t)s->n_ctrl + 1, sizeof(double));
  work_t w;
  if (!uval || work_init(&w, s->n)) {
    free(uval);
    return ORC_ENOMEM;
  }
  controls_at(s, t, uval);
  lindblad(s, uval, (const cplx *)y, (cplx *)out, &w);
  work_free(&w);
  free(uval);
  return ORC_OK;
}

int orc_apply_Ldag(const orc_system *s, double t, const double *x, double *out) {
  int rc = check_system(s);
  if (rc) return rc;
  double *uval = (double *)calloc((size_t)s->n_ctrl + 1, sizeof(double));
  work_t w;
  if (!uval || work_init(&w, s->n)) {
    free(uval);
    return ORC_ENOMEM;
  }
  controls_at(s, t, uval);
  lindblad_dag(s, uval, (const cplx *)x, (cplx *)out, &w);
  work_free(&w);
  free(uval);
  return ORC_OK;
}

int orc_expect(const orc_system *s, const double *rho, double *out) {
  int rc = check_system(s);
  if (rc) return rc;
  for (int m = 0; m < s->n_e; ++m) {
    const cplx e = trace_prod(s->n, &s->E[m], (const cplx *)rho);
    out[2 * m] = creal(e);
    out[2 * m + 1] = cimag(e);
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Fixed-step RK4                                                             */
/* ------------------------------------------------------------------------- */

/* Index m with |t - (t0 + m h)| <= 1e-6 h, or -1 if t is not on the grid. */
static long grid_index(double t, double t0, double h) {
  const double x = (t - t0) / h;
  const long m = lround(x);
  if (fabs(t - (t0 + (double)m * h)) > 1e-6 * fabs(h)) return -1;
  return m;
}

/* Checks the output times and the control edges against the uniform grid
 * t0 + m h, m = 0..nsteps, and fills out_step[k] = m for tlist[k]. */
static int rk4_grid(const orc_system *s, int32_t n_t, const double *tlist,
                    int32_t nsteps, double h, long *out_step) {
  const double t0 = tlist[0];
  out_step[0] = 0;
  for (int k = 1; k < n_t; ++k) {
    if (!(tlist[k] > tlist[k - 1])) return ORC_EINVAL;
    const long m = grid_index(tlist[k], t0, h);
    if (m < 0 || m > nsteps) return ORC_EGRID;
    out_step[k] = m;
  }
  if (n_t > 1 && out_step[n_t - 1] != nsteps) return ORC_EGRID;
  const double t1 = tlist[n_t - 1];
  for (int q = 0; q <= s->n_seg && s->n_seg > 0 && !s->fn; ++q) {
    const double e = s->edges[q];
    if (e > t0 && e < t1 && grid_index(e, t0, h) < 0) return ORC_EGRID;
  }
  return ORC_OK;
}

/* One classic RK4 step: rho <- rho + h/6 (k1 + 2 k2 + 2 k3 + k4).  The stages
 * use the amplitudes u1 (k1), u2 (k2, k3) and u4 (k4). */
static void rk4_step3(const orc_system *s, const double *u1, const double *u2, const double *u4,
                      double h, cplx *rho, cplx *y, cplx *k, cplx *acc, work_t *w) {
  const size_t n2 = (size_t)s->n * s->n;
  lindblad(s, u1, rho, k, w); /* k1 */
  for (size_t e = 0; e < n2; ++e) {
    acc[e] = k[e];
    y[e] = rho[e] + (0.5 * h) * k[e];
  }
  lindblad(s, u2, y, k, w); /* k2 */
  for (size_t e = 0; e < n2; ++e) {
    acc[e] += 2.0 * k[e];
    y[e] = rho[e] + (0.5 * h) * k[e];
  }
  lindblad(s, u2, y, k, w); /* k3 */
  for (size_t e = 0; e < n2; ++e) {
    acc[e] += 2.0 * k[e];
    y[e] = rho[e] + h * k[e];
  }
  lindblad(s, u4, y, k, w); /* k4 */
  for (size_t e = 0; e < n2; ++e) {
    acc[e] += k[e];
    rho[e] += (h / 6.0) * acc[e];
  }
}

static void rk4_step(const orc_system *s, const double *uval, double h, cplx *rho,
                     cplx *y, cplx *k, cplx *acc, work_t *w) {
  rk4_step3(s, uval, uval, uval, h, rho, y, k, acc, w);
}

int orc_rk4(const orc_system *s, const double *rho0, int32_t n_t,
            const double *tlist, int32_t nsteps, double *expect, double *states) {
  int rc = check_system(s);
  if (rc) return rc;
  if (!rho0 || !tlist || n_t < 1 || (s->n_e > 0 && !expect)) return ORC_EINVAL;
  if (n_t > 1 && nsteps < 1) return ORC_EINVAL;
  const int n = s->n;
  const size_t n2 = (size_t)n * n;
  const double t0 = tlist[0];
  const double h = n_t > 1 ? (tlist[n_t - 1] - t0) / nsteps : 0.0;

  long *out_step = (long *)malloc(sizeof(long) * (size_t)n_t);
  cplx *buf = (cplx *)malloc(4 * n2 * sizeof(cplx));
  double *uval = (double *)calloc(3 * ((size_t)s->n_ctrl + 1), sizeof(double));
  work_t w;
  if (!out_step || !buf || !uval || work_init(&w, n)) {
    free(out_step);
    free(buf);
    free(uval);
    return ORC_ENOMEM;
  }
  double *uval2 = uval + s->n_ctrl + 1, *uval4 = uval2 + s->n_ctrl + 1;
  if (n_t > 1) rc = rk4_grid(s, n_t, tlist, nsteps, h, out_step);
  if (rc) goto done;

  cplx *rho = buf, *y = buf + n2, *k = buf + 2 * n2, *acc = buf + 3 * n2;
  memcpy(rho, rho0, n2 * sizeof(cplx));
  record(s, rho, n_t, 0, expect, states);
  int next = 1;
  for (long st = 0; st < (n_t > 1 ? nsteps : 0); ++st) {
    if (s->fn) {
      /* function amplitudes: each stage at its own time */
      const double ts = t0 + (double)st * h;
      controls_at(s, ts, uval);
      controls_at(s, ts + 0.5 * h, uval2);
      controls_at(s, ts + h, uval4);
      rk4_step3(s, uval, uval2, uval4, h, rho, y, k, acc, &w);
    } else {
      /* every stage of a step uses the controls of the segment holding the
         step's midpoint (steps never straddle an edge) */
      controls_at(s, t0 + ((double)st + 0.5) * h, uval);
      rk4_step(s, uval, h, rho, y, k, acc, &w);
    }
    while (next < n_t && out_step[next] == st + 1) {
      if (!all_finite(rho, n2)) {
        rc = ORC_ENONFINITE;
        goto done;
      }
      record(s, rho, n_t, next, expect, states);
      ++next;
    }
  }
done:
  work_free(&w);
  free(out_step);
  free(buf);
  free(uval);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Dormand-Prince 5(4)                                                         */
/* ------------------------------------------------------------------------- */

/* Dormand & Prince (1980) coefficients: stage matrix a (lower triangle),
 * fifth-order weights b (equal to the last row of a, FSAL) and fourth-order
 * embedded weights bh.  The nodes c are not needed: within one step the
 * right-hand side does not depend on time (controls are constant on a step). */
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double DP_B[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192,
                               -2187.0 / 6784, 11.0 / 84, 0};
static const double DP_BH[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

/* RMS over the n^2 complex moduli of v / sc. */
static double rms_scaled(size_t n2, const cplx *v, const double *sc) {
  double acc = 0.0;
  for (size_t e = 0; e < n2; ++e) {
    const double r = cabs(v[e]) / sc[e];
    acc += r * r;
  }
  return sqrt(acc / (double)n2);
}

/* Stages 1..7 from (y, k[0] = f(y) given); writes y5 and the error vector. */
static void dp_stages(const orc_system *s, const double *uval, double h,
                      const cplx *y, cplx *const *k, cplx *tmp, cplx *y5,
                      cplx *err, work_t *w) {
  const size_t n2 = (size_t)s->n * s->n;
  for (int i = 1; i < 7; ++i) {
    for (size_t e = 0; e < n2; ++e) {
      cplx acc = 0.0;
      for (int j = 0; j < i; ++j) acc += DP_A[i][j] * k[j][e];
      tmp[e] = y[e] + h * acc;
    }
    if (i == 6) memcpy(y5, tmp, n2 * sizeof(cplx)); /* row 7 of a is b */
    lindblad(s, uval, tmp, k[i], w);
  }
  for (size_t e = 0; e < n2; ++e) {
    cplx acc = 0.0;
    for (int j = 0; j < 7; ++j) acc += (DP_B[j] - DP_BH[j]) * k[j][e];
    err[e] = h * acc;
  }
}

int orc_dopri5_step(const orc_system *s, double t, double h, const double *y,
                    double *y5, double *err) {
  int rc = check_system(s);
  if (rc) return rc;
  if (s->fn) return ORC_EINVAL;
  const size_t n2 = (size_t)s->n * s->n;
  cplx *buf = (cplx *)malloc(8 * n2 * sizeof(cplx));
  double *uval = (double *)calloc((size_t)s->n_ctrl + 1, sizeof(double));
  work_t w;
  if (!buf || !uval || work_init(&w, s->n)) {
    free(buf);
    free(uval);
    return ORC_ENOMEM;
  }
  cplx *k[7];
  for (int i = 0; i < 7; ++i) k[i] = buf + (size_t)i * n2;
  cplx *tmp = buf + 7 * n2;
  controls_at(s, t + 0.5 * h, uval);
  lindblad(s, uval, (const cplx *)y, k[0], &w);
  dp_stages(s, uval, h, (const cplx *)y, k, tmp, (cplx *)y5, (cplx *)err, &w);
  work_free(&w);
  free(buf);
  free(uval);
  return ORC_OK;
}

static int cmp_double(const void *a, const void *b) {
  const double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

int orc_dopri5(const orc_system *s, const double *rho0, int32_t n_t,
               const double *tlist, double rtol, double atol, double h0,
               double h_min, int64_t max_steps, double *expect, double *states,
               int64_t *counts, double *h_log, int64_t h_log_cap) {
  int rc = check_system(s);
  if (rc) return rc;
  if (!rho0 || !tlist || n_t < 1 || (s->n_e > 0 && !expect) || s->fn) return ORC_EINVAL;
  if (!(rtol > 0.0) || !(atol >= 0.0) || max_steps < 1 || !(h_min >= 0.0))
    return ORC_EINVAL;
  for (int k = 1; k < n_t; ++k)
    if (!(tlist[k] > tlist[k - 1])) return ORC_EINVAL;

  const int n = s->n;
  const size_t n2 = (size_t)n * n;
  const double t0 = tlist[0], t_end = tlist[n_t - 1];
  int64_t n_acc = 0, n_rej = 0;

  /* Stop points: every output time after t0 and every control edge inside
     (t0, t_end), sorted, duplicates removed. */
  const int max_stops = n_t + s->n_seg + 1;
  double *stops = (double *)malloc(sizeof(double) * (size_t)max_stops);
  int *stop_is_out = (int *)malloc(sizeof(int) * (size_t)max_stops);
  cplx *buf = (cplx *)malloc(11 * n2 * sizeof(cplx));
  double *sc = (double *)malloc(n2 * sizeof(double));
  double *uval = (double *)calloc((size_t)s->n_ctrl + 1, sizeof(double));
  work_t w;
  if (!stops || !stop_is_out || !buf || !sc || !uval || work_init(&w, n)) {
    free(stops);
    free(stop_is_out);
    free(buf);
    free(sc);
    free(uval);
    return ORC_ENOMEM;
  }
  int n_stops = 0;
  for (int k = 1; k < n_t; ++k) stops[n_stops++] = tlist[k];
  for (int q = 0; q <= s->n_seg && s->n_seg > 0; ++q)
    if (s->edges[q] > t0 && s->edges[q] < t_end) stops[n_stops++] = s->edges[q];
  qsort(stops, (size_t)n_stops, sizeof(double), cmp_double);
  {
    int m = 0;
    for (int i = 0; i < n_stops; ++i)
      if (m == 0 || stops[i] != stops[m - 1]) stops[m++] = stops[i];
    n_stops = m;
  }
  {
    int k = 1;
    for (int i = 0; i < n_stops; ++i) {
      while (k < n_t && tlist[k] < stops[i]) ++k;
      stop_is_out[i] = (k < n_t && tlist[k] == stops[i]);
    }
  }

  cplx *rho = buf, *tmp = buf + n2, *y5 = buf + 2 * n2, *err = buf + 3 * n2;
  cplx *k[7];
  for (int i = 0; i < 7; ++i) k[i] = buf + (size_t)(4 + i) * n2;
  memcpy(rho, rho0, n2 * sizeof(cplx));
  record(s, rho, n_t, 0, expect, states);
  if (n_t == 1) goto done;

  double t = t0;
  int stop = 0, out_k = 1;
  double h;
  int k1_seg = -2; /* segment k[0] was evaluated with; -2 = not valid */

  if (h0 > 0.0) {
    h = h0;
  } else {
    /* Starting step (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4),
       in the same scaled RMS norm, exponent 1/5. */
    const int q = controls_at(s, t0 + 0.5 * (stops[0] - t0), uval);
    lindblad(s, uval, rho, k[0], &w);
    k1_seg = q;
    for (size_t e = 0; e < n2; ++e) sc[e] = atol + rtol * cabs(rho[e]);
    const double d0 = rms_scaled(n2, rho, sc);
    const double d1 = rms_scaled(n2, k[0], sc);
    double hs = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    for (size_t e = 0; e < n2; ++e) tmp[e] = rho[e] + hs * k[0][e];
    lindblad(s, uval, tmp, k[1], &w);
    for (size_t e = 0; e < n2; ++e) y5[e] = k[1][e] - k[0][e];
    const double d2 = rms_scaled(n2, y5, sc) / hs;
    const double dm = d1 > d2 ? d1 : d2;
    const double h1 = (dm <= 1e-15) ? fmax(1e-6, hs * 1e-3) : pow(0.01 / dm, 0.2);
    h = fmin(100.0 * hs, h1);
  }

  int prev_rejected = 0;
  for (;;) {
    if (n_acc + n_rej >= max_steps) {
      rc = ORC_EMAXSTEPS;
      break;
    }
    if (h < h_min) {
      rc = ORC_ESTEPUNDERFLOW;
      break;
    }
    const double t_stop = stops[stop];
    int landing = 0;
    double h_try = h;
    if (h_try >= t_stop - t) {
      h_try = t_stop - t;
      landing = 1;
    }
    const int q = controls_at(s, t + 0.5 * h_try, uval);
    if (k1_seg != q) {
      lindblad(s, uval, rho, k[0], &w);
      k1_seg = q;
    }
    dp_stages(s, uval, h_try, rho, k, tmp, y5, err, &w);
    for (size_t e = 0; e < n2; ++e) {
      const double a = cabs(rho[e]), b = cabs(y5[e]);
      sc[e] = atol + rtol * (a > b ? a : b);
    }
    const double en = rms_scaled(n2, err, sc);
    if (!isfinite(en)) {
      rc = ORC_ENONFINITE;
      break;
    }
    if (en <= 1.0) {
      if (h_log && n_acc < h_log_cap) h_log[n_acc] = h_try;
      ++n_acc;
      memcpy(rho, y5, n2 * sizeof(cplx));
      /* FSAL: the last stage is f at the new point */
      cplx *sw = k[0];
      k[0] = k[6];
      k[6] = sw;
      double fac = (en == 0.0) ? 10.0 : 0.9 * pow(en, -0.2);
      fac = fac < 0.2 ? 0.2 : (fac > 10.0 ? 10.0 : fac);
      if (prev_rejected && fac > 1.0) fac = 1.0;
      prev_rejected = 0;
      h = h_try * fac;
      if (landing) {
        t = t_stop;
        if (stop_is_out[stop]) {
          record(s, rho, n_t, out_k, expect, states);
          ++out_k;
        }
        ++stop;
        if (stop == n_stops) break;
      } else {
        t = t + h_try;
      }
    } else {
      ++n_rej;
      double fac = 0.9 * pow(en, -0.2);
      if (fac < 0.2) fac = 0.2;
      prev_rejected = 1;
      h = h_try * fac;
    }
  }
done:
  if (counts) {
    counts[0] = n_acc;
    counts[1] = n_rej;
  }
  work_free(&w);
  free(stops);
  free(stop_is_out);
  free(buf);
  free(sc);
  free(uval);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Discrete adjoint of fixed-step RK4                                          */
/* ------------------------------------------------------------------------- */

/* Re Tr(X^+ Y) = Re sum_ij conj(X_ij) Y_ij */
static double hs_real(size_t n2, const cplx *X, const cplx *Y) {
  double acc = 0.0;
  for (size_t e = 0; e < n2; ++e) acc += creal(conj(X[e]) * Y[e]);
  return acc;
}

int orc_rk4_cost_grad(const orc_system *s, const double *rho0, const double *O,
                      double t0, double t1, int32_t nsteps, double *cost,
                      double *grad) {
  int rc = check_system(s);
  if (rc) return rc;
  if (!rho0 || !O || !cost || nsteps < 1 || !(t1 > t0) || s->fn) return ORC_EINVAL;
  if (s->n_ctrl > 0 && s->n_seg > 0 && !grad) return ORC_EINVAL;
  const int n = s->n;
  const size_t n2 = (size_t)n * n;
  const double h = (t1 - t0) / nsteps;
  for (int q = 0; q <= s->n_seg && s->n_seg > 0; ++q) {
    const double e = s->edges[q];
    if (e > t0 && e < t1 && grid_index(e, t0, h) < 0) return ORC_EGRID;
  }

  cplx *R = (cplx *)malloc((size_t)(nsteps + 1) * n2 * sizeof(cplx));
  cplx *buf = (cplx *)malloc(13 * n2 * sizeof(cplx));
  double *uval = (double *)calloc((size_t)s->n_ctrl + 1, sizeof(double));
  work_t w;
  if (!R || !buf || !uval || work_init(&w, n)) {
    free(R);
    free(buf);
    free(uval);
    return ORC_ENOMEM;
  }
  cplx *y = buf, *k = buf + n2, *acc = buf + 2 * n2, *lam = buf + 3 * n2;
  cplx *Y[4], *kap[4];
  for (int i = 0; i < 4; ++i) {
    Y[i] = buf + (size_t)(4 + i) * n2;
    kap[i] = buf + (size_t)(8 + i) * n2;
  }
  cplx *comm = buf + 12 * n2;

  /* forward pass, keeping every step's starting state */
  memcpy(R, rho0, n2 * sizeof(cplx));
  for (long st = 0; st < nsteps; ++st) {
    memcpy(R + (size_t)(st + 1) * n2, R + (size_t)st * n2, n2 * sizeof(cplx));
    controls_at(s, t0 + ((double)st + 0.5) * h, uval);
    rk4_step(s, uval, h, R + (size_t)(st + 1) * n2, y, k, acc, &w);
  }
  /* J = Re Tr(O rho_N) = Re sum_il O_il rho_li */
  {
    const cplx *Oc = (const cplx *)O;
    const cplx *rN = R + (size_t)nsteps * n2;
    cplx tr = 0.0;
    for (int i = 0; i < n; ++i)
      for (int l = 0; l < n; ++l) tr += Oc[(size_t)i * n + l] * rN[(size_t)l * n + i];
    *cost = creal(tr);
    /* dJ/drho_N in the real inner product Re Tr(X^+ Y) is O^+ */
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) lam[(size_t)i * n + j] = conj(Oc[(size_t)j * n + i]);
  }
  if (grad)
    for (int j = 0; j < s->n_ctrl * s->n_seg; ++j) grad[j] = 0.0;

  /* backward pass */
  for (long st = nsteps - 1; st >= 0; --st) {
    const int q = controls_at(s, t0 + ((double)st + 0.5) * h, uval);
    const cplx *rs = R + (size_t)st * n2;
    /* stage inputs of this step */
    memcpy(Y[0], rs, n2 * sizeof(cplx));
    lindblad(s, uval, Y[0], k, &w);
    for (size_t e = 0; e < n2; ++e) Y[1][e] = rs[e] + (0.5 * h) * k[e];
    lindblad(s, uval, Y[1], k, &w);
    for (size_t e = 0; e < n2; ++e) Y[2][e] = rs[e] + (0.5 * h) * k[e];
    lindblad(s, uval, Y[2], k, &w);
    for (size_t e = 0; e < n2; ++e) Y[3][e] = rs[e] + h * k[e];
    /* kap_i = dJ/dk_i, w_i = L^+ kap_i = dJ/dY_i:
       rho' = rho + h (k1 + 2k2 + 2k3 + k4)/6, Y2 = rho + h/2 k1,
       Y3 = rho + h/2 k2, Y4 = rho + h k3 */
    for (size_t e = 0; e < n2; ++e) kap[3][e] = (h / 6.0) * lam[e];
    lindblad_dag(s, uval, kap[3], acc, &w); /* w4 in acc */
    for (size_t e = 0; e < n2; ++e) kap[2][e] = (h / 3.0) * lam[e] + h * acc[e];
    for (size_t e = 0; e < n2; ++e) y[e] = acc[e]; /* y accumulates sum w_i */
    lindblad_dag(s, uval, kap[2], acc, &w); /* w3 */
    for (size_t e = 0; e < n2; ++e) {
      kap[1][e] = (h / 3.0) * lam[e] + (0.5 * h) * acc[e];
      y[e] += acc[e];
    }
    lindblad_dag(s, uval, kap[1], acc, &w); /* w2 */
    for (size_t e = 0; e < n2; ++e) {
      kap[0][e] = (h / 6.0) * lam[e] + (0.5 * h) * acc[e];
      y[e] += acc[e];
    }
    lindblad_dag(s, uval, kap[0], acc, &w); /* w1 */
    for (size_t e = 0; e < n2; ++e) y[e] += acc[e];
    /* dJ/du_j += sum_i Re Tr(kap_i^+ (dL/du_j) Y_i), (dL/du_j) Y = -i[H_j, Y] */
    if (grad && q >= 0)
      for (int j = 0; j < s->n_ctrl; ++j) {
        double g = 0.0;
        for (int i = 0; i < 4; ++i) {
          memset(comm, 0, n2 * sizeof(cplx));
          mul_csr_dense(n, &s->Hc[j], Y[i], -I, comm);
          mul_dense_csr(n, Y[i], &s->Hc[j], I, comm);
          g += hs_real(n2, kap[i], comm);
        }
        grad[(size_t)j * s->n_seg + q] += g;
      }
    for (size_t e = 0; e < n2; ++e) lam[e] += y[e];
  }
  work_free(&w);
  free(R);
  free(buf);
  free(uval);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Propagator and steady state                                                 */
/* ------------------------------------------------------------------------- */

int orc_propagator(const orc_system *s, double t0, double t1, int32_t nsteps, double *U) {
  int rc = check_system(s);
  if (rc) return rc;
  if (!U || nsteps < 1 || !(t1 > t0)) return ORC_EINVAL;
  const int n = s->n;
  const size_t n2 = (size_t)n * n;
  cplx *basis = (cplx *)calloc(n2, sizeof(cplx));
  cplx *states = (cplx *)malloc(2 * n2 * sizeof(cplx));
  double *ex = (double *)malloc(4 * ((size_t)s->n_e + 1) * sizeof(double));
  if (!basis || !states || !ex) {
    free(basis);
    free(states);
    free(ex);
    return ORC_ENOMEM;
  }
  const double tl[2] = {t0, t1};
  for (size_t c = 0; c < n2 && rc == ORC_OK; ++c) {
    basis[c] = 1.0; /* |i><j| with c = i*n + j */
    rc = orc_rk4(s, (const double *)basis, 2, tl, nsteps, ex, (double *)states);
    basis[c] = 0.0;
    if (rc == ORC_OK) memcpy((cplx *)U + c * n2, states + n2, n2 * sizeof(cplx));
  }
  free(basis);
  free(states);
  free(ex);
  return rc;
}

int orc_steadystate(const orc_system *s, double *rho) {
  int rc = check_system(s);
  if (rc) return rc;
  if (!rho || s->n_ctrl != 0) return ORC_EINVAL;
  const int n = s->n;
  const size_t N = (size_t)n * n;
  cplx *M = (cplx *)calloc(N * N, sizeof(cplx)); /* row-major M[r*N + c] */
  cplx *x = (cplx *)calloc(N, sizeof(cplx));
  cplx *out = (cplx *)malloc(N * sizeof(cplx));
  double *uval = (double *)calloc((size_t)s->n_ctrl + 1, sizeof(double));
  work_t w;
  if (!M || !x || !out || !uval || work_init(&w, n)) {
    free(M);
    free(x);
    free(out);
    free(uval);
    return ORC_ENOMEM;
  }
  /* column c of the superoperator: L applied to the basis matrix |i><j| */
  for (size_t c = 0; c < N; ++c) {
    x[c] = 1.0;
    lindblad(s, uval, x, out, &w);
    x[c] = 0.0;
    for (size_t r = 0; r < N; ++r) M[r * N + c] = out[r];
  }
  /* the trace condition replaces row 0: sum_i rho_ii = 1 */
  cplx *b = x; /* right-hand side, reused */
  for (size_t c = 0; c < N; ++c) M[c] = 0.0;
  for (int i = 0; i < n; ++i) M[(size_t)i * n + i] = 1.0;
  memset(b, 0, N * sizeof(cplx));
  b[0] = 1.0;
  /* Gaussian elimination with partial pivoting */
  for (size_t k = 0; k < N && rc == ORC_OK; ++k) {
    size_t p = k;
    double best = cabs(M[k * N + k]);
    for (size_t r = k + 1; r < N; ++r)
      if (cabs(M[r * N + k]) > best) {
        best = cabs(M[r * N + k]);
        p = r;
      }
    if (!(best > 0.0)) {
      rc = ORC_ENONFINITE; /* singular: no unique steady state */
      break;
    }
    if (p != k) {
      for (size_t c = 0; c < N; ++c) {
        const cplx tmp = M[k * N + c];
        M[k * N + c] = M[p * N + c];
        M[p * N + c] = tmp;
      }
      const cplx tb = b[k];
      b[k] = b[p];
      b[p] = tb;
    }
    for (size_t r = k + 1; r < N; ++r) {
      const cplx f = M[r * N + k] / M[k * N + k];
      if (f == 0.0) continue;
      for (size_t c = k; c < N; ++c) M[r * N + c] -= f * M[k * N + c];
      b[r] -= f * b[k];
    }
  }
  if (rc == ORC_OK) {
    for (size_t k = N; k-- > 0;) {
      cplx acc = b[k];
      for (size_t c = k + 1; c < N; ++c) acc -= M[k * N + c] * out[c];
      out[k] = acc / M[k * N + k];
    }
    memcpy(rho, out, N * sizeof(cplx));
  }
  work_free(&w);
  free(M);
  free(x);
  free(out);
  free(uval);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Two-time correlation functions (quantum regression theorem)                 */
/* ------------------------------------------------------------------------- */

int orc_correlation(const orc_system *s, const double *rho0, int32_t n_t, const double *tlist,
                    int32_t nsteps, int32_t n_tau, const double *taulist, int32_t tau_nsteps,
                    const orc_csr *B, double *corr) {
  int rc = check_system(s);
  if (rc) return rc;
  if (s->n_ctrl != 0 || !rho0 || !tlist || !taulist || !B || !corr || n_t < 1 || n_tau < 1)
    return ORC_EINVAL;
  if ((rc = check_csr(B, s->n))) return rc;
  if (taulist[0] != 0.0) return ORC_EINVAL;
  const int n = s->n;
  const size_t n2 = (size_t)n * n;
  cplx *states = (cplx *)malloc((size_t)n_t * n2 * sizeof(cplx));
  cplx *sigma = (cplx *)malloc(n2 * sizeof(cplx));
  double *ex_t = (double *)malloc(2 * ((size_t)s->n_e + 1) * n_t * sizeof(double));
  double *ex_tau = (double *)malloc(2 * ((size_t)s->n_e + 1) * n_tau * sizeof(double));
  if (!states || !sigma || !ex_t || !ex_tau) {
    rc = ORC_ENOMEM;
    goto done;
  }
  /* rho(t_i) at every t_i */
  if ((rc = orc_rk4(s, rho0, n_t, tlist, nsteps, ex_t, (double *)states))) goto done;
  for (int i = 0; i < n_t; ++i) {
    /* sigma = B rho(t_i) */
    memset(sigma, 0, n2 * sizeof(cplx));
    mul_csr_dense(n, B, states + (size_t)i * n2, 1.0, sigma);
    /* Tr(E_m V(tau_j) sigma) */
    if ((rc = orc_rk4(s, (const double *)sigma, n_tau, taulist, tau_nsteps, ex_tau, NULL)))
      goto done;
    for (int m = 0; m < s->n_e; ++m)
      for (int j = 0; j < n_tau; ++j) {
        const size_t o = 2 * (((size_t)i * s->n_e + m) * n_tau + j);
        corr[o] = ex_tau[2 * ((size_t)m * n_tau + j)];
        corr[o + 1] = ex_tau[2 * ((size_t)m * n_tau + j) + 1];
      }
  }
done:
  free(states);
  free(sigma);
  free(ex_t);
  free(ex_tau);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Monte-Carlo wave-function trajectories (Sec. 3.2)                           */
/* ------------------------------------------------------------------------- */

/* out += alpha * M x */
static void csr_vec(int n, const orc_csr *M, const cplx *x, cplx alpha, cplx *out) {
  const cplx *mv = cval(M);
  for (int i = 0; i < n; ++i)
    for (int p = M->row_ptr[i]; p < M->row_ptr[i + 1]; ++p) out[i] += alpha * mv[p] * x[M->col[p]];
}

/* out += alpha * M^+ x,  (M^+ x)_i = sum_l conj(M_li) x_l */
static void csrdag_vec(int n, const orc_csr *M, const cplx *x, cplx alpha, cplx *out) {
  const cplx *mv = cval(M);
  for (int l = 0; l < n; ++l)
    for (int p = M->row_ptr[l]; p < M->row_ptr[l + 1]; ++p)
      out[M->col[p]] += alpha * conj(mv[p]) * x[l];
}

static double norm2_vec(int n, const cplx *x) {
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
  return acc;
}

/* out = -i H_eff psi with H_eff = H0 - (i/2) sum_n C_n^+ C_n (Eq. (heff), hbar = 1),
 * i.e. out = -i H0 psi - 1/2 sum_n C_n^+ (C_n psi). */
static void heff_rhs(const orc_system *s, const cplx *psi, cplx *out, cplx *tmp) {
  const int n = s->n;
  memset(out, 0, (size_t)n * sizeof(cplx));
  csr_vec(n, &s->H0, psi, -I, out);
  for (int k = 0; k < s->n_c; ++k) {
    memset(tmp, 0, (size_t)n * sizeof(cplx));
    csr_vec(n, &s->C[k], psi, 1.0, tmp);
    csrdag_vec(n, &s->C[k], tmp, -0.5, out);
  }
}

typedef struct {
  cplx *k, *y, *acc, *tmp;
} mc_work;

/* out = the classic RK4 step of length h of d psi/dt = -i H_eff psi from psi. */
static void rk4_vec(const orc_system *s, double h, const cplx *psi, cplx *out, mc_work *w) {
  const int n = s->n;
  heff_rhs(s, psi, w->k, w->tmp); /* k1 */
  for (int i = 0; i < n; ++i) {
    w->acc[i] = w->k[i];
    w->y[i] = psi[i] + (0.5 * h) * w->k[i];
  }
  heff_rhs(s, w->y, w->k, w->tmp); /* k2 */
  for (int i = 0; i < n; ++i) {
    w->acc[i] += 2.0 * w->k[i];
    w->y[i] = psi[i] + (0.5 * h) * w->k[i];
  }
  heff_rhs(s, w->y, w->k, w->tmp); /* k3 */
  for (int i = 0; i < n; ++i) {
    w->acc[i] += 2.0 * w->k[i];
    w->y[i] = psi[i] + h * w->k[i];
  }
  heff_rhs(s, w->y, w->k, w->tmp); /* k4 */
  for (int i = 0; i < n; ++i) {
    w->acc[i] += w->k[i];
    out[i] = psi[i] + (h / 6.0) * w->acc[i];
  }
}

/* <psi|E psi> / <psi|psi> for every expectation operator into ex[m] (complex). */
static void mc_record(const orc_system *s, const cplx *psi, cplx *tmp, cplx *ex) {
  const int n = s->n;
  const double nn = norm2_vec(n, psi);
  for (int m = 0; m < s->n_e; ++m) {
    memset(tmp, 0, (size_t)n * sizeof(cplx));
    csr_vec(n, &s->E[m], psi, 1.0, tmp);
    cplx acc = 0.0;
    for (int i = 0; i < n; ++i) acc += conj(psi[i]) * tmp[i];
    ex[m] = acc / nn;
  }
}

/* One trajectory: steps I-IV of Sec. 3.2.  ex: [n_e][n_t] complex. */
static int mc_trajectory(const orc_system *s, const cplx *psi0, int32_t n_t, const double *tlist,
                         int32_t nsteps, const long *out_step, const double *draws,
                         int32_t max_jumps, cplx *ex, int32_t *n_jumps, double *jump_t,
                         int32_t *jump_op) {
  const int n = s->n;
  const double t0 = tlist[0];
  const double h = n_t > 1 ? (tlist[n_t - 1] - t0) / nsteps : 0.0;
  cplx *buf = (cplx *)malloc(7 * (size_t)n * sizeof(cplx));
  cplx *exk = (cplx *)malloc(((size_t)s->n_e + 1) * sizeof(cplx));
  if (!buf || !exk) {
    free(buf);
    free(exk);
    return ORC_ENOMEM;
  }
  mc_work w = {buf, buf + n, buf + 2 * (size_t)n, buf + 3 * (size_t)n};
  cplx *psi = buf + 4 * (size_t)n, *trial = buf + 5 * (size_t)n, *cpsi = buf + 6 * (size_t)n;
  int rc = ORC_OK;
  int jumps = 0;
  /* the initial state, normalised */
  const double nn0 = norm2_vec(n, psi0);
  if (!(nn0 > 0.0) || !isfinite(nn0)) {
    rc = ORC_EINVAL;
    goto done;
  }
  for (int i = 0; i < n; ++i) psi[i] = psi0[i] / sqrt(nn0);
  mc_record(s, psi, w.tmp, exk);
  for (int m = 0; m < s->n_e; ++m) ex[(size_t)m * n_t] = exk[m];

  double r = draws[0]; /* step I: the first waiting period's threshold */
  int next = 1;
  for (long st = 0; st < (n_t > 1 ? nsteps : 0); ++st) {
    double t = t0 + (double)st * h; /* time of the current state */
    double left = h;                  /* the rest of this grid step */
    while (left > 0.0) {
      /* step II: integrate; does the norm reach r within the rest of the step? */
      rk4_vec(s, left, psi, trial, &w);
      const double nt = norm2_vec(n, trial);
      if (!isfinite(nt)) {
        rc = ORC_ENONFINITE;
        goto done;
      }
      if (nt > r) {
        memcpy(psi, trial, (size_t)n * sizeof(cplx));
        break;
      }
      /* the jump time: tau in (0, left] with |RK4(psi, tau)|^2 = r, by bisection
         (the norm is above r at 0 and at most r at `left`) */
      double lo = 0.0, hi = left;
      for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        rk4_vec(s, mid, psi, trial, &w);
        if (norm2_vec(n, trial) <= r)
          hi = mid;
        else
          lo = mid;
      }
      const double tau = hi;
      rk4_vec(s, tau, psi, trial, &w);
      /* step III: probabilities P_i = <psi|C_i^+ C_i|psi> / sum (Eq. (pcn)) and
         the smallest n with P_1 + ... + P_n >= r' (Eq. (mc3)) */
      if (jumps >= max_jumps) {
        rc = ORC_EDRAWS;
        goto done;
      }
      const double r2 = draws[2 * (size_t)jumps + 1];
      double total = 0.0;
      for (int k = 0; k < s->n_c; ++k) {
        memset(cpsi, 0, (size_t)n * sizeof(cplx));
        csr_vec(n, &s->C[k], trial, 1.0, cpsi);
        total += norm2_vec(n, cpsi);
      }
      if (!(total > 0.0) || !isfinite(total)) {
        rc = ORC_ENONFINITE;
        goto done;
      }
      int chosen = -1, last_nonzero = -1;
      double cum = 0.0, w_chosen = 0.0;
      for (int k = 0; k < s->n_c && chosen < 0; ++k) {
        memset(cpsi, 0, (size_t)n * sizeof(cplx));
        csr_vec(n, &s->C[k], trial, 1.0, cpsi);
        const double wk = norm2_vec(n, cpsi);
        if (wk > 0.0) last_nonzero = k;
        cum += wk / total;
        if (cum >= r2 && wk > 0.0) {
          chosen = k;
          w_chosen = wk;
        }
      }
      if (chosen < 0) { /* r' above the rounded cumulative sum: the last channel */
        chosen = last_nonzero;
        memset(cpsi, 0, (size_t)n * sizeof(cplx));
        csr_vec(n, &s->C[chosen], trial, 1.0, cpsi);
        w_chosen = norm2_vec(n, cpsi);
      }
      /* the projected, renormalised state (Eq. (project)) */
      memset(cpsi, 0, (size_t)n * sizeof(cplx));
      csr_vec(n, &s->C[chosen], trial, 1.0, cpsi);
      for (int i = 0; i < n; ++i) psi[i] = cpsi[i] / sqrt(w_chosen);
      t += tau;
      if (jump_t) jump_t[jumps] = t;
      if (jump_op) jump_op[jumps] = chosen;
      ++jumps;
      /* step IV: a new random number; continue from the jump time with the
         rest of the grid step */
      r = draws[2 * (size_t)jumps];
      left -= tau;
    }
    while (next < n_t && out_step[next] == st + 1) {
      mc_record(s, psi, w.tmp, exk);
      for (int m = 0; m < s->n_e; ++m) ex[(size_t)m * n_t + next] = exk[m];
      ++next;
    }
  }
done:
  if (n_jumps) *n_jumps = jumps;
  free(buf);
  free(exk);
  return rc;
}

typedef struct {
  const orc_system *s;
  const cplx *psi0;
  int32_t n_t;
  const double *tlist;
  int32_t nsteps;
  const long *out_step;
  const double *draws;
  int32_t max_jumps;
  cplx *ex_all; /* [n_traj][n_e][n_t] */
  int32_t *n_jumps;
  double *jump_t;
  int32_t *jump_op;
  int32_t *status;
  int32_t n_traj;
  int next;
} mc_job;

static void *mc_worker(void *arg) {
  mc_job *j = (mc_job *)arg;
  const size_t per = (size_t)j->s->n_e * j->n_t;
  for (;;) {
    const int b = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
    if (b >= j->n_traj) break;
    int32_t nj = 0;
    j->status[b] = mc_trajectory(
        j->s, j->psi0, j->n_t, j->tlist, j->nsteps, j->out_step,
        j->draws + 2 * (size_t)b * ((size_t)j->max_jumps + 1), j->max_jumps, j->ex_all + per * b,
        &nj, j->jump_t ? j->jump_t + (size_t)b * j->max_jumps : NULL,
        j->jump_op ? j->jump_op + (size_t)b * j->max_jumps : NULL);
    if (j->n_jumps) j->n_jumps[b] = nj;
  }
  return NULL;
}

int orc_mc(const orc_system *s, const double *psi0, int32_t n_t, const double *tlist,
           int32_t nsteps, int32_t n_traj, const double *draws, int32_t max_jumps,
           double *expect_avg, double *expect_traj, int32_t *n_jumps, double *jump_t,
           int32_t *jump_op, int32_t *status, int32_t n_threads) {
  int rc = check_system(s);
  if (rc) return rc;
  if (s->n_ctrl != 0 || !psi0 || !tlist || n_t < 1 || n_traj < 1 || !draws || max_jumps < 0 ||
      n_threads < 1)
    return ORC_EINVAL;
  if (n_t > 1 && nsteps < 1) return ORC_EINVAL;
  const double h = n_t > 1 ? (tlist[n_t - 1] - tlist[0]) / nsteps : 0.0;
  long *out_step = (long *)malloc(sizeof(long) * (size_t)n_t);
  const size_t per = (size_t)s->n_e * n_t;
  cplx *ex_all = (cplx *)calloc(per * n_traj + 1, sizeof(cplx));
  int32_t *st = (int32_t *)calloc((size_t)n_traj, sizeof(int32_t));
  if (!out_step || !ex_all || !st) {
    free(out_step);
    free(ex_all);
    free(st);
    return ORC_ENOMEM;
  }
  if (n_t > 1) rc = rk4_grid(s, n_t, tlist, nsteps, h, out_step);
  else out_step[0] = 0;
  if (rc) goto done;
  {
    mc_job job = {s, (const cplx *)psi0, n_t, tlist, nsteps, out_step, draws, max_jumps, ex_all,
                  n_jumps, jump_t, jump_op, st, n_traj, 0};
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    int started = 0;
    if (th)
      for (int i = 0; i < n_threads; ++i)
        if (pthread_create(&th[i], NULL, mc_worker, &job) == 0) ++started;
    if (started == 0) mc_worker(&job);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    free(th);
  }
  for (int b = 0; b < n_traj; ++b)
    if (st[b] != ORC_OK) rc = st[b];
  if (status) memcpy(status, st, sizeof(int32_t) * (size_t)n_traj);
  if (expect_traj) memcpy(expect_traj, ex_all, per * n_traj * sizeof(cplx));
  if (expect_avg) {
    /* mean over trajectories, in trajectory order */
    cplx *avg = (cplx *)expect_avg;
    for (size_t e = 0; e < per; ++e) {
      cplx acc = 0.0;
      for (int b = 0; b < n_traj; ++b) acc += ex_all[per * b + e];
      avg[e] = acc / (double)n_traj;
    }
  }
done:
  free(out_step);
  free(ex_all);
  free(st);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Many instances on host threads                                             */
/* ------------------------------------------------------------------------- */

typedef struct {
  int32_t n_inst;
  const orc_system *systems;
  const double *const *rho0;
  int32_t n_t;
  const double *tlist;
  int32_t nsteps;
  double *const *expect;
  int32_t *rc;
  int next; /* shared work counter */
} batch_job;

static void *batch_worker(void *arg) {
  batch_job *job = (batch_job *)arg;
  for (;;) {
    const int b = __atomic_fetch_add(&job->next, 1, __ATOMIC_RELAXED);
    if (b >= job->n_inst) break;
    job->rc[b] = orc_rk4(&job->systems[b], job->rho0[b], job->n_t, job->tlist,
                         job->nsteps, job->expect[b], NULL);
  }
  return NULL;
}

int orc_rk4_batch(int32_t n_inst, const orc_system *systems,
                  const double *const *rho0, int32_t n_t, const double *tlist,
                  int32_t nsteps, double *const *expect, int32_t n_threads,
                  int32_t *rc) {
  if (n_inst < 0 || n_threads < 1 || !rc) return ORC_EINVAL;
  batch_job job = {n_inst, systems, rho0, n_t, tlist, nsteps, expect, rc, 0};
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!th) return ORC_ENOMEM;
  int started = 0;
  for (int i = 0; i < n_threads; ++i)
    if (pthread_create(&th[i], NULL, batch_worker, &job) == 0) ++started;
  if (started == 0) batch_worker(&job);
  for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
  free(th);
  int worst = ORC_OK;
  for (int b = 0; b < n_inst; ++b)
    if (rc[b] != ORC_OK) worst = rc[b];
  return worst;
}
