/*
 * lme.h -- C ABI of the MI355X (gfx950) Lindblad master-equation library.
 *
 * What is computed (Johansson, Nation & Nori, arXiv:1110.0573):
 *   Sec. 3.1, Eq. (master_equation), hbar = 1:
 *     drho/dt = L(t) rho = -i[H(t), rho]
 *               + sum_k ( C_k rho C_k^+ - 1/2 rho C_k^+ C_k - 1/2 C_k^+ C_k rho )
 *   with H(t) = H0 + sum_j u_j(t) H_j (Sec. 4.4 gives a time-dependent
 *   Hamiltonian as constant operators times scalar functions of time; here
 *   the u_j are piecewise constant on a fixed set of segment edges).
 *   Sec. 4 (odesolve): the solver returns expectation values Tr(E rho(t)) at
 *   every requested output time, the first output time being the initial
 *   time, or the density matrices themselves.
 * The paper names no integrator.  Two are provided: classic fixed-step RK4
 * and the adaptive Dormand-Prince 5(4) pair.
 *
 * Conventions used throughout:
 *   - complex numbers are two consecutive doubles (re, im) ("complex128");
 *   - a density matrix of dimension n is n*n complex128, row-major
 *     (element (i, j) at i*n + j);
 *   - a batch of instances (possibly of different n) is one packed device
 *     buffer: instance b occupies [offset[b], offset[b] + n_b^2) in units of
 *     complex128, offsets in instance order without gaps (lme_layout);
 *   - operators are handed over as host CSR (lme_csr) and COPIED at create:
 *     the caller may free them as soon as lme_create* returns;
 *   - every device pointer argument is caller-owned device memory
 *     (e.g. a torch tensor's data_ptr()); the library only reads or writes it
 *     on the given HIP stream, asynchronously; it must stay valid until the
 *     work queued on that stream has completed;
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *
 * Errors: every entry point returns an lme_status.  Arguments are validated
 * on the host before any HIP call is made, so a malformed argument never
 * reaches the GPU.  lme_last_error() gives a human-readable message for the
 * last failing call on the calling thread.  No C++ exception crosses the ABI.
 * Failures that can only be detected on the device during integration
 * (step budget, step underflow, non-finite values) are reported per instance
 * through the optional `status_dev` array.
 *
 * Thread safety: distinct handles may be used concurrently; one handle must
 * not be used by two host threads at the same time.
 */
#ifndef LME_H
#define LME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LME_ABI_VERSION 1

typedef enum lme_status {
  LME_OK = 0,
  LME_EINVAL = 1,          /* malformed argument (CSR, sizes, options, times) */
  LME_EGRID = 2,           /* RK4: an output time or a control edge is not on
                              the uniform step grid                          */
  LME_EMAXSTEPS = 3,       /* adaptive: max_steps attempts used up (device)   */
  LME_ESTEPUNDERFLOW = 4,  /* adaptive: step size fell below h_min (device)   */
  LME_ENONFINITE = 5,      /* NaN/Inf in an error norm or expectation (device)*/
  LME_ENOMEM = 6,          /* host or device allocation failed                */
  LME_EHIP = 7,            /* a HIP runtime call failed (no device, launch)   */
  LME_ENOTSUP = 8,         /* valid input outside what this build supports    */
  LME_ENOTHERM = 9,        /* hermitian option with a non-Hermitian rho0 of
                              that instance (device, per instance)            */
  LME_EDRAWS = 10          /* Monte-Carlo: a trajectory needed more jumps than
                              its random draws cover (device, per trajectory)*/
} lme_status;

typedef struct lme_ctx *lme_handle;

typedef enum lme_method { LME_RK4 = 0, LME_DOPRI5 = 1 } lme_method;

/* Which kernel family integrates the batch. */
typedef enum lme_path {
  LME_PATH_AUTO = 0,       /* resident when every instance fits, else streamed */
  LME_PATH_RESIDENT = 1,   /* one workgroup owns a pack of instances for the
                              whole integration; stage input held in LDS      */
  LME_PATH_STREAMED = 2    /* one grid-wide kernel per stage; state in HBM    */
} lme_path;

/* Thread-to-element layout of the resident kernels. */
typedef enum lme_layout_kind {
  LME_LAYOUT_AUTO = 0,
  LME_LAYOUT_ROW = 1,      /* thread t owns elements t, t+T, ... of the pack  */
  LME_LAYOUT_COLUMN = 2    /* thread owns one column; its operator entries
                              stay in registers                               */
} lme_layout_kind;

/* Form of the Liouvillian application used by lme_apply. */
typedef enum lme_form {
  LME_FORM_OPERATOR = 0,   /* sparse H, C_k applied to the dense n x n matrix;
                              stage input staged in LDS: whole instances when
                              they fit a workgroup, else blocks of rows (every
                              instance 128 <= n <= 1024), else read from HBM */
  LME_FORM_SUPEROP = 1,    /* explicit n^2 x n^2 CSR superoperator SpMV       */
  LME_FORM_OPERATOR_STREAMED = 2  /* operator form read straight from HBM     */
} lme_form;

/* Square sparse matrix in CSR form, host memory.
 *   row_ptr[n+1] (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz),
 *   col[nnz] (0 <= col < n; duplicates within a row are summed),
 *   val[2*nnz] complex128.  Explicit zeros are dropped at create. */
typedef struct lme_csr {
  int32_t n;
  int32_t nnz;
  const int32_t *row_ptr;
  const int32_t *col;
  const double *val;
} lme_csr;

/* One open system.  H0 (Hermitian), the batch-wide number n_ctrl of control
 * Hamiltonians H_ctrl[n_ctrl] (Hermitian), n_c collapse operators C[n_c]
 * (arbitrary; n_c may differ between instances) and the batch-wide number
 * n_e of expectation operators E[n_e] (arbitrary).  All of dimension n. */
typedef struct lme_instance {
  const lme_csr *H0;
  const lme_csr *H_ctrl;
  int32_t n_c;
  const lme_csr *C;
  const lme_csr *E;
} lme_instance;

/* Piecewise-constant control segments shared by the batch: u_j(t) takes its
 * segment value on [edges[s], edges[s+1]) and is 0 outside [edges[0],
 * edges[n_seg]).  A step never straddles an edge: with RK4 every edge inside
 * the integration interval must lie on the step grid (else LME_EGRID); the
 * adaptive stepper stops on every edge.  Within one step the amplitudes of
 * the segment holding the step's midpoint are used. */
typedef struct lme_segments {
  int32_t n_seg;           /* 0: no controls                                  */
  const double *edges;     /* host, [n_seg+1], strictly increasing            */
} lme_segments;

typedef struct lme_options {
  int32_t method;          /* lme_method                                      */
  int32_t path;            /* lme_path                                        */
  int32_t nsteps;          /* RK4: equal steps from tlist[0] to tlist[n_t-1];
                              every output time must be on this grid          */
  int32_t block;           /* resident path: threads per workgroup; 0 = tuned
                              default.  RK4 row layout: 256, 512 or 1024;
                              RK4 column layout: 512 or 768.  DOPRI5: 512, or
                              1024 in the column layout                       */
  int32_t layout;          /* resident path, thread-to-element layout:
                              LME_LAYOUT_AUTO, LME_LAYOUT_ROW (any operator)
                              or LME_LAYOUT_COLUMN (monomial collapse
                              operators, at most 2 off-diagonal entries per
                              row of H, at most 3 collapse operators and 1
                              control term); both give identical results.
                              DOPRI5 has the row layout at 512 threads and
                              the column layout at 1024 threads (4 rows per
                              thread) or 512 (8 or 16); AUTO takes the column
                              layout when 4 or 8 rows per thread suffice    */
  double rtol, atol;       /* DOPRI5: per-element tolerance
                              atol + rtol*max(|rho|, |rho_new|)               */
  double h0;               /* DOPRI5: first step; <= 0 selects it
                              automatically (Hairer-Norsett-Wanner rule)      */
  double h_min;            /* DOPRI5: smallest allowed step                   */
  int64_t max_steps;       /* DOPRI5: attempts (accepted + rejected) per
                              instance                                        */
  int32_t hermitian;       /* 1: rho0 is Hermitian (a density matrix).  The
                              Lindblad generator maps Hermitian matrices to
                              Hermitian matrices, so every stage input and
                              every state stays Hermitian; the resident RK4
                              column-layout kernel then computes each pair
                              {i, j} once and writes its mirror as the
                              conjugate (half the arithmetic).  rho0 is read
                              as its Hermitian part; an instance with
                              |rho_ij - conj(rho_ji)| > 1e-12 sqrt(2(|rho_ij|^2
                              + |rho_ji|^2)) for some pair gets status
                              LME_ENOTHERM (and is integrated from that
                              Hermitian part).  Other paths ignore the flag
                              and compute every element.  0: no assumption  */
  int32_t reserved;        /* unused; set to 0                                */
} lme_options;

/* Fills defaults: RK4, AUTO path, nsteps 0 (must be set), block 0, layout 0,
 * rtol 1e-6, atol 1e-9, h0 0, h_min 0, max_steps 10^7, hermitian 0. */
void lme_default_options(lme_options *opt);

/* Create a handle for a batch of n_inst independent systems (Sec. 3.1,
 * Eq. (master_equation): each system is its Hamiltonian, its collapse
 * operators C_n = sqrt(gamma_n) A_n and, as in the solver call of Sec. 4,
 * the operators whose expectation values are returned).
 *   inst[n_inst]: the systems (host, copied);
 *   n_ctrl, n_e: batch-wide counts of control and expectation operators;
 *   seg: control segments (NULL or n_seg == 0 when n_ctrl == 0);
 *   u_host: default control amplitudes, host, [n_inst][n_ctrl][n_seg]
 *           (NULL = all zero); lme_evolve may override them per call.
 * Builds the operator tables (A = -iH0 - 1/2 sum_k C_k^+ C_k, the control
 * terms -iH_j, the jump tables and their adjoints) and uploads them to the
 * current HIP device (on a machine without a device, at the handle's first
 * device call instead).  *out receives the handle (NULL on failure).
 * Errors: LME_EINVAL, LME_ENOTSUP (an operator row with more than 64
 * non-zeros, or n > 4096), LME_ENOMEM, LME_EHIP. */
int lme_create_batch(int32_t n_inst, const lme_instance *inst, int32_t n_ctrl,
                     int32_t n_e, const lme_segments *seg, const double *u_host,
                     lme_handle *out);

/* Single-instance form of lme_create_batch (Sec. 3.1, Eq.
 * (master_equation); the argument order follows the solver call of Sec. 4:
 * Hamiltonian, its time-dependent terms, collapse operators, expectation
 * operators):
 *   lme_create(H0, {H_j}, segments + amplitudes, {C_k}, {E_m}). */
int lme_create(const lme_csr *H0, int32_t n_ctrl, const lme_csr *H_ctrl,
               const lme_segments *seg, const double *u_host, int32_t n_c,
               const lme_csr *C, int32_t n_e, const lme_csr *E, lme_handle *out);

/* Closed-form amplitudes (Sec. 4.4: a time-dependent Hamiltonian given as
 * constant operators times scalar functions of time, such as the
 * Landau-Zener sweep H0 + t H1 of Eq. (lz-hamiltonian)).
 *   fn_host: host double [n_inst][n_ctrl][7] = (c0, c1, c2, c3, a, w, phi),
 *            u_j(t) = c0 + c1 t + c2 t^2 + c3 t^3 + a cos(w t + phi) for
 *            control term j of each instance; copied.  NULL returns the
 *            handle to its piecewise-constant segments.
 * While set, lme_evolve integrates with fixed-step RK4 on the resident
 * kernels, every stage evaluating the amplitudes at its own time (t,
 * t + h/2, t + h/2, t + h); segment edges no longer constrain the grid; the
 * u_dev override is refused; lme_apply evaluates the amplitudes at its t.
 * LME_ENOTSUP from lme_evolve with LME_DOPRI5 or the streamed path, and from
 * lme_cost_grad (its gradient is with respect to segment amplitudes).
 * Errors: LME_EINVAL (NULL handle, no control terms, non-finite values),
 * LME_ENOMEM, LME_EHIP. */
int lme_set_coeff_fn(lme_handle h, const double *fn_host);

/* Releases the handle and every device buffer it owns.  NULL is a no-op.
 * Work already queued on a stream that uses the handle must have completed. */
void lme_destroy(lme_handle h);

/* Message for the last failing call made by this host thread ("" if none). */
const char *lme_last_error(void);

/* Number of instances, total packed state size (complex128 elements), and
 * the per-instance layout: offsets[n_inst] (elements) and dims[n_inst].
 * Either output array may be NULL. */
int lme_layout(lme_handle h, int32_t *n_inst, int64_t *state_elems,
               int64_t *offsets, int32_t *dims);

/* Time integration (Sec. 4, odesolve) of every instance from tlist[0].
 *   opt: method and its parameters (see lme_options);
 *   n_t, tlist: host, strictly increasing output times (n_t >= 1);
 *   rho0_dev: packed initial states (complex128, lme_layout);
 *   u_dev: device [n_inst][n_ctrl][n_seg] control amplitudes, or NULL to
 *          use those given at create;
 * outputs (each may be NULL):
 *   expect_dev: complex128 [n_inst][n_e][n_t], Tr(E_m rho(tlist[k]));
 *   states_dev: complex128 [n_t][state_elems], rho at every output time;
 *   rho_out_dev: complex128 [state_elems], rho at tlist[n_t-1];
 *   counts_dev: int64 [n_inst][2], accepted and rejected steps;
 *   status_dev: int32 [n_inst], LME_OK or the device-detected failure of
 *               that instance (LME_EMAXSTEPS, LME_ESTEPUNDERFLOW,
 *               LME_ENONFINITE); a failed instance stops integrating and
 *               its later outputs are left untouched.
 * The call is asynchronous on `stream` except that the adaptive stepper on
 * the streamed path polls a device flag from the host between step batches.
 * Host-side errors: LME_EINVAL, LME_EGRID, LME_ENOTSUP, LME_ENOMEM, LME_EHIP. */
int lme_evolve(lme_handle h, const lme_options *opt, int32_t n_t,
               const double *tlist, const void *rho0_dev, const double *u_dev,
               void *expect_dev, void *states_dev, void *rho_out_dev,
               int64_t *counts_dev, int32_t *status_dev, void *stream);

/* lme_evolve without any device allocation, for callers that cannot
 * allocate device memory during a call: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results
 * and errors as lme_evolve (bit for bit: the same kernels run), restricted
 * to the resident kernels (LME_ENOTSUP for path = LME_PATH_STREAMED or a
 * batch the automatic path would stream).  The step or stop tables, the pack
 * tables and, with LME_DOPRI5, the stage derivatives (112 bytes per state
 * element) live in one library-owned device array of 64 MiB per GPU instead
 * of handle-owned buffers; a call that needs more returns LME_ENOTSUP before
 * any device work.  The tables are copied into the array with
 * hipMemcpyAsync on `stream` from a host image the handle keeps until its
 * next such call.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or host threads) race; calls queued
 * on one stream are ordered.  The handle must have been created while a
 * device was present (its operators are uploaded at create then);
 * LME_EINVAL otherwise. */
int lme_evolve_noalloc(lme_handle h, const lme_options *opt, int32_t n_t,
                       const double *tlist, const void *rho0_dev, const double *u_dev,
                       void *expect_dev, void *states_dev, void *rho_out_dev,
                       int64_t *counts_dev, int32_t *status_dev, void *stream);

/* One application of the Liouvillian (Eq. (master_equation)) or, with
 * adjoint != 0, of its adjoint under the Hilbert-Schmidt inner product
 * L^+ x = i[H, x] + sum_k (C_k^+ x C_k - 1/2 {C_k^+ C_k, x}),
 * to every instance of a packed batch at time t:
 *   out_dev = L(t) y_dev   (both complex128, packed; must not overlap).
 *   form: lme_form (LME_FORM_SUPEROP assembles the n^2 x n^2 CSR
 *         superoperator on first use; forward only).
 *   u_dev: as in lme_evolve (NULL = amplitudes given at create). */
int lme_apply(lme_handle h, int32_t form, int32_t adjoint, double t,
              const double *u_dev, const void *y_dev, void *out_dev,
              void *stream);

/* Two-time correlation functions by the quantum regression theorem (the
 * correlation_ode entry of the paper's function table, Appendix A):
 *   corr[b][i][m][j] = Tr( E_m V(tau_j) [ B_b rho_b(t_i) ] ),
 * rho(t) the solution of Eq. (master_equation) from rho0, V(tau) the same
 * evolution over a delay tau; for E_m = A this is <A(t_i + tau_j) B(t_i)>.
 * rho(t) is integrated with opt (fixed-step RK4, opt->nsteps over tlist,
 * every tlist entry on the grid); every B rho(t_i) with RK4 in tau_nsteps
 * steps over taulist (taulist[0] = 0, increasing), all n_inst * n_t of them
 * as one batch on the general (non-Hermitian) kernels.
 *   B: host CSR [n_inst], B_b of dimension n_b (copied);
 *   rho0_dev: packed initial states (lme_layout);
 *   corr_dev: device complex128 [n_inst][n_t][n_e][n_tau];
 *   status_dev: device int32 [n_inst] or NULL: the first device-detected
 *               failure of the instance's evolutions.
 * Needs a time-independent generator: LME_ENOTSUP with control terms or
 * LME_DOPRI5.  The handle keeps a workspace of 2 n_t state copies and a
 * batch repeated n_t times.  Asynchronous on `stream`.
 * Errors: LME_EINVAL, LME_EGRID, LME_ENOTSUP, LME_ENOMEM, LME_EHIP. */
int lme_correlation(lme_handle h, const lme_options *opt, int32_t n_t, const double *tlist,
                    int32_t n_tau, const double *taulist, int32_t tau_nsteps, const lme_csr *B,
                    const void *rho0_dev, void *corr_dev, int32_t *status_dev, void *stream);

/* Cost and gradient for optimal control of piecewise-constant drives.
 * Integrates every instance with fixed-step RK4 (nsteps equal steps on
 * [t0, t1]; every control edge inside must be on that grid, else LME_EGRID)
 * and returns J_b = Re Tr(O_b rho_b(t1)) and dJ_b/du_b[j][s] for every control
 * term j and segment s: the exact derivative of the discrete RK4 map,
 * obtained by its adjoint (backward recurrence with L^+, the Hilbert-Schmidt
 * adjoint of the Liouvillian of Eq. (master_equation)).  A checkpoint of rho
 * is kept every ckpt_every steps; the stage inputs of one checkpoint interval
 * are recomputed during the backward pass.
 *   rho0_dev, O_dev: packed complex128 (lme_layout); O_b is any n x n matrix
 *                    (a projector |target><target| gives the fidelity);
 *   u_dev: device [n_inst][n_ctrl][n_seg], or NULL for the create-time values;
 *   cost_dev: device double [n_inst]; grad_dev: device double
 *             [n_inst][n_ctrl][n_seg] (overwritten).
 * Needs 1 <= n_ctrl <= 2 control terms and n_seg >= 1 (LME_ENOTSUP /
 * LME_EINVAL otherwise).  Device scratch: (ceil(nsteps/ckpt_every) +
 * 4 ckpt_every) x 16 x state_elems bytes, owned by the handle.
 * Asynchronous on `stream`. */
int lme_cost_grad(lme_handle h, int32_t nsteps, int32_t ckpt_every, double t0, double t1,
                  const void *rho0_dev, const void *O_dev, const double *u_dev,
                  double *cost_dev, double *grad_dev, void *stream);

/* Tuning knobs of a handle (schedules only: every setting gives identical
 * results).  0 in a field means "library default".
 *   rk4_layout, rk4_block: used by lme_evolve (RK4) when the options leave
 *                          layout = LME_LAYOUT_AUTO and block = 0;
 *   herm_layout, herm_block: the same for runs with options.hermitian = 1;
 *   apply_cap: elements per workgroup of the LDS-staged application
 *              (lme_apply, LME_FORM_OPERATOR, general operators), 256 .. 65536;
 *   apply_lds_kb: see the field; 0 or 16 .. 160;
 *   apply_block: threads per workgroup of the column-layout application
 *                (256, 512 or 1024; 0 = 1024);
 *   apply_path: column-layout application as pipelined tiles (0: one
 *               persistent workgroup per CU streaming row tiles through two
 *               LDS stages) or as packs of whole instances (1);
 *   grad_layout: layout of lme_cost_grad, LME_LAYOUT_AUTO (the column layout
 *                where it applies), LME_LAYOUT_ROW or LME_LAYOUT_COLUMN (one
 *                control term, real structure, monomial jumps, one
 *                off-diagonal per row of A; else LME_ENOTSUP). */
typedef struct lme_tuning {
  int32_t rk4_layout;
  int32_t rk4_block;
  int32_t apply_cap;
  int32_t apply_lds_kb;     /* LDS budget of one application workgroup (KB);
                               0 = the device maximum; instances larger than
                               the budget run alone                        */
  double rk4_ms_per_step;   /* lme_autotune: best trial time per RK4 step      */
  double apply_us;          /* lme_autotune: best trial time per application  */
  int32_t herm_layout;
  int32_t herm_block;       /* column layout: 512 or 768                       */
  double herm_ms_per_step;  /* lme_autotune (hermitian = 1): best trial time   */
  int32_t apply_block;
  int32_t apply_path;
  int32_t grad_layout;
} lme_tuning;

int lme_get_tuning(lme_handle h, lme_tuning *t);
int lme_set_tuning(lme_handle h, const lme_tuning *t);

/* Autotuner.  Times every eligible RK4 configuration (layout x workgroup
 * size) on a trial of min(opt->nsteps, 40) steps of this batch from rho0_dev,
 * and every pack size of the LDS-staged application, with HIP events on
 * `stream`; stores the fastest in the handle and in *result (may be NULL).
 * With opt->hermitian = 1 the RK4 trials use the Hermitian kernels and fill
 * herm_layout / herm_block / herm_ms_per_step instead of the rk4_ fields.
 * Synchronises the stream.  Uses a device scratch of two states.
 * Errors as lme_evolve. */
int lme_autotune(lme_handle h, const lme_options *opt, const void *rho0_dev, void *stream,
                 lme_tuning *result);

/* ---------------------------------------------------------------------------
 * Monte-Carlo wave-function trajectories (Sec. 3.2, steps I-IV).
 *
 * Each trajectory evolves a ket under the non-Hermitian effective Hamiltonian
 * of Eq. (heff), d psi/dt = -i H_eff psi with H_eff = H - (i/2) sum_n C_n^+ C_n,
 * until its squared norm falls to the drawn number r (step II); it then jumps
 * with the collapse operator C_k for the smallest k with
 * P_1 + ... + P_k >= r' (Eqs. (pcn), (mc3); r' is a second, independent
 * draw), P_i = <psi|C_i^+ C_i|psi> / sum_j <psi|C_j^+ C_j|psi>, is
 * renormalised (Eq. (project)) and continues with the next draw (step IV).
 * The paper names no integrator: classic RK4 on the uniform grid
 * h = (tlist[n_t-1] - tlist[0]) / nsteps (every output time on the grid,
 * LME_EGRID otherwise); between grid points the state is the RK4 step of the
 * partial length, and the jump time solves |psi(tau)|^2 = r on it.
 * --------------------------------------------------------------------------- */
typedef struct lme_mc_ctx *lme_mc_handle;

/* One system for Monte-Carlo trajectories: Hamiltonian H (n x n, n <= 8192),
 * n_c <= 16 collapse operators C[n_c] and n_e expectation operators E[n_e]
 * (host CSR, copied; Sec. 4.3 passes the same arguments as the master
 * equation solver).  Builds -i H_eff as diagonal + ELL tables, the collapse
 * and expectation operators as ELL tables, and uploads them to the current
 * device (at the first device call on a machine without one).
 * Errors: LME_EINVAL, LME_ENOTSUP (n, row widths > 64, n_c), LME_ENOMEM,
 * LME_EHIP. */
int lme_mc_create(const lme_csr *H, int32_t n_c, const lme_csr *C, int32_t n_e,
                  const lme_csr *E, lme_mc_handle *out);

/* Releases the handle and its device buffers.  NULL is a no-op. */
void lme_mc_destroy(lme_mc_handle h);

/* n_traj trajectories from psi0 (device complex128 [n], normalised by the
 * call) over tlist (host, strictly increasing, n_t >= 1, tlist[0] the
 * initial time) in nsteps RK4 steps.
 *   draws_dev: device double [n_traj][max_jumps + 1][2], uniform numbers in
 *              [0, 1): entry [b][j][0] is the threshold r of trajectory b's
 *              j-th waiting period, [b][j][1] the number r' that chooses the
 *              collapse operator of its j-th jump.  A trajectory that needs
 *              more than max_jumps jumps stops with status LME_EDRAWS.
 * outputs (device; each may be NULL):
 *   expect_dev:      complex128 [n_e][n_t], the mean over trajectories of
 *                    <psi|E_m|psi> / <psi|psi> (summed in trajectory order);
 *   expect_traj_dev: complex128 [n_traj][n_e][n_t], each trajectory's values
 *                    (a stopped trajectory's later values are 0);
 *   n_jumps_dev:     int32 [n_traj];
 *   jump_t_dev, jump_op_dev: double / int32 [n_traj][max_jumps], time and
 *                    collapse-operator index of every jump;
 *   status_dev:      int32 [n_traj], LME_OK, LME_EDRAWS or LME_ENONFINITE.
 * The handle owns a scratch of 64 n bytes per trajectory slot in flight (the
 * Taylor vectors of a step with a jump) and, when expect_traj_dev is NULL,
 * the per-trajectory outputs.  Asynchronous on `stream`.
 * Host-side errors: LME_EINVAL, LME_EGRID, LME_ENOTSUP, LME_ENOMEM, LME_EHIP. */
int lme_mc_evolve(lme_mc_handle h, int32_t n_t, const double *tlist, int32_t nsteps,
                  const void *psi0_dev, int32_t n_traj, const double *draws_dev,
                  int32_t max_jumps, void *expect_dev, void *expect_traj_dev,
                  int32_t *n_jumps_dev, double *jump_t_dev, int32_t *jump_op_dev,
                  int32_t *status_dev, void *stream);

/* Propagator (the propagator entry of the paper's function table,
 * Appendix A): for every instance the n^2 x n^2 matrix U_b with
 * vec(rho(t1)) = U_b vec(rho(t0)), vec row-major (element i n + j of vec is
 * rho[i][j]) and U the fixed-step RK4 map of Eq. (master_equation) in
 * opt->nsteps steps.  Column c = i n + j of U_b is the solution from the
 * basis matrix |i><j|.  The map is linear, so the n^2 Hermitian matrices
 * |a><a|, |a><b| + |b><a| and i(|b><a| - |a><b|) (a < b) are evolved
 * instead, as one batch of all instances on the Hermitian kernels, and
 * recombined: U|a><b| = (U X - i U Y)/2, U|b><a| = (U X + i U Y)/2.
 *   U_dev: device complex128, instance blocks of n_b^4 elements one after
 *          another (block b at sum_{b'<b} n_{b'}^4), each column-major:
 *          U_b[r][c] at element c n_b^2 + r of the block;
 *   status_dev: device int32 [n_inst] or NULL: the first device-detected
 *               failure among the instance's basis evolutions.
 * Needs a time-independent generator (no control terms: LME_ENOTSUP) and
 * opt->method LME_RK4; n_b <= 128.  The handle keeps the batch repeated
 * n_b^2 times.  Asynchronous on `stream`.
 * Errors: LME_EINVAL, LME_ENOTSUP, LME_ENOMEM, LME_EHIP. */
int lme_propagator(lme_handle h, const lme_options *opt, double t0, double t1, void *U_dev,
                   int32_t *status_dev, void *stream);

/* Steady state (the steadystate and propagator_steadystate entries of the
 * paper's function table, Appendix A): the density matrix rho_ss with
 * L rho_ss = 0 and Tr rho_ss = 1, as the limit of repeated propagation.
 * U = U(T) as in lme_propagator over [0, T] (opt->nsteps RK4 steps), then
 * U <- U U (complex FP64 products on the matrix cores) until, for every
 * instance, max |U_new - U_old| <= tol max |U_new| or max_squarings products
 * are done; the columns of the limit are Tr(X) rho_ss, and rho_ss is column
 * 0 (the image of |0><0|) divided by its trace.  The fixed points of the
 * RK4 map are exactly the null space of L, so the limit carries no
 * time-step error; T sets the convergence rate (the gap of L times T
 * 2^k).
 *   T > 0; max_squarings in [0, 200]; tol >= 0 (0 means 1e-12);
 *   rho_ss_dev: packed states (lme_layout), written for every instance;
 *   status_dev: device int32 [n_inst] or NULL: LME_OK (converged),
 *               LME_EMAXSTEPS (not within max_squarings; rho_ss_dev holds
 *               the last iterate) or LME_ENONFINITE;
 *   squarings: host int32 or NULL, the number of products done.
 * Synchronises `stream` once per product (the convergence test).  The
 * handle keeps two propagator sets.
 * Errors: LME_EINVAL, LME_ENOTSUP, LME_ENOMEM, LME_EHIP. */
int lme_steadystate(lme_handle h, const lme_options *opt, double T, int32_t max_squarings,
                    double tol, void *rho_ss_dev, int32_t *status_dev, int32_t *squarings,
                    void *stream);

#ifdef __cplusplus
}
#endif
#endif
