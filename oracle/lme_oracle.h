/*
 * lme_oracle.h -- plain FP64 CPU oracle for Lindblad master-equation evolution.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; it is
 * called by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark, and by nothing else.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Paper: Johansson, Nation, Nori, "QuTiP: An open-source Python framework for
 * the dynamics of open quantum systems" (arXiv:1110.0573).
 *   - Lindblad equation: Sec. 3.1, Eq. (master_equation), hbar = 1 (Sec. 2,
 *     Eq. (twolevel) convention), C_n = sqrt(gamma_n) A_n.
 *   - Time-dependent Hamiltonian as a sum of terms: Sec. 4.4 (Landau-Zener
 *     callback H0 + t*H1), generalised here to H0 + sum_j u_j(t) H_j with
 *     piecewise-constant u_j.
 *   - Expectation values at the output times: Sec. 4 (odesolve with e_ops).
 *
 * Storage conventions (all arrays are host memory, owned by the caller):
 *   - complex numbers are two consecutive doubles (re, im);
 *   - a density matrix is n*n complex numbers, row-major: rho[i*n + j];
 *   - operators are CSR: row_ptr[n+1], col[nnz], val[2*nnz].
 *
 * Return codes: ORC_OK and the ORC_E* values below.
 */
#ifndef LME_ORACLE_H
#define LME_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_EINVAL = 1,          /* malformed argument                              */
  ORC_EGRID = 2,           /* output time / control edge off the RK4 grid      */
  ORC_EMAXSTEPS = 3,       /* adaptive: step budget exhausted                  */
  ORC_ESTEPUNDERFLOW = 4,  /* adaptive: step size fell below h_min             */
  ORC_ENONFINITE = 5,      /* NaN/Inf met in the state or the error norm       */
  ORC_ENOMEM = 6,
  ORC_EDRAWS = 7           /* Monte-Carlo: a trajectory used up its draws      */
};

typedef struct {
  int32_t n, nnz;
  const int32_t *row_ptr, *col;
  const double *val;               /* 2*nnz doubles */
} orc_csr;

typedef struct {
  int32_t n;
  orc_csr H0;
  int32_t n_ctrl;  const orc_csr *Hc;   /* control Hamiltonians H_j            */
  int32_t n_c;     const orc_csr *C;    /* collapse operators C_k              */
  int32_t n_e;     const orc_csr *E;    /* expectation operators               */
  int32_t n_seg;   const double *edges; /* n_seg+1 increasing times            */
  const double *u;                      /* u[j*n_seg + s]: amplitude of H_j on
                                           [edges[s], edges[s+1])            */
  const double *fn;                     /* NULL, or fn[7*j .. 7*j+6] =
                                           (c0, c1, c2, c3, a, w, phi): the
                                           amplitude of H_j is the function
                                           c0 + c1 t + c2 t^2 + c3 t^3
                                           + a cos(w t + phi) (segments then
                                           unused)                           */
} orc_system;

/* out = L(t) y, the right-hand side of the Lindblad equation. */
int orc_apply_L(const orc_system *s, double t, const double *y, double *out);
/* out = L(t)^dagger x, adjoint w.r.t. the Hilbert-Schmidt inner product. */
int orc_apply_Ldag(const orc_system *s, double t, const double *x, double *out);
/* Tr(E_m rho) for every expectation operator; out[2*m], out[2*m+1]. */
int orc_expect(const orc_system *s, const double *rho, double *out);

/* Classic fixed-step RK4 from tlist[0] to tlist[n_t-1] in nsteps equal steps.
 * Piecewise-constant amplitudes: every stage of a step uses the segment
 * holding the step's midpoint.  Function amplitudes (fn): each stage uses
 * the amplitudes at its own time t, t + h/2, t + h/2, t + h (the classic
 * scheme for a time-dependent right-hand side).
 * expect: [n_e][n_t] complex (may be NULL when n_e == 0);
 * states: [n_t][n*n] complex or NULL. */
int orc_rk4(const orc_system *s, const double *rho0, int32_t n_t,
            const double *tlist, int32_t nsteps, double *expect, double *states);

/* Dormand-Prince 5(4) with per-step error control; steps stop exactly on every
 * output time and control edge (ORC_EINVAL with function amplitudes).  h_log (may be NULL) receives the accepted step
 * sizes, at most h_log_cap of them.  counts[0] = accepted, counts[1] = rejected. */
int orc_dopri5(const orc_system *s, const double *rho0, int32_t n_t,
               const double *tlist, double rtol, double atol, double h0,
               double h_min, int64_t max_steps, double *expect, double *states,
               int64_t *counts, double *h_log, int64_t h_log_cap);

/* One Dormand-Prince step from (t, y) with step h: y5 = fifth-order solution,
 * err = h * sum_i (b_i - bhat_i) k_i (the embedded error estimate). */
int orc_dopri5_step(const orc_system *s, double t, double h, const double *y,
                    double *y5, double *err);

/* Fixed-step RK4 cost J = Re Tr(O rho(t1)) and its exact gradient with
 * respect to the piecewise-constant amplitudes, grad[j*n_seg + s], by the
 * discrete adjoint of the RK4 map. */
int orc_rk4_cost_grad(const orc_system *s, const double *rho0, const double *O,
                      double t0, double t1, int32_t nsteps, double *cost,
                      double *grad);

/* Monte-Carlo wave-function trajectories (Sec. 3.2, steps I-IV).
 * Each trajectory starts from psi0 (normalised here) at tlist[0] and evolves
 * under the non-Hermitian effective Hamiltonian of Eq. (heff),
 *   d psi/dt = -i H_eff psi,   H_eff = H0 - (i/2) sum_n C_n^+ C_n,
 * with classic RK4 on the grid tlist[0] + m h, h = (tlist[n_t-1] - tlist[0])
 * / nsteps (every output time on the grid).  Between grid points the
 * solution is the RK4 step of the partial length.  Random numbers are an
 * input: draws[(traj*(max_jumps+1) + j)*2 + 0] is the number r of step I for
 * the j-th waiting period, draws[... + 1] the number that chooses the
 * collapse operator of the j-th jump (step III).  A trajectory that would
 * need more than max_jumps jumps stops with ORC_EDRAWS.
 * Outputs (each may be NULL): expect_avg [n_e][n_t] complex, the mean over
 * trajectories of <psi|E|psi>/<psi|psi>; expect_traj [n_traj][n_e][n_t]
 * complex; n_jumps [n_traj]; jump_t, jump_op [n_traj][max_jumps] (time and
 * collapse-operator index of every jump); status [n_traj]. */
int orc_mc(const orc_system *s, const double *psi0, int32_t n_t, const double *tlist,
           int32_t nsteps, int32_t n_traj, const double *draws, int32_t max_jumps,
           double *expect_avg, double *expect_traj, int32_t *n_jumps, double *jump_t,
           int32_t *jump_op, int32_t *status, int32_t n_threads);

/* Two-time correlation functions by the quantum regression theorem (the
 * paper's correlation_ode, Table A1): with rho(t) the master-equation state,
 *   corr[i][m][j] = Tr( E_m V(tau_j) [ B rho(t_i) ] ),
 * V(tau) the evolution of Eq. (master_equation) over tau.  rho(t) comes from
 * orc_rk4 over tlist in nsteps steps; every B rho(t_i) is evolved by orc_rk4
 * over taulist (taulist[0] = 0, increasing) in tau_nsteps steps.  B is CSR;
 * the system must have no control terms.  corr: [n_t][n_e][n_tau] complex. */
int orc_correlation(const orc_system *s, const double *rho0, int32_t n_t, const double *tlist,
                    int32_t nsteps, int32_t n_tau, const double *taulist, int32_t tau_nsteps,
                    const orc_csr *B, double *corr);

/* Propagator (the paper's propagator, Table A1): the linear map U with
 * rho(t1) = U rho(t0), as the n^2 x n^2 matrix acting on row-major vec(rho):
 * column c = i*n + j is vec of the RK4 solution (nsteps steps) from
 * rho(t0) = |i><j|.  U: n^2 * n^2 complex, column-major (U[c*n^2 + r]). */
int orc_propagator(const orc_system *s, double t0, double t1, int32_t nsteps, double *U);

/* Steady state (the paper's steadystate, Table A1): the density matrix with
 * L rho = 0 and Tr rho = 1, from the explicit n^2 x n^2 superoperator of
 * Eq. (master_equation) (time-independent: no control terms) with the
 * trace condition in place of its first row, solved by Gaussian
 * elimination with partial pivoting.  rho: n*n complex. */
int orc_steadystate(const orc_system *s, double *rho);

/* RK4 over many independent instances on n_threads host threads (dynamic
 * scheduling); used for timing the oracle on the host. rc[b] per instance. */
int orc_rk4_batch(int32_t n_inst, const orc_system *systems,
                  const double *const *rho0, int32_t n_t, const double *tlist,
                  int32_t nsteps, double *const *expect, int32_t n_threads,
                  int32_t *rc);

#ifdef __cplusplus
}
#endif
#endif
