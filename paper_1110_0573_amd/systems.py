"""Seeded synthetic inputs shaped like the paper's example systems.

This module builds operators and initial states only (standard matrices of the
paper's operator library, Table A1: destroy, sigma-, sigma-z, tensor products)
and draws the random parameters of each workload from a numpy Generator.  It
holds none of the evolution arithmetic: both the GPU library and the CPU oracle
receive what it returns.

Conventions (fixed readings where the paper leaves them open):
  * cavity (x) qubit, basis index = 2 * photon_number + q, as in the paper's
    ``tensor(destroy(N), qeye(2))`` (Sec. 2, Jaynes-Cummings example);
  * qubit basis (g, e) = (0, 1); sigma- = |g><e|, sigma-z = |e><e| - |g><g|;
  * spin chains: site 1 is the most significant bit.

Workloads (all sizes are those of the headline configurations):
  * ``jc_single``   Jaynes-Cummings, N=10 (dim 20), fixed-step RK4, t in [0, 25],
                    2500 steps, <a^+a> and <sigma_z> at 101 times;
  * ``kerr_single`` driven damped Kerr cavity, N=60, Dormand-Prince rtol 1e-8;
  * ``jc_sweep``    4096 Jaynes-Cummings instances with cutoffs N in {5..40},
                    fixed-step RK4, 1000 steps;
  * ``jc_drive``    256 driven qubit x cavity instances (N=20), piecewise
                    constant drive on 100 segments, RK4 with 1000 steps;
  * ``tfim``        dissipative transverse-field Ising chain, 8 spins, 64
                    disorder realizations, Dormand-Prince rtol 1e-7;
  * ``trilinear``   three coupled modes of 17 states (dim 4913) for the
                    Monte-Carlo solver, with ``mc_draws`` supplying the
                    random numbers of every trajectory.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

TWO_PI = 2.0 * np.pi


# --------------------------------------------------------------------------
# standard operators (paper, Table A1)
# --------------------------------------------------------------------------

def destroy(N):
    """Bosonic annihilation operator a on N Fock states."""
    return sp.diags(np.sqrt(np.arange(1, N, dtype=np.float64)), 1,
                    shape=(N, N), format="csr").astype(np.complex128)


def qeye(N):
    return sp.identity(N, dtype=np.complex128, format="csr")


def sigmam():
    """|g><e| in the basis (g, e)."""
    return sp.csr_matrix(np.array([[0, 1], [0, 0]], dtype=np.complex128))


def sigmaz():
    """|e><e| - |g><g| in the basis (g, e)."""
    return sp.csr_matrix(np.array([[-1, 0], [0, 1]], dtype=np.complex128))


def sigmax():
    return sp.csr_matrix(np.array([[0, 1], [1, 0]], dtype=np.complex128))


def sigmay():
    return sp.csr_matrix(np.array([[0, -1j], [1j, 0]], dtype=np.complex128))


def tensor(*ops):
    out = ops[0]
    for o in ops[1:]:
        out = sp.kron(out, o, format="csr")
    return sp.csr_matrix(out, dtype=np.complex128)


def dag(m):
    return sp.csr_matrix(m.conj().T)


def ket(dim, idx):
    v = np.zeros(dim, np.complex128)
    v[idx] = 1.0
    return v


def ket2dm(psi):
    psi = np.asarray(psi, np.complex128).reshape(-1)
    return np.outer(psi, psi.conj())


def tidy(m):
    """CSR with explicit zeros removed and sorted column indices."""
    m = sp.csr_matrix(m, dtype=np.complex128)
    m.eliminate_zeros()
    m.sort_indices()
    return m


# --------------------------------------------------------------------------
# a system description understood by both the GPU binding and the oracle
# --------------------------------------------------------------------------

@dataclass
class System:
    """One open system: H(t) = H0 + sum_j u_j(t) H_ctrl[j], collapse ops C,
    expectation ops E, initial state rho0, piecewise-constant controls on
    ``edges`` with amplitudes ``u[j, seg]``."""
    H0: sp.csr_matrix
    C: list
    E: list
    rho0: np.ndarray
    H_ctrl: list = field(default_factory=list)
    edges: np.ndarray | None = None
    u: np.ndarray | None = None
    meta: dict = field(default_factory=dict)
    fn: np.ndarray | None = None    # [n_ctrl, 7] closed-form amplitudes (see coeff_fn)

    @property
    def n(self):
        return self.H0.shape[0]


@dataclass
class Workload:
    name: str
    systems: list
    tlist: np.ndarray
    method: str                 # "rk4" or "dopri5"
    nsteps: int = 0
    rtol: float = 0.0
    atol: float = 0.0
    extra: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# Jaynes-Cummings family
# --------------------------------------------------------------------------

def jc_ops(N):
    a = tensor(destroy(N), qeye(2))
    sm = tensor(qeye(N), sigmam())
    sz = tensor(qeye(N), sigmaz())
    return a, sm, sz


def jc_system(N, wc=1.0, wa=1.0, g=0.05 * TWO_PI, kappa=0.005, gamma=0.05,
              n_th=0.0, psi0=(1, 0), phase=0.0):
    """H = wc a^+a + wa sigma+sigma- + g (e^{i phase} a^+ sigma- + h.c.);
    C = sqrt(kappa(1+n_th)) a, [sqrt(kappa n_th) a^+], sqrt(gamma) sigma-;
    E = a^+a, sigma_z; rho0 = |n_photon, q><..| with psi0 = (n_photon, q)."""
    a, sm, sz = jc_ops(N)
    ad, sp_ = dag(a), dag(sm)
    cp = np.exp(1j * phase)
    H = tidy(wc * (ad @ a) + wa * (sp_ @ sm) + g * (cp * (ad @ sm) + np.conj(cp) * (a @ sp_)))
    C = [tidy(np.sqrt(kappa * (1.0 + n_th)) * a)]
    if n_th > 0:
        C.append(tidy(np.sqrt(kappa * n_th) * ad))
    C.append(tidy(np.sqrt(gamma) * sm))
    E = [tidy(ad @ a), tidy(sz)]
    dim = 2 * N
    rho0 = ket2dm(ket(dim, 2 * psi0[0] + psi0[1]))
    return System(H, C, E, rho0, meta=dict(N=N, wc=wc, wa=wa, g=g, kappa=kappa,
                                           gamma=gamma, n_th=n_th))


def jc_single():
    """Qubit x cavity, N=10, g = 0.05*2pi, kappa 0.005, gamma 0.05, rho0=|1,g>,
    RK4 over [0, 25] in 2500 steps, outputs at 101 times."""
    s = jc_system(10, wc=1.0, wa=1.0, g=0.05 * TWO_PI, kappa=0.005, gamma=0.05)
    return Workload("jc_single_N10", [s], np.linspace(0.0, 25.0, 101), "rk4",
                    nsteps=2500)


def jc_sweep(n_inst=4096, seed=3, nsteps=1000, t_end=25.0, n_out=101,
             coherent=False):
    """Parameter sweep: N ~ U{5..40}, g ~ U[0.01, 0.2]*2pi, detuning
    delta ~ U[-0.5, 0.5] (wc = 1, wa = 1 + delta), kappa, gamma log-uniform in
    [1e-3, 1e-1]; rho0 = |1, g> (or a coherent cavity state with alpha = 1
    when ``coherent``, which populates every matrix element)."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(5, 41, size=n_inst)
    gs = rng.uniform(0.01, 0.2, size=n_inst) * TWO_PI
    ds = rng.uniform(-0.5, 0.5, size=n_inst)
    ks = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), size=n_inst))
    gm = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), size=n_inst))
    systems = []
    for b in range(n_inst):
        s = jc_system(int(Ns[b]), wc=1.0, wa=1.0 + ds[b], g=gs[b], kappa=ks[b],
                      gamma=gm[b])
        if coherent:
            s.rho0 = ket2dm(np.kron(coherent_ket(int(Ns[b]), 1.0), ket(2, 1)))
        systems.append(s)
    return Workload(f"jc_sweep_{n_inst}", systems, np.linspace(0.0, t_end, n_out),
                    "rk4", nsteps=nsteps)


def coherent_ket(N, alpha):
    """Truncated coherent state, normalised in the truncated space."""
    n = np.arange(N)
    from math import lgamma
    logfact = np.array([lgamma(k + 1) for k in n])
    amp = np.exp(-0.5 * abs(alpha) ** 2 + n * np.log(abs(alpha) + 1e-300)
                 - 0.5 * logfact) * np.exp(1j * np.angle(alpha) * n)
    amp = amp.astype(np.complex128)
    return amp / np.linalg.norm(amp)


def jc_drive(n_inst=256, seed=4, N=20, n_seg=100, t_end=10.0, steps_per_seg=10,
             sigma_u=0.1):
    """Driven qubit x cavity: H0 = JC at N=20 (w = 1, g = 0.05*2pi),
    H_1 = a + a^+ with amplitudes u ~ N(0, 0.1) on n_seg equal segments,
    C = sqrt(0.005) a, sqrt(0.05) sigma-; rho0 = |0, e>; target |1, g>."""
    rng = np.random.default_rng(seed)
    u = rng.normal(0.0, sigma_u, size=(n_inst, 1, n_seg))
    a, sm, sz = jc_ops(N)
    edges = np.linspace(0.0, t_end, n_seg + 1)
    V = tidy(a + dag(a))
    systems = []
    for b in range(n_inst):
        s = jc_system(N, g=0.05 * TWO_PI, kappa=0.005, gamma=0.05, psi0=(0, 1))
        s.H_ctrl = [V]
        s.edges = edges
        s.u = u[b]
        systems.append(s)
    target = ket(2 * N, 2 * 1 + 0)
    return Workload(f"jc_drive_{n_inst}", systems, np.array([0.0, t_end]), "rk4",
                    nsteps=n_seg * steps_per_seg,
                    extra=dict(target=ket2dm(target), u=u, edges=edges,
                               ckpt_every=steps_per_seg))


# --------------------------------------------------------------------------
# Kerr cavity
# --------------------------------------------------------------------------

def kerr_single(N=60, seed=2, n_th=0.1, t_end=50.0, n_out=101):
    """H = Delta a^+a + K a^+a^+aa + E (a + a^+) with (Delta, K, E, kappa) drawn
    in that order from U[0.1, 1]; C = sqrt(kappa(1+n_th)) a, sqrt(kappa n_th) a^+;
    rho0 = vacuum; E-ops a^+a and a; Dormand-Prince rtol 1e-8, atol 1e-11."""
    rng = np.random.default_rng(seed)
    delta, K, E, kappa = rng.uniform(0.1, 1.0, size=4)
    s = kerr_system(N, delta, K, E, kappa, n_th)
    return Workload(f"kerr_N{N}", [s], np.linspace(0.0, t_end, n_out), "dopri5",
                    rtol=1e-8, atol=1e-11)


def kerr_system(N, delta, K, E, kappa, n_th=0.1):
    a = destroy(N)
    ad = dag(a)
    H = tidy(delta * (ad @ a) + K * (ad @ ad @ a @ a) + E * (a + ad))
    C = [tidy(np.sqrt(kappa * (1 + n_th)) * a), tidy(np.sqrt(kappa * n_th) * ad)]
    Eo = [tidy(ad @ a), tidy(a)]
    rho0 = ket2dm(ket(N, 0))
    return System(H, C, Eo, rho0, meta=dict(N=N, delta=delta, K=K, E=E,
                                            kappa=kappa, n_th=n_th))


# --------------------------------------------------------------------------
# dissipative transverse-field Ising chain
# --------------------------------------------------------------------------

def site_op(op, i, M):
    return tensor(*[op if k == i else qeye(2) for k in range(M)])


def tfim_system(h, J=1.0, g_minus=0.05, g_z=0.02):
    """H = -1/2 sum_i h_i sigma_x^i - 1/2 J sum_{i<M} sigma_z^i sigma_z^{i+1}
    (the paper's chain form, Eq. spinchain, with J_x = J_y = 0 and a transverse
    field); C = sqrt(g_minus) sigma-_i, sqrt(g_z) sigma_z^i; rho0 = |e g ... g>."""
    M = len(h)
    sx = [site_op(sigmax(), i, M) for i in range(M)]
    sz = [site_op(sigmaz(), i, M) for i in range(M)]
    sm = [site_op(sigmam(), i, M) for i in range(M)]
    H = sum(-0.5 * h[i] * sx[i] for i in range(M))
    H = H + sum(-0.5 * J * (sz[i] @ sz[i + 1]) for i in range(M - 1))
    C = [tidy(np.sqrt(g_minus) * sm[i]) for i in range(M)]
    C += [tidy(np.sqrt(g_z) * sz[i]) for i in range(M)]
    dim = 2 ** M
    rho0 = ket2dm(ket(dim, 1 << (M - 1)))
    return System(tidy(H), C, [tidy(z) for z in sz], rho0, meta=dict(h=list(h), J=J))


def tfim(n_inst=64, seed=5, M=8, t_end=20.0, n_out=201):
    rng = np.random.default_rng(seed)
    hs = rng.uniform(0.5, 1.5, size=(n_inst, M))
    systems = [tfim_system(hs[b]) for b in range(n_inst)]
    return Workload(f"tfim_{M}x{n_inst}", systems, np.linspace(0.0, t_end, n_out),
                    "dopri5", rtol=1e-7, atol=1e-10)


# --------------------------------------------------------------------------
# other paper examples and random small systems for tests
# --------------------------------------------------------------------------

def damped_cavity(N=5, kappa=1.0 / 0.129, n_th=0.0, n0=1):
    """Cavity H = a^+a with thermal damping (paper Sec. 3.2 example, Fig. 4)."""
    a = destroy(N)
    ad = dag(a)
    C = [tidy(np.sqrt(kappa * (1 + n_th)) * a)]
    if n_th > 0:
        C.append(tidy(np.sqrt(kappa * n_th) * ad))
    return System(tidy(ad @ a), C, [tidy(ad @ a)], ket2dm(ket(N, n0)),
                  meta=dict(kappa=kappa, n_th=n_th))


# --------------------------------------------------------------------------
# time-dependent Hamiltonians in closed form (Sec. 4.4)
# --------------------------------------------------------------------------

def coeff_fn(c0=0.0, c1=0.0, c2=0.0, c3=0.0, a=0.0, w=0.0, phi=0.0):
    """Parameters of the amplitude u(t) = c0 + c1 t + c2 t^2 + c3 t^3
    + a cos(w t + phi), in the order both sides read them."""
    return np.array([c0, c1, c2, c3, a, w, phi], np.float64)


def landau_zener(delta=0.5 * TWO_PI, v=2.0 * TWO_PI, gamma=0.0):
    """Landau-Zener two-level system (Sec. 4.4, Eq. (lz-hamiltonian)):
    H(t) = delta/2 sigma_x + (v t / 2) sigma_z, written as H0 = delta/2 sigma_x
    plus the control term sigma_z with amplitude u(t) = v t / 2; optional
    relaxation C = sqrt(gamma) sigma-.  rho0 = |0><0| (the paper's basis(2, 0),
    the first basis state); E-ops: the population of |1>, sigma_x, sigma_y,
    sigma_z (the paper's sm^+ sm, sx, sy, sz with sm = destroy(2))."""
    sm = destroy(2)
    H0 = tidy(0.5 * delta * sigmax())
    C = [tidy(np.sqrt(gamma) * sm)] if gamma > 0 else []
    E = [tidy(dag(sm) @ sm), tidy(sigmax()), tidy(sigmay()), tidy(sigmaz())]
    s = System(H0, C, E, ket2dm(ket(2, 0)), H_ctrl=[tidy(sigmaz())],
               fn=coeff_fn(c1=0.5 * v)[None, :], meta=dict(delta=delta, v=v, gamma=gamma))
    return s


def landau_zener_sweep(n_inst=4096, seed=8, t0=-10.0, t1=10.0, n_out=1500, steps_per_out=20):
    """A sweep of Landau-Zener problems: delta = 0.5 * 2pi, sweep rates v
    log-uniform in [0.5, 8] * 2pi (final-state probability from near 0 to
    near 1), relaxation gamma log-uniform in [1e-4, 1e-2]; RK4 on the paper's
    grid t in [-10, 10] with 1500 outputs, steps_per_out steps between
    outputs."""
    rng = np.random.default_rng(seed)
    vs = np.exp(rng.uniform(np.log(0.5), np.log(8.0), size=n_inst)) * TWO_PI
    gs = np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), size=n_inst))
    systems = [landau_zener(v=vs[b], gamma=gs[b]) for b in range(n_inst)]
    return Workload(f"landau_zener_{n_inst}", systems, np.linspace(t0, t1, n_out), "rk4",
                    nsteps=(n_out - 1) * steps_per_out)


def jc_correlation_sweep(n_inst=64, seed=9, n_t=26, n_tau=101):
    """First-order coherence <a^+(t + tau) a(t)> of a sweep of damped JC
    systems (the JC sweep's parameter draws, N ~ U{5..20}), rho0 = |1, g>:
    first times t on [0, 25] (n_t points), delays tau on [0, 25] (n_tau
    points), RK4 with h = 0.025 on both axes; B = a, E-ops a^+ (and a^+a,
    sigma_z kept from the JC system for context)."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(5, 21, size=n_inst)
    gs = rng.uniform(0.01, 0.2, size=n_inst) * TWO_PI
    ds = rng.uniform(-0.5, 0.5, size=n_inst)
    ks = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), size=n_inst))
    gm = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), size=n_inst))
    systems, Bs = [], []
    for b in range(n_inst):
        s = jc_system(int(Ns[b]), wc=1.0, wa=1.0 + ds[b], g=gs[b], kappa=ks[b], gamma=gm[b])
        a = jc_ops(int(Ns[b]))[0]
        s.E = [tidy(dag(a))] + s.E
        systems.append(s)
        Bs.append(tidy(a))
    return Workload(f"jc_correlation_{n_inst}", systems, np.linspace(0.0, 25.0, n_t), "rk4",
                    nsteps=1000, extra=dict(B=Bs, taulist=np.linspace(0.0, 25.0, n_tau),
                                            tau_nsteps=1000))


def jc_steady_sweep(n_inst=16, seed=10, N=16, T=10.0, nsteps=200):
    """Steady states of a sweep of thermal Jaynes-Cummings systems (the
    cavity of Sec. 3.2 at a thermal occupation, coupled to a two-level atom):
    N photon states (dimension 2N, propagators of (2N)^2 = 1024 rows for
    N = 16), wa in [0.9, 1.1], g in [0.02, 0.08] 2pi, kappa and gamma in
    [0.05, 0.2], n_th in [0.05, 0.5].  U(T) from RK4 (nsteps steps over
    [0, T]), then repeated squaring."""
    rng = np.random.default_rng(seed)
    wa = rng.uniform(0.9, 1.1, size=n_inst)
    gs = rng.uniform(0.02, 0.08, size=n_inst) * TWO_PI
    ks = rng.uniform(0.05, 0.2, size=n_inst)
    gm = rng.uniform(0.05, 0.2, size=n_inst)
    nth = rng.uniform(0.05, 0.5, size=n_inst)
    systems = [jc_system(N, wc=1.0, wa=wa[b], g=gs[b], kappa=ks[b], gamma=gm[b], n_th=nth[b])
               for b in range(n_inst)]
    return Workload(f"jc_steady_{n_inst}", systems, np.array([0.0, T]), "rk4", nsteps=nsteps)


# --------------------------------------------------------------------------
# Monte-Carlo workloads (Sec. 3.2 and Sec. 4.3)
# --------------------------------------------------------------------------

def mc_draws(n_traj, max_jumps, seed):
    """Uniform numbers in [0, 1) for the Monte-Carlo trajectories, shape
    [n_traj, max_jumps + 1, 2]: per waiting period j the norm threshold r of
    step I and the number that picks the collapse operator of the j-th jump
    (step III).  Drawn once here and handed to both the GPU and the oracle."""
    rng = np.random.default_rng(seed)
    return rng.random((n_traj, max_jumps + 1, 2))


def thermal_cavity_mc(N=5, kappa=1.0 / 0.129, n_th=0.063):
    """Single-photon cavity decay in a thermal environment (Sec. 3.2 example,
    Fig. 4): H = a^+a, C_1 = sqrt((1 + n_th) kappa) a, C_2 = sqrt(n_th kappa) a^+,
    psi0 = |1>, <a^+a> at 100 times on [0, 0.6]."""
    s = damped_cavity(N=N, kappa=kappa, n_th=n_th, n0=1)
    s.meta["psi0"] = ket(N, 1)
    return s


def trilinear(N=17, alpha=np.sqrt(10.0), g=(0.1, 0.4, 0.1)):
    """Trilinear Hamiltonian (Sec. 4.3, Eq. (trilinear), K = 1, hbar = 1):
    H = i (a b^+ c^+ - a^+ b c) on three modes of N states each (pump a,
    signal b, idler c, in that tensor order), C_k = sqrt(2 g_k) a_k,
    psi0 = |alpha> |0> |0> (coherent pump), E-ops the three number operators."""
    a0 = tensor(destroy(N), qeye(N), qeye(N))
    a1 = tensor(qeye(N), destroy(N), qeye(N))
    a2 = tensor(qeye(N), qeye(N), destroy(N))
    H = tidy(1j * (a0 @ dag(a1) @ dag(a2) - dag(a0) @ a1 @ a2))
    C = [tidy(np.sqrt(2.0 * gk) * ak) for gk, ak in zip(g, (a0, a1, a2))]
    E = [tidy(dag(ak) @ ak) for ak in (a0, a1, a2)]
    psi0 = np.kron(np.kron(coherent_ket(N, alpha), ket(N, 0)), ket(N, 0))
    s = System(H, C, E, None, meta=dict(N=N, alpha=alpha, g=g))
    s.meta["psi0"] = psi0
    return s


def trilinear_mc_workload(n_traj=1000, seed=6, max_jumps=128):
    """Sec. 4.3 trilinear Hamiltonian (N = 17, dim 4913), 1000 trajectories,
    201 outputs on [0, 4], RK4 with h = 0.004 (1000 steps; the no-jump
    propagator is reproduced to 1e-9 at this step), draws seeded."""
    s = trilinear()
    return Workload(f"trilinear_mc_{n_traj}", [s], np.linspace(0.0, 4.0, 201), "mc",
                    nsteps=1000, extra=dict(draws=mc_draws(n_traj, max_jumps, seed)))


def random_system(n, n_c=2, n_ctrl=0, n_e=2, density=0.4, seed=0, n_seg=0,
                  t_end=1.0, hermitian_rho=True):
    """Random sparse Hermitian H, general sparse C_k, random controls and a
    random density matrix (or a random non-Hermitian matrix)."""
    rng = np.random.default_rng(seed)

    def rand_sparse(herm):
        m = (rng.random((n, n)) < density) * (rng.normal(size=(n, n))
                                               + 1j * rng.normal(size=(n, n)))
        if herm:
            m = 0.5 * (m + m.conj().T)
        return tidy(m)

    H = rand_sparse(True)
    C = [tidy(0.3 * rand_sparse(False).toarray()) for _ in range(n_c)]
    E = [rand_sparse(False) for _ in range(n_e)]
    Hc = [rand_sparse(True) for _ in range(n_ctrl)]
    X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    if hermitian_rho:
        rho = X @ X.conj().T
        rho /= np.trace(rho).real
    else:
        rho = X
    s = System(H, C, E, rho, H_ctrl=Hc)
    if n_ctrl and n_seg:
        s.edges = np.linspace(0.0, t_end, n_seg + 1)
        s.u = rng.normal(size=(n_ctrl, n_seg))
    return s
