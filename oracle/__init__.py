"""Plain FP64 CPU oracle for Lindblad master-equation evolution.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package.  It shares no code with the GPU
library (``paper_1110_0573_amd``) and never imports it: systems are passed in
as plain objects with the attributes listed in :func:`_marshal`.

The numerics live in ``lme_oracle.c`` (textbook sparse-times-dense loops, see
its header for the paper passages each routine follows); this module only
builds that file with gcc and marshals numpy / scipy arrays through ctypes.

Functions without a pin of their own are marked "parity unpinned" in their
docstring; every other function is pinned by ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lme_oracle.c")
_LIBPATH = os.path.join(_HERE, "liblme_oracle.so")
_LOCK = threading.Lock()
_LIB = None

OK, EINVAL, EGRID, EMAXSTEPS, ESTEPUNDERFLOW, ENONFINITE, ENOMEM, EDRAWS = range(8)
CODE_NAMES = {0: "OK", 1: "EINVAL", 2: "EGRID", 3: "EMAXSTEPS",
              4: "ESTEPUNDERFLOW", 5: "ENONFINITE", 6: "ENOMEM", 7: "EDRAWS"}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed: {CODE_NAMES.get(code, code)}")
        self.code = code


def build(force: bool = True, path: str | None = None, native: bool = False) -> str:
    """Compile lme_oracle.c into liblme_oracle.so (gcc -O3).  The in-tree copy
    uses the generic x86-64 ISA, because it is built on one machine and loaded
    on another (the GPU host); ``native=True`` adds -march=native for a copy
    built and timed on the same host (``path``)."""
    path = path or _LIBPATH
    if not force and os.path.exists(path):
        return path
    tmp = path + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O3", "-std=c11", "-Wall", "-shared", "-fPIC"] + \
        (["-march=native"] if native else []) + ["-o", tmp, _SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, path)
    return path


def use_native_build(workdir: str) -> str:
    """Builds an -O3 -march=native copy of the oracle in ``workdir`` and makes
    every following call use it (for timing the oracle on the host it runs
    on).  Returns its path."""
    global _LIB, _LIBPATH
    path = build(path=os.path.join(workdir, "liblme_oracle_native.so"), native=True)
    with _LOCK:
        _LIB = None
        _LIBPATH = path
    _lib()
    return path


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class _System(C.Structure):
    _fields_ = [("n", C.c_int32), ("H0", _Csr),
                ("n_ctrl", C.c_int32), ("Hc", C.POINTER(_Csr)),
                ("n_c", C.c_int32), ("C", C.POINTER(_Csr)),
                ("n_e", C.c_int32), ("E", C.POINTER(_Csr)),
                ("n_seg", C.c_int32), ("edges", C.POINTER(C.c_double)),
                ("u", C.POINTER(C.c_double)), ("fn", C.POINTER(C.c_double))]


_PD = C.POINTER(C.c_double)
_PI64 = C.POINTER(C.c_int64)


def _lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(_LIBPATH) or (
                    os.path.getmtime(_LIBPATH) < os.path.getmtime(_SRC)):
                build(path=_LIBPATH)
            lib = C.CDLL(_LIBPATH)
            P = C.POINTER(_System)
            lib.orc_apply_L.argtypes = [P, C.c_double, _PD, _PD]
            lib.orc_apply_Ldag.argtypes = [P, C.c_double, _PD, _PD]
            lib.orc_expect.argtypes = [P, _PD, _PD]
            lib.orc_rk4.argtypes = [P, _PD, C.c_int32, _PD, C.c_int32, _PD, _PD]
            lib.orc_dopri5.argtypes = [P, _PD, C.c_int32, _PD, C.c_double,
                                       C.c_double, C.c_double, C.c_double,
                                       C.c_int64, _PD, _PD, _PI64, _PD, C.c_int64]
            lib.orc_dopri5_step.argtypes = [P, C.c_double, C.c_double, _PD, _PD, _PD]
            lib.orc_rk4_cost_grad.argtypes = [P, _PD, _PD, C.c_double, C.c_double,
                                              C.c_int32, _PD, _PD]
            lib.orc_mc.argtypes = [P, _PD, C.c_int32, _PD, C.c_int32, C.c_int32, _PD,
                                   C.c_int32, _PD, _PD, C.POINTER(C.c_int32), _PD,
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32]
            lib.orc_propagator.argtypes = [P, C.c_double, C.c_double, C.c_int32, _PD]
            lib.orc_steadystate.argtypes = [P, _PD]
            lib.orc_correlation.argtypes = [P, _PD, C.c_int32, _PD, C.c_int32, C.c_int32,
                                            _PD, C.c_int32, C.POINTER(_Csr), _PD]
            lib.orc_rk4_batch.argtypes = [C.c_int32, P, C.POINTER(_PD), C.c_int32,
                                          _PD, C.c_int32, C.POINTER(_PD), C.c_int32,
                                          C.POINTER(C.c_int32)]
            _LIB = lib
    return _LIB


def _dptr(a):
    return a.ctypes.data_as(_PD) if a is not None else None


class _Marshalled:
    """ctypes view of one system; keeps every numpy buffer alive."""

    def __init__(self, system, u=None):
        keep = []

        def csr(m):
            m = sp.csr_matrix(m, dtype=np.complex128)
            m.sort_indices()
            rp = np.ascontiguousarray(m.indptr, dtype=np.int32)
            ci = np.ascontiguousarray(m.indices, dtype=np.int32)
            va = np.ascontiguousarray(m.data, dtype=np.complex128).view(np.float64)
            keep.extend([rp, ci, va])
            return _Csr(m.shape[0], m.nnz, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                        ci.ctypes.data_as(C.POINTER(C.c_int32)), va.ctypes.data_as(_PD))

        def csr_array(ops):
            arr = (_Csr * max(1, len(ops)))(*[csr(o) for o in ops])
            keep.append(arr)
            return arr

        H_ctrl = list(getattr(system, "H_ctrl", []) or [])
        edges = getattr(system, "edges", None)
        if u is None:
            u = getattr(system, "u", None)
        n_seg = 0
        e_arr = u_arr = None
        if H_ctrl and edges is not None and len(edges) > 1:
            e_arr = np.ascontiguousarray(edges, dtype=np.float64)
            n_seg = len(e_arr) - 1
            u_arr = np.ascontiguousarray(
                np.zeros((len(H_ctrl), n_seg)) if u is None else u,
                dtype=np.float64).reshape(len(H_ctrl), n_seg)
            keep.extend([e_arr, u_arr])
        fn = getattr(system, "fn", None)
        fn_arr = None
        if fn is not None:
            fn_arr = np.ascontiguousarray(fn, dtype=np.float64).reshape(len(H_ctrl), 7)
            keep.append(fn_arr)
        self.n = system.H0.shape[0]
        self.n_e = len(system.E)
        self.n_ctrl = len(H_ctrl)
        self.n_seg = n_seg
        self.s = _System(self.n, csr(system.H0),
                         len(H_ctrl), csr_array(H_ctrl),
                         len(system.C), csr_array(list(system.C)),
                         len(system.E), csr_array(list(system.E)),
                         n_seg, _dptr(e_arr), _dptr(u_arr), _dptr(fn_arr))
        self.keep = keep


def _marshal(system, u=None):
    """``system`` needs: H0 (n x n sparse/dense), C (list), E (list) and,
    optionally, H_ctrl (list), edges (n_seg+1,), u (n_ctrl, n_seg), or fn
    (n_ctrl, 7): closed-form amplitudes c0 + c1 t + c2 t^2 + c3 t^3
    + a cos(w t + phi)."""
    return _Marshalled(system, u)


def _cplx(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape != shape:
        a = a.reshape(shape)
    return a


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def apply_L(system, y, t=0.0, u=None):
    """L(t) y: the Lindblad right-hand side (Eq. master_equation)."""
    m = _marshal(system, u)
    y = _cplx(y, (m.n, m.n))
    out = np.zeros((m.n, m.n), np.complex128)
    _check(_lib().orc_apply_L(C.byref(m.s), t, _dptr(y.view(np.float64)),
                              _dptr(out.view(np.float64))), "apply_L")
    return out


def apply_Ldag(system, x, t=0.0, u=None):
    """L(t)^+ x, the Hilbert-Schmidt adjoint of apply_L."""
    m = _marshal(system, u)
    x = _cplx(x, (m.n, m.n))
    out = np.zeros((m.n, m.n), np.complex128)
    _check(_lib().orc_apply_Ldag(C.byref(m.s), t, _dptr(x.view(np.float64)),
                                 _dptr(out.view(np.float64))), "apply_Ldag")
    return out


def expect(system, rho):
    """[Tr(E_m rho) for m] as complex numbers."""
    m = _marshal(system)
    rho = _cplx(rho, (m.n, m.n))
    out = np.zeros(max(1, m.n_e), np.complex128)
    _check(_lib().orc_expect(C.byref(m.s), _dptr(rho.view(np.float64)),
                             _dptr(out.view(np.float64))), "expect")
    return out[:m.n_e]


def rk4(system, rho0, tlist, nsteps, store_states=False, u=None):
    """Fixed-step classic RK4.  Returns (expect[n_e, n_t], states[n_t,n,n] or None)."""
    m = _marshal(system, u)
    rho0 = _cplx(rho0, (m.n, m.n))
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    n_t = len(tl)
    ex = np.zeros((max(1, m.n_e), n_t), np.complex128)
    st = np.zeros((n_t, m.n, m.n), np.complex128) if store_states else None
    rc = _lib().orc_rk4(C.byref(m.s), _dptr(rho0.view(np.float64)), n_t, _dptr(tl),
                        int(nsteps), _dptr(ex.view(np.float64)),
                        _dptr(st.view(np.float64)) if st is not None else None)
    _check(rc, "rk4")
    return ex[:m.n_e], st


def dopri5(system, rho0, tlist, rtol, atol, h0=0.0, h_min=0.0, max_steps=10**7,
           store_states=False, h_log_cap=0, u=None, raise_on_error=True):
    """Dormand-Prince 5(4).  Returns dict with expect, states, counts, h_log, rc."""
    m = _marshal(system, u)
    rho0 = _cplx(rho0, (m.n, m.n))
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    n_t = len(tl)
    ex = np.zeros((max(1, m.n_e), n_t), np.complex128)
    st = np.zeros((n_t, m.n, m.n), np.complex128) if store_states else None
    counts = np.zeros(2, np.int64)
    hl = np.zeros(max(1, h_log_cap), np.float64)
    rc = _lib().orc_dopri5(C.byref(m.s), _dptr(rho0.view(np.float64)), n_t, _dptr(tl),
                           rtol, atol, h0, h_min, int(max_steps),
                           _dptr(ex.view(np.float64)),
                           _dptr(st.view(np.float64)) if st is not None else None,
                           counts.ctypes.data_as(_PI64), _dptr(hl), int(h_log_cap))
    if raise_on_error:
        _check(rc, "dopri5")
    nl = min(int(counts[0]), h_log_cap)
    return {"expect": ex[:m.n_e], "states": st, "counts": counts, "h_log": hl[:nl],
            "rc": rc}


def dopri5_step(system, y, t, h, u=None):
    """One Dormand-Prince step: (fifth-order y5, embedded error vector)."""
    m = _marshal(system, u)
    y = _cplx(y, (m.n, m.n))
    y5 = np.zeros((m.n, m.n), np.complex128)
    err = np.zeros((m.n, m.n), np.complex128)
    _check(_lib().orc_dopri5_step(C.byref(m.s), t, h, _dptr(y.view(np.float64)),
                                  _dptr(y5.view(np.float64)),
                                  _dptr(err.view(np.float64))), "dopri5_step")
    return y5, err


def rk4_cost_grad(system, rho0, O, t0, t1, nsteps, u=None):
    """J = Re Tr(O rho(t1)) under fixed-step RK4 and dJ/du[j, seg] (discrete adjoint)."""
    m = _marshal(system, u)
    rho0 = _cplx(rho0, (m.n, m.n))
    O = _cplx(O, (m.n, m.n))
    cost = np.zeros(1, np.float64)
    grad = np.zeros((max(1, m.n_ctrl), max(1, m.n_seg)), np.float64)
    _check(_lib().orc_rk4_cost_grad(C.byref(m.s), _dptr(rho0.view(np.float64)),
                                    _dptr(O.view(np.float64)), t0, t1, int(nsteps),
                                    _dptr(cost), _dptr(grad)), "rk4_cost_grad")
    return float(cost[0]), grad[:m.n_ctrl, :m.n_seg]


def rk4_batch(systems, rho0s, tlist, nsteps, n_threads):
    """RK4 over many instances on n_threads host threads.  Returns list of expect arrays."""
    ms = [_marshal(s) for s in systems]
    B = len(ms)
    arr = (_System * max(1, B))(*[m.s for m in ms])
    rhos = [_cplx(r, (m.n, m.n)) for r, m in zip(rho0s, ms)]
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    n_t = len(tl)
    exs = [np.zeros((max(1, m.n_e), n_t), np.complex128) for m in ms]
    rho_p = (_PD * max(1, B))(*[_dptr(r.view(np.float64)) for r in rhos])
    ex_p = (_PD * max(1, B))(*[_dptr(e.view(np.float64)) for e in exs])
    rc = np.zeros(max(1, B), np.int32)
    worst = _lib().orc_rk4_batch(B, arr, rho_p, n_t, _dptr(tl), int(nsteps), ex_p,
                                 int(n_threads), rc.ctypes.data_as(C.POINTER(C.c_int32)))
    _check(worst, "rk4_batch")
    return [e[:m.n_e] for e, m in zip(exs, ms)]


def mc(system, psi0, tlist, nsteps, draws, n_threads=1, raise_on_error=True):
    """Monte-Carlo wave-function trajectories (Sec. 3.2, steps I-IV), one per
    row of ``draws`` ([n_traj, max_jumps + 1, 2] uniform numbers: the norm
    threshold r of each waiting period and the number that picks the
    collapse operator of each jump).  Fixed-step RK4 on the effective
    Hamiltonian of Eq. (heff); jump times located on the RK4 step of partial
    length by bisection.  Returns a dict: expect (mean over trajectories,
    [n_e, n_t]), expect_traj [n_traj, n_e, n_t], n_jumps, jump_t, jump_op
    ([n_traj, max_jumps]), status [n_traj], rc."""
    m = _marshal(system)
    psi0 = np.ascontiguousarray(np.asarray(psi0, np.complex128).reshape(m.n))
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    n_t = len(tl)
    draws = np.ascontiguousarray(draws, dtype=np.float64)
    n_traj, mj1 = draws.shape[0], draws.shape[1]
    assert draws.shape == (n_traj, mj1, 2)
    max_jumps = mj1 - 1
    ne = max(1, m.n_e)
    avg = np.zeros((ne, n_t), np.complex128)
    per = np.zeros((n_traj, ne, n_t), np.complex128)
    nj = np.zeros(n_traj, np.int32)
    jt = np.zeros((n_traj, max(1, max_jumps)), np.float64)
    jo = np.full((n_traj, max(1, max_jumps)), -1, np.int32)
    st = np.zeros(n_traj, np.int32)
    PI = C.POINTER(C.c_int32)
    rc = _lib().orc_mc(C.byref(m.s), _dptr(psi0.view(np.float64)), n_t, _dptr(tl), int(nsteps),
                       n_traj, _dptr(draws), max_jumps, _dptr(avg.view(np.float64)),
                       _dptr(per.view(np.float64)), nj.ctypes.data_as(PI), _dptr(jt),
                       jo.ctypes.data_as(PI), st.ctypes.data_as(PI), int(n_threads))
    if raise_on_error:
        _check(rc, "mc")
    return {"expect": avg[:m.n_e], "expect_traj": per[:, :m.n_e], "n_jumps": nj,
            "jump_t": jt[:, :max_jumps], "jump_op": jo[:, :max_jumps], "status": st, "rc": rc}


def correlation(system, rho0, tlist, nsteps, taulist, tau_nsteps, B):
    """Two-time correlations by the quantum regression theorem:
    corr[i, m, j] = Tr(E_m V(tau_j)[B rho(t_i)]), rho(t) and V from RK4
    (nsteps over tlist, tau_nsteps over taulist, taulist[0] = 0)."""
    m = _marshal(system)
    rho0 = _cplx(rho0, (m.n, m.n))
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    ta = np.ascontiguousarray(taulist, dtype=np.float64)
    Bm = sp.csr_matrix(B, dtype=np.complex128)
    Bm.sort_indices()
    rp = np.ascontiguousarray(Bm.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(Bm.indices, dtype=np.int32)
    va = np.ascontiguousarray(Bm.data, dtype=np.complex128).view(np.float64)
    Bc = _Csr(m.n, Bm.nnz, rp.ctypes.data_as(C.POINTER(C.c_int32)),
              ci.ctypes.data_as(C.POINTER(C.c_int32)), va.ctypes.data_as(_PD))
    out = np.zeros((len(tl), max(1, m.n_e), len(ta)), np.complex128)
    _check(_lib().orc_correlation(C.byref(m.s), _dptr(rho0.view(np.float64)), len(tl), _dptr(tl),
                                  int(nsteps), len(ta), _dptr(ta), int(tau_nsteps), C.byref(Bc),
                                  _dptr(out.view(np.float64))), "correlation")
    return out[:, :m.n_e]


def propagator(system, t0, t1, nsteps):
    """U with vec(rho(t1)) = U vec(rho(t0)) (row-major vec), from RK4 on each
    basis matrix; returned as an n^2 x n^2 array."""
    m = _marshal(system)
    N = m.n * m.n
    U = np.zeros((N, N), np.complex128)          # column-major storage: U.T here
    _check(_lib().orc_propagator(C.byref(m.s), float(t0), float(t1), int(nsteps),
                                 _dptr(U.view(np.float64))), "propagator")
    return U.T.copy()


def steadystate(system):
    """The density matrix with L rho = 0 and Tr rho = 1 (Gaussian elimination
    on the explicit superoperator with the trace condition)."""
    m = _marshal(system)
    rho = np.zeros((m.n, m.n), np.complex128)
    _check(_lib().orc_steadystate(C.byref(m.s), _dptr(rho.view(np.float64))), "steadystate")
    return rho
