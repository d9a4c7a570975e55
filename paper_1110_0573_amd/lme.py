"""Thin ctypes binding of liblme.so (include/lme.h).

Argument marshalling only: every step of the integration runs in the HIP
kernels of liblme.so.  PyTorch provides device memory and the current stream.
There is no fallback: if liblme.so is missing or no GPU is present, the calls
raise.
"""
from __future__ import annotations

import ctypes as C
import ctypes as C_
import os

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "liblme.so")

LME_OK, LME_EINVAL, LME_EGRID, LME_EMAXSTEPS, LME_ESTEPUNDERFLOW, LME_ENONFINITE, \
    LME_ENOMEM, LME_EHIP, LME_ENOTSUP, LME_ENOTHERM, LME_EDRAWS = range(11)
STATUS_NAMES = {0: "LME_OK", 1: "LME_EINVAL", 2: "LME_EGRID", 3: "LME_EMAXSTEPS",
                4: "LME_ESTEPUNDERFLOW", 5: "LME_ENONFINITE", 6: "LME_ENOMEM",
                7: "LME_EHIP", 8: "LME_ENOTSUP", 9: "LME_ENOTHERM", 10: "LME_EDRAWS"}
LME_RK4, LME_DOPRI5 = 0, 1
LME_PATH_AUTO, LME_PATH_RESIDENT, LME_PATH_STREAMED = 0, 1, 2
LME_FORM_OPERATOR, LME_FORM_SUPEROP, LME_FORM_OPERATOR_STREAMED = 0, 1, 2
LME_LAYOUT_AUTO, LME_LAYOUT_ROW, LME_LAYOUT_COLUMN = 0, 1, 2

# every symbol include/lme.h declares
EXPORTS = ["lme_default_options", "lme_create_batch", "lme_create", "lme_destroy",
           "lme_last_error", "lme_layout", "lme_evolve", "lme_evolve_noalloc", "lme_apply",
           "lme_set_coeff_fn", "lme_correlation", "lme_propagator", "lme_steadystate",
           "lme_cost_grad", "lme_get_tuning", "lme_set_tuning", "lme_autotune",
           "lme_mc_create", "lme_mc_destroy", "lme_mc_evolve"]


class LmeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class Instance(C.Structure):
    _fields_ = [("H0", C.POINTER(Csr)), ("H_ctrl", C.POINTER(Csr)), ("n_c", C.c_int32),
                ("C", C.POINTER(Csr)), ("E", C.POINTER(Csr))]


class Segments(C.Structure):
    _fields_ = [("n_seg", C.c_int32), ("edges", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("method", C.c_int32), ("path", C.c_int32), ("nsteps", C.c_int32),
                ("block", C.c_int32), ("layout", C.c_int32), ("rtol", C.c_double), ("atol", C.c_double),
                ("h0", C.c_double), ("h_min", C.c_double), ("max_steps", C.c_int64),
                ("hermitian", C.c_int32), ("reserved", C.c_int32)]


_LIB = None
_PD = C.POINTER(C.c_double)


def load():
    """Loads liblme.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with "
                               "`python -m paper_1110_0573_amd.build`")
        lib = C.CDLL(LIBPATH)
        H = C.c_void_p
        lib.lme_default_options.argtypes = [C.POINTER(Options)]
        lib.lme_default_options.restype = None
        lib.lme_create_batch.argtypes = [C.c_int32, C.POINTER(Instance), C.c_int32, C.c_int32,
                                         C.POINTER(Segments), _PD, C.POINTER(H)]
        lib.lme_create.argtypes = [C.POINTER(Csr), C.c_int32, C.POINTER(Csr),
                                   C.POINTER(Segments), _PD, C.c_int32, C.POINTER(Csr),
                                   C.c_int32, C.POINTER(Csr), C.POINTER(H)]
        lib.lme_set_coeff_fn.argtypes = [H, _PD]
        lib.lme_correlation.argtypes = [H, C.POINTER(Options), C.c_int32, _PD, C.c_int32, _PD,
                                        C.c_int32, C.POINTER(Csr), C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
        lib.lme_propagator.argtypes = [H, C.POINTER(Options), C.c_double, C.c_double,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
        lib.lme_steadystate.argtypes = [H, C.POINTER(Options), C.c_double, C.c_int32,
                                        C.c_double, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_int32), C.c_void_p]
        lib.lme_destroy.argtypes = [H]
        lib.lme_destroy.restype = None
        lib.lme_last_error.argtypes = []
        lib.lme_last_error.restype = C.c_char_p
        lib.lme_layout.argtypes = [H, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        lib.lme_evolve.argtypes = [H, C.POINTER(Options), C.c_int32, _PD, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
        lib.lme_evolve_noalloc.argtypes = lib.lme_evolve.argtypes
        lib.lme_apply.argtypes = [H, C.c_int32, C.c_int32, C.c_double, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]
        lib.lme_cost_grad.argtypes = [H, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]
        lib.lme_get_tuning.argtypes = [H, C.POINTER(Tuning)]
        lib.lme_set_tuning.argtypes = [H, C.POINTER(Tuning)]
        lib.lme_autotune.argtypes = [H, C.POINTER(Options), C.c_void_p, C.c_void_p,
                                     C.POINTER(Tuning)]
        lib.lme_mc_create.argtypes = [C.POINTER(Csr), C.c_int32, C.POINTER(Csr), C.c_int32,
                                      C.POINTER(Csr), C.POINTER(H)]
        lib.lme_mc_destroy.argtypes = [H]
        lib.lme_mc_destroy.restype = None
        lib.lme_mc_evolve.argtypes = [H, C.c_int32, _PD, C.c_int32, C.c_void_p, C.c_int32,
                                      C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _LIB = lib
    return _LIB


def _check(rc, what):
    if rc != LME_OK:
        raise LmeError(rc, f"{what}: {load().lme_last_error().decode()}")


def default_options(**kw):
    o = Options()
    load().lme_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Tuning(C.Structure):
    _fields_ = [("rk4_layout", C.c_int32), ("rk4_block", C.c_int32), ("apply_cap", C.c_int32),
                ("apply_lds_kb", C.c_int32), ("rk4_ms_per_step", C.c_double),
                ("apply_us", C.c_double), ("herm_layout", C.c_int32), ("herm_block", C.c_int32),
                ("herm_ms_per_step", C.c_double), ("apply_block", C.c_int32),
                ("apply_path", C.c_int32), ("grad_layout", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _CsrKeep:
    """Builds an lme_csr view of a scipy matrix and keeps its arrays alive."""

    def __init__(self):
        self.keep = []

    def csr(self, m):
        m = sp.csr_matrix(m, dtype=np.complex128)
        m.sort_indices()
        rp = np.ascontiguousarray(m.indptr, np.int32)
        ci = np.ascontiguousarray(m.indices, np.int32)
        va = np.ascontiguousarray(m.data, np.complex128).view(np.float64)
        self.keep += [rp, ci, va]
        return Csr(m.shape[0], m.nnz, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                   ci.ctypes.data_as(C.POINTER(C.c_int32)), va.ctypes.data_as(_PD))

    def array(self, ops):
        arr = (Csr * max(1, len(ops)))(*[self.csr(o) for o in ops])
        self.keep.append(arr)
        return arr


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_tensor(t, dtype, numel, what, optional=False):
    """Raises LmeError(LME_EINVAL) unless ``t`` is a contiguous device tensor
    of ``dtype`` with exactly ``numel`` elements: the library cannot see the
    size of a device buffer, so every buffer is checked here before its
    pointer crosses the C ABI."""
    import torch
    if t is None:
        if optional:
            return
        raise LmeError(LME_EINVAL, f"{what} is missing")
    if not isinstance(t, torch.Tensor):
        raise LmeError(LME_EINVAL, f"{what} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise LmeError(LME_EINVAL, f"{what} has dtype {t.dtype}, expected {dtype}")
    if t.numel() != numel:
        raise LmeError(LME_EINVAL, f"{what} has {t.numel()} elements, expected {numel}")
    if not t.is_contiguous():
        raise LmeError(LME_EINVAL, f"{what} must be contiguous")
    if not t.is_cuda:
        raise LmeError(LME_EINVAL, f"{what} must be a device tensor, got device {t.device}")


class Handle:
    """A batch of systems uploaded to the current GPU (lme_create_batch).

    ``systems`` is a list of objects with attributes H0, C, E and optionally
    H_ctrl, edges, u (see :class:`paper_1110_0573_amd.systems.System`).  All
    systems must share the number of control and expectation operators and,
    with controls, the segment edges."""

    def __init__(self, systems):
        lib = load()
        keep = _CsrKeep()
        n_inst = len(systems)
        n_ctrl = len(getattr(systems[0], "H_ctrl", []) or [])
        n_e = len(systems[0].E)
        edges = getattr(systems[0], "edges", None) if n_ctrl else None
        insts = (Instance * n_inst)()
        for b, s in enumerate(systems):
            H0 = keep.array([s.H0])
            insts[b] = Instance(C.cast(H0, C.POINTER(Csr)),
                                C.cast(keep.array(list(getattr(s, "H_ctrl", []) or [])),
                                       C.POINTER(Csr)),
                                len(s.C), C.cast(keep.array(list(s.C)), C.POINTER(Csr)),
                                C.cast(keep.array(list(s.E)), C.POINTER(Csr)))
        seg = None
        u_host = None
        self.n_seg = 0
        if edges is not None and n_ctrl:
            e = np.ascontiguousarray(edges, np.float64)
            keep.keep.append(e)
            self.n_seg = len(e) - 1
            seg = Segments(self.n_seg, e.ctypes.data_as(_PD))
            u = np.zeros((n_inst, n_ctrl, self.n_seg))
            for b, s in enumerate(systems):
                if getattr(s, "u", None) is not None:
                    u[b] = np.asarray(s.u).reshape(n_ctrl, self.n_seg)
            u_host = np.ascontiguousarray(u)
            keep.keep.append(u_host)
        h = C.c_void_p()
        rc = lib.lme_create_batch(n_inst, insts, n_ctrl, n_e,
                                  C.byref(seg) if seg is not None else None,
                                  u_host.ctypes.data_as(_PD) if u_host is not None else None,
                                  C.byref(h))
        _check(rc, "lme_create_batch")
        self._h = h
        self.n_inst, self.n_ctrl, self.n_e = n_inst, n_ctrl, n_e
        ni = C.c_int32()
        tot = C.c_int64()
        self.offsets = np.zeros(n_inst, np.int64)
        self.dims = np.zeros(n_inst, np.int32)
        _check(lib.lme_layout(h, C.byref(ni), C.byref(tot),
                              self.offsets.ctypes.data_as(C.POINTER(C.c_int64)),
                              self.dims.ctypes.data_as(C.POINTER(C.c_int32))), "lme_layout")
        self.state_elems = int(tot.value)
        fns = [getattr(s, "fn", None) for s in systems]
        if n_ctrl and any(f is not None for f in fns):
            if any(f is None for f in fns):
                raise LmeError(LME_EINVAL, "closed-form amplitudes must be given for every "
                                           "instance or none")
            self.set_coeff_fn(np.stack([np.asarray(f, np.float64).reshape(n_ctrl, 7)
                                        for f in fns]))

    def set_coeff_fn(self, fn):
        """lme_set_coeff_fn: fn [n_inst, n_ctrl, 7] = (c0, c1, c2, c3, a, w,
        phi) per control term, u(t) = c0 + c1 t + c2 t^2 + c3 t^3
        + a cos(w t + phi); None returns to the piecewise-constant segments."""
        if fn is None:
            _check(load().lme_set_coeff_fn(self._h, None), "lme_set_coeff_fn")
            return
        arr = np.ascontiguousarray(fn, np.float64)
        if arr.size != self.n_inst * self.n_ctrl * 7:
            raise LmeError(LME_EINVAL, f"fn has {arr.size} values, expected "
                                       f"{self.n_inst * self.n_ctrl * 7}")
        _check(load().lme_set_coeff_fn(self._h, arr.ctypes.data_as(_PD)), "lme_set_coeff_fn")

    def close(self):
        if getattr(self, "_h", None):
            load().lme_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks (before any pointer reaches the C ABI) ---------------
    def _check_state(self, t, what):
        import torch
        _check_tensor(t, torch.complex128, self.state_elems, what)

    def _check_u(self, u):
        import torch
        if u is not None and self.n_ctrl * self.n_seg == 0:
            raise LmeError(LME_EINVAL, "u given but the batch has no control segments")
        _check_tensor(u, torch.float64, self.n_inst * self.n_ctrl * self.n_seg, "u",
                      optional=True)

    # -- packed state helpers (marshalling only) ------------------------------
    def pack(self, mats, device="cuda"):
        import torch
        buf = np.zeros(self.state_elems, np.complex128)
        for b, m in enumerate(mats):
            n = int(self.dims[b])
            buf[self.offsets[b]:self.offsets[b] + n * n] = np.asarray(m, np.complex128).reshape(-1)
        return torch.from_numpy(buf).to(device)

    def unpack(self, t):
        a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
        out = []
        for b in range(self.n_inst):
            n = int(self.dims[b])
            out.append(a[..., self.offsets[b]:self.offsets[b] + n * n].reshape(a.shape[:-1] + (n, n)))
        return out

    # -- entry points ----------------------------------------------------------
    def evolve(self, rho0, tlist, method="rk4", nsteps=0, rtol=1e-6, atol=1e-9, h0=0.0,
               h_min=0.0, max_steps=10**7, path=LME_PATH_AUTO, block=0, layout=0, u=None,
               want_expect=True, want_states=False, want_rho=True, hermitian=False,
               stream=None, noalloc=False):
        """Runs lme_evolve (lme_evolve_noalloc with ``noalloc``).  rho0:
        complex128 device tensor [state_elems].  hermitian: rho0 is Hermitian
        (options.hermitian).
        Returns a dict of device tensors (expect, states, rho, counts, status)."""
        import torch
        self._check_state(rho0, "rho0")
        self._check_u(u)
        dev = rho0.device
        tl = np.ascontiguousarray(tlist, np.float64)
        n_t = len(tl)
        opt = default_options(method=LME_RK4 if method == "rk4" else LME_DOPRI5,
                              path=path, nsteps=int(nsteps), block=int(block),
                              layout=int(layout), rtol=rtol,
                              atol=atol, h0=h0, h_min=h_min, max_steps=int(max_steps),
                              hermitian=1 if hermitian else 0)
        out = {}
        out["expect"] = (torch.zeros((self.n_inst, self.n_e, n_t), dtype=torch.complex128,
                                     device=dev) if want_expect and self.n_e else None)
        out["states"] = (torch.zeros((n_t, self.state_elems), dtype=torch.complex128,
                                     device=dev) if want_states else None)
        out["rho"] = (torch.zeros(self.state_elems, dtype=torch.complex128, device=dev)
                      if want_rho else None)
        out["counts"] = torch.zeros((self.n_inst, 2), dtype=torch.int64, device=dev)
        out["status"] = torch.full((self.n_inst,), -1, dtype=torch.int32, device=dev)
        fn = load().lme_evolve_noalloc if noalloc else load().lme_evolve
        rc = fn(self._h, C.byref(opt), n_t, tl.ctypes.data_as(_PD),
                _ptr(rho0), _ptr(u), _ptr(out["expect"]), _ptr(out["states"]),
                _ptr(out["rho"]), _ptr(out["counts"]), _ptr(out["status"]),
                _stream_ptr(stream))
        _check(rc, "lme_evolve_noalloc" if noalloc else "lme_evolve")
        return out

    def autotune(self, rho0, nsteps, hermitian=False, stream=None):
        """lme_autotune: picks the fastest schedule for this batch; returns it."""
        self._check_state(rho0, "rho0")
        t = Tuning()
        opt = default_options(method=LME_RK4, nsteps=int(nsteps),
                              hermitian=1 if hermitian else 0)
        _check(load().lme_autotune(self._h, C.byref(opt), _ptr(rho0), _stream_ptr(stream),
                                   C.byref(t)), "lme_autotune")
        return t.as_dict()

    def get_tuning(self):
        t = Tuning()
        _check(load().lme_get_tuning(self._h, C.byref(t)), "lme_get_tuning")
        return t

    def set_tuning(self, **kw):
        t = self.get_tuning()
        for k, v in kw.items():
            setattr(t, k, v)
        _check(load().lme_set_tuning(self._h, C.byref(t)), "lme_set_tuning")

    def correlation(self, rho0, tlist, nsteps, taulist, tau_nsteps, B, hermitian=False,
                    stream=None):
        """lme_correlation: corr[b, i, m, j] = Tr(E_m V(tau_j)[B_b rho_b(t_i)])
        (quantum regression theorem).  B: one matrix per instance (or one for
        all).  Returns (corr device tensor [n_inst, n_t, n_e, n_tau], status)."""
        import torch
        self._check_state(rho0, "rho0")
        tl = np.ascontiguousarray(tlist, np.float64)
        ta = np.ascontiguousarray(taulist, np.float64)
        Bs = list(B) if isinstance(B, (list, tuple)) else [B] * self.n_inst
        if len(Bs) != self.n_inst:
            raise LmeError(LME_EINVAL, f"{len(Bs)} B matrices for {self.n_inst} instances")
        keep = _CsrKeep()
        Barr = keep.array([sp.csr_matrix(b, dtype=np.complex128) for b in Bs])
        opt = default_options(method=LME_RK4, nsteps=int(nsteps),
                              hermitian=1 if hermitian else 0)
        corr = torch.zeros((self.n_inst, len(tl), self.n_e, len(ta)), dtype=torch.complex128,
                           device=rho0.device)
        status = torch.full((self.n_inst,), -1, dtype=torch.int32, device=rho0.device)
        rc = load().lme_correlation(self._h, C.byref(opt), len(tl), tl.ctypes.data_as(_PD),
                                    len(ta), ta.ctypes.data_as(_PD), int(tau_nsteps),
                                    C.cast(Barr, C.POINTER(Csr)), _ptr(rho0), _ptr(corr),
                                    _ptr(status), _stream_ptr(stream))
        _check(rc, "lme_correlation")
        return corr, status

    def propagator(self, t0, t1, nsteps, device="cuda", stream=None):
        """lme_propagator: the RK4 maps U_b (vec(rho(t1)) = U_b vec(rho(t0)),
        row-major vec) of every instance.  Returns ([U_b as n^2 x n^2 device
        tensors], status)."""
        import torch
        sizes = [int(n) ** 4 for n in self.dims]
        flat = torch.empty(sum(sizes), dtype=torch.complex128, device=device)
        status = torch.full((self.n_inst,), -1, dtype=torch.int32, device=device)
        opt = default_options(method=LME_RK4, nsteps=int(nsteps))
        rc = load().lme_propagator(self._h, C.byref(opt), float(t0), float(t1), _ptr(flat),
                                   _ptr(status), _stream_ptr(stream))
        _check(rc, "lme_propagator")
        out, o = [], 0
        for n, sz in zip(self.dims, sizes):
            N = int(n) ** 2
            out.append(flat[o:o + sz].view(N, N).t())   # stored column-major
            o += sz
        return out, status

    def steadystate(self, T, nsteps, max_squarings=60, tol=1e-12, device="cuda", stream=None):
        """lme_steadystate: rho_ss of every instance as the limit of U(T)^(2^k).
        Returns (packed rho_ss device tensor, status, number of products)."""
        import torch
        rho = torch.empty(self.state_elems, dtype=torch.complex128, device=device)
        status = torch.full((self.n_inst,), -1, dtype=torch.int32, device=device)
        k = C.c_int32(-1)
        opt = default_options(method=LME_RK4, nsteps=int(nsteps))
        rc = load().lme_steadystate(self._h, C.byref(opt), float(T), int(max_squarings),
                                    float(tol), _ptr(rho), _ptr(status), C.byref(k),
                                    _stream_ptr(stream))
        _check(rc, "lme_steadystate")
        return rho, status, k.value

    def apply(self, y, t=0.0, adjoint=False, form=LME_FORM_OPERATOR, u=None, stream=None):
        """out = L(t) y (or L^+ y) for every instance of the packed batch."""
        import torch
        self._check_state(y, "y")
        self._check_u(u)
        out = torch.empty(self.state_elems, dtype=torch.complex128, device=y.device)
        rc = load().lme_apply(self._h, form, 1 if adjoint else 0, float(t), _ptr(u), _ptr(y),
                              _ptr(out), _stream_ptr(stream))
        _check(rc, "lme_apply")
        return out


class _Spec:
    """One system for :func:`evolve` (the attributes Handle reads)."""

    def __init__(self, H0, C, E, H_ctrl=(), edges=None, u=None, fn=None):
        self.H0, self.C, self.E = H0, list(C), list(E)
        self.H_ctrl, self.edges, self.u, self.fn = list(H_ctrl), edges, u, fn


def evolve(H0, c_ops, rho0, tlist, e_ops, controls=None, method="rk4", nsteps=None,
           rtol=1e-6, atol=None, hermitian=None, device="cuda"):
    """Master-equation evolution of one system on the GPU, in the calling
    convention of the paper's solver (Sec. 4: Hamiltonian, initial state, times,
    collapse and expectation operators; tlist[0] is the initial time and is
    part of the output).

    H0, c_ops, e_ops: square matrices (NumPy or SciPy sparse).  rho0: a ket
    (converted to |psi><psi|) or a density matrix.  controls: optional
    (H_ctrl list, edges[n_seg + 1], u[n_ctrl][n_seg]) for piecewise-constant
    u_j(t), or (H_ctrl list, fn[n_ctrl][7]) for closed-form amplitudes
    c0 + c1 t + c2 t^2 + c3 t^3 + a cos(w t + phi) (Sec. 4.4: e.g. the
    Landau-Zener sweep, H_ctrl = [v/2 sigma_z] with fn = [(0, 1, 0, ...)]).  method "rk4" takes nsteps equal steps over [tlist[0], tlist[-1]]
    (every output time on that grid); "dopri5" adapts its steps to rtol/atol
    (atol defaults to 1e-3 rtol).  hermitian: use the Hermitian RK4 path
    (default: whenever rho0 is Hermitian).

    Returns expectation values [len(e_ops)][len(tlist)] (real for Hermitian
    e_ops, complex otherwise); with no e_ops, the states rho(t) instead, as
    an array [len(tlist)][n][n]."""
    import torch

    def m(a):
        return sp.csr_matrix(a, dtype=np.complex128)

    H0 = m(H0)
    n = H0.shape[0]
    r = np.asarray(rho0.toarray() if sp.issparse(rho0) else rho0, np.complex128)
    if r.ndim == 1 or 1 in r.shape:
        psi = r.reshape(-1)
        r = np.outer(psi, psi.conj())
    if r.shape != (n, n):
        raise LmeError(LME_EINVAL, f"rho0 has shape {r.shape}, expected ({n}, {n})")
    E = [m(e) for e in e_ops]
    want_states = len(E) == 0
    if want_states:  # the batch needs one expectation operator; its values are dropped
        E = [sp.identity(n, dtype=np.complex128, format="csr")]
    fn = None
    if controls is None:
        hc, edges, u = (), None, None
    elif len(controls) == 2:      # (H_ctrl, fn[n_ctrl][7]): closed-form amplitudes
        hc, fn = controls
        edges, u = None, None
        fn = np.asarray(fn, np.float64).reshape(len(hc), 7)
    else:
        hc, edges, u = controls
    spec = _Spec(H0, [m(c) for c in c_ops], E, [m(x) for x in hc], edges,
                 None if u is None else np.asarray(u, np.float64), fn)
    tlist = np.asarray(tlist, np.float64)
    if method == "rk4" and nsteps is None:
        raise LmeError(LME_EINVAL, "rk4 needs nsteps")
    if hermitian is None:
        hermitian = method == "rk4" and np.array_equal(r, r.conj().T)
    h = Handle([spec])
    try:
        y = h.pack([r], device=device)
        out = h.evolve(y, tlist, method=method, nsteps=nsteps or 0, rtol=rtol,
                       atol=1e-3 * rtol if atol is None else atol, hermitian=bool(hermitian),
                       want_states=want_states)
        torch.cuda.synchronize()
        st = int(out["status"].cpu().numpy()[0])
        if st != 0:
            raise LmeError(st, f"evolve: instance status {STATUS_NAMES.get(st, st)}")
        if want_states:
            return np.stack([h.unpack(out["states"][k])[0] for k in range(len(tlist))])
        ex = out["expect"].cpu().numpy()[0]
        herm = [abs(e - e.conj().T).max() == 0 if e.nnz else True for e in E]
        return np.stack([ex[k].real if herm[k] else ex[k] for k in range(len(E))]) \
            if all(herm) else ex
    finally:
        h.close()


def _cost_grad(handle, rho0, O, u, t0, t1, nsteps, ckpt_every, stream=None):
    import torch
    handle._check_state(rho0, "rho0")
    handle._check_state(O, "O")
    handle._check_u(u)
    dev = rho0.device
    cost = torch.empty(handle.n_inst, dtype=torch.float64, device=dev)
    grad = torch.empty((handle.n_inst, handle.n_ctrl, handle.n_seg), dtype=torch.float64,
                       device=dev)
    rc = load().lme_cost_grad(handle._h, int(nsteps), int(ckpt_every), float(t0), float(t1),
                              _ptr(rho0), _ptr(O), _ptr(u), _ptr(cost), _ptr(grad),
                              _stream_ptr(stream))
    _check(rc, "lme_cost_grad")
    return cost, grad


class _CostFn:
    """Holder for the torch.autograd.Function, built on first use."""
    fn = None


def _cost_function():
    if _CostFn.fn is None:
        import torch

        class ExpectationCost(torch.autograd.Function):
            """J(u) = Re Tr(O rho(t1)) per instance; backward multiplies the
            gradient computed by lme_cost_grad (the discrete adjoint) with the
            incoming gradient."""

            @staticmethod
            def forward(ctx, u, handle, rho0, O, t0, t1, nsteps, ckpt_every):
                cost, grad = _cost_grad(handle, rho0, O, u.detach().contiguous(), t0, t1,
                                        nsteps, ckpt_every)
                ctx.save_for_backward(grad)
                return cost

            @staticmethod
            def backward(ctx, g):
                (grad,) = ctx.saved_tensors
                return (g[:, None, None] * grad, None, None, None, None, None, None, None)

        _CostFn.fn = ExpectationCost
    return _CostFn.fn


def expectation_cost(u, handle, rho0, O, t0, t1, nsteps, ckpt_every=10):
    """Differentiable J_b(u) = Re Tr(O_b rho_b(t1)) (torch.autograd.Function).
    u: float64 device tensor [n_inst, n_ctrl, n_seg]; returns [n_inst]."""
    import torch
    _check_tensor(u.detach().contiguous() if isinstance(u, torch.Tensor) else u,
                  torch.float64, handle.n_inst * handle.n_ctrl * handle.n_seg, "u")
    return _cost_function().apply(u, handle, rho0, O, t0, t1, nsteps, ckpt_every)


def raw_create_batch(systems, n_ctrl=None, n_e=None):
    """Calls lme_create_batch and returns (rc, message); for argument-validation
    tests.  Destroys the handle on success."""
    lib = load()
    keep = _CsrKeep()
    n_ctrl = len(getattr(systems[0], "H_ctrl", []) or []) if n_ctrl is None else n_ctrl
    n_e = len(systems[0].E) if n_e is None else n_e
    insts = (Instance * len(systems))()
    for b, s in enumerate(systems):
        insts[b] = Instance(C.cast(keep.array([s.H0]), C.POINTER(Csr)),
                            C.cast(keep.array(list(getattr(s, "H_ctrl", []) or [])),
                                   C.POINTER(Csr)),
                            len(s.C), C.cast(keep.array(list(s.C)), C.POINTER(Csr)),
                            C.cast(keep.array(list(s.E)), C.POINTER(Csr)))
    h = C.c_void_p()
    rc = lib.lme_create_batch(len(systems), insts, n_ctrl, n_e, None, None, C.byref(h))
    msg = lib.lme_last_error().decode()
    if rc == LME_OK:
        lib.lme_destroy(h)
    return rc, msg


# ---------------------------------------------------------------------------
# Monte-Carlo wave-function trajectories (Sec. 3.2)
# ---------------------------------------------------------------------------

class McHandle:
    """One system for Monte-Carlo trajectories (lme_mc_create): Hamiltonian H,
    collapse operators C, expectation operators E (square matrices)."""

    def __init__(self, H, C, E):
        lib = load()
        keep = _CsrKeep()
        Hc = keep.array([H])
        Cs = keep.array(list(C))
        Es = keep.array(list(E))
        h = C_.c_void_p()
        rc = lib.lme_mc_create(C_.cast(Hc, C_.POINTER(Csr)), len(C), C_.cast(Cs, C_.POINTER(Csr)),
                               len(E), C_.cast(Es, C_.POINTER(Csr)), C_.byref(h))
        _check(rc, "lme_mc_create")
        self._h = h
        self.n = sp.csr_matrix(H).shape[0]
        self.n_c, self.n_e = len(C), len(E)

    def close(self):
        if getattr(self, "_h", None):
            load().lme_mc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def evolve(self, psi0, tlist, nsteps, draws, want_traj=True, want_jumps=True, stream=None):
        """lme_mc_evolve.  psi0: complex128 device tensor [n]; draws: float64
        device tensor [n_traj, max_jumps + 1, 2].  Returns a dict of device
        tensors: expect [n_e, n_t] (mean), expect_traj [n_traj, n_e, n_t],
        n_jumps, jump_t, jump_op [n_traj, max_jumps], status [n_traj]."""
        import torch
        _check_tensor(psi0, torch.complex128, self.n, "psi0")
        if not isinstance(draws, torch.Tensor) or draws.dim() != 3 or draws.shape[2] != 2:
            raise LmeError(LME_EINVAL, "draws must be a tensor [n_traj, max_jumps + 1, 2]")
        n_traj, mj = int(draws.shape[0]), int(draws.shape[1]) - 1
        _check_tensor(draws, torch.float64, n_traj * (mj + 1) * 2, "draws")
        tl = np.ascontiguousarray(tlist, np.float64)
        n_t = len(tl)
        dev = psi0.device
        out = {"expect": torch.zeros((self.n_e, n_t), dtype=torch.complex128, device=dev),
               "expect_traj": (torch.zeros((n_traj, self.n_e, n_t), dtype=torch.complex128,
                                           device=dev) if want_traj else None),
               "status": torch.full((n_traj,), -1, dtype=torch.int32, device=dev)}
        if want_jumps:
            out["n_jumps"] = torch.zeros(n_traj, dtype=torch.int32, device=dev)
            out["jump_t"] = torch.zeros((n_traj, max(mj, 1)), dtype=torch.float64, device=dev)
            out["jump_op"] = torch.full((n_traj, max(mj, 1)), -1, dtype=torch.int32, device=dev)
        g = out.get
        rc = load().lme_mc_evolve(self._h, n_t, tl.ctypes.data_as(_PD), int(nsteps), _ptr(psi0),
                                  n_traj, _ptr(draws), mj, _ptr(g("expect")),
                                  _ptr(g("expect_traj")), _ptr(g("n_jumps")), _ptr(g("jump_t")),
                                  _ptr(g("jump_op")), _ptr(g("status")), _stream_ptr(stream))
        _check(rc, "lme_mc_evolve")
        return out


def mcsolve(H, psi0, tlist, ntraj, c_ops, e_ops, nsteps, seed=0, max_jumps=64, device="cuda",
            draws=None):
    """Monte-Carlo solver in the calling convention of the paper (Sec. 4.3:
    Hamiltonian, initial ket, times, number of trajectories, collapse and
    expectation operators).  The random numbers of every trajectory are drawn
    once from ``numpy.random.default_rng(seed)`` (or given as ``draws``,
    [ntraj, max_jumps + 1, 2]).  Returns the trajectory-averaged expectation
    values [len(e_ops)][len(tlist)] (real for Hermitian e_ops)."""
    import torch
    from . import systems
    E = [sp.csr_matrix(e, dtype=np.complex128) for e in e_ops]
    h = McHandle(H, [sp.csr_matrix(c, dtype=np.complex128) for c in c_ops], E)
    try:
        psi = torch.from_numpy(np.ascontiguousarray(np.asarray(psi0, np.complex128).reshape(-1)))
        d = systems.mc_draws(ntraj, max_jumps, seed) if draws is None else np.asarray(draws)
        out = h.evolve(psi.to(device), tlist, nsteps, torch.from_numpy(np.ascontiguousarray(d)).to(device),
                       want_traj=False, want_jumps=False)
        torch.cuda.synchronize()
        st = out["status"].cpu().numpy()
        if (st != 0).any():
            bad = int(st[st != 0][0])
            raise LmeError(bad, f"mcsolve: {int((st != 0).sum())} trajectories stopped "
                                f"({STATUS_NAMES.get(bad, bad)})")
        ex = out["expect"].cpu().numpy()
        herm = [abs(e - e.conj().T).max() == 0 if e.nnz else True for e in E]
        return np.stack([ex[k].real if herm[k] else ex[k] for k in range(len(E))]) if E else ex
    finally:
        h.close()
