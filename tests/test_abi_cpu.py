"""The C ABI on a machine without a GPU: the library loads, exports every
symbol the header declares, and rejects malformed input before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1110_0573_amd import lme, systems as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "lme.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lme_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = lme.load()
    declared = header_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(lme.EXPORTS) == declared


def test_default_options():
    o = lme.default_options()
    assert o.method == lme.LME_RK4 and o.path == lme.LME_PATH_AUTO
    assert o.rtol == 1e-6 and o.atol == 1e-9 and o.max_steps == 10**7
    assert o.hermitian == 0
    # the ctypes mirrors have the C layout (fields appended at the end)
    assert C.sizeof(lme.Options) == 72 and lme.Options.hermitian.offset == 64
    assert C.sizeof(lme.Tuning) == 64 and lme.Tuning.apply_block.offset == 48
    assert lme.Tuning.grad_layout.offset == 56


def _jc():
    return S.jc_system(3)


def _bad(system, attr, value):
    s = S.System(system.H0, list(system.C), list(system.E), system.rho0)
    setattr(s, attr, value)
    return s


def test_create_rejects_dimension_mismatch():
    s = _jc()
    bad = _bad(s, "C", [sp.identity(5, dtype=np.complex128, format="csr")])
    rc, msg = lme.raw_create_batch([bad])
    assert rc == lme.LME_EINVAL and "expected" in msg


def test_create_rejects_out_of_range_column():
    s = _jc()
    m = sp.csr_matrix(s.H0)
    # hand-built CSR with a bad column index
    keep = lme._CsrKeep()
    rp = np.array(m.indptr, np.int32)
    ci = np.array(m.indices, np.int32)
    ci[0] = 99
    va = np.array(m.data, np.complex128).view(np.float64)
    csr = lme.Csr(m.shape[0], m.nnz, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                  ci.ctypes.data_as(C.POINTER(C.c_int32)), va.ctypes.data_as(C.POINTER(C.c_double)))
    inst = lme.Instance(C.pointer(csr), None, 0, None, None)
    h = C.c_void_p()
    rc = lme.load().lme_create_batch(1, C.byref(inst), 0, 0, None, None, C.byref(h))
    assert rc == lme.LME_EINVAL
    assert "out of range" in lme.load().lme_last_error().decode()
    del keep


def test_create_rejects_decreasing_row_ptr_and_nan():
    s = _jc()
    m = sp.csr_matrix(s.H0)
    rp = np.array(m.indptr, np.int32)
    rp[2], rp[3] = rp[3], rp[2] - 1 if rp[2] > 0 else 0
    ci = np.array(m.indices, np.int32)
    va = np.array(m.data, np.complex128).view(np.float64)
    csr = lme.Csr(m.shape[0], m.nnz, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                  ci.ctypes.data_as(C.POINTER(C.c_int32)), va.ctypes.data_as(C.POINTER(C.c_double)))
    h = C.c_void_p()
    inst = lme.Instance(C.pointer(csr), None, 0, None, None)
    assert lme.load().lme_create_batch(1, C.byref(inst), 0, 0, None, None, C.byref(h)) == lme.LME_EINVAL
    s2 = _jc()
    H = sp.csr_matrix(s2.H0).copy()
    H.data[0] = np.nan
    rc, msg = lme.raw_create_batch([_bad(s2, "H0", H)])
    assert rc == lme.LME_EINVAL and "non-finite" in msg


def test_create_rejects_empty_batch_and_null_out():
    lib = lme.load()
    h = C.c_void_p()
    assert lib.lme_create_batch(0, None, 0, 0, None, None, C.byref(h)) == lme.LME_EINVAL
    assert lib.lme_create_batch(1, None, 0, 0, None, None, None) == lme.LME_EINVAL


def test_create_rejects_too_wide_rows():
    n = 80
    H = sp.csr_matrix(np.ones((n, n), np.complex128))
    s = S.System(H, [], [], np.eye(n))
    rc, msg = lme.raw_create_batch([s])
    assert rc == lme.LME_ENOTSUP


def test_destroy_null_is_noop():
    lme.load().lme_destroy(None)


def _handle():
    w = S.jc_sweep(n_inst=3, nsteps=10, t_end=1.0, n_out=3)
    return lme.Handle(w.systems), w


def test_layout_packs_instances_in_order():
    h, w = _handle()
    dims = [s.n for s in w.systems]
    assert list(h.dims) == dims
    assert list(h.offsets) == list(np.cumsum([0] + [d * d for d in dims])[:-1])
    assert h.state_elems == sum(d * d for d in dims)


def _evolve_rc(h, tlist, **opt):
    o = lme.default_options(**opt)
    tl = np.ascontiguousarray(tlist, np.float64)
    rc = lme.load().lme_evolve(h._h, C.byref(o), len(tl), tl.ctypes.data_as(C.POINTER(C.c_double)),
                               C.c_void_p(16), None, None, None, None, None, None, None)
    return rc, lme.load().lme_last_error().decode()


def test_evolve_validation_precedes_device_use():
    h, w = _handle()
    assert _evolve_rc(h, [0.0, 0.5, 0.4], nsteps=10)[0] == lme.LME_EINVAL     # not increasing
    assert _evolve_rc(h, [0.0, 1.0], nsteps=0)[0] == lme.LME_EINVAL           # no steps
    assert _evolve_rc(h, [0.0, 0.33, 1.0], nsteps=10)[0] == lme.LME_EGRID     # off grid
    assert _evolve_rc(h, [0.0, 1.0], nsteps=10, block=300)[0] == lme.LME_EINVAL
    assert _evolve_rc(h, [0.0, np.nan], nsteps=10)[0] == lme.LME_EINVAL
    assert _evolve_rc(h, [0.0, 1.0], nsteps=10, method=7)[0] == lme.LME_EINVAL
    assert _evolve_rc(h, [0.0, 1.0], nsteps=10, hermitian=2)[0] == lme.LME_EINVAL
    rc, msg = _evolve_rc(h, [0.0, 1.0], nsteps=10)
    import torch
    if not torch.cuda.is_available():
        assert rc == lme.LME_EHIP, msg


def test_dopri5_validation_precedes_device_use():
    """Adaptive-stepper options and the layout/block combinations are checked
    on the host, before any HIP call."""
    h, w = _handle()
    D = lme.LME_DOPRI5
    tl = [0.0, 1.0]
    assert _evolve_rc(h, tl, method=D, rtol=0.0)[0] == lme.LME_EINVAL
    assert _evolve_rc(h, tl, method=D, atol=-1.0)[0] == lme.LME_EINVAL
    assert _evolve_rc(h, tl, method=D, max_steps=0)[0] == lme.LME_EINVAL
    assert _evolve_rc(h, tl, method=D, block=768)[0] == lme.LME_EINVAL
    # a batch outside the column kernels' operator shapes
    g = lme.Handle([S.random_system(6, n_c=2, density=0.9, seed=1)])
    rc, msg = _evolve_rc(g, tl, method=D, layout=lme.LME_LAYOUT_COLUMN)
    assert rc == lme.LME_ENOTSUP, msg
    rc, msg = _evolve_rc(h, tl, method=D)
    import torch
    if not torch.cuda.is_available():
        assert rc == lme.LME_EHIP, msg


def test_evolve_grid_check_for_control_edges():
    w = S.jc_drive(n_inst=2, N=3, n_seg=3, t_end=1.0, steps_per_seg=2)
    h = lme.Handle(w.systems)
    assert _evolve_rc(h, [0.0, 1.0], nsteps=10)[0] == lme.LME_EGRID   # edges at 1/3, 2/3
    rc, _ = _evolve_rc(h, [0.0, 1.0], nsteps=6)
    assert rc in (lme.LME_OK, lme.LME_EHIP)


def test_null_handle_is_rejected():
    lib = lme.load()
    o = lme.default_options(nsteps=1)
    tl = np.array([0.0, 1.0])
    assert lib.lme_evolve(None, C.byref(o), 2, tl.ctypes.data_as(C.POINTER(C.c_double)),
                          C.c_void_p(16), None, None, None, None, None, None, None) == lme.LME_EINVAL
    assert lib.lme_apply(None, 0, 0, 0.0, None, C.c_void_p(16), C.c_void_p(32), None) == lme.LME_EINVAL
    assert lib.lme_layout(None, None, None, None, None) == lme.LME_EINVAL


def test_dopri5_rejects_unknown_layout_before_device_use():
    h, w = _handle()
    for bad in (-1, 3):
        rc, msg = _evolve_rc(h, [0.0, 1.0], method=lme.LME_DOPRI5, layout=bad)
        assert rc == lme.LME_EINVAL and "layout" in msg, msg


def test_binding_checks_every_buffer_before_the_c_call():
    """dtype, size and contiguity of every tensor are checked in the binding
    (the C side cannot see the size of a device buffer); all of these raise
    LME_EINVAL without any HIP call, so they run on a machine without a GPU."""
    import torch
    h, w = _handle()
    good = torch.zeros(h.state_elems, dtype=torch.complex128)
    cases = [
        torch.zeros(h.state_elems, dtype=torch.complex64),          # wrong dtype
        torch.zeros(h.state_elems - 1, dtype=torch.complex128),     # too short
        torch.zeros(h.state_elems + 5, dtype=torch.complex128),     # too long
        torch.zeros(2 * h.state_elems, dtype=torch.complex128)[::2],  # not contiguous
        np.zeros(h.state_elems, np.complex128),                      # not a tensor
        good,                                                        # not on the device
    ]
    for bad in cases:
        with pytest.raises(lme.LmeError) as e:
            h.evolve(bad, np.array([0.0, 1.0]), nsteps=10)
        assert e.value.code == lme.LME_EINVAL
        with pytest.raises(lme.LmeError) as e:
            h.apply(bad)
        assert e.value.code == lme.LME_EINVAL
    # control amplitudes: float64, n_inst * n_ctrl * n_seg elements
    wd = S.jc_drive(n_inst=2, N=3, n_seg=4, t_end=1.0, steps_per_seg=2)
    hd = lme.Handle(wd.systems)
    rho = torch.zeros(hd.state_elems, dtype=torch.complex128)
    for bad_u in (torch.zeros((2, 1, 4), dtype=torch.float32),
                  torch.zeros((2, 1, 3), dtype=torch.float64)):
        with pytest.raises(lme.LmeError) as e:
            hd.evolve(rho, np.array([0.0, 1.0]), nsteps=8, u=bad_u)
        assert e.value.code == lme.LME_EINVAL and "u" in str(e.value)
        with pytest.raises(lme.LmeError) as e:
            lme._cost_grad(hd, rho, rho, bad_u, 0.0, 1.0, 8, 2)
        assert e.value.code == lme.LME_EINVAL
        with pytest.raises(lme.LmeError) as e:
            lme.expectation_cost(bad_u, hd, rho, rho, 0.0, 1.0, 8)
        assert e.value.code == lme.LME_EINVAL
    with pytest.raises(lme.LmeError):   # controls given to a batch without segments
        h.evolve(torch.zeros(h.state_elems, dtype=torch.complex128), np.array([0.0, 1.0]),
                 nsteps=10, u=torch.zeros(3, dtype=torch.float64))
    with pytest.raises(lme.LmeError) as e:   # O of the wrong size
        lme._cost_grad(hd, rho, torch.zeros(hd.state_elems - 1, dtype=torch.complex128),
                       torch.zeros((2, 1, 4), dtype=torch.float64), 0.0, 1.0, 8, 2)
    assert e.value.code == lme.LME_EINVAL


def test_mc_create_and_evolve_validation_before_device_use():
    """Monte-Carlo entry points: operator validation at create, time grid and
    argument checks before any HIP call."""
    lib = lme.load()
    s = S.thermal_cavity_mc()
    with pytest.raises(lme.LmeError) as e:      # collapse operator of the wrong dimension
        lme.McHandle(s.H0, [sp.identity(3, dtype=np.complex128, format="csr")], s.E)
    assert e.value.code == lme.LME_EINVAL
    with pytest.raises(lme.LmeError) as e:      # too many collapse operators
        lme.McHandle(s.H0, [s.C[0]] * 17, s.E)
    assert e.value.code == lme.LME_ENOTSUP
    h = lme.McHandle(s.H0, s.C, s.E)

    def rc_of(tl, nsteps, n_traj=4, max_jumps=2, psi=16, draws=32):
        tl = np.ascontiguousarray(tl, np.float64)
        return lib.lme_mc_evolve(h._h, len(tl), tl.ctypes.data_as(C.POINTER(C.c_double)), nsteps,
                                 C.c_void_p(psi), n_traj, C.c_void_p(draws), max_jumps, None,
                                 None, None, None, None, None, None)
    assert rc_of([0.0, 0.5, 0.4], 10) == lme.LME_EINVAL           # not increasing
    assert rc_of([0.0, 0.33, 1.0], 10) == lme.LME_EGRID           # off the grid
    assert rc_of([0.0, 1.0], 0) == lme.LME_EINVAL                 # no steps
    assert rc_of([0.0, 1.0], 10, n_traj=0) == lme.LME_EINVAL
    assert rc_of([0.0, 1.0], 10, max_jumps=-1) == lme.LME_EINVAL
    assert rc_of([0.0, 1.0], 10, psi=0) == lme.LME_EINVAL
    assert lib.lme_mc_evolve(None, 1, None, 0, None, 1, None, 0, None, None, None, None, None,
                             None, None) == lme.LME_EINVAL
    import torch
    if not torch.cuda.is_available():
        assert rc_of([0.0, 1.0], 10) == lme.LME_EHIP
        with pytest.raises(lme.LmeError) as e:    # the binding checks tensors first
            h.evolve(torch.zeros(4, dtype=torch.complex128), [0.0, 1.0], 10,
                     torch.zeros((2, 3, 2), dtype=torch.float64))
        assert e.value.code == lme.LME_EINVAL
    lib.lme_mc_destroy(None)
    h.close()


def test_set_coeff_fn_validation():
    lib = lme.load()
    assert lib.lme_set_coeff_fn(None, None) == lme.LME_EINVAL
    h, w = _handle()                       # no control terms
    with pytest.raises(lme.LmeError) as e:
        h.set_coeff_fn(np.zeros((3, 1, 7)))
    assert e.value.code == lme.LME_EINVAL
    wd = S.jc_drive(n_inst=2, N=3, n_seg=2, t_end=1.0, steps_per_seg=2)
    hd = lme.Handle(wd.systems)
    bad = np.zeros((2, 1, 7))
    bad[1, 0, 4] = np.inf
    with pytest.raises(lme.LmeError) as e:
        hd.set_coeff_fn(bad)
    assert e.value.code == lme.LME_EINVAL
    hd.set_coeff_fn(np.zeros((2, 1, 7)))
    # closed-form amplitudes lift the edge grid constraint, refuse DOPRI5
    assert _evolve_rc(hd, [0.0, 1.0], nsteps=7)[0] in (lme.LME_OK, lme.LME_EHIP)
    assert _evolve_rc(hd, [0.0, 1.0], method=lme.LME_DOPRI5)[0] == lme.LME_ENOTSUP
    hd.set_coeff_fn(None)
    assert _evolve_rc(hd, [0.0, 1.0], nsteps=7)[0] == lme.LME_EGRID


def test_correlation_validation_before_device_use():
    lib = lme.load()
    h, w = _handle()
    o = lme.default_options(nsteps=10)
    tl = np.array([0.0, 1.0])
    keep = lme._CsrKeep()
    Bs = keep.array([S.jc_ops(s.n // 2)[0] for s in w.systems])

    def rc(ta, B=Bs, opt=o, tns=10):
        ta = np.ascontiguousarray(ta, np.float64)
        return lib.lme_correlation(h._h, C.byref(opt), 2, tl.ctypes.data_as(C.POINTER(C.c_double)),
                                   len(ta), ta.ctypes.data_as(C.POINTER(C.c_double)), tns,
                                   C.cast(B, C.POINTER(lme.Csr)) if B is not None else None,
                                   C.c_void_p(16), C.c_void_p(32), None, None)
    assert rc([0.5, 1.0]) == lme.LME_EINVAL                 # delays must start at 0
    assert rc([0.0, 1.0], B=None) == lme.LME_EINVAL
    assert rc([0.0, 1.0], tns=0) == lme.LME_EINVAL
    assert rc([0.0, 1.0], opt=lme.default_options(method=lme.LME_DOPRI5)) == lme.LME_ENOTSUP
    bad = keep.array([S.jc_ops(2)[0]] * 3)                  # wrong dimensions
    assert rc([0.0, 1.0], B=bad) == lme.LME_EINVAL
    import torch
    if not torch.cuda.is_available():
        assert rc([0.0, 1.0]) == lme.LME_EHIP


def test_propagator_and_steadystate_validation_before_device_use():
    lib = lme.load()
    h, w = _handle()
    o = lme.default_options(nsteps=10)
    P = C.c_void_p(16)
    prop = lambda opt=o, t0=0.0, t1=1.0, U=P: lib.lme_propagator(h._h, C.byref(opt), t0, t1, U,
                                                                 None, None)
    ss = lambda opt=o, T=1.0, k=10, tol=0.0, r=P: lib.lme_steadystate(
        h._h, C.byref(opt), T, k, tol, r, None, None, None)
    assert lib.lme_propagator(None, C.byref(o), 0.0, 1.0, P, None, None) == lme.LME_EINVAL
    assert prop(t1=0.0) == lme.LME_EINVAL                      # t1 must exceed t0
    assert prop(t1=float("nan")) == lme.LME_EINVAL
    assert prop(U=None) == lme.LME_EINVAL
    assert prop(opt=lme.default_options(nsteps=0)) == lme.LME_EINVAL
    assert prop(opt=lme.default_options(method=lme.LME_DOPRI5)) == lme.LME_ENOTSUP
    assert ss(T=-1.0) == lme.LME_EINVAL
    assert ss(k=-1) == lme.LME_EINVAL and ss(k=201) == lme.LME_EINVAL
    assert ss(tol=float("inf")) == lme.LME_EINVAL and ss(tol=-1.0) == lme.LME_EINVAL
    assert ss(r=None) == lme.LME_EINVAL
    wd = S.jc_drive(n_inst=2, N=3, n_seg=2, t_end=1.0, steps_per_seg=2)
    hd = lme.Handle(wd.systems)                                # control terms
    assert lib.lme_propagator(hd._h, C.byref(o), 0.0, 1.0, P, None, None) == lme.LME_ENOTSUP
    big = lme.Handle([S.random_system(130, n_c=1, n_e=1, seed=1, density=0.02)])
    assert lib.lme_propagator(big._h, C.byref(o), 0.0, 1.0, P, None, None) == lme.LME_ENOTSUP
    assert lib.lme_steadystate(big._h, C.byref(o), 1.0, 5, 0.0, P, None, None,
                               None) == lme.LME_ENOTSUP
    import torch
    if not torch.cuda.is_available():
        assert prop() == lme.LME_EHIP and ss() == lme.LME_EHIP


def test_tuning_grad_layout_roundtrip_and_range():
    """lme_set_tuning takes grad_layout in {AUTO, ROW, COLUMN} and rejects
    anything else without touching the handle's settings."""
    h = lme.Handle([S.jc_system(3)])
    h.set_tuning(grad_layout=lme.LME_LAYOUT_ROW)
    assert h.get_tuning().grad_layout == lme.LME_LAYOUT_ROW
    for bad in (-1, 3):
        with pytest.raises(lme.LmeError) as e:
            h.set_tuning(grad_layout=bad)
        assert e.value.code == lme.LME_EINVAL
    assert h.get_tuning().grad_layout == lme.LME_LAYOUT_ROW
