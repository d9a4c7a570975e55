#!/usr/bin/env python3
"""Benchmark: batched FP64 Lindblad evolution on one MI355X.

Workload (one "step" = one pass of the whole hot path over the batch): the
Jaynes-Cummings parameter sweep, 4096 instances with cavity cutoffs N in
{5..40} (dims 10..80), fixed-step RK4, 1000 steps over t in [0, 25],
<a^+a> and <sigma_z> at 101 output times, every instance's state resident in
HBM before the timed region.

Prints one JSON line with the headline throughput (instance-RK-steps/s), the
roofline position of the dominant kernel (measured with HIP events on the
stream the kernel runs on), the batched-vs-plain speedup (the same instances
integrated one per launch) and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "instance-RK-steps/sec + HBM GB/s, batched vs plain, at 1e-10 trace distance"
# HBM bytes per launch of the timed kernels from the FETCH_SIZE / WRITE_SIZE passes
# (rocprofv3 --pmc, scaled by a 256 MiB copy: x2.0 and x1.0; profiles/README.md), valid
# only while the kernel's source file has the SHA-256 recorded with them; any other
# source reports null.
TRAFFIC_SOURCES = {
    "lme_kernels.hip": "5c1c6e4612d8bbb6f71a8e1cdcc9befa366c5c42b067f6889e915b74ae7e1d59",
    "lme_mc.hip": "430556a8477c37b2518b1ef033bf9e5d02253ea52ef0d06223e0015092f8d385",
    "lme_prop.hip": "1cb74cb326de73396be2810a8f7bc6a348ad3fa4957b14d9137df9ade952e57d",
}
TRAFFIC = {
    "rk4_herm_kernel": ("lme_kernels.hip", 192.1e6 + 178.2e6),
    "rk4_colown_kernel": ("lme_kernels.hip", 217.2e6 + 234.0e6),
    "apply_pipe_kernel": ("lme_kernels.hip", 184.5e6 + 158.3e6),
    "apply_rows_kernel": ("lme_kernels.hip", 154.7e6 + 104.9e6),
    "mc_kernel": ("lme_mc.hip", 2332.6e6 + 3173.0e6),
    "zgemm_kernel": ("lme_prop.hip", 2450.9e6 + 268.4e6),
}


def kernel_traffic(name):
    """Counter-measured bytes per launch of `name`, or None if its source changed."""
    import hashlib
    if name not in TRAFFIC:
        return None
    src, nbytes = TRAFFIC[name]
    with open(os.path.join(ROOT, "paper_1110_0573_amd", "csrc", src), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    return nbytes if digest == TRAFFIC_SOURCES[src] else None


FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CUs x 4 SIMD x 16 lanes x 2 flop/FMA x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def apply_flops(s):
    """Algorithmic FP64 flops of one Liouvillian application in operator form
    (complex multiply-add = 8 flops): A y and y A^+ over the off-diagonal
    entries of A = -iH - 1/2 sum C^+C, the diagonal term (D_i + conj D_j) y_ij,
    and C_k y C_k^+ (nnz(C_k)^2 products per instance)."""
    import scipy.sparse as sp
    n = s.n
    A = sp.csr_matrix(-1j * s.H0)
    for c in s.C:
        A = A - 0.5 * (c.conj().T @ c)
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    off = A.nnz - np.count_nonzero(A.diagonal())
    jumps = sum(int(sp.csr_matrix(c).nnz) ** 2 for c in s.C)
    return 8.0 * (2 * n * off + n * n + jumps)


def survey_apply_flops(s):
    """The scope table's count of one application, operator form:
    8 n nnz(A) + 2 n^2 + 8 n^2 K (A = -iH - 1/2 sum C^+C with its diagonal,
    K collapse operators)."""
    import scipy.sparse as sp
    n = s.n
    A = sp.csr_matrix(-1j * s.H0)
    for c in s.C:
        A = A - 0.5 * (c.conj().T @ c)
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    return 8.0 * n * A.nnz + 2.0 * n * n + 8.0 * n * n * len(s.C)


def herm_lds_bytes_per_element_stage(s):
    """LDS bytes one element-stage of the Hermitian resident kernel moves
    (row data in registers): the y gathers of A y, y A^+ (one per
    off-diagonal entry of A on each side) and C_k y C_k^+ (one per monomial
    collapse operator), 16 bytes each, plus the stage input stored twice
    (the element and its conjugate mirror)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(-1j * s.H0)
    for c in s.C:
        A = A - 0.5 * (c.conj().T @ c)
    A = sp.csr_matrix(A)
    A.setdiag(0)
    A.eliminate_zeros()
    wo = int(np.max(np.diff(A.indptr))) if A.nnz else 0
    return 16.0 * (2 * wo + len(s.C)) + 32.0


def lds_peak_tbs(lme, torch, reps=5):
    """Measured LDS read bandwidth of the chip (TB/s): the probe kernel,
    two 1024-thread workgroups per CU, ds_read_b128 without bank conflicts."""
    import ctypes as C
    lib = lme.load()
    lib.lme_internal_probe_lds.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    grid, iters = 2 * n_cu, 8192
    sink = torch.zeros(grid, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    for _ in range(2):
        assert lib.lme_internal_probe_lds(grid, iters, lme._ptr(sink), lme._stream_ptr(stream)) == 0
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        lib.lme_internal_probe_lds(grid, iters, lme._ptr(sink), lme._stream_ptr(stream))
    b.record(stream)
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3 / reps
    return grid * 1024.0 * iters * 16.0 / sec / 1e12


def rk4_step_flops(s):
    """One RK4 step: four applications plus the stage combinations
    (2 complex-by-real axpys per stage and the final update: 36 flops/element)."""
    return 4.0 * apply_flops(s) + 36.0 * s.n * s.n


def rk4_step_flops_hermitian(s):
    """The same step when rho is Hermitian: each of the n(n+1)/2 pairs {i, j}
    is computed once (the element flops above scale with the elements)."""
    return rk4_step_flops(s) * (s.n + 1) / (2.0 * s.n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, sample, nsteps_full, systems, with_configs=True):
    """The oracle (plain C, gcc -O3 -march=native, built here on the host it
    is timed on) on bounded samples: the headline sweep (one instance per
    host thread, median of 3 runs) and, single-threaded or one instance per
    thread, the other configurations and the Monte-Carlo workload."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    try:
        oracle.use_native_build(tempfile.mkdtemp(prefix="oracle_native_"))
        build = "gcc -O3 -march=native"
    except Exception as e:  # pragma: no cover - no compiler on the host
        build = f"gcc -O3 (generic; native build failed: {e})"
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    rng = np.random.default_rng(123)
    idx = rng.choice(len(w.systems), sample, replace=False)
    sub = [w.systems[i] for i in idx]
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.rk4_batch(sub, [s.rho0 for s in sub], w.tlist, nsteps_full, cores)
        runs.append(time.perf_counter() - t0)
    dt = float(np.median(runs))
    rec = {"value": sample * nsteps_full / dt, "unit": "instance-RK-steps/s", "cores": cores,
           "kind": "oracle", "cpu": cpu_model(), "build": build,
           "sample": f"{sample} random instances of the 4096-instance sweep, full 1000 RK4 "
                     f"steps each, one instance per thread on {cores} host threads; median of "
                     f"3 runs ({', '.join(f'{r:.2f}' for r in runs)} s)"}
    if not with_configs:
        return rec
    cfg = {}
    ws = systems.jc_single()
    s = ws.systems[0]
    t0 = time.perf_counter()
    oracle.rk4(s, s.rho0, ws.tlist, ws.nsteps)
    d = time.perf_counter() - t0
    cfg["jc_single_N10_rk4_2500"] = {"steps_per_s": ws.nsteps / d, "threads": 1,
                                     "sample": "the full run", "s": d}
    wk = systems.kerr_single()
    s = wk.systems[0]
    tl = np.linspace(0.0, 5.0, 11)
    t0 = time.perf_counter()
    r = oracle.dopri5(s, s.rho0, tl, wk.rtol, wk.atol)
    d = time.perf_counter() - t0
    cfg["kerr_N60_dopri5"] = {"accepted_steps_per_s": float(r["counts"][0]) / d, "threads": 1,
                              "sample": f"t in [0, 5] ({int(r['counts'][0])} accepted steps) of "
                                        "the t in [0, 50] run", "s": d}
    wd = systems.jc_drive()
    nd = min(cores, 16)
    O = wd.extra["target"]

    def grad_one(b):
        sy = wd.systems[b]
        return oracle.rk4_cost_grad(sy, sy.rho0, O, 0.0, 10.0, wd.nsteps)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(nd) as ex:
        list(ex.map(grad_one, range(nd)))
    d = time.perf_counter() - t0
    cfg["jc_drive_cost_grad"] = {"forward_instance_steps_per_s": nd * wd.nsteps / d,
                                 "threads": nd, "sample": f"{nd} of the 256 instances, full "
                                 "1000-step cost and gradient each", "s": d}
    wt = systems.tfim()
    nt = min(cores, 8)
    tlt = np.linspace(0.0, 1.0, 11)

    def tfim_one(b):
        sy = wt.systems[b]
        return oracle.dopri5(sy, sy.rho0, tlt, wt.rtol, wt.atol)["counts"][0]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(nt) as ex:
        acc = sum(ex.map(tfim_one, range(nt)))
    d = time.perf_counter() - t0
    cfg["tfim_8spin_dopri5"] = {"accepted_instance_steps_per_s": float(acc) / d, "threads": nt,
                                "sample": f"{nt} of the 64 realizations on t in [0, 1] "
                                          "(of [0, 20])", "s": d}
    wm = systems.trilinear_mc_workload()
    sm = wm.systems[0]
    nm = 2 * cores
    t0 = time.perf_counter()
    oracle.mc(sm, sm.meta["psi0"], wm.tlist, wm.nsteps, wm.extra["draws"][:nm], n_threads=cores)
    d = time.perf_counter() - t0
    cfg["trilinear_mc"] = {"trajectory_steps_per_s": nm * wm.nsteps / d, "threads": cores,
                           "sample": f"{nm} of the 1000 trajectories, full 1000 steps each",
                           "s": d}
    rec["configs"] = cfg
    return rec


def mc_trilinear_bench(lme, systems, torch, reps=3):
    """Monte-Carlo trajectories of the trilinear Hamiltonian (Sec. 4.3): 1000
    trajectories of dimension 4913, 1000 RK4 steps, 201 outputs.  Kernel
    time with HIP events on the launch stream (median of the timed runs)."""
    import scipy.sparse as sp
    w = systems.trilinear_mc_workload()
    s = w.systems[0]
    h = lme.McHandle(s.H0, s.C, s.E)
    psi0 = torch.from_numpy(s.meta["psi0"]).cuda()
    draws = torch.from_numpy(w.extra["draws"]).cuda()
    stream = torch.cuda.current_stream()
    out = h.evolve(psi0, w.tlist, w.nsteps, draws, want_traj=False)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out = h.evolve(psi0, w.tlist, w.nsteps, draws, want_traj=False)
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    st = out["status"].cpu().numpy()
    jumps = out["n_jumps"].cpu().numpy()
    n_traj = len(w.extra["draws"])
    kms = float(np.median(ms))
    # algorithmic flops per trajectory-step: four sparse products with A
    # (8 per complex multiply-add over nnz(A)), the 1/k scalings and the
    # running-sum updates (2 + 4 per element each) and the squared norm
    A = sp.csr_matrix(-1j * s.H0)
    for c in s.C:
        A = A - 0.5 * (c.conj().T @ c)
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    n = s.n
    f_step = 4 * (8.0 * A.nnz + 6.0 * n) + 4.0 * n
    flops = f_step * n_traj * w.nsteps
    return {"workload": "trilinear Hamiltonian, 3 modes x 17 states (dim 4913), 1000 "
                        "trajectories, 1000 RK4 steps on [0, 4], 201 outputs",
            "ms": kms, "ms_runs": ms, "trajectory_steps_per_s": n_traj * w.nsteps / (kms * 1e-3),
            "jumps_mean": float(jumps.mean()), "status_ok": bool((st == 0).all()),
            "algorithmic_flops": flops, "achieved_tflops": flops / (kms * 1e-3) / 1e12,
            "frac_fp64_peak": flops / (kms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "kernel": "mc_kernel", "traffic": kernel_traffic("mc_kernel")}


FP64_MFMA_PEAK_TFLOPS = 78.6


def steady_state_bench(lme, systems, torch, reps=3):
    """Steady states of 16 thermal JC systems (dimension 32): the propagator
    U(10) of each (its 1024 basis matrices as one RK4 batch), then squarings
    on the matrix cores.  Timed with HIP events on the launch stream: the
    propagator, the whole steady-state call (it synchronises once per
    product for the convergence test), and one launch of the complex product
    alone on the same operands (the matrix-core roofline)."""
    import ctypes
    w = systems.jc_steady_sweep()
    T = float(w.tlist[-1])
    h = lme.Handle(w.systems)
    stream = torch.cuda.current_stream()

    def ev_ms(fn):
        fn()
        torch.cuda.synchronize()
        ms, out = [], None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            out = fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return float(np.median(ms)), out

    p_ms, (Us, pst) = ev_ms(lambda: h.propagator(0.0, T, w.nsteps, stream=stream))
    s_ms, (rho, st, k) = ev_ms(lambda: h.steadystate(T, w.nsteps, stream=stream))
    # one product on the propagators just formed
    dims = [int(n) for n in h.dims]
    Ns = [n * n for n in dims]
    off4 = np.concatenate([[0], np.cumsum([N * N for N in Ns])]).astype(np.int64)
    tiles = np.array([(b, i, j, 0) for b, N in enumerate(Ns)
                      for i in range((N + 63) // 64) for j in range((N + 63) // 64)],
                     np.int32).reshape(-1)
    A = torch.cat([U.t().contiguous().reshape(-1) for U in Us])
    Cm = torch.empty_like(A)
    t_tiles, t_off = torch.from_numpy(tiles).cuda(), torch.from_numpy(off4).cuda()
    t_dims = torch.tensor(dims, dtype=torch.int32, device="cuda")
    f = lme.load().lme_internal_launch_zgemm
    f.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 6
    f.restype = ctypes.c_int

    def gemm():
        rc = f(t_tiles.data_ptr(), len(tiles) // 4, t_off.data_ptr(), t_dims.data_ptr(),
               A.data_ptr(), A.data_ptr(), Cm.data_ptr(), stream.cuda_stream)
        assert rc == 0
    g_ms, _ = ev_ms(gemm)
    flops = float(sum(8.0 * N ** 3 for N in Ns))
    n_basis = sum(Ns)
    return {"workload": "jc_steady_sweep: 16 thermal JC systems, N = 16 (dim 32), U(10) by "
                        "RK4 in 200 steps over the 1024 basis matrices, then squarings",
            "propagator_ms": p_ms,
            "propagator_instance_steps_per_s": n_basis * w.nsteps / (p_ms * 1e-3),
            "steadystate_ms": s_ms, "squarings": int(k),
            "status_ok": bool((st.cpu().numpy() == 0).all()),
            "zgemm": {"kernel": "zgemm_kernel", "ms": g_ms, "algorithmic_flops": flops,
                      "achieved_tflops": flops / (g_ms * 1e-3) / 1e12,
                      "peak": FP64_MFMA_PEAK_TFLOPS, "bound": "mfma",
                      "frac": flops / (g_ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS,
                      "traffic": kernel_traffic("zgemm_kernel"),
                      "note": "8 N^3 real flops per complex N x N product, N = 1024"}}


def streamed_apply_bench(lme, systems, torch, reps=20):
    """HBM roofline of the streamed Liouvillian application (stage input read
    from HBM, result written back): algorithmic bytes 32 n^2 per instance,
    for the operator form and the explicit superoperator form."""
    w = systems.jc_sweep()
    h = lme.Handle(w.systems)
    y = h.pack([s.rho0 for s in w.systems], device="cuda:0")
    tuned = h.autotune(y, w.nsteps)          # picks the application's LDS budget
    out = torch.empty_like(y)
    nbytes = 32.0 * h.state_elems
    stream = torch.cuda.current_stream()
    res = {"workload": f"jc_sweep batch, 4096 instances ({16 * h.state_elems / 1e6:.1f} MB per "
                       f"state copy)",
           "algorithmic_bytes": nbytes, "apply_lds_kb": tuned["apply_lds_kb"],
           "apply_block": tuned["apply_block"]}
    for name, form in (("operator_lds", lme.LME_FORM_OPERATOR),
                       ("operator_global", lme.LME_FORM_OPERATOR_STREAMED),
                       ("superop", lme.LME_FORM_SUPEROP)):
        for _ in range(2):
            lme.load().lme_apply(h._h, form, 0, 0.0, None, lme._ptr(y), lme._ptr(out),
                                 lme._stream_ptr(stream))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            rc = lme.load().lme_apply(h._h, form, 0, 0.0, None, lme._ptr(y), lme._ptr(out),
                                      lme._stream_ptr(stream))
            assert rc == 0
        b.record(stream)
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / reps
        gbs = nbytes / (us * 1e-6) / 1e9
        res[name] = {"us_per_apply": us, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    res["operator_lds"]["kernel"] = "apply_pipe_kernel" if tuned["apply_path"] == 0 else \
        "apply_col_kernel"
    res["operator_lds"]["traffic"] = kernel_traffic(res["operator_lds"]["kernel"])
    # device copy of the same bytes (one state read, one written) for reference
    src = torch.empty_like(y)
    for _ in range(2):
        out.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        out.copy_(src)
    b.record(stream)
    torch.cuda.synchronize()
    cus = a.elapsed_time(b) * 1e3 / reps
    res["device_copy"] = {"us": cus, "GBs": nbytes / (cus * 1e-6) / 1e9}
    res["operator_lds"]["frac_of_copy"] = res["device_copy"]["us"] / res["operator_lds"]["us_per_apply"]
    return res


def tfim_apply_bench(lme, systems, torch, reps=10):
    """HBM roofline of the Liouvillian application on 8-spin chains (n = 256,
    1 MiB per state): 64 realizations (134 MB per application) and 512 (1.07
    GB, past the last-level cache).  Algorithmic bytes 32 n^2 per instance.
    The default form runs the row-block kernel; the plain streamed kernel
    (every gather from memory) and a device copy of the same bytes are timed
    beside it."""
    res = {}
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(2):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e3 / reps

    for n_inst in (64, 512):
        w = systems.tfim(n_inst=n_inst)
        h = lme.Handle(w.systems)
        y = h.pack([s.rho0 for s in w.systems], device="cuda:0")
        y.copy_(torch.randn_like(y))   # every element populated
        out = torch.empty_like(y)
        nbytes = 32.0 * h.state_elems
        r = {"algorithmic_bytes": nbytes}
        for name, form in (("row_blocks", lme.LME_FORM_OPERATOR),
                           ("plain_streamed", lme.LME_FORM_OPERATOR_STREAMED)):
            def go(form=form):
                rc = lme.load().lme_apply(h._h, form, 0, 0.0, None, lme._ptr(y), lme._ptr(out),
                                          lme._stream_ptr(stream))
                assert rc == 0
            us = timed(go)
            gbs = nbytes / (us * 1e-6) / 1e9
            r[name] = {"us_per_apply": us, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
        src = torch.empty_like(y)
        cus = timed(lambda: out.copy_(src))
        r["row_blocks"]["kernel"] = "apply_rows_kernel"
        if n_inst == 64:
            r["row_blocks"]["traffic"] = kernel_traffic("apply_rows_kernel")
        r["device_copy"] = {"us": cus, "GBs": nbytes / (cus * 1e-6) / 1e9}
        r["row_blocks"]["frac_of_copy"] = cus / r["row_blocks"]["us_per_apply"]
        res[f"tfim_8spin_x{n_inst}"] = r
        del h, y, out, src
        torch.cuda.empty_cache()
    return res


def other_configs(lme, systems, torch):
    """Wall time of each of the other headline configurations, one run after a
    warm-up (HIP events on the launch stream; the adaptive streamed path
    includes its host polling)."""
    stream = torch.cuda.current_stream()
    res = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b), out

    w = systems.jc_single()
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    ms, _ = timed(lambda: h.evolve(r0, w.tlist, nsteps=w.nsteps, hermitian=True))
    ms_full, _ = timed(lambda: h.evolve(r0, w.tlist, nsteps=w.nsteps))
    res["jc_single_N10_rk4_2500"] = {"ms": ms, "instance_steps_per_s": w.nsteps / (ms * 1e-3),
                                     "path": "hermitian", "full_path_ms": ms_full}

    w = systems.kerr_single()
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    ms, out = timed(lambda: h.evolve(r0, w.tlist, method="dopri5", rtol=w.rtol, atol=w.atol))
    acc, rej = (int(x) for x in out["counts"].cpu().numpy()[0])
    res["kerr_N60_dopri5_t50"] = {"ms": ms, "accepted": acc, "rejected": rej,
                                  "instance_steps_per_s": acc / (ms * 1e-3)}

    w = systems.jc_drive()
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    O = h.pack([w.extra["target"]] * len(w.systems))
    u = torch.from_numpy(w.extra["u"]).cuda()
    ms, _ = timed(lambda: lme._cost_grad(h, r0, O, u, 0.0, 10.0, w.nsteps, 10))
    res["jc_drive_256_cost_grad"] = {"ms": ms, "forward_instance_steps_per_s":
                                     len(w.systems) * w.nsteps / (ms * 1e-3)}

    w = systems.tfim()
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    ms, out = timed(lambda: h.evolve(r0, w.tlist, method="dopri5", rtol=w.rtol, atol=w.atol))
    acc = out["counts"].cpu().numpy()[:, 0]
    res["tfim_8spin_64_dopri5_t20"] = {"ms": ms, "accepted_mean": float(acc.mean()),
                                       "instance_steps_per_s": float(acc.sum()) / (ms * 1e-3),
                                       "path": "streamed"}

    w = systems.landau_zener_sweep()
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    ms, _ = timed(lambda: h.evolve(r0, w.tlist, nsteps=w.nsteps, hermitian=True))
    res["landau_zener_4096_rk4"] = {"ms": ms, "instance_steps_per_s":
                                    len(w.systems) * w.nsteps / (ms * 1e-3),
                                    "amplitudes": "closed form, evaluated per stage"}

    w = systems.jc_correlation_sweep()
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    ms, _ = timed(lambda: h.correlation(r0, w.tlist, w.nsteps, w.extra["taulist"],
                                        w.extra["tau_nsteps"], w.extra["B"], hermitian=True))
    n_evol = len(w.systems) * (1 + len(w.tlist))
    res["jc_correlation_64x26x101"] = {"ms": ms, "instance_steps_per_s":
                                       n_evol * w.nsteps / (ms * 1e-3)}
    res["jc_steady_16_dim32"] = steady_state_bench(lme, systems, torch)
    return res


def pmc_pass(lme, systems, torch):
    """One dispatch of each kernel of interest plus a copy of known size."""
    w = systems.jc_sweep()
    h = lme.Handle(w.systems)
    rho0 = h.pack([s.rho0 for s in w.systems], device="cuda:0")
    h.set_tuning(rk4_layout=lme.LME_LAYOUT_COLUMN, rk4_block=768, apply_cap=8192,
                 herm_layout=lme.LME_LAYOUT_COLUMN, herm_block=768)
    h.evolve(rho0, w.tlist, method="rk4", nsteps=w.nsteps)
    h.evolve(rho0, w.tlist, method="rk4", nsteps=w.nsteps, hermitian=True)
    out = torch.empty_like(rho0)
    for form in (lme.LME_FORM_OPERATOR, lme.LME_FORM_OPERATOR_STREAMED, lme.LME_FORM_SUPEROP):
        rc = lme.load().lme_apply(h._h, form, 0, 0.0, None, lme._ptr(rho0), lme._ptr(out),
                                  lme._stream_ptr(None))
        assert rc == 0
    # the row-block application on 64 8-spin chains
    wt = systems.tfim(n_inst=64)
    ht = lme.Handle(wt.systems)
    yt = ht.pack([s.rho0 for s in wt.systems], device="cuda:0")
    yt.copy_(torch.randn_like(yt))
    ot = torch.empty_like(yt)
    rc = lme.load().lme_apply(ht._h, lme.LME_FORM_OPERATOR, 0, 0.0, None, lme._ptr(yt),
                              lme._ptr(ot), lme._stream_ptr(None))
    assert rc == 0
    # the other configurations' kernels, on short horizons
    wk = systems.kerr_single()
    hk = lme.Handle(wk.systems)
    hk.evolve(hk.pack([s.rho0 for s in wk.systems]), np.linspace(0.0, 5.0, 11), method="dopri5",
              rtol=wk.rtol, atol=wk.atol)
    wt5 = systems.tfim()
    ht5 = lme.Handle(wt5.systems)
    ht5.evolve(ht5.pack([s.rho0 for s in wt5.systems]), np.linspace(0.0, 1.0, 11),
               method="dopri5", rtol=wt5.rtol, atol=wt5.atol)
    wd = systems.jc_drive()
    hd = lme.Handle(wd.systems)
    lme._cost_grad(hd, hd.pack([s.rho0 for s in wd.systems]),
                   hd.pack([wd.extra["target"]] * len(wd.systems)),
                   torch.from_numpy(wd.extra["u"]).cuda(), 0.0, 10.0, wd.nsteps, 10)
    wm = systems.trilinear_mc_workload()
    sm = wm.systems[0]
    hm = lme.McHandle(sm.H0, sm.C, sm.E)
    hm.evolve(torch.from_numpy(sm.meta["psi0"]).cuda(), wm.tlist, wm.nsteps,
              torch.from_numpy(wm.extra["draws"]).cuda(), want_traj=False)
    ws = systems.jc_steady_sweep()
    lme.Handle(ws.systems).steadystate(float(ws.tlist[-1]), ws.nsteps)
    src = torch.ones(32 * 2**20, dtype=torch.float64, device="cuda:0")   # 256 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_pass": "done", "copy_bytes_each_way": src.numel() * 8,
                      "state_bytes": 16 * h.state_elems,
                      "tfim_state_bytes": 16 * ht.state_elems}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--layout", type=int, default=0)
    ap.add_argument("--full", action="store_true",
                    help="headline without the Hermitian path (every element computed)")
    ap.add_argument("--plain-sample", type=int, default=32)
    ap.add_argument("--cpu-sample", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the timings of the other headline configurations")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="run one of each kernel (and a 256 MiB device copy as the counter "
                         "reference) for a rocprofv3 --pmc pass, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the batch of "
                          "independent instances would shard by instance across GPUs with no "
                          "communication; only the single-GPU share is measured",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1110_0573_amd import lme, systems

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.pmc_pass:
        pmc_pass(lme, systems, torch)
        return
    w = systems.jc_sweep()
    n_inst = len(w.systems)
    h = lme.Handle(w.systems)
    rho0 = h.pack([s.rho0 for s in w.systems], device="cuda:0")
    stream = torch.cuda.current_stream()

    herm = not args.full   # density matrices: rho0 is Hermitian
    tuning = None
    if args.block == 0 and args.layout == 0:
        # outside the timed region; the full-path tuning serves the comparison
        tuning = h.autotune(rho0, w.nsteps, hermitian=herm, stream=stream)
        if herm:
            h.autotune(rho0, w.nsteps, hermitian=False, stream=stream)

    def one(hermitian=herm):
        return h.evolve(rho0, w.tlist, method="rk4", nsteps=w.nsteps, block=args.block,
                        layout=args.layout, hermitian=hermitian, stream=stream)

    def timed_steps(hermitian):
        for _ in range(args.warmup):
            one(hermitian)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            out = one(hermitian)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert (out["status"].cpu().numpy() == 0).all()
        return wall * 1e3 / args.steps, [a.elapsed_time(b) for a, b in ev]

    ms_per_step, kern_ms = timed_steps(herm)
    inst_steps = n_inst * w.nsteps
    value = inst_steps / (ms_per_step * 1e-3)
    full_path = None
    if herm:
        f_ms, f_kern = timed_steps(False)
        f_flops = sum(rk4_step_flops(s) for s in w.systems) * w.nsteps
        f_kms = float(np.mean(f_kern))
        full_path = {"value": inst_steps / (f_ms * 1e-3), "ms_per_step": f_ms,
                     "kernel_ms": f_kms,
                     "achieved_tflops": f_flops / (f_kms * 1e-3) / 1e12,
                     "frac": f_flops / (f_kms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS}

    step_flops = rk4_step_flops_hermitian if herm else rk4_step_flops
    flops = sum(step_flops(s) for s in w.systems) * w.nsteps
    survey_flops = sum(4.0 * survey_apply_flops(s) for s in w.systems) * w.nsteps
    k_ms = float(np.mean(kern_ms))
    achieved = flops / (k_ms * 1e-3) / 1e12
    survey_tflops = survey_flops / (k_ms * 1e-3) / 1e12
    # LDS: the resident kernel's own bound (its state never leaves the chip)
    if herm:
        elem_stages = [4.0 * w.nsteps * s.n * (s.n + 1) / 2 for s in w.systems]
        lds_bytes = sum(e * herm_lds_bytes_per_element_stage(s)
                        for e, s in zip(elem_stages, w.systems))
    else:
        lds_bytes = None
    lds_peak = lds_peak_tbs(lme, torch)
    # HBM bytes the path must move: rho0 in, final rho out, expectations out
    hbm_bytes = 2 * 16 * h.state_elems + 16 * n_inst * 2 * len(w.tlist)

    # plain: the same instances integrated one per launch
    rng = np.random.default_rng(7)
    pidx = rng.choice(n_inst, args.plain_sample, replace=False)
    plain = [lme.Handle([w.systems[i]]) for i in pidx]
    prho = [p.pack([w.systems[i].rho0], device="cuda:0") for p, i in zip(plain, pidx)]
    for p, r in zip(plain, prho):
        p.evolve(r, w.tlist, method="rk4", nsteps=w.nsteps, block=args.block,
                 layout=args.layout, hermitian=herm, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for p, r in zip(plain, prho):
        p.evolve(r, w.tlist, method="rk4", nsteps=w.nsteps, block=args.block,
                 layout=args.layout, hermitian=herm, stream=stream)
    torch.cuda.synchronize()
    plain_rate = args.plain_sample * w.nsteps / (time.perf_counter() - t1)

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "instance-RK-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "jc_sweep: 4096 Jaynes-Cummings instances, N in {5..40} "
                               "(dims 10..80), fixed-step RK4, 1000 steps, 101 outputs",
                   "instances": n_inst, "rk_steps": w.nsteps, "outputs": len(w.tlist),
                   "state_MB": 16 * h.state_elems / 1e6, "path": "resident",
                   "hermitian": herm,
                   "block": args.block or "tuned", "layout": args.layout or "tuned",
                   "tuning": tuning},
        "roofline": ({"bound": "lds", "achieved": lds_bytes / (k_ms * 1e-3) / 1e12,
                      "peak": lds_peak, "unit": "TB/s",
                      "frac": lds_bytes / (k_ms * 1e-3) / 1e12 / lds_peak,
                      "algorithmic_lds_bytes": lds_bytes,
                      "lds_bytes_per_element_stage": herm_lds_bytes_per_element_stage(w.systems[0]),
                      "peak_source": "measured: LDS read probe (ds_read_b128, no bank conflicts)"}
                     if herm else
                     {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                      "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS}) | {
                     "traffic": kernel_traffic("rk4_herm_kernel" if herm else "rk4_colown_kernel"),
                     "kernel": "rk4_herm_kernel" if herm else "rk4_colown_kernel",
                     "kernel_ms": k_ms,
                     "flops": {"scope_table_count": survey_flops,
                               "achieved_tflops": survey_tflops, "peak": FP64_VECTOR_PEAK_TFLOPS,
                               "frac": survey_tflops / FP64_VECTOR_PEAK_TFLOPS,
                               "path_count": flops, "path_achieved_tflops": achieved,
                               "path_frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                               "note": "scope_table_count: 4 x (8 n nnz(A) + 2 n^2 + 8 n^2 K) "
                                       "per step; path_count: the elements this path computes "
                                       "(n(n+1)/2 per instance on the Hermitian path)"}},
        "hbm": {"algorithmic_bytes": hbm_bytes, "GBs": hbm_bytes / (k_ms * 1e-3) / 1e9,
                "note": "state stays on chip for all steps; HBM moves rho0, rho, outputs"},
        "batched_vs_plain": {"plain_value": plain_rate, "speedup": value / plain_rate,
                             "plain_sample": int(args.plain_sample)},
    }
    if full_path:
        rec["full_path"] = full_path
    rec["streamed_apply"] = streamed_apply_bench(lme, systems, torch)
    rec["mc_trilinear"] = mc_trilinear_bench(lme, systems, torch)
    rec["streamed_apply_tfim"] = tfim_apply_bench(lme, systems, torch)
    if not args.no_configs:
        rec["other_configs"] = other_configs(lme, systems, torch)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_sample, w.nsteps, systems,
                                           with_configs=not args.no_configs)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
