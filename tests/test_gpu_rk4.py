"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: fixed-step RK4 states within trace distance 1e-10 of the oracle,
expectation values within 1e-10 absolute; Liouvillian application within
1e-12 relative to the largest entry.  Batched and single runs, runs with
different workgroup sizes and repeated runs must agree bit for bit (every
element is computed by the same arithmetic in the same order).
"""
import numpy as np
import pytest

import oracle
from paper_1110_0573_amd import systems as S
from tests import brute

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1110_0573_amd import lme  # noqa: E402

TD_BAR = 1e-10


def run(systems, tlist, nsteps, **kw):
    h = lme.Handle(systems)
    rho0 = h.pack([s.rho0 for s in systems])
    out = h.evolve(rho0, tlist, method="rk4", nsteps=nsteps, **kw)
    torch.cuda.synchronize()
    return h, out


def td(a, b):
    return brute.trace_distance(a, b)


# --------------------------------------------------------------------------
# Liouvillian application
# --------------------------------------------------------------------------

@pytest.mark.parametrize("adjoint", [False, True])
def test_apply_matches_oracle_random_batch(adjoint):
    systems = [S.random_system(n, n_c=nc, n_ctrl=2, n_seg=3, seed=100 + n, t_end=1.0,
                               hermitian_rho=False)
               for n, nc in [(1, 1), (3, 0), (5, 2), (7, 3), (12, 2), (5, 1)]]
    h = lme.Handle(systems)
    y = h.pack([s.rho0 for s in systems])
    t = 0.5
    out = h.unpack(h.apply(y, t=t, adjoint=adjoint))
    for s, got in zip(systems, out):
        f = oracle.apply_Ldag if adjoint else oracle.apply_L
        want = f(s, s.rho0, t=t)
        assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


def test_apply_jc_sweep_tiles():
    w = S.jc_sweep(n_inst=40, seed=11, coherent=True)
    h = lme.Handle(w.systems)
    y = h.pack([s.rho0 for s in w.systems])
    out = h.unpack(h.apply(y))
    for s, got in zip(w.systems, out):
        want = oracle.apply_L(s, s.rho0)
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("adjoint", [False, True])
def test_apply_streamed_matches_oracle(adjoint):
    systems = [S.random_system(n, n_c=nc, n_ctrl=2, n_seg=3, seed=400 + n, t_end=1.0,
                               hermitian_rho=False)
               for n, nc in [(1, 1), (3, 0), (47, 2), (7, 3), (64, 2)]]
    h = lme.Handle(systems)
    y = h.pack([s.rho0 for s in systems])
    out = h.unpack(h.apply(y, t=0.7, adjoint=adjoint, form=lme.LME_FORM_OPERATOR_STREAMED))
    for s, got in zip(systems, out):
        f = oracle.apply_Ldag if adjoint else oracle.apply_L
        want = f(s, s.rho0, t=0.7)
        assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


def test_apply_superoperator_matches_oracle():
    systems = [S.random_system(n, n_c=nc, seed=500 + n, hermitian_rho=False)
               for n, nc in [(1, 1), (4, 0), (9, 3), (30, 2)]]
    systems += S.jc_sweep(n_inst=6, seed=5, coherent=True).systems
    h = lme.Handle(systems)
    y = h.pack([s.rho0 for s in systems])
    out = h.unpack(h.apply(y, form=lme.LME_FORM_SUPEROP))
    for s, got in zip(systems, out):
        want = oracle.apply_L(s, s.rho0)
        assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


def test_apply_large_instance_routes_to_streamed():
    """n = 2*72 = 144: the stage input (324 KB) exceeds LDS."""
    s = S.jc_system(72, g=0.2, kappa=0.01, gamma=0.02)
    s.rho0 = S.ket2dm(np.kron(S.coherent_ket(72, 2.0), S.ket(2, 1)))
    h = lme.Handle([s])
    out = h.unpack(h.apply(h.pack([s.rho0])))[0]
    want = oracle.apply_L(s, s.rho0)
    assert np.max(np.abs(out - want)) <= 1e-12 * np.max(np.abs(want))


# --------------------------------------------------------------------------
# fixed-step RK4
# --------------------------------------------------------------------------

def test_rk4_jc_single_all_output_states():
    """Headline single instance: N=10, 2500 steps, 101 outputs."""
    w = S.jc_single()
    s = w.systems[0]
    h, out = run([s], w.tlist, w.nsteps, want_states=True)
    st = h.unpack(out["states"])[0]
    ex = out["expect"].cpu().numpy()[0]
    oex, ost = oracle.rk4(s, s.rho0, w.tlist, w.nsteps, store_states=True)
    worst = max(td(a, b) for a, b in zip(st, ost))
    assert worst <= TD_BAR, worst
    assert np.max(np.abs(ex - oex)) <= TD_BAR
    assert out["status"].cpu().numpy()[0] == 0
    assert tuple(out["counts"].cpu().numpy()[0]) == (w.nsteps, 0)


def test_rk4_sweep_ragged_batch_matches_oracle():
    """64 instances, cutoffs 5..40 (dims 10..80): many packs, ragged tails."""
    w = S.jc_sweep(n_inst=64, seed=21, nsteps=200, t_end=5.0, n_out=21)
    h, out = run(w.systems, w.tlist, w.nsteps)
    ex = out["expect"].cpu().numpy()
    rho = h.unpack(out["rho"])
    oex = oracle.rk4_batch(w.systems, [s.rho0 for s in w.systems], w.tlist, w.nsteps, 8)
    for b, s in enumerate(w.systems):
        assert np.max(np.abs(ex[b] - oex[b])) <= TD_BAR
    # final states of a sample
    for b in range(0, 64, 7):
        s = w.systems[b]
        _, ost = oracle.rk4(s, s.rho0, w.tlist, w.nsteps, store_states=True)
        assert td(rho[b], ost[-1]) <= TD_BAR


def test_rk4_coherent_state_full_occupancy():
    w = S.jc_sweep(n_inst=10, seed=31, nsteps=100, t_end=2.5, n_out=11, coherent=True)
    h, out = run(w.systems, w.tlist, w.nsteps)
    rho = h.unpack(out["rho"])
    for b, s in enumerate(w.systems):
        _, ost = oracle.rk4(s, s.rho0, w.tlist, w.nsteps, store_states=True)
        assert td(rho[b], ost[-1]) <= TD_BAR


def test_rk4_piecewise_constant_controls():
    w = S.jc_drive(n_inst=6, N=5, n_seg=10, t_end=2.0, steps_per_seg=4, sigma_u=0.5)
    tl = np.linspace(0.0, 2.0, 11)
    h, out = run(w.systems, tl, w.nsteps)
    ex = out["expect"].cpu().numpy()
    rho = h.unpack(out["rho"])
    for b, s in enumerate(w.systems):
        oex, ost = oracle.rk4(s, s.rho0, tl, w.nsteps, store_states=True)
        assert np.max(np.abs(ex[b] - oex)) <= TD_BAR
        assert td(rho[b], ost[-1]) <= TD_BAR
    # amplitudes given per call override those given at create
    u = np.random.default_rng(3).normal(size=(6, 1, 10))
    out2 = h.evolve(h.pack([s.rho0 for s in w.systems]), tl, nsteps=w.nsteps,
                    u=torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    ex2 = out2["expect"].cpu().numpy()
    for b, s in enumerate(w.systems):
        oex, _ = oracle.rk4(s, s.rho0, tl, w.nsteps, u=u[b])
        assert np.max(np.abs(ex2[b] - oex)) <= TD_BAR


def test_rk4_random_general_operators_and_edge_dims():
    systems = [S.random_system(n, n_c=nc, n_e=2, seed=200 + n) for n, nc in
               [(1, 1), (2, 0), (4, 3), (9, 2)]]
    tl = np.linspace(0.0, 1.0, 6)
    h, out = run(systems, tl, 50, want_states=True)
    st = h.unpack(out["states"])
    ex = out["expect"].cpu().numpy()
    for b, s in enumerate(systems):
        oex, ost = oracle.rk4(s, s.rho0, tl, 50, store_states=True)
        assert max(td(a, c) for a, c in zip(st[b], ost)) <= TD_BAR
        assert np.max(np.abs(ex[b] - oex)) <= TD_BAR


def test_rk4_single_output_time_no_steps():
    w = S.jc_sweep(n_inst=3, seed=41)
    h, out = run(w.systems, np.array([1.5]), 0)
    ex = out["expect"].cpu().numpy()
    for b, s in enumerate(w.systems):
        want = [np.trace(e.toarray() @ s.rho0) for e in s.E]
        np.testing.assert_allclose(ex[b, :, 0], want, atol=1e-14)
    rho = h.unpack(out["rho"])
    for b, s in enumerate(w.systems):
        np.testing.assert_array_equal(rho[b], s.rho0)


def test_rk4_batched_equals_single_and_layouts_bitwise():
    """Row layout (block 256/512/1024), column layout (block 512/768) and
    single-instance runs give identical bits."""
    w = S.jc_sweep(n_inst=24, seed=51, nsteps=60, t_end=1.5, n_out=7)
    _, ref = run(w.systems, w.tlist, w.nsteps, block=512, layout=lme.LME_LAYOUT_ROW)
    ref_ex = ref["expect"].cpu().numpy()
    ref_rho = ref["rho"].cpu().numpy()
    variants = [(256, lme.LME_LAYOUT_ROW), (1024, lme.LME_LAYOUT_ROW),
                (512, lme.LME_LAYOUT_COLUMN), (768, lme.LME_LAYOUT_COLUMN), (0, 0)]
    for block, layout in variants:
        _, o = run(w.systems, w.tlist, w.nsteps, block=block, layout=layout)
        assert np.array_equal(o["expect"].cpu().numpy(), ref_ex), (block, layout)
        assert np.array_equal(o["rho"].cpu().numpy(), ref_rho), (block, layout)
    h_all = lme.Handle(w.systems)
    rho_all = h_all.unpack(torch.from_numpy(ref_rho))
    for b in (0, 5, 23):
        hs, o = run([w.systems[b]], w.tlist, w.nsteps)
        assert np.array_equal(o["expect"].cpu().numpy()[0], ref_ex[b])
        assert np.array_equal(hs.unpack(o["rho"])[0], rho_all[b])


def test_rk4_column_layout_with_controls_and_thermal_jumps():
    """Column layout with one control term and three collapse operators."""
    w = S.jc_drive(n_inst=5, N=6, n_seg=5, t_end=1.0, steps_per_seg=4, sigma_u=0.7)
    for s in w.systems:
        s.C.append(S.tidy(np.sqrt(0.02) * S.dag(S.jc_ops(6)[0])))
    tl = np.linspace(0.0, 1.0, 6)
    h, out = run(w.systems, tl, w.nsteps, layout=lme.LME_LAYOUT_COLUMN)
    _, ref = run(w.systems, tl, w.nsteps, layout=lme.LME_LAYOUT_ROW)
    assert np.array_equal(out["rho"].cpu().numpy(), ref["rho"].cpu().numpy())
    rho = h.unpack(out["rho"])
    for b, s in enumerate(w.systems):
        _, ost = oracle.rk4(s, s.rho0, tl, w.nsteps, store_states=True)
        assert td(rho[b], ost[-1]) <= TD_BAR


def test_rk4_column_layout_complex_coupling():
    """A complex coupling phase makes the off-diagonal of A non-imaginary: the
    column layout takes its general-complex specialisation."""
    systems = [S.jc_system(N, g=0.3, kappa=0.02, gamma=0.04, phase=0.7 + 0.1 * N,
                           n_th=0.1) for N in (3, 7, 12, 20)]
    tl = np.linspace(0.0, 2.0, 5)
    h, out = run(systems, tl, 80, layout=lme.LME_LAYOUT_COLUMN)
    _, ref = run(systems, tl, 80, layout=lme.LME_LAYOUT_ROW)
    assert np.array_equal(out["rho"].cpu().numpy(), ref["rho"].cpu().numpy())
    rho = h.unpack(out["rho"])
    for b, s in enumerate(systems):
        _, ost = oracle.rk4(s, s.rho0, tl, 80, store_states=True)
        assert td(rho[b], ost[-1]) <= TD_BAR


def test_rk4_column_layout_rejects_general_jumps():
    s = S.random_system(4, n_c=2, seed=5)
    h = lme.Handle([s])
    with pytest.raises(lme.LmeError) as e:
        h.evolve(h.pack([s.rho0]), np.array([0.0, 1.0]), nsteps=4, layout=lme.LME_LAYOUT_COLUMN)
    assert e.value.code == lme.LME_ENOTSUP


def test_autotune_keeps_results_and_tuning_roundtrip():
    w = S.jc_sweep(n_inst=40, seed=91, nsteps=50, t_end=1.25, n_out=6)
    h = lme.Handle(w.systems)
    rho0 = h.pack([s.rho0 for s in w.systems])
    ref = h.evolve(rho0, w.tlist, nsteps=w.nsteps, layout=lme.LME_LAYOUT_ROW, block=512)
    ref_apply = h.apply(rho0)
    t = h.autotune(rho0, w.nsteps)
    assert t["rk4_block"] in (256, 512, 768, 1024) and t["apply_cap"] >= 256
    assert t["apply_lds_kb"] in (0, 27, 40, 53, 80) and t["apply_block"] in (256, 512, 1024)
    assert t["rk4_ms_per_step"] > 0 and t["apply_us"] > 0
    out = h.evolve(rho0, w.tlist, nsteps=w.nsteps)
    torch.cuda.synchronize()
    assert torch.equal(out["rho"], ref["rho"]) and torch.equal(out["expect"], ref["expect"])
    assert torch.equal(h.apply(rho0), ref_apply)
    h.set_tuning(apply_cap=1024, rk4_block=256, rk4_layout=lme.LME_LAYOUT_ROW)
    tt = h.get_tuning()
    assert tt.apply_cap == 1024 and tt.rk4_block == 256
    with pytest.raises(lme.LmeError):
        h.set_tuning(apply_cap=7)


def test_rk4_deterministic_repeat():
    w = S.jc_sweep(n_inst=16, seed=61, nsteps=40, t_end=1.0, n_out=5)
    _, a = run(w.systems, w.tlist, w.nsteps)
    _, b = run(w.systems, w.tlist, w.nsteps)
    assert np.array_equal(a["expect"].cpu().numpy(), b["expect"].cpu().numpy())
    assert np.array_equal(a["rho"].cpu().numpy(), b["rho"].cpu().numpy())


def test_rk4_nonfinite_input_sets_status():
    w = S.jc_sweep(n_inst=3, seed=71, nsteps=20, t_end=0.5, n_out=3)
    rhos = [s.rho0.copy() for s in w.systems]
    rhos[1][0, 0] = np.nan
    h = lme.Handle(w.systems)
    out = h.evolve(h.pack(rhos), w.tlist, nsteps=w.nsteps)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert st[1] == lme.LME_ENONFINITE and st[0] == 0 and st[2] == 0


def test_rk4_sweep_full_size_sampled():
    """The full sweep (4096 instances, 1000 steps) in the launch configuration
    the benchmark times; sampled instances against the oracle."""
    w = S.jc_sweep()
    h, out = run(w.systems, w.tlist, w.nsteps)
    ex = out["expect"].cpu().numpy()
    rho = h.unpack(out["rho"])
    st = out["status"].cpu().numpy()
    assert (st == 0).all()
    rng = np.random.default_rng(0)
    dims = np.array([s.n for s in w.systems])
    sample = list(rng.choice(4096, 10, replace=False)) + [int(np.argmax(dims)), int(np.argmin(dims))]
    for b in sample:
        s = w.systems[b]
        oex, ost = oracle.rk4(s, s.rho0, w.tlist, w.nsteps, store_states=True)
        assert np.max(np.abs(ex[b] - oex)) <= TD_BAR
        assert td(rho[b], ost[-1]) <= TD_BAR
    # every instance: trace preserved, Hermitian, closed-form first output
    for b in range(0, 4096, 97):
        r = rho[b]
        assert abs(np.trace(r) - 1) < 1e-12
        assert np.max(np.abs(r - r.conj().T)) < 1e-13


# --------------------------------------------------------------------------
# streamed RK4 (state in HBM, graph of 16 steps replayed)
# --------------------------------------------------------------------------

def test_rk4_streamed_bitwise_equals_resident_across_replays():
    w = S.jc_sweep(n_inst=10, seed=111, nsteps=37, t_end=0.925, n_out=38)
    _, ref = run(w.systems, w.tlist, w.nsteps, layout=lme.LME_LAYOUT_ROW, block=512)
    ref_ex, ref_rho = ref["expect"].cpu().numpy(), ref["rho"].cpu().numpy()
    h = lme.Handle(w.systems)
    rho0 = h.pack([s.rho0 for s in w.systems])
    for rep in range(3):
        o = h.evolve(rho0, w.tlist, nsteps=w.nsteps, path=lme.LME_PATH_STREAMED)
        torch.cuda.synchronize()
        assert np.array_equal(o["expect"].cpu().numpy(), ref_ex), rep
        assert np.array_equal(o["rho"].cpu().numpy(), ref_rho), rep
        assert (o["status"].cpu().numpy() == 0).all()
        assert (o["counts"].cpu().numpy()[:, 0] == w.nsteps).all()
        # eager work on the same handle between graph replays (re-captures the graph)
        h.evolve(rho0, w.tlist[:2], nsteps=1, path=lme.LME_PATH_STREAMED)
        h.apply(rho0)
        torch.cuda.synchronize()


def test_rk4_streamed_controls():
    w = S.jc_drive(n_inst=4, N=5, n_seg=10, t_end=2.0, steps_per_seg=4, sigma_u=0.5)
    tl = np.linspace(0.0, 2.0, 11)
    h, out = run(w.systems, tl, w.nsteps, path=lme.LME_PATH_STREAMED)
    _, ref = run(w.systems, tl, w.nsteps, layout=lme.LME_LAYOUT_ROW)
    assert np.array_equal(out["rho"].cpu().numpy(), ref["rho"].cpu().numpy())
    ex = out["expect"].cpu().numpy()
    for b, s in enumerate(w.systems):
        oex, _ = oracle.rk4(s, s.rho0, tl, w.nsteps)
        assert np.max(np.abs(ex[b] - oex)) <= TD_BAR


def test_rk4_large_instance_routes_to_streamed():
    """N = 72 (dim 144, 324 KB per state): too large for a resident workgroup."""
    s = S.jc_system(72, g=0.2, kappa=0.01, gamma=0.02)
    s.rho0 = S.ket2dm(np.kron(S.coherent_ket(72, 2.0), S.ket(2, 1)))
    tl = np.linspace(0.0, 0.5, 3)
    h, out = run([s], tl, 50, want_states=True)
    st = h.unpack(out["states"])[0]
    _, ost = oracle.rk4(s, s.rho0, tl, 50, store_states=True)
    assert max(td(a, b) for a, b in zip(st, ost)) <= TD_BAR
