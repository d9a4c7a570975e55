"""GPU parity of closed-form time-dependent amplitudes (Sec. 4.4) against
the oracle: u(t) = c0 + c1 t + c2 t^2 + c3 t^3 + a cos(w t + phi), every RK4
stage at its own time.  Bar: trace distance 1e-10 at every output time (the
fixed-step bar), all kernel layouts bit for bit equal."""
import numpy as np
import pytest

import oracle
from paper_1110_0573_amd import systems as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1110_0573_amd import lme  # noqa: E402
from tests import brute  # noqa: E402

TD = 1e-10


def evolve(systems, tlist, nsteps, **kw):
    h = lme.Handle(systems)
    out = h.evolve(h.pack([s.rho0 for s in systems]), tlist, nsteps=nsteps, want_states=True,
                   **kw)
    torch.cuda.synchronize()
    assert (out["status"].cpu().numpy() == 0).all()
    return h, out


def check(h, out, systems, tlist, nsteps, every=1):
    st = h.unpack(out["states"])
    ex = out["expect"].cpu().numpy()
    for b, s in enumerate(systems):
        if b % every:
            continue
        oex, ost = oracle.rk4(s, s.rho0, tlist, nsteps, store_states=True)
        td = max(brute.trace_distance(st[b][k], ost[k]) for k in range(len(tlist)))
        assert td <= TD, (b, td)
        assert np.max(np.abs(ex[b] - oex)) <= TD


def test_landau_zener_sweep_matches_oracle():
    """Landau-Zener problems with different sweep rates and relaxation, the
    paper's time grid (t in [-10, 10], 1500 outputs), 20 steps per output."""
    w = S.landau_zener_sweep(n_inst=48, seed=31)
    h, out = evolve(w.systems, w.tlist, w.nsteps)
    check(h, out, w.systems, w.tlist, w.nsteps, every=4)


def test_driven_jc_all_layouts_bitwise_and_oracle():
    """Qubit x cavity (N = 5) with a drive a + a^+ whose amplitude is a cubic
    plus a cosine: row layout, column layout and the Hermitian kernel agree
    bit for bit (full paths) or to rounding (Hermitian), and with the oracle."""
    systems = []
    for k in range(6):
        s = S.jc_system(5, g=0.3 + 0.05 * k, kappa=0.05, gamma=0.02, psi0=(k % 2, 1))
        a = S.jc_ops(5)[0]
        s.H_ctrl = [S.tidy(a + S.dag(a))]
        s.fn = S.coeff_fn(0.05 * k, 0.1, -0.02, 0.003, 0.3, 1.7 + 0.1 * k, 0.2 * k)[None, :]
        systems.append(s)
    tl = np.linspace(-1.0, 3.0, 9)
    ns = 800
    hr, row = evolve(systems, tl, ns, layout=lme.LME_LAYOUT_ROW)
    hc, col = evolve(systems, tl, ns, layout=lme.LME_LAYOUT_COLUMN)
    for k in ("expect", "states", "rho"):
        assert torch.equal(row[k], col[k]), k
    check(hr, row, systems, tl, ns)
    hh, herm = evolve(systems, tl, ns, hermitian=True)
    assert torch.max(torch.abs(herm["states"] - row["states"])).item() < 1e-13
    # the handle can return to piecewise-constant segments (all zero here)
    hr.set_coeff_fn(None)
    zero = hr.evolve(hr.pack([s.rho0 for s in systems]), tl, nsteps=ns)
    torch.cuda.synchronize()
    base = [S.System(s.H0, s.C, s.E, s.rho0) for s in systems]
    hb, ref = evolve(base, tl, ns)
    assert torch.max(torch.abs(zero["rho"] - ref["rho"])).item() < 1e-14


def test_apply_at_time_t_and_refusals():
    """lme_apply evaluates the amplitudes at its t; the adaptive stepper,
    the streamed path, the gradient and a u override refuse them."""
    systems = [S.random_system(5, n_c=2, n_ctrl=2, seed=40 + k, hermitian_rho=False)
               for k in range(3)]
    for k, s in enumerate(systems):
        s.fn = np.array([S.coeff_fn(0.1 * k, 0.4, -0.2, 0.01, 0.8, 2.0, 0.3),
                         S.coeff_fn(-0.3, 0.0, 0.1, 0.0, 0.5, 0.9, -0.7)])
    h = lme.Handle(systems)
    y = h.pack([s.rho0 for s in systems])
    for t in (0.0, 0.37, -1.25):
        out = h.unpack(h.apply(y, t=t))
        for b, s in enumerate(systems):
            want = oracle.apply_L(s, s.rho0, t=t)
            assert np.max(np.abs(out[b] - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))
    tl = np.array([0.0, 1.0])
    for kw, code in ((dict(method="dopri5"), lme.LME_ENOTSUP),
                     (dict(nsteps=10, path=lme.LME_PATH_STREAMED), lme.LME_ENOTSUP),
                     (dict(nsteps=10, u=torch.zeros(0, dtype=torch.float64, device="cuda")),
                      lme.LME_EINVAL)):
        with pytest.raises(lme.LmeError) as e:
            h.evolve(y, tl, **kw)
        assert e.value.code == code, kw
    with pytest.raises(lme.LmeError) as e:
        lme._cost_grad(h, y, y, None, 0.0, 1.0, 10, 2)
    assert e.value.code in (lme.LME_ENOTSUP, lme.LME_EINVAL)


def test_landau_zener_sweep_as_benchmarked_sampled():
    """The benchmark's sweep (4096 problems, 1500 outputs, 29 980 RK4 steps):
    every instance finishes, a seeded sample of 8 matches the oracle."""
    w = S.landau_zener_sweep()
    h = lme.Handle(w.systems)
    out = h.evolve(h.pack([s.rho0 for s in w.systems]), w.tlist, nsteps=w.nsteps,
                   hermitian=True)
    torch.cuda.synchronize()
    assert (out["status"].cpu().numpy() == 0).all()
    ex = out["expect"].cpu().numpy()
    rho = h.unpack(out["rho"])
    for b in np.sort(np.random.default_rng(5).choice(len(w.systems), 8, replace=False)):
        s = w.systems[b]
        oex, ost = oracle.rk4(s, s.rho0, w.tlist, w.nsteps, store_states=True)
        assert brute.trace_distance(rho[b], ost[-1]) <= TD
        assert np.max(np.abs(ex[b] - oex)) <= TD


def test_small_instances_lane_kernel_bitwise_row_kernel():
    """Batches of instances with n^2 <= 64 run one element per lane (one
    wavefront per pack, the stage input exchanged between lanes, no LDS in a
    stage); they give the bits of the row kernel at 256 threads: Landau-Zener
    problems with closed-form amplitudes, and qubit x cavity systems
    (N = 2..4) with two piecewise-constant controls and three collapse
    operators, which also match the oracle."""
    w = S.landau_zener_sweep(n_inst=40, seed=5, n_out=51, steps_per_out=120)
    _, lane = evolve(w.systems, w.tlist, w.nsteps)
    _, row = evolve(w.systems, w.tlist, w.nsteps, block=256)
    for k in ("expect", "states", "rho"):
        assert torch.equal(lane[k], row[k]), k
    rng = np.random.default_rng(23)
    systems = []
    for b in range(10):
        N = 2 + b % 3
        s = S.jc_system(N, g=0.3 + 0.02 * b, kappa=0.1, gamma=0.05, n_th=0.2, psi0=(b % 2, 1))
        a = S.jc_ops(N)[0]
        s.H_ctrl = [S.tidy(a + S.dag(a)), S.tidy(1j * (S.dag(a) - a))]
        s.edges = np.linspace(0.0, 2.0, 5)
        s.u = rng.normal(0.0, 0.5, size=(2, 4))
        systems.append(s)
    tl = np.linspace(0.0, 2.0, 11)
    hl, lane = evolve(systems, tl, 400)
    _, row = evolve(systems, tl, 400, block=256)
    for k in ("expect", "states", "rho"):
        assert torch.equal(lane[k], row[k]), k
    check(hl, lane, systems, tl, 400, every=3)
