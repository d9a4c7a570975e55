"""lme_evolve_noalloc (no device allocation during the call) against
lme_evolve on the same inputs: the same kernels run, so every output must be
bitwise equal.  Two calls in a row, the second with a smaller input, check
that what the shared scratch array keeps from one call cannot leak into the
next.  Runs alone or after the other GPU tests."""
import numpy as np
import pytest

from paper_1110_0573_amd import systems as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1110_0573_amd import lme  # noqa: E402

KEYS = ("expect", "rho", "counts", "status")


def both(systems, tlist, **kw):
    h = lme.Handle(systems)
    r0 = h.pack([s.rho0 for s in systems])
    ref = h.evolve(r0, tlist, **kw)
    got = h.evolve(r0, tlist, noalloc=True, **kw)
    torch.cuda.synchronize()
    return ref, got


def assert_same(ref, got):
    for k in KEYS:
        assert torch.equal(ref[k], got[k]), k
    assert (got["status"].cpu().numpy() == 0).all()


def test_noalloc_dopri5_twice_second_smaller():
    """Adaptive stepper: stage derivatives in the scratch array.  First a
    ragged batch of 24 instances, then a smaller batch of 3."""
    w = S.jc_sweep(n_inst=24, seed=91, t_end=2.0, n_out=5, coherent=True)
    ref, got = both(w.systems, w.tlist, method="dopri5", rtol=1e-7, atol=1e-10)
    assert_same(ref, got)
    w2 = S.jc_sweep(n_inst=3, seed=92, t_end=1.0, n_out=3)
    ref2, got2 = both(w2.systems, w2.tlist, method="dopri5", rtol=1e-8, atol=1e-11)
    assert_same(ref2, got2)


def test_noalloc_rk4_twice_second_smaller_both_layouts():
    """Fixed step: step tables and pack tables in the scratch array; full and
    Hermitian column kernels, then a smaller batch on the row kernel, then
    small instances with two control terms on the one-element-per-lane
    kernel."""
    w = S.jc_sweep(n_inst=64, seed=93, nsteps=200, t_end=5.0, n_out=11)
    for herm in (False, True):
        ref, got = both(w.systems, w.tlist, method="rk4", nsteps=w.nsteps, hermitian=herm)
        assert_same(ref, got)
    w2 = S.jc_sweep(n_inst=5, seed=94, nsteps=50, t_end=1.0, n_out=3)
    ref2, got2 = both(w2.systems, w2.tlist, method="rk4", nsteps=w2.nsteps,
                      layout=lme.LME_LAYOUT_ROW)
    assert_same(ref2, got2)
    rng = np.random.default_rng(97)
    small = []
    for b in range(6):
        N = 2 + b % 3
        s = S.jc_system(N, g=0.3, kappa=0.1, gamma=0.05, psi0=(b % 2, 1))
        a = S.jc_ops(N)[0]
        s.H_ctrl = [S.tidy(a + S.dag(a)), S.tidy(1j * (S.dag(a) - a))]
        s.edges = np.linspace(0.0, 1.0, 3)
        s.u = rng.normal(0.0, 0.5, size=(2, 2))
        small.append(s)
    ref3, got3 = both(small, np.linspace(0.0, 1.0, 5), method="rk4", nsteps=100)
    assert_same(ref3, got3)


def test_noalloc_kerr_dopri5_matches():
    w = S.kerr_single()
    tl = np.linspace(0.0, 2.0, 5)
    ref, got = both(w.systems, tl, method="dopri5", rtol=w.rtol, atol=w.atol)
    assert_same(ref, got)


def test_noalloc_rejects_what_does_not_fit():
    """A DOPRI5 batch whose stage derivatives exceed the 64 MiB array, and a
    forced streamed path, are refused on the host before any device work."""
    w = S.jc_sweep(n_inst=1024, seed=95, t_end=1.0, n_out=2)
    h = lme.Handle(w.systems)
    assert 112 * h.state_elems > 64 << 20
    r0 = h.pack([s.rho0 for s in w.systems])
    with pytest.raises(lme.LmeError) as e:
        h.evolve(r0, w.tlist, method="dopri5", rtol=1e-6, atol=1e-9, noalloc=True)
    assert e.value.code == lme.LME_ENOTSUP and "scratch" in str(e.value)
    s = [S.jc_system(3)]
    h2 = lme.Handle(s)
    with pytest.raises(lme.LmeError) as e:
        h2.evolve(h2.pack([s[0].rho0]), np.array([0.0, 1.0]), nsteps=10,
                  path=lme.LME_PATH_STREAMED, noalloc=True)
    assert e.value.code == lme.LME_ENOTSUP
