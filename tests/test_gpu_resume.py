"""Resuming a fixed-step integration: RK4 over [0, T] in 2k steps gives
bit for bit the state of RK4 over [0, T/2] in k steps followed by RK4 over
[T/2, T] in k steps from that state (the step h = T / 2k is the same, and
every step is the same map of its input).  With piecewise-constant controls
whose edges fall on T/2 the segment of every step is the same too."""
import numpy as np
import pytest

from paper_1110_0573_amd import systems as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1110_0573_amd import lme  # noqa: E402


def halves(h, rho0, T, k, **kw):
    full = h.evolve(rho0, [0.0, 0.5 * T, T], nsteps=2 * k, **kw)
    a = h.evolve(rho0, [0.0, 0.5 * T], nsteps=k, **kw)
    mid = a["rho"].clone()
    b = h.evolve(mid, [0.5 * T, T], nsteps=k, **kw)
    torch.cuda.synchronize()
    for o in (full, a, b):
        assert (o["status"].cpu().numpy() == 0).all()
    return full["rho"].cpu().numpy(), b["rho"].cpu().numpy(), full, a, b


@pytest.mark.parametrize("hermitian", [False, True])
def test_resume_ragged_jc_batch_bitwise(hermitian):
    w = S.jc_sweep(n_inst=24, seed=12, nsteps=200, t_end=4.0, n_out=3)
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    f, r, full, a, b = halves(h, r0, 4.0, 100, hermitian=hermitian)
    assert np.array_equal(f.view(np.uint64), r.view(np.uint64))
    # the expectation values at T/2 and T agree bit for bit as well
    fe = full["expect"].cpu().numpy()
    ae, be = a["expect"].cpu().numpy(), b["expect"].cpu().numpy()
    assert np.array_equal(fe[..., 1], ae[..., 1]) and np.array_equal(fe[..., 2], be[..., 1])


def test_resume_with_piecewise_controls_bitwise():
    """Driven JC batch, 10 segments on [0, 10]: T/2 = 5 is an edge."""
    w = S.jc_drive(n_inst=8, N=6, n_seg=10, t_end=10.0, steps_per_seg=20)
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    f, r, *_ = halves(h, r0, 10.0, 100)
    assert np.array_equal(f.view(np.uint64), r.view(np.uint64))


def test_resume_streamed_path_bitwise():
    """Instances too large for a resident workgroup (8-spin chains, n = 256)
    take the streamed stepper; it resumes bit for bit too."""
    w = S.tfim(n_inst=2, seed=5, M=8, t_end=0.2, n_out=2)
    h = lme.Handle(w.systems)
    r0 = h.pack([s.rho0 for s in w.systems])
    f, r, *_ = halves(h, r0, 0.2, 4)
    assert np.array_equal(f.view(np.uint64), r.view(np.uint64))
