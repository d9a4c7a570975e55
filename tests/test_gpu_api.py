"""The one-call interface lme.evolve (the paper's solver convention: H,
initial state, times, collapse and expectation operators) against the
oracle.  Bars as for the batch interface: 1e-10 for RK4 expectation values
and trace distance, 1e-6 relative for DOPRI5.
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


def test_evolve_ket_rk4_expectations_and_states():
    s = S.jc_system(10, g=0.05 * 2 * np.pi, kappa=0.005, gamma=0.05)
    psi = np.kron(S.coherent_ket(10, 0.8), S.ket(2, 1))
    tl = np.linspace(0.0, 2.0, 11)
    ex = lme.evolve(s.H0, s.C, psi, tl, s.E, nsteps=200)
    rho0 = np.outer(psi, psi.conj())
    oex, ost = oracle.rk4(s, rho0, tl, 200, store_states=True)
    assert ex.dtype == np.float64 and ex.shape == (len(s.E), len(tl))
    assert np.max(np.abs(ex - oex.real)) <= 1e-10
    states = lme.evolve(s.H0, s.C, psi, tl, [], nsteps=200)
    assert states.shape == (len(tl), s.n, s.n)
    for k in (0, 5, 10):
        assert brute.trace_distance(states[k], ost[k]) <= 1e-10
    # the full (non-Hermitian) path gives the same to rounding
    ex2 = lme.evolve(s.H0, s.C, psi, tl, s.E, nsteps=200, hermitian=False)
    assert np.max(np.abs(ex2 - ex)) <= 1e-13


def test_evolve_dopri5_and_controls():
    s = S.kerr_system(15, delta=0.5, K=0.3, E=0.4, kappa=0.6)
    tl = np.linspace(0.0, 3.0, 7)
    ex = lme.evolve(s.H0, s.C, s.rho0, tl, s.E, method="dopri5", rtol=1e-8, atol=1e-11)
    r = oracle.dopri5(s, s.rho0, tl, 1e-8, 1e-11)
    want = r["expect"]
    for k in range(len(s.E)):
        scale = np.max(np.abs(want[k]))
        assert np.max(np.abs(ex[k] - want[k])) <= 1e-6 * scale
    c = S.random_system(5, n_c=2, n_ctrl=1, n_e=2, seed=9, n_seg=4, t_end=1.0)
    tl = np.linspace(0.0, 1.0, 5)
    ex = lme.evolve(c.H0, c.C, c.rho0, tl, c.E, controls=(c.H_ctrl, c.edges, c.u), nsteps=40)
    oex, _ = oracle.rk4(c, c.rho0, tl, 40)
    assert np.max(np.abs(np.asarray(ex) - oex)) <= 1e-10
