"""GPU parity of the cost / adjoint-gradient path.

Bars: cost within 1e-12 of the oracle; gradient within 1e-10 of the largest
oracle gradient entry (both are the exact derivative of the same discrete RK4
map); against central finite differences (h = 1e-6) through the GPU's own cost,
|g - g_FD| <= 1e-7 + 1e-5 |g_FD|.
"""
import numpy as np
import pytest

import oracle
from paper_1110_0573_amd import systems as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1110_0573_amd import lme  # noqa: E402


def gpu_cost_grad(systems, O, t1, nsteps, ckpt, u=None):
    h = lme.Handle(systems)
    rho0 = h.pack([s.rho0 for s in systems])
    Od = h.pack([O] * len(systems) if not isinstance(O, list) else O)
    ud = None if u is None else torch.from_numpy(np.ascontiguousarray(u)).cuda()
    cost, grad = lme._cost_grad(h, rho0, Od, ud, 0.0, t1, nsteps, ckpt)
    torch.cuda.synchronize()
    return h, cost.cpu().numpy(), grad.cpu().numpy()


def check_against_oracle(systems, O, t1, nsteps, ckpt):
    _, cost, grad = gpu_cost_grad(systems, O, t1, nsteps, ckpt)
    for b, s in enumerate(systems):
        Ob = O[b] if isinstance(O, list) else O
        J, g = oracle.rk4_cost_grad(s, s.rho0, Ob, 0.0, t1, nsteps)
        assert abs(cost[b] - J) <= 1e-12
        assert np.max(np.abs(grad[b] - g)) <= 1e-10 * max(1e-3, np.max(np.abs(g))), b


def test_grad_small_driven_jc_matches_oracle():
    w = S.jc_drive(n_inst=6, N=4, n_seg=10, t_end=2.0, steps_per_seg=4, sigma_u=0.3)
    check_against_oracle(w.systems, w.extra["target"], 2.0, w.nsteps, 4)


def test_grad_checkpoints_misaligned_with_segments():
    w = S.jc_drive(n_inst=3, N=3, n_seg=5, t_end=1.0, steps_per_seg=4, sigma_u=0.5)
    check_against_oracle(w.systems, w.extra["target"], 1.0, w.nsteps, 3)
    check_against_oracle(w.systems, w.extra["target"], 1.0, w.nsteps, 7)
    check_against_oracle(w.systems, w.extra["target"], 1.0, w.nsteps, 100)


def test_grad_two_controls_and_general_observable():
    rng = np.random.default_rng(9)
    systems = []
    for b in range(4):
        s = S.jc_system(3 + b, g=0.4, kappa=0.1, gamma=0.05, psi0=(0, 1))
        a = S.jc_ops(3 + b)[0]
        s.H_ctrl = [S.tidy(a + S.dag(a)), S.tidy(1j * (S.dag(a) - a))]
        s.edges = np.linspace(0.0, 1.5, 7)
        s.u = rng.normal(0, 0.4, size=(2, 6))
        systems.append(s)
    Os = []
    for s in systems:
        n = s.n
        X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        Os.append(X)
    check_against_oracle(systems, Os, 1.5, 30, 5)


def test_grad_full_size_sample_and_finite_differences():
    """256 driven instances, N=20, 100 segments, 1000 steps, checkpoint every 10."""
    w = S.jc_drive()
    O = w.extra["target"]
    h, cost, grad = gpu_cost_grad(w.systems, O, 10.0, w.nsteps, 10)
    assert np.all(np.isfinite(grad)) and grad.shape == (256, 1, 100)
    for b in (0, 137):
        s = w.systems[b]
        J, g = oracle.rk4_cost_grad(s, s.rho0, O, 0.0, 10.0, w.nsteps)
        assert abs(cost[b] - J) <= 1e-12
        assert np.max(np.abs(grad[b] - g)) <= 1e-10 * np.max(np.abs(g))
    # central differences through the GPU cost for a few segments of instance 3
    u = w.extra["u"].copy()
    hfd = 1e-6
    for q in (0, 41, 99):
        up, dn = u.copy(), u.copy()
        up[3, 0, q] += hfd
        dn[3, 0, q] -= hfd
        _, cp, _ = gpu_cost_grad(w.systems, O, 10.0, w.nsteps, 10, u=up)
        _, cm, _ = gpu_cost_grad(w.systems, O, 10.0, w.nsteps, 10, u=dn)
        fd = (cp[3] - cm[3]) / (2 * hfd)
        assert abs(grad[3, 0, q] - fd) <= 1e-7 + 1e-5 * abs(fd), (q, grad[3, 0, q], fd)


def test_grad_cost_equals_evolved_expectation():
    w = S.jc_drive(n_inst=5, N=5, n_seg=8, t_end=1.6, steps_per_seg=5)
    O = w.extra["target"]
    h, cost, _ = gpu_cost_grad(w.systems, O, 1.6, w.nsteps, 5)
    h2 = lme.Handle(w.systems)
    out = h2.evolve(h2.pack([s.rho0 for s in w.systems]), np.array([0.0, 1.6]),
                    nsteps=w.nsteps)
    torch.cuda.synchronize()
    rho = h2.unpack(out["rho"])
    for b in range(5):
        assert abs(cost[b] - np.real(np.trace(O @ rho[b]))) <= 1e-13


def test_autograd_function():
    w = S.jc_drive(n_inst=4, N=4, n_seg=6, t_end=1.2, steps_per_seg=5)
    h = lme.Handle(w.systems)
    rho0 = h.pack([s.rho0 for s in w.systems])
    O = h.pack([w.extra["target"]] * 4)
    u = torch.from_numpy(w.extra["u"].copy()).cuda().requires_grad_(True)
    J = lme.expectation_cost(u, h, rho0, O, 0.0, 1.2, w.nsteps, 5)
    loss = (1.0 - J).sum()
    loss.backward()
    _, g = lme._cost_grad(h, rho0, O, u.detach(), 0.0, 1.2, w.nsteps, 5)
    assert torch.equal(u.grad, -g)


def test_grad_column_layout_bitwise_row_layout_ragged():
    """The column layout (each thread's column of the forward and adjoint
    operators in registers) gives the bits of the row layout, on a ragged
    batch (N = 3..10, several instances per pack) with a general observable;
    asking for the column layout where it does not apply is an error."""
    rng = np.random.default_rng(21)
    systems, Os = [], []
    for b in range(9):
        N = 3 + (b * 5) % 8
        s = S.jc_system(N, g=0.3, kappa=0.02, gamma=0.05, psi0=(0, 1))
        a = S.jc_ops(N)[0]
        s.H_ctrl = [S.tidy(a + S.dag(a))]
        s.edges = np.linspace(0.0, 1.2, 5)
        s.u = rng.normal(0, 0.4, size=(1, 4))
        systems.append(s)
        X = rng.normal(size=(s.n, s.n)) + 1j * rng.normal(size=(s.n, s.n))
        Os.append(X + X.conj().T)
    out = {}
    for layout in (lme.LME_LAYOUT_COLUMN, lme.LME_LAYOUT_ROW, 0):
        h = lme.Handle(systems)
        h.set_tuning(grad_layout=layout)
        cost, grad = lme._cost_grad(h, h.pack([s.rho0 for s in systems]), h.pack(Os), None,
                                    0.0, 1.2, 24, 5)
        torch.cuda.synchronize()
        out[layout] = (cost.cpu().numpy(), grad.cpu().numpy())
    for layout in (lme.LME_LAYOUT_ROW, 0):
        assert np.array_equal(out[layout][0], out[lme.LME_LAYOUT_COLUMN][0])
        assert np.array_equal(out[layout][1], out[lme.LME_LAYOUT_COLUMN][1])
    for b in (0, 4, 8):
        J, g = oracle.rk4_cost_grad(systems[b], systems[b].rho0, Os[b], 0.0, 1.2, 24)
        assert abs(out[0][0][b] - J) <= 1e-12
        assert np.max(np.abs(out[0][1][b] - g)) <= 1e-10 * max(1e-3, np.max(np.abs(g)))
    # two control terms: no column layout
    s2 = S.jc_system(3, g=0.4, kappa=0.1, gamma=0.05, psi0=(0, 1))
    a = S.jc_ops(3)[0]
    s2.H_ctrl = [S.tidy(a + S.dag(a)), S.tidy(1j * (S.dag(a) - a))]
    s2.edges = np.linspace(0.0, 1.0, 3)
    s2.u = np.zeros((2, 2))
    h = lme.Handle([s2])
    h.set_tuning(grad_layout=lme.LME_LAYOUT_COLUMN)
    with pytest.raises(lme.LmeError):
        lme._cost_grad(h, h.pack([s2.rho0]), h.pack([np.eye(6)]), None, 0.0, 1.0, 4, 2)
