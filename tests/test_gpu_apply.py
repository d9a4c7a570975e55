"""GPU parity of the pipelined column application (apply_path 0): row tiles
of the batch streamed through two LDS stages by one persistent workgroup per
CU.  Bars: 1e-12 relative to the largest entry against the oracle's L(y), and
identical bits to the whole-instance pack path (apply_path 1), which computes
every element with the same arithmetic in the same order.
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


def both_paths(systems, rhos=None, t=0.0, u=None):
    h = lme.Handle(systems)
    y = h.pack(rhos if rhos is not None else [s.rho0 for s in systems])
    h.set_tuning(apply_path=0)
    a = h.apply(y, t=t, u=u)
    h.set_tuning(apply_path=1, apply_block=1024, apply_lds_kb=0)
    b = h.apply(y, t=t, u=u)
    torch.cuda.synchronize()
    return h, a, b


def check_oracle(h, out, systems, rhos=None, t=0.0, u=None):
    got = h.unpack(out)
    for k, s in enumerate(systems):
        r = rhos[k] if rhos is not None else s.rho0
        want = oracle.apply_L(s, r, t=t, u=None if u is None else u[k])
        assert np.max(np.abs(got[k] - want)) <= 1e-12 * max(1.0, np.max(np.abs(want))), k


def test_pipe_sweep_whole_and_row_tiles():
    """Dims 10..80: small instances go several to a tile, the largest are cut
    into row tiles with their band."""
    w = S.jc_sweep(n_inst=48, seed=13, coherent=True)
    h, a, b = both_paths(w.systems)
    assert torch.equal(a, b)
    check_oracle(h, a, w.systems)


def test_pipe_large_and_odd_instances():
    """n = 2*72 = 144 (a stage holds a few dozen of its rows) and Kerr
    oscillators of odd cutoff up to n = 101 (two off-diagonals per row)."""
    systems = [S.jc_system(72, g=0.2, kappa=0.01, gamma=0.02)]
    systems[0].rho0 = S.ket2dm(np.kron(S.coherent_ket(72, 2.0), S.ket(2, 1)))
    rng = np.random.default_rng(4)
    for N in (7, 33, 61, 101):
        d, K, E, kap = rng.uniform(0.1, 1.0, 4)
        s = S.kerr_system(N, d, K, E, kap)
        s.rho0 = S.ket2dm(S.coherent_ket(N, 1.5))
        systems.append(s)
    h, a, b = both_paths(systems)
    assert torch.equal(a, b)
    check_oracle(h, a, systems)


def test_pipe_controls_thermal_and_complex_coupling():
    w = S.jc_drive(n_inst=7, N=9, n_seg=5, t_end=1.0, steps_per_seg=4, sigma_u=0.7)
    u = np.random.default_rng(5).normal(size=(7, 1, 5))
    rhos = [S.random_system(s.n, n_c=0, seed=30 + k, hermitian_rho=False).rho0
            for k, s in enumerate(w.systems)]
    h, a, b = both_paths(w.systems, rhos=rhos, t=0.45, u=torch.from_numpy(u).cuda())
    assert torch.equal(a, b)
    check_oracle(h, a, w.systems, rhos=rhos, t=0.45, u=u)

    systems = [S.jc_system(N, g=0.3, kappa=0.02, gamma=0.04, phase=0.7 + 0.1 * N, n_th=0.1)
               for N in (3, 12, 30, 45)]
    for N, s in zip((3, 12, 30, 45), systems):
        s.rho0 = S.ket2dm(np.kron(S.coherent_ket(N, 0.9), S.ket(2, 0)))
    h, a, b = both_paths(systems)
    assert torch.equal(a, b)
    check_oracle(h, a, systems)


def test_pipe_repeat_is_deterministic_and_tuning_roundtrip():
    w = S.jc_sweep(n_inst=20, seed=17, coherent=True)
    h = lme.Handle(w.systems)
    y = h.pack([s.rho0 for s in w.systems])
    x1 = h.apply(y)
    x2 = h.apply(y)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)
    assert h.get_tuning().apply_path == 0
    with pytest.raises(lme.LmeError):
        h.set_tuning(apply_path=2)
