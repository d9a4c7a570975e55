"""GPU parity of propagators and steady states against the oracle.

The propagator is the fixed-step RK4 map, built on the GPU from the n^2
basis matrices, so the bar is the fixed-step one (1e-12 of the largest
entry).  The steady state is the limit of U(T)^(2^k) (complex FP64 products
on the matrix cores); its fixed point is exactly the null space of L, so it
is compared with the oracle's direct solve of L rho = 0, Tr rho = 1 and with
closed forms, to 1e-10 (the iteration stops at a relative change of 1e-13;
what remains is rounding amplified by the inverse gap of L)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1110_0573_amd import systems as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1110_0573_amd import lme  # noqa: E402


def test_zgemm_matrix_core_layout():
    """The batched complex product on its own (the lane layout of the FP64
    matrix-core instruction, the LDS panels): ragged blocks of N = 9, 25,
    64, 100, 169 (partial 64 x 64 tiles, several k-panels) against numpy."""
    lib = lme.load()
    f = lib.lme_internal_launch_zgemm
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    dims = [3, 5, 8, 10, 13]
    rng = np.random.default_rng(17)
    As, Bs, off4, tiles = [], [], [0], []
    for b, n in enumerate(dims):
        N = n * n
        As.append(rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)))
        Bs.append(rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)))
        off4.append(off4[-1] + N * N)
        nt = (N + 63) // 64
        tiles += [(b, i, j, 0) for i in range(nt) for j in range(nt)]
    # column-major blocks: element r + c N holds M[r, c]
    flat = lambda Ms: torch.tensor(np.concatenate([M.T.reshape(-1) for M in Ms]),
                                   device="cuda")
    A, B = flat(As), flat(Bs)
    Cm = torch.full_like(A, complex(np.nan, np.nan))
    t_tiles = torch.tensor(np.array(tiles, np.int32).reshape(-1), device="cuda")
    t_off = torch.tensor(np.array(off4, np.int64), device="cuda")
    t_dims = torch.tensor(np.array(dims, np.int32), device="cuda")
    rc = f(t_tiles.data_ptr(), len(tiles), t_off.data_ptr(), t_dims.data_ptr(), A.data_ptr(),
           B.data_ptr(), Cm.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    got = Cm.cpu().numpy()
    for b, n in enumerate(dims):
        N = n * n
        Cb = got[off4[b]:off4[b + 1]].reshape(N, N).T
        want = As[b] @ Bs[b]
        assert np.max(np.abs(Cb - want)) <= 1e-13 * np.max(np.abs(want)), b


def test_propagator_ragged_vs_oracle():
    systems = [S.random_system(n, n_c=2, seed=60 + n) for n in (2, 3, 5, 7)]
    h = lme.Handle(systems)
    Us, st = h.propagator(0.3, 1.1, 64)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for s, U in zip(systems, Us):
        want = oracle.propagator(s, 0.3, 1.1, 64)
        got = U.cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_propagator_jc_maps_states():
    """U applied to a state equals the state's own RK4 evolution."""
    s = S.jc_system(4)
    h = lme.Handle([s])
    (U,), st = h.propagator(0.0, 2.0, 100)
    got = (U.cpu().numpy() @ s.rho0.reshape(-1)).reshape(s.n, s.n)
    want = oracle.rk4(S.System(s.H0, s.C, [], s.rho0), s.rho0, [0.0, 2.0], 100,
                      store_states=True)[1][-1]
    assert np.max(np.abs(got - want)) < 1e-13


def steady(systems, T, nsteps, max_sq=60, tol=1e-13):
    h = lme.Handle(systems)
    rho, st, k = h.steadystate(T, nsteps, max_squarings=max_sq, tol=tol)
    torch.cuda.synchronize()
    return h, h.unpack(rho), st.cpu().numpy(), k


def test_steadystate_closed_forms_ragged_batch():
    nth = 0.3
    cav = S.damped_cavity(N=6, kappa=0.8, n_th=nth)
    D, Om, G = 0.7, 1.3, 0.9
    tls = S.System(S.tidy(0.5 * D * S.sigmaz() + 0.5 * Om * S.sigmax()),
                   [S.tidy(np.sqrt(G) * S.sigmam())], [S.tidy(S.sigmaz())], np.eye(2) / 2)
    _, (r_cav, r_tls), st, k = steady([cav, tls], 4.0, 200)
    assert (st == 0).all() and 1 <= k < 60
    q = (nth / (1 + nth)) ** np.arange(6)
    np.testing.assert_allclose(r_cav, np.diag(q / q.sum()), atol=1e-10)
    assert abs(r_tls[1, 1] - (Om ** 2 / 4) / (D ** 2 + G ** 2 / 4 + Om ** 2 / 2)) < 1e-10
    np.testing.assert_allclose(r_tls, oracle.steadystate(tls), atol=1e-10)


def test_steadystate_random_vs_oracle():
    systems = [S.random_system(n, n_c=3, seed=90 + n) for n in (3, 4, 6, 9)]
    _, rhos, st, k = steady(systems, 6.0, 300)
    assert (st == 0).all()
    for s, r in zip(systems, rhos):
        want = oracle.steadystate(s)
        assert np.max(np.abs(r - want)) < 1e-10
        assert abs(np.trace(r) - 1) < 1e-13


def test_steadystate_jc_thermal_vs_oracle():
    """Jaynes-Cummings with cavity and atom damping at a thermal occupation
    (the paper's Sec. 3.2 cavity coupled to a two-level atom): n = 2 N = 24,
    N^2 = 576 (36 tiles a side)."""
    s = S.jc_system(12, n_th=0.2)
    _, (r,), st, k = steady([s], 60.0, 3000)
    assert st[0] == 0
    want = oracle.steadystate(s)
    assert np.max(np.abs(r - want)) < 1e-10


def test_steadystate_not_converged_status():
    s = S.random_system(4, n_c=2, seed=7)
    _, (r,), st, k = steady([s], 0.5, 20, max_sq=1, tol=0.0)
    assert k == 1 and st[0] == lme.LME_EMAXSTEPS
    assert abs(np.trace(r) - 1) < 1e-13     # the last iterate, normalised


def test_steadystate_sweep_as_benchmarked_sampled():
    """The benchmark's workload (16 thermal JC systems, dimension 32,
    propagators of 1024 rows): every instance converges, a seeded sample of
    2 matches the oracle's direct solve."""
    w = S.jc_steady_sweep()
    _, rhos, st, k = steady(w.systems, w.tlist[-1], w.nsteps)
    assert (st == 0).all() and k < 60
    for b in np.sort(np.random.default_rng(4).choice(len(w.systems), 2, replace=False)):
        assert np.max(np.abs(rhos[b] - oracle.steadystate(w.systems[b]))) < 1e-10
