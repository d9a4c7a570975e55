"""GPU parity of the row-block application (instances with 128 <= n <= 1024,
too large for a resident pack): rows of one instance staged in LDS, source
rows outside the block read from memory.  Bars: 1e-12 relative to the
largest entry against the oracle's L(y) (and L^+ x), and agreement with the
plain streamed kernel (every gather from memory, same per-element order) to
rounding.
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


def random_states(systems, seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(s.n, s.n)) + 1j * rng.normal(size=(s.n, s.n)) for s in systems]


def check(h, out, systems, ys, fn, **kw):
    got = h.unpack(out)
    for k, s in enumerate(systems):
        want = fn(s, ys[k], **{a: (v[k] if a == "u" and v is not None else v)
                               for a, v in kw.items()})
        assert np.max(np.abs(got[k] - want)) <= 1e-12 * np.max(np.abs(want)), k


def test_rows_tfim_batch_16_row_blocks():
    """8-spin chains (n = 256): bit flips of the four high bits and their
    jumps read rows of other blocks."""
    w = S.tfim(n_inst=3, seed=11)
    ys = random_states(w.systems, 1)
    h = lme.Handle(w.systems)
    y = h.pack(ys)
    a = h.apply(y)
    b = h.apply(y, form=lme.LME_FORM_OPERATOR_STREAMED)
    torch.cuda.synchronize()
    check(h, a, w.systems, ys, oracle.apply_L)
    assert torch.max(torch.abs(a - b)).item() <= 1e-14 * torch.max(torch.abs(b)).item()
    x = h.apply(y, adjoint=True)
    torch.cuda.synchronize()
    check(h, x, w.systems, ys, oracle.apply_Ldag)


def test_rows_general_operators_controls_4_row_blocks():
    """Complex operators of dimension 300 and 131 (4-row blocks, a ragged last
    block) with a control term inside and outside its segments."""
    systems = [S.random_system(300, n_c=2, n_ctrl=1, density=0.006, seed=3, n_seg=4),
               S.random_system(131, n_c=1, n_ctrl=1, density=0.012, seed=4, n_seg=4)]
    ys = random_states(systems, 2)
    h = lme.Handle(systems)
    y = h.pack(ys)
    u = np.stack([s.u for s in systems])
    ut = torch.from_numpy(u).cuda()
    for t in (0.3, 1.5):
        a = h.apply(y, t=t, u=ut)
        b = h.apply(y, t=t, u=ut, form=lme.LME_FORM_OPERATOR_STREAMED)
        torch.cuda.synchronize()
        check(h, a, systems, ys, oracle.apply_L, t=t, u=u)
        assert torch.max(torch.abs(a - b)).item() <= 1e-14 * torch.max(torch.abs(b)).item()
    x = h.apply(y, t=0.3, u=ut, adjoint=True)
    torch.cuda.synchronize()
    check(h, x, systems, ys, oracle.apply_Ldag, t=0.3, u=u)


def test_rows_not_used_below_128_still_correct():
    """A batch with a small instance keeps the plain streamed kernel."""
    systems = S.tfim(n_inst=1, seed=12).systems + [S.random_system(150, density=0.01, seed=5, n_e=8),
                                                    S.random_system(20, seed=6, n_e=8)]
    ys = random_states(systems, 3)
    h = lme.Handle(systems)
    a = h.apply(h.pack(ys))
    torch.cuda.synchronize()
    check(h, a, systems, ys, oracle.apply_L)
