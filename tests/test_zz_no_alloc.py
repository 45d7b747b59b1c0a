"""The allocation-free one-shot solve (spaqr_apply_noalloc) against
spaqr_apply, through the C-ABI: both run the same kernels in the same
order, so their outputs must agree bit for bit.  Two calls in a row share
the library's static scratch array, the second on a smaller problem, so a
stale or misplaced part of the array would show up there."""
import numpy as np
import pytest

import paper_2102_09878_amd as pk
from synth import grid_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solver(grid, extra, seed, depth, skip, precision):
    p = grid_ls(grid, extra, seed)
    s = pk.Solver.from_problem(p, depth, skip, precision=precision)
    s.factorize(1e-2)
    return p, s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_apply_equals_apply(precision):
    big = _solver((40, 36), 40 * 36, 11, 5, 2, precision)
    small = _solver((16, 12), 150, 12, 3, 1, precision)
    for p, s in (big, small):  # the second call is on the smaller problem
        b = torch.as_tensor(p.b, device="cuda")
        ref = s.apply(b).cpu().numpy()
        x = torch.full((p.N,), np.nan, dtype=torch.float64, device="cuda")
        s.apply_noalloc(b, x)
        got = x.cpu().numpy()
        assert np.isfinite(ref).all() and np.linalg.norm(ref) > 0
        assert np.array_equal(got, ref), float(np.abs(got - ref).max())
    # the larger problem again, after the smaller one left its data in the array
    p, s = big
    b = torch.as_tensor(p.b, device="cuda")
    x = torch.empty(p.N, dtype=torch.float64, device="cuda")
    s.apply_noalloc(b, x)
    assert np.array_equal(x.cpu().numpy(), s.apply(b).cpu().numpy())
    for _, s in (big, small):
        s.close()
