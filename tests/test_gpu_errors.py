"""Error returns of the C-ABI that need a GPU: SPAQR_ERANK when an
interface's scaling block is numerically rank deficient (A without full
column rank, Section 1's assumption), and SPAQR_NOCONV when CGLS stops at
max_iter (x still written)."""
import ctypes

import numpy as np
import pytest

import paper_2102_09878_amd as pk
from paper_2102_09878_amd import spaqr as b
from rankdef import duplicated_column_problem
from synth import grid_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rank_deficient_interface_returns_erank(precision):
    p, j1, j2 = duplicated_column_problem()
    s = pk.Solver.from_problem(p, 4, 1, precision=precision)
    lib = b.load()
    rc = lib.spaqr_factorize(s.h, 1e-2)
    assert rc == b.ERANK, (rc, lib.spaqr_last_error(s.h))
    assert b"rank deficient" in lib.spaqr_last_error(s.h)
    # no factor is left behind: solving is a call-order error
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    bb = torch.as_tensor(p.b, device="cuda")
    info = b.CglsInfo()
    assert lib.spaqr_cgls(s.h, b._ptr(bb), 1e-10, 10, b._ptr(x), ctypes.byref(info)) == b.ESTATE
    s.close()


def test_cgls_iteration_limit_returns_noconv():
    p = grid_ls((32, 32), 1024, 0)
    s = pk.Solver.from_problem(p, 4, 1)
    s.factorize(1e-1)
    lib = b.load()
    bb = torch.as_tensor(p.b, device="cuda")
    x = torch.full((p.N,), np.nan, dtype=torch.float64, device="cuda")
    info = b.CglsInfo()
    rc = lib.spaqr_cgls(s.h, b._ptr(bb), 1e-15, 1, b._ptr(x), ctypes.byref(info))
    assert rc == b.NOCONV
    assert info.iters == 1 and info.converged == 0
    xh = x.cpu().numpy()
    assert np.isfinite(xh).all() and np.linalg.norm(xh) > 0
    # the same solve with room to converge returns OK
    rc = lib.spaqr_cgls(s.h, b._ptr(bb), 1e-10, 200, b._ptr(x), ctypes.byref(info))
    assert rc == b.OK and info.converged == 1
    s.close()
