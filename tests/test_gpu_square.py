"""GPU parity on square systems (M = N, Section 2.1's spaQR: step 2 only)
against the oracle: rank decisions, factor ops at the oracle's ranks,
and the solution of the linear system after CGLS and after refined
seminormal equations."""
import numpy as np
import pytest

import paper_2102_09878_amd as pk
from oracle import solve as osolve
from oracle import spaqr as osp
from synth import grid_square

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [((32, 32), 4, 1, 1e-2), ((64, 48), 5, 2, 1e-3), ((12, 12, 12), 4, 1, 1e-2)]


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("grid,depth,skip,eps", CASES)
def test_square_parity(grid, depth, skip, eps):
    p = grid_square(grid, 9)
    f = osp.factorize(osp.analyze(p, depth), eps, skip)
    s = pk.Solver.from_problem(p, depth, skip)
    s.factorize(eps)
    assert s.ranks() == f.ranks
    s.factorize(eps, ranks=f.ranks)
    assert s.stats()["num_ops"] == len(f.ops)
    worst = 0.0
    for i, o in enumerate(f.ops):
        g = s.op(i)
        ref = o[3] if o[0] == "elim" else o[2]
        assert g["kind"] == o[0] and np.array_equal(g["slots"], o[1]), i
        assert g["mat"].shape == ref.shape, i
        if ref.size:
            e = np.abs(g["mat"] - ref).max() / max(1.0, np.abs(ref).max())
            worst = max(worst, e)
            assert e <= 1e-10, (i, o[0], e)
    xs = np.linalg.solve(p.dense(), p.b) if p.N <= 4096 else None
    xo, io = osolve.cgls(osolve.Operator(f), p.b, tol=1e-12)
    x, info = s.cgls(dev(p.b), tol=1e-12)
    x = x.cpu().numpy()
    print(f"square {grid}: worst op difference {worst:.2e}, cgls {info['iters']} (oracle {io['iters']})")
    assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    if xs is not None:
        assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    xc, ic = s.csne(dev(p.b), tol=1e-12)
    assert ic["converged"] and np.linalg.norm(xc.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()


def test_square_fp32_form():
    p = grid_square((64, 64), 10)
    s = pk.Solver.from_problem(p, 6, 2, precision="fp32")
    s.factorize(1e-2)
    x, info = s.cgls(dev(p.b), tol=1e-12)
    A = p.scipy()
    import scipy.sparse.linalg as spla
    xs = spla.spsolve(A.tocsc(), p.b)
    assert info["converged"] and np.linalg.norm(x.cpu().numpy() - xs) <= 1e-8 * np.linalg.norm(xs)
    s.close()
