"""GPU parity on matrices handed over without a grid (graph nested
dissection and max-product matching in the analysis): rank decisions,
factor ops at the oracle's ranks and x after CGLS against the oracle."""
import numpy as np
import pytest

import paper_2102_09878_amd as pk
from oracle import solve as osolve
from oracle import spaqr as osp
from synth import general_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("grid,depth,skip,eps", [((32, 32), 4, 1, 1e-2), ((64, 48), 5, 2, 1e-3),
                                                 ((12, 12, 12), 3, 1, 1e-2)])
def test_general_parity(grid, depth, skip, eps):
    p = general_ls(grid, int(np.prod(grid)), 12)
    f = osp.factorize(osp.analyze(p, depth), eps, skip)
    s = pk.Solver(p.row_ptr, p.col_idx, p.vals, p.M, p.N, None, depth, skip)
    s.factorize(eps)
    assert s.ranks() == f.ranks
    s.factorize(eps, ranks=f.ranks)
    worst = 0.0
    for i, o in enumerate(f.ops):
        g = s.op(i)
        ref = o[3] if o[0] == "elim" else o[2]
        assert g["kind"] == o[0] and np.array_equal(g["slots"], o[1]) and g["mat"].shape == ref.shape, i
        if ref.size:
            e = np.abs(g["mat"] - ref).max() / max(1.0, np.abs(ref).max())
            worst = max(worst, e)
            assert e <= 1e-10, (i, o[0], e)
    xo, io = osolve.cgls(osolve.Operator(f), p.b, tol=1e-12)
    x, info = s.cgls(dev(p.b), tol=1e-12)
    print(f"general {grid}: {len(f.ops)} ops, worst {worst:.1e}, cgls {info['iters']} (oracle {io['iters']})")
    assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()
