"""GPU parity on the inverse-Poisson least-squares problems (Appendices A
and B, aspect ratios about 2, 1.5 and 1.05): rank decisions, factor ops at
the oracle's ranks, and x after CGLS, against the oracle."""
import numpy as np
import pytest

import paper_2102_09878_amd as pk
from oracle import solve as osolve
from oracle import spaqr as osp
from synth import default_depth, inverse_poisson

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("n,dim,alpha,eps,seed", [(64, 2, 2.0, 1e-2, 5), (64, 2, 1.5, 1e-2, 5),
                                                  (64, 2, 1.05, 1e-4, 5), (12, 3, 1.5, 1e-2, 5),
                                                  (12, 3, 1.5, 1e-2, 6), (16, 3, 2.0, 1e-2, 5)])
def test_inverse_poisson_parity(n, dim, alpha, eps, seed):
    p = inverse_poisson(n, dim, alpha, seed=seed)
    depth = default_depth(p.N)
    f = osp.factorize(osp.analyze(p, depth), eps, 2)
    s = pk.Solver.from_problem(p, depth, 2)
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
    print(f"inverse Poisson {dim}D n={n} alpha={p.M / p.N:.3f}: ops {len(f.ops)} worst {worst:.1e}, "
          f"cgls {info['iters']} (oracle {io['iters']})")
    assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()
