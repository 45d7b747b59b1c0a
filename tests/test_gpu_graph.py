"""The CGLS iterations replay one captured HIP graph per factorization.
Its kernels are the eager path's, in the same order, so every replay must
give the eager result bit for bit: checked over repeated solves with eager
work and synchronisations between the replays, after a refactorization
(the graph is recorded again) and on a batch handle."""
import os

import numpy as np
import pytest

import paper_2102_09878_amd as pk
from synth import CONFIGS, config_problem, grid_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _solve(s, b, eager, tol=1e-12, each=False):
    if eager:
        os.environ["SPAQR_NO_GRAPH"] = "1"
    try:
        if each:
            x, infos = s.cgls_each(b, tol=tol)
            return x.cpu().numpy(), [i["iters"] for i in infos]
        x, info = s.cgls(b, tol=tol)
        return x.cpu().numpy(), info["iters"]
    finally:
        os.environ.pop("SPAQR_NO_GRAPH", None)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_equal_eager(precision):
    c = CONFIGS[1]
    p = config_problem(1)
    s = pk.Solver.from_problem(p, c["depth"], c["skip"], precision=precision)
    b = dev(p.b)
    for eps in (c["eps"], 1e-1):
        s.factorize(eps)
        xe, ie = _solve(s, b, True)
        for rep in range(3):
            xg, ig = _solve(s, b, False)
            assert ig == ie and np.array_equal(xg, xe), (eps, rep)
            # eager work between replays: an eager solve of another right-hand side
            _solve(s, dev(np.ones(p.M)), True)
            torch.cuda.synchronize()
    s.close()


def test_graph_batch_handle():
    grids = [(16, 16), (23, 17), (12, 20)]
    probs = [grid_ls(g, g[0] * g[1], 80 + i) for i, g in enumerate(grids)]
    bs = pk.BatchSolver.from_problems(probs, [4, 4, 3], skip=1)
    bs.factorize(1e-2)
    b = dev(np.concatenate([p.b for p in probs]))
    xe, ie = _solve(bs, b, True, each=True)
    for _ in range(2):
        xg, ig = _solve(bs, b, False, each=True)
        assert ig == ie and np.array_equal(xg, xe)
    bs.close()
