"""GPU parity of the corrected seminormal equations with iterative
refinement (spaqr_csne, Section 1) against the oracle's csne_refined."""
import numpy as np
import pytest

import paper_2102_09878_amd as pk
from oracle import solve as osolve
from oracle import spaqr as osp
from synth import CONFIGS, config_problem, grid_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("case", ["config1", "ragged"])
def test_csne_matches_oracle(case):
    if case == "config1":
        c = CONFIGS[1]
        p = config_problem(1)
        depth, skip, eps = c["depth"], c["skip"], c["eps"]
    else:
        p = grid_ls((17, 23), 17 * 23 // 2 + 7, 11)
        depth, skip, eps = 4, 1, 1e-1
    f = osp.factorize(osp.analyze(p, depth), eps, skip)
    op = osolve.Operator(f)
    xo, io = osolve.csne_refined(op, p.b, tol=1e-12)
    s = pk.Solver.from_problem(p, depth, skip)
    s.factorize(eps)
    x, info = s.csne(dev(p.b), tol=1e-12)
    x = x.cpu().numpy()
    print(f"{case}: steps {info['steps']} (oracle {io['steps']}), residual {info['residual']:.2e}")
    assert info["converged"] and abs(info["steps"] - io["steps"]) <= 1
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    # at the benchmark's tolerance
    x2, info2 = s.csne(dev(p.b), tol=1e-10)
    A = p.scipy()
    r = p.b - A @ x2.cpu().numpy()
    assert info2["converged"] and np.linalg.norm(A.T @ r) <= 1.0001e-10 * info2["norm_a"] * np.linalg.norm(p.b)
    s.close()


def test_csne_zero_steps_is_the_one_shot_solve():
    p = config_problem(1)
    c = CONFIGS[1]
    s = pk.Solver.from_problem(p, c["depth"], c["skip"])
    s.factorize(c["eps"])
    b = dev(p.b)
    x, info = s.csne(b, tol=0.0, max_steps=0)
    assert info["steps"] == 0 and not info["converged"]
    assert np.array_equal(x.cpu().numpy(), s.apply(b).cpu().numpy())
    s.close()


def test_csne_exact_factor_and_fp32_form():
    p = grid_ls((16, 16), 256, 3)
    s = pk.Solver.from_problem(p, 4, 1)
    s.factorize(0.0)
    x, info = s.csne(dev(p.b), tol=1e-12)
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert info["steps"] <= 1 and np.linalg.norm(x.cpu().numpy() - xs) <= 1e-11 * np.linalg.norm(xs)
    s.close()
    p = config_problem(1)
    c = CONFIGS[1]
    s = pk.Solver.from_problem(p, c["depth"], c["skip"], precision="fp32")
    s.factorize(c["eps"])
    x, info = s.csne(dev(p.b), tol=1e-12)
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert info["converged"] and np.linalg.norm(x.cpu().numpy() - xs) <= 1e-8 * np.linalg.norm(xs)
    s.close()


def test_csne_batch_handle():
    grids = [(16, 16), (23, 17), (12, 20)]
    probs = [grid_ls(g, g[0] * g[1], 70 + i) for i, g in enumerate(grids)]
    bs = pk.BatchSolver.from_problems(probs, [4, 4, 3], skip=1)
    bs.factorize(1e-2)
    x, info = bs.csne(dev(np.concatenate([p.b for p in probs])), tol=1e-11)
    x = x.cpu().numpy()
    assert info["converged"]
    for g, p in enumerate(probs):
        c0, c1 = int(bs.col_off[g]), int(bs.col_off[g + 1])
        xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
        assert np.linalg.norm(x[c0:c1] - xs) <= 1e-8 * np.linalg.norm(xs), g
    bs.close()
