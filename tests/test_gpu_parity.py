"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

* factor ops element by element when both sides take the same ranks
  (forced-rank mode), with identical slot lists (integer parity);
* rank decisions of the free run equal the oracle's;
* W^-1, W^-T applied by the GPU equal the oracle's;
* x from GPU CGLS equals the oracle's to 1e-8 and meets the residual bound;
* exact recovery at eps = 0, ragged and 3D grids, full-size configurations.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import paper_2102_09878_amd as pk
from oracle import solve as osolve
from oracle import spaqr as osp
from synth import CONFIGS, config_problem, grid_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _oracle(p, depth, eps, skip):
    an = osp.analyze(p, depth)
    f = osp.factorize(an, eps, skip)
    return an, f


def _res(p, x):
    A = p.scipy()
    r = p.b - A @ x
    nA = spla.svds(A, k=1, return_singular_vectors=False)[0] if min(A.shape) > 2 else np.linalg.norm(A.toarray(), 2)
    return np.linalg.norm(A.T @ r) / (nA * np.linalg.norm(p.b))


def _compare_ops(f, s, tol):
    assert s.stats()["num_ops"] == len(f.ops)
    worst = 0.0
    for i, o in enumerate(f.ops):
        g = s.op(i)
        assert g["kind"] == o[0], i
        assert (g["slots"] == o[1]).all(), i
        if o[0] == "elim":
            assert (g["nslots"] == o[2]).all(), i
            ref = o[3]
        elif o[0] == "scale":
            ref = o[2]
        else:
            ref = o[2]
            assert g["mat"].shape == ref.shape, i
            if ref.shape[1]:
                assert np.abs(g["tau"] - o[3]).max() <= tol, i
        scale = max(1.0, np.abs(ref).max()) if ref.size else 1.0
        err = np.abs(g["mat"] - ref).max() / scale if ref.size else 0.0
        worst = max(worst, err)
        assert err <= tol, (i, o[0], err)
    return worst


@pytest.fixture(scope="module")
def cfg1():
    c = CONFIGS[1]
    p = config_problem(1)
    an, f = _oracle(p, c["depth"], c["eps"], c["skip"])
    return c, p, an, f


def test_config1_ranks_match_oracle(cfg1):
    c, p, an, f = cfg1
    s = pk.Solver.from_problem(p, c["depth"], c["skip"])
    s.factorize(c["eps"])
    assert s.ranks() == f.ranks
    s.close()


def test_config1_factor_parity_forced_ranks(cfg1):
    c, p, an, f = cfg1
    s = pk.Solver.from_problem(p, c["depth"], c["skip"])
    s.factorize(c["eps"], ranks=f.ranks)
    worst = _compare_ops(f, s, 1e-10)
    print(f"config1 worst relative factor difference {worst:.3e}")
    s.close()


@pytest.mark.parametrize("grid,depth,skip,eps", [((32, 32), 4, 1, 1e-2), ((48, 40), 5, 2, 1e-2)])
def test_fp32_factor_close_to_oracle(grid, depth, skip, eps):
    """FP32 fronts and factors, same ranks as the FP64 oracle: every factor
    op within about a hundred FP32 roundings of the oracle's."""
    p = grid_ls(grid, grid[0] * grid[1], 31)
    an, f = _oracle(p, depth, eps, skip)
    s = pk.Solver.from_problem(p, depth, skip, precision="fp32")
    s.factorize(eps, ranks=f.ranks)
    worst = _compare_ops(f, s, 2e-5)
    print(f"fp32 {grid}: worst relative factor difference {worst:.3e}")
    s.close()


def test_config1_factor_deterministic(cfg1):
    c, p, an, f = cfg1
    s = pk.Solver.from_problem(p, c["depth"], c["skip"])
    s.factorize(c["eps"])
    a = [s.op(i)["mat"].copy() for i in range(s.stats()["num_ops"])]
    s.factorize(c["eps"])
    b2 = [s.op(i)["mat"] for i in range(s.stats()["num_ops"])]
    assert all((x == y).all() for x, y in zip(a, b2))
    s.close()


def test_config1_apply_matches_oracle(cfg1):
    c, p, an, f = cfg1
    s = pk.Solver.from_problem(p, c["depth"], c["skip"])
    s.factorize(c["eps"], ranks=f.ranks)
    rng = np.random.default_rng(1)
    for _ in range(3):
        v = rng.standard_normal(p.N)
        for op, fn in ((pk.spaqr.WINV, osolve.apply_winv), (pk.spaqr.WINVT, osolve.apply_winvt)):
            got = host(s.apply_op(op, dev(v)))
            ref = fn(f.ops, v)
            assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), op
    s.close()


def test_config1_cgls_matches_oracle(cfg1):
    c, p, an, f = cfg1
    xo, io = osolve.cgls(osolve.Operator(f), p.b, tol=1e-12)
    s = pk.Solver.from_problem(p, c["depth"], c["skip"])
    s.factorize(c["eps"])
    x, info = s.cgls(dev(p.b), tol=1e-12)
    x = host(x)
    assert info["converged"] and info["residual"] <= 1e-12
    assert abs(info["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    x2, info2 = s.cgls(dev(p.b), tol=1e-10)
    assert _res(p, host(x2)) <= 1e-10
    # one-shot seminormal solve equals the oracle's
    xs = host(s.apply(dev(p.b)))
    assert np.linalg.norm(xs - osolve.csne(osolve.Operator(f), p.b)) <= 1e-10 * np.linalg.norm(xs)
    s.close()


@pytest.mark.parametrize("grid,depth,skip", [((4, 4), 2, 1), ((16, 16), 4, 1), ((17, 23), 4, 1),
                                             ((6, 6, 6), 3, 1), ((9, 10, 11), 4, 1)])
def test_eps0_exact_recovery(grid, depth, skip):
    p = grid_ls(grid, int(np.prod(grid)), 3)
    s = pk.Solver.from_problem(p, depth, skip)
    s.factorize(0.0)
    x, info = s.cgls(dev(p.b), tol=1e-13)
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert info["iters"] <= 1
    assert np.linalg.norm(host(x) - xs) <= 1e-11 * np.linalg.norm(xs)
    s.close()


@pytest.mark.parametrize("grid,depth,skip,eps", [((17, 23), 4, 1, 1e-2), ((40, 24), 5, 2, 1e-3),
                                                 ((9, 10, 11), 4, 1, 1e-2), ((12, 12, 12), 4, 1, 1e-1)])
def test_ragged_and_3d_parity(grid, depth, skip, eps):
    p = grid_ls(grid, int(np.prod(grid)) // 2 + 7, 11)
    an, f = _oracle(p, depth, eps, skip)
    s = pk.Solver.from_problem(p, depth, skip)
    s.factorize(eps, ranks=f.ranks)
    _compare_ops(f, s, 1e-9)
    xo, io = osolve.cgls(osolve.Operator(f), p.b, tol=1e-12)
    x, info = s.cgls(dev(p.b), tol=1e-12)
    assert np.linalg.norm(host(x) - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()


def _full_config(cfg, precision, tol=1e-10):
    c = CONFIGS[cfg]
    p = config_problem(cfg)
    s = pk.Solver.from_problem(p, c["depth"], c["skip"], precision=precision)
    s.factorize(c["eps"])
    x, info = s.cgls(dev(p.b), tol=tol, max_iter=500)
    st = s.stats()
    s.close()
    return p, host(x), info, st


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config2_full_size(precision):
    p, x, info, st = _full_config(2, precision, tol=1e-12)
    print(f"config2 {precision}: iters {info['iters']} residual {info['residual']:.2e} "
          f"factor {st['factor_seconds']:.4f}s cgls {info['seconds']:.4f}s")
    assert info["converged"]
    assert _res(p, x) <= 1e-10
    A = p.scipy()
    xs = spla.spsolve((A.T @ A).tocsc(), A.T @ p.b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config3_full_size(precision):
    p, x, info, st = _full_config(3, precision)
    print(f"config3 {precision}: iters {info['iters']} residual {info['residual']:.2e} "
          f"factor {st['factor_seconds']:.4f}s cgls {info['seconds']:.4f}s")
    assert info["converged"]
    assert _res(p, x) <= 1e-10
