"""GPU parity of the batching form: independent problems factorized in one
handle (same-level fronts of all members in the same launches) and solved
by per-member CGLS, against each member factorized alone, against the
oracle's factor of each member (FP64) and against the least-squares
solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import paper_2102_09878_amd as pk
from oracle import adjoint as oadj
from oracle import spaqr as osp
from synth import batch_problem, batch_sides, grid_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _member_ops(bs, c0, c1):
    """Ops of the batch whose slots fall in [c0, c1), in creation order."""
    out = []
    for i in range(bs.stats()["num_ops"]):
        o = bs.op(i)
        if c0 <= o["slots"][0] < c1:
            assert ((o["slots"] >= c0) & (o["slots"] < c1)).all()
            out.append(o)
    return out


def _lsq_res(p, x):
    A = p.scipy()
    nA = spla.svds(A, k=1, return_singular_vectors=False)[0]
    return np.linalg.norm(A.T @ (p.b - A @ x)) / (nA * np.linalg.norm(p.b))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_members_equal_standalone(precision):
    grids = [(16, 16), (23, 17), (30, 30), (12, 20), (26, 21)]
    probs = [grid_ls(g, g[0] * g[1], 60 + i) for i, g in enumerate(grids)]
    depths = [4, 4, 5, 3, 4]
    eps = 1e-2
    bs = pk.BatchSolver.from_problems(probs, depths, skip=1, precision=precision)
    bs.factorize(eps)
    b_all = dev(np.concatenate([p.b for p in probs]))
    x_all, infos = bs.cgls_each(b_all, tol=1e-12)
    x_all = host(x_all)
    for g, (p, d) in enumerate(zip(probs, depths)):
        c0, c1 = int(bs.col_off[g]), int(bs.col_off[g + 1])
        s = pk.Solver.from_problem(p, d, 1, precision=precision)
        s.factorize(eps)
        mine = _member_ops(bs, c0, c1)
        assert len(mine) == s.stats()["num_ops"], g
        for i, o in enumerate(mine):
            r = s.op(i)
            assert o["kind"] == r["kind"] and (o["slots"] - c0 == r["slots"]).all(), (g, i)
            if o["kind"] == "elim":
                assert (o["nslots"] - c0 == r["nslots"]).all(), (g, i)
            scale = max(1.0, np.abs(r["mat"]).max()) if r["mat"].size else 1.0
            assert np.abs(o["mat"] - r["mat"]).max(initial=0.0) <= 1e-12 * scale, (g, i)
        if precision == "fp64":
            # the member's ops taken from the batch handle against the oracle
            f = osp.factorize(osp.analyze(p, d), eps, 1)
            assert len(f.ops) == len(mine), g
            for i, (o, fo) in enumerate(zip(mine, f.ops)):
                ref = fo[3] if fo[0] == "elim" else fo[2]
                assert o["kind"] == fo[0] and np.array_equal(o["slots"] - c0, fo[1]), (g, i)
                assert o["mat"].shape == ref.shape, (g, i)
                if ref.size:
                    assert np.abs(o["mat"] - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max()), (g, i)
        x, info = s.cgls(dev(p.b), tol=1e-12)
        assert infos[g]["converged"] and infos[g]["iters"] == info["iters"], (g, infos[g], info)
        assert np.abs(x_all[c0:c1] - host(x)).max() <= 1e-10 * np.abs(host(x)).max()
        xs = oadj.lstsq_solution(p.row_ptr, p.col_idx, p.vals, p.b, p.M, p.N)
        assert np.linalg.norm(x_all[c0:c1] - xs) <= 1e-8 * np.linalg.norm(xs)
        s.close()
    bs.close()


def test_batch_of_64_fp32():
    """64 grids of side 48..160 (M = 2N, eps 1e-2), FP32 factor, per-member
    CGLS to 1e-12 (the x check needs both sides converged well below the
    1e-10 bound); sampled members checked against the normal equations."""
    sides = batch_sides()
    probs = [batch_problem(i, sides) for i in range(len(sides))]
    depths = [p.meta["depth"] for p in probs]
    bs = pk.BatchSolver.from_problems(probs, depths, skip=2, precision="fp32")
    bs.factorize(1e-2)
    st = bs.stats()
    b_all = dev(np.concatenate([p.b for p in probs]))
    x_all, infos = bs.cgls_each(b_all, tol=1e-12)
    x_all = host(x_all)
    its = [i["iters"] for i in infos]
    print(f"batch64: N {bs.N} factor {st['factor_seconds']:.3f}s launches {st['launches']} syncs {st['syncs']} "
          f"phases {st['phase_seconds']} "
          f"iters {min(its)}..{max(its)} worst residual {max(i['residual'] for i in infos):.2e}")
    assert all(i["converged"] and i["residual"] <= 1e-10 for i in infos)
    for g in (0, 17, 40, 63):
        p = probs[g]
        c0, c1 = int(bs.col_off[g]), int(bs.col_off[g + 1])
        x = x_all[c0:c1]
        assert _lsq_res(p, x) <= 1e-10
        xs = oadj.lstsq_solution(p.row_ptr, p.col_idx, p.vals, p.b, p.M, p.N)
        assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs), g
    bs.close()
