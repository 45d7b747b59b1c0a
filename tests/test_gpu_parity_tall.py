"""GPU parity on the kernel paths that only large fronts take.

The benchmark's fronts reach several thousand rows and its rank-revealing
QRs over a thousand, which the small parity grids never do.  These problems
are shaped so that the paths of the large workloads run against the FP64
oracle at oracle-friendly sizes:

* a 34 x 64 grid with a two-level tree: both leaf fronts have more than 2048
  rows (tall Householder panels: the cooperative FP32 panel, the FP64
  two-launch panel with Gram and T kernels, trailing updates over several
  1024-row segments) and their rows below the diagonal are rank-revealing
  QRs of more than 1024 rows (the pivot step's memory path);
* a 64 x 48 grid with a three-level tree: rank-revealing QRs of 700-730
  rows (register windows of 12 rows per lane), then a sparsified level;
* a 48 x 96 grid with a four-level tree and eps 1e-3: taller leaves and
  scaled / sparsified interfaces of a few hundred rows.

Every case compares the factor ops element by element with the oracle's at
the oracle's ranks (1e-10 of the block's largest entry, FP64), checks that
the free FP64 run takes the oracle's rank decisions, and compares x after
CGLS (1e-8) and the iteration counts (within one).  In FP32 the leaf-level
eliminations are compared (2e-5) and x after CGLS (1e-8).
"""
import numpy as np
import pytest

import paper_2102_09878_amd as pk
from oracle import solve as osolve
from oracle import spaqr as osp
from synth import grid_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "tall2": ((34, 64), 2, 1, 1e-2),
    "win12": ((64, 48), 3, 1, 1e-2),
    "deep4": ((48, 96), 4, 1, 1e-3),
}


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


@pytest.fixture(scope="module")
def oracle_runs():
    out = {}
    for name, (grid, depth, skip, eps) in CASES.items():
        p = grid_ls(grid, int(np.prod(grid)), 5)
        an = osp.analyze(p, depth)
        log = []
        f = osp.factorize(an, eps, skip, log=log)
        out[name] = (p, an, f, log)
    return out


def _compare(f, s, tol):
    assert s.stats()["num_ops"] == len(f.ops)
    worst = 0.0
    for i, o in enumerate(f.ops):
        g = s.op(i)
        assert g["kind"] == o[0], i
        assert np.array_equal(g["slots"], o[1]), i
        ref = o[3] if o[0] == "elim" else o[2]
        if o[0] == "elim":
            assert np.array_equal(g["nslots"], o[2]), i
        if o[0] == "sparsify" and ref.shape[1]:
            assert np.abs(g["tau"] - o[3]).max() <= tol, i
        assert g["mat"].shape == ref.shape, i
        if ref.size:
            err = np.abs(g["mat"] - ref).max() / max(1.0, np.abs(ref).max())
            worst = max(worst, err)
            assert err <= tol, (i, o[0], err)
    return worst


def test_cases_reach_the_large_paths(oracle_runs):
    """The shapes the cases are meant to exercise (a check on the cases)."""
    p, an, f, log = oracle_runs["tall2"]
    elim = [o for o in f.ops if o[0] == "elim"]
    ras = [r for r in log if r["kind"] == "reassign"]
    # leaf front rows >= owned rows = c_s + rows below the diagonal
    assert max(e[3].shape[0] + r["m"] for e, r in zip(elim, ras)) > 2048
    assert max(r["m"] for r in ras) > 1024
    p, an, f, log = oracle_runs["win12"]
    assert any(640 < r["m"] <= 768 for r in log if r["kind"] == "reassign")
    p, an, f, log = oracle_runs["deep4"]
    assert any(r["kind"] == "step1" and r["m"] > 200 for r in log)
    assert any(r["kind"] == "step2" and r["n"] > 500 for r in log)


@pytest.mark.parametrize("name", list(CASES))
def test_large_paths_forced_rank_parity(oracle_runs, name):
    grid, depth, skip, eps = CASES[name]
    p, an, f, log = oracle_runs[name]
    s = pk.Solver.from_problem(p, depth, skip)
    s.factorize(eps, ranks=f.ranks)
    worst = _compare(f, s, 1e-10)
    print(f"{name} fp64: worst relative op difference {worst:.3e} over {len(f.ops)} ops")
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_large_paths_fp32(oracle_runs, name):
    """FP32 fronts: the leaf-level eliminations (tall FP32 panels and MFMA
    trailing updates, inputs taken straight from A) within 2e-5 of the
    oracle's; past the first rank-revealing QR the FP32 form keeps its own
    decisions (its numerical-rank floor is the FP32 one), so there the
    check is x after CGLS against the FP64 oracle's x."""
    grid, depth, skip, eps = CASES[name]
    p, an, f, log = oracle_runs[name]
    s = pk.Solver.from_problem(p, depth, skip, precision="fp32")
    s.factorize(eps)
    n = 0
    worst = 0.0
    for i, o in enumerate(f.ops):
        g = s.op(i)
        if o[0] != "elim" or g["level"] != depth:
            break
        assert g["kind"] == "elim" and np.array_equal(g["slots"], o[1]) and np.array_equal(g["nslots"], o[2])
        err = np.abs(g["mat"] - o[3]).max() / max(1.0, np.abs(o[3]).max())
        worst = max(worst, err)
        assert err <= 2e-5, (i, err)
        n += 1
    assert n == sum(1 for o in f.ops[:n] if o[0] == "elim") and n >= 2
    xo, io = osolve.cgls(osolve.Operator(f), p.b, tol=1e-12)
    x, info = s.cgls(dev(p.b), tol=1e-12)
    x = x.cpu().numpy()
    err_x = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"{name} fp32: {n} leaf ops, worst {worst:.2e}; CGLS iters {info['iters']} (oracle {io['iters']}), "
          f"x error {err_x:.1e}")
    assert info["converged"] and err_x <= 1e-8
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_large_paths_free_run(oracle_runs, name):
    grid, depth, skip, eps = CASES[name]
    p, an, f, log = oracle_runs[name]
    s = pk.Solver.from_problem(p, depth, skip)
    s.factorize(eps)
    assert s.ranks() == f.ranks
    xo, io = osolve.cgls(osolve.Operator(f), p.b, tol=1e-12)
    x, info = s.cgls(dev(p.b), tol=1e-12)
    x = x.cpu().numpy()
    assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1, (info["iters"], io["iters"])
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()
