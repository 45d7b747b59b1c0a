"""The launch-shape autotuner (spaqr_autotune): it times factorizations of
the handle's problem, caches its choice by problem signature, and its knobs
change no result of the per-step pivoted QR (poll interval, register
window: same sums in the same order) and keep the tall-panel forms within
the oracle's tolerances."""
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


def _ops(s):
    return [s.op(i)["mat"].copy() for i in range(s.stats()["num_ops"])]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_knobs_keep_the_factor(precision):
    p = grid_ls((48, 40), 48 * 40, 31)
    s = pk.Solver.from_problem(p, 5, 2, precision=precision)
    s.factorize(1e-3)
    ref, rr = _ops(s), s.ranks()
    for poll, rows in ((1, 1024), (64, 256), (7, 0), (16, 512)):
        s.set_tune(pqr_poll=poll, pqr_reg_rows=rows)
        s.factorize(1e-3)
        assert s.ranks() == rr
        assert all(np.array_equal(a, b) for a, b in zip(_ops(s), ref)), (poll, rows)
    s.close()


def test_split_tall_panels_fp32_match_oracle():
    """Two-launch tall FP32 panels (the tuner's other choice) on fronts over
    2048 rows: leaf eliminations within 2e-5 of the oracle, x within 1e-8."""
    p = grid_ls((34, 64), 34 * 64, 5)
    f = osp.factorize(osp.analyze(p, 2), 1e-2, 1)
    s = pk.Solver.from_problem(p, 2, 1, precision="fp32")
    s.set_tune(tall_coop=0)
    s.factorize(1e-2)
    for i in range(2):
        g, o = s.op(i), f.ops[i]
        assert o[0] == "elim" and np.abs(g["mat"] - o[3]).max() <= 2e-5 * max(1.0, np.abs(o[3]).max())
    xo, _ = osolve.cgls(osolve.Operator(f), p.b, tol=1e-12)
    x, info = s.cgls(dev(p.b), tol=1e-12)
    assert info["converged"] and np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()


@pytest.mark.parametrize("coop", [1, 0])
def test_fp64_tall_panel_forms_match_oracle(coop):
    """FP64 fronts over 1024 rows, with tall panels in one cooperative launch
    (the default) or in two launches per column: with the oracle's ranks,
    every op within 1e-10 of the oracle's, then x within 1e-8."""
    p = grid_ls((34, 64), 34 * 64, 5)
    f = osp.factorize(osp.analyze(p, 2), 1e-2, 1)
    s = pk.Solver.from_problem(p, 2, 1, precision="fp64")
    s.set_tune(tall_coop=coop)
    s.factorize(1e-2, ranks=f.ranks)
    assert s.stats()["num_ops"] == len(f.ops)
    for i, o in enumerate(f.ops):
        g = s.op(i)
        ref = o[3] if o[0] == "elim" else o[2]
        assert g["mat"].shape == ref.shape, i
        if ref.size:
            assert np.abs(g["mat"] - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max()), (i, o[0])
    s.factorize(1e-2)
    assert s.ranks() == f.ranks
    xo, _ = osolve.cgls(osolve.Operator(f), p.b, tol=1e-12)
    x, info = s.cgls(dev(p.b), tol=1e-12)
    assert info["converged"] and np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()


def test_autotune_caches_and_reloads(tmp_path):
    c = CONFIGS[1]
    p = config_problem(1)
    cache = str(tmp_path / "tune.txt")
    s = pk.Solver.from_problem(p, c["depth"], c["skip"], precision="fp32")
    t1 = s.autotune(c["eps"], reps=1, cache_path=cache)
    assert not t1["from_cache"] and t1["evaluations"] == 6 and t1["seconds_best"] <= t1["seconds_default"]
    assert open(cache).read().count("\n") == 1
    x, info = s.cgls(dev(p.b), tol=1e-10)
    assert info["converged"]
    s.close()
    s = pk.Solver.from_problem(p, c["depth"], c["skip"], precision="fp32")
    t2 = s.autotune(c["eps"], reps=1, cache_path=cache)
    assert t2["from_cache"]
    assert (t2["pqr_poll"], t2["pqr_reg_rows"], t2["tall_coop"]) == (t1["pqr_poll"], t1["pqr_reg_rows"],
                                                                     t1["tall_coop"])
    assert s.get_tune()["pqr_poll"] == t1["pqr_poll"]
    s.close()
