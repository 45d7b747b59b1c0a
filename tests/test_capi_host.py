"""Host-side checks of libspaqr: it loads, exports every symbol of
include/spaqr.h, its analysis matches the oracle's exactly (integer work:
column order and row owners), and it reports errors with clean codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2102_09878_amd as pk
from paper_2102_09878_amd import spaqr as b
from oracle import spaqr as osp
from synth import CONFIGS, batch_problem, config_problem, grid_ls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_library_exports_every_declared_symbol():
    lib = b.load()
    header = open(os.path.join(ROOT, "include", "spaqr.h")).read()
    declared = set(re.findall(r"\b(spaqr_[a-z_]+)\s*\(", header))
    assert declared == set(b.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
def test_analysis_matches_oracle(cfg):
    c = CONFIGS[cfg]
    p = config_problem(cfg)
    s = pk.Solver.from_problem(p, c["depth"], c["skip"])
    perm, owner = s.ordering()
    an = osp.analyze(p, c["depth"])
    assert (perm == an.col_perm).all()
    assert (owner == an.row_owner).all()
    s.close()


@pytest.mark.parametrize("grid,depth", [((32, 32), 4), ((48, 40), 5), ((12, 12, 12), 3), ((64, 64), 6)])
def test_graph_analysis_matches_oracle(grid, depth):
    """Matrices without a grid: graph nested dissection, interfaces and the
    max-product matching decide the column order and the row owners, which
    must equal the oracle's exactly."""
    from synth import general_ls
    p = general_ls(grid, int(np.prod(grid)), 9)
    s = pk.Solver(p.row_ptr, p.col_idx, p.vals, p.M, p.N, None, depth, -1)
    perm, owner = s.ordering()
    an = osp.analyze(p, depth)
    assert (perm == an.col_perm).all()
    assert (owner == an.row_owner).all()
    s.close()


def test_graph_analysis_rejects_too_deep_tree():
    from synth import general_ls
    p = general_ls((8, 8), 64, 1)
    with pytest.raises(pk.SpaqrError) as e:
        pk.Solver(p.row_ptr, p.col_idx, p.vals, p.M, p.N, None, 8, -1)
    assert e.value.code == b.EARG


@pytest.mark.parametrize("i", [0, 17, 63])
def test_analysis_matches_oracle_batch_members(i):
    p = batch_problem(i)
    d = p.meta["depth"]
    s = pk.Solver.from_problem(p, d, 2)
    perm, owner = s.ordering()
    an = osp.analyze(p, d)
    assert (perm == an.col_perm).all() and (owner == an.row_owner).all()


def _analyze_rc(rp, ci, va, M, N, grid, depth=2):
    lib = b.load()
    g = list(grid) + [1] * (3 - len(grid))
    opt = b.Options(depth, -1, (ctypes.c_int32 * 3)(*g), 0, 0, 0, None)
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    va = np.ascontiguousarray(va, dtype=np.float64)
    rc = lib.spaqr_analyze(b._ptr(rp), b._ptr(ci), b._ptr(va), M, N, ctypes.byref(opt), ctypes.byref(h))
    msg = lib.spaqr_last_error(None).decode()
    if rc == 0:
        lib.spaqr_destroy(h)
    return rc, msg


def test_error_codes_for_bad_input():
    p = grid_ls((8, 8), 64, 0)
    rp, ci, va = p.row_ptr, p.col_idx, p.vals
    assert _analyze_rc(rp, ci, va, p.M, p.N, p.grid)[0] == b.OK
    # M < N
    assert _analyze_rc(rp[:40], ci[:rp[39]], va[:rp[39]], 39, p.N, p.grid)[0] == b.EARG
    # unsorted columns in a row
    ci2 = ci.copy()
    ci2[rp[0]], ci2[rp[0] + 1] = ci2[rp[0] + 1], ci2[rp[0]]
    assert _analyze_rc(rp, ci2, va, p.M, p.N, p.grid)[0] == b.EARG
    # column index out of range
    ci3 = ci.copy()
    ci3[-1] = p.N
    assert _analyze_rc(rp, ci3, va, p.M, p.N, p.grid)[0] == b.EARG
    # empty column
    va4 = va.copy()
    va4[ci == 5] = 0.0
    rc, msg = _analyze_rc(rp, ci, va4, p.M, p.N, p.grid)
    assert rc == b.EARG and "empty" in msg
    # grid that does not match N, depth too large for the grid
    assert _analyze_rc(rp, ci, va, p.M, p.N, (8, 7))[0] == b.EARG
    assert _analyze_rc(rp, ci, va, p.M, p.N, p.grid, depth=6)[0] == b.EARG
    # one-plane separators cannot separate radius-1 rows
    lib = b.load()
    opt = b.Options(3, -1, (ctypes.c_int32 * 3)(32, 32, 1), 1, 0, 0, None)
    q = grid_ls((32, 32), 1024, 0)
    h = ctypes.c_void_p()
    rc = lib.spaqr_analyze(b._ptr(q.row_ptr), b._ptr(q.col_idx), b._ptr(q.vals), q.M, q.N,
                           ctypes.byref(opt), ctypes.byref(h))
    assert rc == b.EARG and "sibling" in lib.spaqr_last_error(None).decode()


def test_call_order_errors_without_gpu_work():
    p = grid_ls((8, 8), 64, 0)
    s = pk.Solver.from_problem(p, 2, 1)
    lib = b.load()
    info = b.CglsInfo()
    dummy = ctypes.c_void_p(16)
    assert lib.spaqr_cgls(s.h, dummy, 1e-10, 10, dummy, ctypes.byref(info)) == b.ESTATE
    st = b.Stats()
    assert lib.spaqr_factor_stats(s.h, ctypes.byref(st)) == b.ESTATE
    assert lib.spaqr_apply_op(s.h, 0, dummy, dummy) == b.ESTATE
    assert lib.spaqr_apply_op(s.h, 7, dummy, dummy) == b.EARG
    assert lib.spaqr_apply_noalloc(s.h, dummy, dummy) == b.ESTATE
    assert lib.spaqr_apply_noalloc(s.h, None, dummy) == b.EARG
    assert lib.spaqr_factorize(s.h, -1.0) == b.EARG
    s.close()


@pytest.mark.skipif(_has_gpu(), reason="checks the no-GPU error path")
def test_factorize_without_gpu_reports_hip_error():
    p = grid_ls((8, 8), 64, 0)
    s = pk.Solver.from_problem(p, 2, 1)
    with pytest.raises(pk.SpaqrError) as e:
        s.factorize(1e-2)
    assert e.value.code == b.EHIP
    s.close()


def test_batch_analysis_is_the_union_of_members():
    """A batch handle orders each member exactly as its own analysis does,
    at the member's column offset (integer parity, host only)."""
    probs = [grid_ls((s, s + 3), s * (s + 3), 40 + s) for s in (9, 14, 11)]
    depths = [3, 4, 3]
    bs = pk.BatchSolver.from_problems(probs, depths, skip=1)
    assert bs.count == 3
    assert list(bs.col_off) == [0] + list(np.cumsum([p.N for p in probs]))
    assert list(bs.row_off) == [0] + list(np.cumsum([p.M for p in probs]))
    perm, owner = bs.ordering()
    fbase = 0
    for g, (p, d) in enumerate(zip(probs, depths)):
        an = osp.analyze(p, d)
        c0, c1 = bs.col_off[g], bs.col_off[g + 1]
        r0, r1 = bs.row_off[g], bs.row_off[g + 1]
        assert (perm[c0:c1] == an.col_perm + c0).all()
        assert (owner[r0:r1] == an.row_owner + fbase).all()
        fbase += int(an.row_owner.max()) + 1
    bs.close()


def test_batch_rejects_mixed_skip_and_bad_member():
    def member(p, grid=None):
        return (p.row_ptr, p.col_idx, p.vals, p.M, p.N, grid or p.grid)

    p1, p2 = grid_ls((24, 24), 576, 1), grid_ls((24, 24), 576, 2)
    # default skip is 1 at depth 4 and 2 at depth 5
    with pytest.raises(pk.SpaqrError) as e:
        pk.BatchSolver([member(p1), member(p2)], [4, 5], skip=-1)
    assert e.value.code == b.EARG and "sparsify_skip" in str(e.value)
    # a member whose grid does not match its N is named in the message
    with pytest.raises(pk.SpaqrError) as e:
        pk.BatchSolver([member(p1), member(p2, (24, 23))], [4, 4], skip=1)
    assert e.value.code == b.EARG and "batch member 1" in str(e.value)


def test_set_tune_validates_without_gpu():
    p = grid_ls((8, 8), 64, 0)
    s = pk.Solver.from_problem(p, 2, 1)
    assert s.get_tune() == dict(pqr_poll=16, pqr_reg_rows=1024, tall_coop=1, from_cache=False, evaluations=0,
                                seconds_default=0.0, seconds_best=0.0)
    for bad in (dict(pqr_poll=0), dict(pqr_reg_rows=2048), dict(tall_coop=3)):
        with pytest.raises(pk.SpaqrError) as e:
            s.set_tune(**bad)
        assert e.value.code == b.EARG
    s.set_tune(pqr_poll=4)
    assert s.get_tune()["pqr_poll"] == 4 and s.get_tune()["pqr_reg_rows"] == 1024
    s.close()

