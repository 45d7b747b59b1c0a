"""The host analysis (analyze.cpp, graph_nd.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer.

The analysis sources are compiled with g++ and -fsanitize=address,undefined
(no recovery: the first report aborts the run) together with the host-only
driver csrc/host_check.cpp, which runs the analysis of every problem and the
block-diagonal union of a batch.  Problems: geometric 2D and 3D grids, a
ragged grid, a general matrix (graph nested dissection and max-product
matching), an inverse-Poisson J^T, a square system, and malformed inputs
that must be refused with an error code (unsorted or repeated columns, a
column index out of range, M < N, a decreasing row pointer, a grid that
does not match N).  The sanitized run must report nothing and return the
same column order and row owners as libspaqr's own build
(spaqr_get_ordering)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import paper_2102_09878_amd as pk
from synth import general_ls, grid_ls, grid_square, inverse_poisson

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_09878_amd", "csrc")
GXX = shutil.which("g++")
ROCM_INC = "/opt/rocm/include"

pytestmark = pytest.mark.skipif(GXX is None or not os.path.isdir(ROCM_INC),
                                reason="needs g++ and the HIP headers")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = tmp_path_factory.mktemp("host_check")
    exe = str(out / "host_check")
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM_INC}",
             f"-I{os.path.join(ROOT, 'include')}"]
    srcs = [os.path.join(CSRC, f) for f in ("host_check.cpp", "analyze.cpp", "graph_nd.cpp")]
    r = subprocess.run([GXX, *flags, *srcs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _problem_bytes(rp, ci, va, M, N, grid, depth, skip, expect_error=False, in_union=False):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    va = np.ascontiguousarray(va, dtype=np.float64)
    hdr = struct.pack("<3q7i", M, N, len(ci), *grid, depth, skip, int(expect_error), int(in_union))
    assert len(rp) == max(M + 1, 0)
    return hdr + rp.tobytes() + ci.tobytes() + va.tobytes()


def _run(driver, tmp_path, items):
    inp = tmp_path / "problems.bin"
    outp = tmp_path / "out.bin"
    with open(inp, "wb") as fh:
        fh.write(struct.pack("<q", len(items)))
        for it in items:
            fh.write(_problem_bytes(**it))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, str(inp), str(outp)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, \
        r.stderr[-4000:]
    buf = open(outp, "rb").read()
    pos = 0
    res = []

    def take(dt, n):
        nonlocal pos
        a = np.frombuffer(buf, dtype=dt, count=n, offset=pos)
        pos += a.nbytes
        return a

    for it in items:
        st = int(take(np.int32, 1)[0])
        if st == 0:
            res.append((st, take(np.int32, it["N"]).copy(), take(np.int32, it["M"]).copy()))
        else:
            res.append((st, None, None))
    st = int(take(np.int32, 1)[0])
    UN, UM = (int(v) for v in take(np.int64, 2))
    union = (st, take(np.int32, UN).copy(), take(np.int32, UM).copy()) if st == 0 and UN else (st, None, None)
    assert pos == len(buf)
    return res, union


def _item(p, depth, skip=-1, geometric=True, **kw):
    grid = tuple(p.grid) + (1,) * (3 - len(p.grid)) if geometric else (0, 0, 0)
    return dict(rp=p.row_ptr, ci=p.col_idx, va=p.vals, M=p.M, N=p.N, grid=grid, depth=depth, skip=skip, **kw)


def _valid_problems():
    probs = [
        (grid_ls((32, 32), 1024, 0), 4, True),
        (grid_ls((23, 17), 300, 3), 4, True),
        (grid_ls((10, 10, 10), 500, 2), 3, True),
        (general_ls((24, 24), 576, 9), 4, False),
        (inverse_poisson(24, 2, 1.5, seed=1), 4, True),
        (grid_square((20, 20), 5), 3, True),
    ]
    return probs


def test_analysis_clean_under_sanitizers(driver, tmp_path):
    probs = _valid_problems()
    items = [_item(p, d, geometric=g, in_union=(i < 3)) for i, (p, d, g) in enumerate(probs)]
    res, union = _run(driver, tmp_path, items)
    for (p, d, g), (st, perm, owner) in zip(probs, res):
        assert st == 0
        s = pk.Solver(p.row_ptr, p.col_idx, p.vals, p.M, p.N, tuple(p.grid) if g else None, d, -1)
        perm_lib, owner_lib = s.ordering()
        s.close()
        assert np.array_equal(perm, perm_lib) and np.array_equal(owner, owner_lib)
    # the batch union: every column and row appears once, problems side by side
    st, perm, owner = union
    assert st == 0
    n_tot = sum(p.N for p, _, _ in probs[:3])
    assert perm is not None and np.array_equal(np.sort(perm), np.arange(n_tot))
    assert owner.min() >= 0


def test_malformed_inputs_refused_under_sanitizers(driver, tmp_path):
    p = grid_ls((8, 8), 64, 1)
    rp, ci, va = p.row_ptr.copy(), p.col_idx.copy(), p.vals.copy()
    bad = []
    # columns of a row out of order
    c2 = ci.copy()
    c2[rp[0]], c2[rp[0] + 1] = c2[rp[0] + 1], c2[rp[0]]
    bad.append(dict(rp=rp, ci=c2, va=va))
    # a repeated column in a row
    c3 = ci.copy()
    c3[rp[0] + 1] = c3[rp[0]]
    bad.append(dict(rp=rp, ci=c3, va=va))
    # a column index out of range (and a negative one)
    c4 = ci.copy()
    c4[-1] = p.N
    bad.append(dict(rp=rp, ci=c4, va=va))
    c5 = ci.copy()
    c5[0] = -1
    bad.append(dict(rp=rp, ci=c5, va=va))
    # a decreasing row pointer
    r6 = rp.copy()
    r6[5] = r6[4] - 1
    bad.append(dict(rp=r6, ci=ci, va=va))
    items = [dict(M=p.M, N=p.N, grid=(8, 8, 1), depth=3, skip=-1, expect_error=True, **b) for b in bad]
    # M < N: the first N - 1 rows of the pattern only
    k = p.N - 1
    items.append(dict(rp=rp[:k + 1], ci=ci[:rp[k]], va=va[:rp[k]], M=k, N=p.N, grid=(8, 8, 1), depth=3,
                      skip=-1, expect_error=True))
    # a grid that does not match N
    items.append(dict(rp=rp, ci=ci, va=va, M=p.M, N=p.N, grid=(8, 7, 1), depth=3, skip=-1, expect_error=True))
    res, union = _run(driver, tmp_path, items)
    assert all(st != 0 for st, _, _ in res)
    assert all(st == pk.spaqr.EARG for st, _, _ in res), [st for st, _, _ in res]
