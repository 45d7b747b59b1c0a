"""The pivot-step loop stops launching steps on the live-matrix count that
the step kernel reports to pinned host memory; when the report does not
advance in time it reads the count through the stream instead.  With
SPAQR_PQR_REPORT_WAIT_MS=0 every wait takes that second path: the factor,
the ranks and the CGLS iterates must be exactly those of the default path
(both stop the same batches at steps whose results are identical), and the
host synchronises more often."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = r"""
import hashlib, json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_2102_09878_amd as pk
from synth import grid_ls
p = grid_ls((40, 36), 40 * 36 + 300, 23)
out = {}
for prec in ("fp64", "fp32"):
    s = pk.Solver.from_problem(p, 5, 1, precision=prec)
    s.factorize(1e-2)
    st = s.stats()
    h = hashlib.sha256()
    for i in range(st["num_ops"]):
        h.update(np.ascontiguousarray(s.op(i)["mat"]).tobytes())
    x, info = s.cgls(torch.as_tensor(p.b, device="cuda"), tol=1e-12)
    out[prec] = dict(ops=h.hexdigest(), ranks=s.ranks(), syncs=st["syncs"],
                     x=hashlib.sha256(x.cpu().numpy().tobytes()).hexdigest(), iters=info["iters"])
    s.close()
print(json.dumps(out))
"""


def _run(env_extra):
    env = dict(os.environ)
    env.pop("SPAQR_PQR_REPORT_WAIT_MS", None)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", CODE, ROOT], env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_stream_read_path_matches_report_path():
    a = _run({})
    b = _run({"SPAQR_PQR_REPORT_WAIT_MS": "0"})
    for prec in ("fp64", "fp32"):
        assert a[prec]["ranks"] == b[prec]["ranks"]
        assert a[prec]["ops"] == b[prec]["ops"]
        assert a[prec]["x"] == b[prec]["x"] and a[prec]["iters"] == b[prec]["iters"]
        assert b[prec]["syncs"] > a[prec]["syncs"]
