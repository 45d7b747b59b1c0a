"""Writes tests/golden/full_size_cfg<k>.json from the FP64 oracle alone.

    python tests/golden/make_full_size.py 2 3

For each workload (the 256 x 256 grid and the 32^3 grid least-squares
problems of synth.CONFIGS) the oracle analyses, factorizes and runs CGLS;
the file keeps what a GPU test can compare at full size without rerunning
the oracle there:

* every rank decision (integer parity) and the kind and shape of every op;
* for a fixed sample of ops, 96 entries each at fixed pseudo-random
  positions (element-wise op parity at the oracle's ranks);
* the CGLS iteration counts to 1e-10 and 1e-12 and the final residuals;
* x (tol 1e-12) at 512 fixed positions, and ||x||.

Only oracle/ and synth/ are used.  Takes about 15-30 minutes per workload
on one core.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import solve, spaqr  # noqa: E402
from synth import CONFIGS, config_problem  # noqa: E402

OP_STRIDE = 11
ENTRIES = 96
X_SAMPLE = 512


def op_matrix(o):
    return o[3] if o[0] == "elim" else o[2]


def main(cfgs):
    for k in cfgs:
        c = CONFIGS[k]
        p = config_problem(k)
        t0 = time.perf_counter()
        an = spaqr.analyze(p, c["depth"])
        t1 = time.perf_counter()
        f = spaqr.factorize(an, c["eps"], c["skip"])
        t2 = time.perf_counter()
        print(f"cfg {k}: analyze {t1 - t0:.1f}s factorize {t2 - t1:.1f}s ops {len(f.ops)}", flush=True)
        op = solve.Operator(f)
        normA = solve.norm2_estimate(op)
        x10, i10 = solve.cgls(op, p.b, tol=1e-10, normA=normA)
        x12, i12 = solve.cgls(op, p.b, tol=1e-12, normA=normA)
        t3 = time.perf_counter()
        print(f"cfg {k}: cgls {t3 - t2:.1f}s iters {i10['iters']} / {i12['iters']}", flush=True)
        shapes = []
        samples = []
        for i, o in enumerate(f.ops):
            R = op_matrix(o)
            shapes.append([o[0], int(R.shape[0]), int(R.shape[1])])
            if i % OP_STRIDE or R.size == 0:
                continue
            rng = np.random.default_rng(1000 + i)
            rr = rng.integers(0, R.shape[0], ENTRIES)
            cc = rng.integers(0, R.shape[1], ENTRIES)
            samples.append(dict(op=i, rows=rr.tolist(), cols=cc.tolist(), vals=R[rr, cc].tolist(),
                                absmax=float(np.abs(R).max())))
        xi = np.random.default_rng(7).choice(p.N, min(X_SAMPLE, p.N), replace=False)
        out = dict(config=k, eps=c["eps"], depth=c["depth"], skip=c["skip"], ranks=[int(r) for r in f.ranks],
                   op_shapes=shapes, op_samples=samples,
                   cgls_1e10=dict(iters=i10["iters"], residual=i10["residual"]),
                   cgls_1e12=dict(iters=i12["iters"], residual=i12["residual"]), normA=normA,
                   x_index=xi.tolist(), x_values=x12[xi].tolist(), x_norm=float(np.linalg.norm(x12)),
                   oracle_seconds=dict(analyze=t1 - t0, factorize=t2 - t1, cgls=t3 - t2))
        path = os.path.join(ROOT, "tests", "golden", f"full_size_cfg{k}.json")
        with open(path, "w") as fh:
            json.dump(out, fh)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [2, 3])
