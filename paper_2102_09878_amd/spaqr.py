"""Thin ctypes binding of libspaqr (the C-ABI declared in include/spaqr.h).

Argument marshalling only: every step of the factorization and of the
solvers runs in the library's HIP kernels.  Device vectors are passed as
torch tensors on the GPU (FP64, contiguous); PyTorch is used for device
memory only.  The binding fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SPAQR_LIB", os.path.join(_HERE, "libspaqr.so"))

OK, NOCONV = 0, 1
EARG, ESTATE, ERANK, EHIP, ENOMEM = -1, -2, -3, -4, -5
FP64, FP32_FACTOR = 0, 1
WINV, WINVT = 0, 1
MAX_LEVELS = 32

EXPORTS = ["spaqr_analyze", "spaqr_get_ordering", "spaqr_set_values", "spaqr_factorize",
           "spaqr_factorize_forced", "spaqr_apply", "spaqr_apply_noalloc", "spaqr_csne", "spaqr_apply_op", "spaqr_cgls", "spaqr_factor_stats",
           "spaqr_get_ranks", "spaqr_get_op", "spaqr_time_kernel", "spaqr_adjoint", "spaqr_batch_analyze",
           "spaqr_batch_info", "spaqr_batch_cgls", "spaqr_autotune", "spaqr_set_tune", "spaqr_get_tune",
           "spaqr_destroy", "spaqr_last_error"]


class Options(ctypes.Structure):
    _fields_ = [("nd_depth", ctypes.c_int32), ("sparsify_skip", ctypes.c_int32),
                ("grid", ctypes.c_int32 * 3), ("sep_width", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("device", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class CglsInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("residual", ctypes.c_double),
                ("paper_residual", ctypes.c_double), ("norm_a", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("num_ops", ctypes.c_int32), ("num_ranks", ctypes.c_int32),
                ("top_cols", ctypes.c_int32), ("top_rows", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("syncs", ctypes.c_int32), ("pad_", ctypes.c_int32), ("mem_factor", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("flops", ctypes.c_double * 5),
                ("bytes", ctypes.c_double * 5), ("phase_seconds", ctypes.c_double * 5),
                ("factor_seconds", ctypes.c_double), ("kernel_calls", ctypes.c_int64),
                ("kernel_seconds", ctypes.c_double), ("kernel_bytes", ctypes.c_double),
                ("kernel_flops", ctypes.c_double),
                ("level_interfaces", ctypes.c_int32 * MAX_LEVELS), ("level_aspect", ctypes.c_double * MAX_LEVELS),
                ("level_cols", ctypes.c_int64 * MAX_LEVELS), ("level_rank1", ctypes.c_int64 * MAX_LEVELS),
                ("level_rank2", ctypes.c_int64 * MAX_LEVELS), ("sync_wait_seconds", ctypes.c_double),
                ("kernel_span_calls", ctypes.c_int64), ("kernel_span_seconds", ctypes.c_double)]


class Tune(ctypes.Structure):
    _fields_ = [("pqr_poll", ctypes.c_int32), ("pqr_reg_rows", ctypes.c_int32), ("tall_coop", ctypes.c_int32),
                ("from_cache", ctypes.c_int32), ("evaluations", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("seconds_default", ctypes.c_double), ("seconds_best", ctypes.c_double)]


class OpDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("round", ctypes.c_int32), ("level", ctypes.c_int32)]


PHASES = ("eliminate", "reassign", "scale", "sparsify", "merge")

_lib = None


def load(path: str = LIB_PATH):
    """Load libspaqr.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libspaqr.so not found at {path}; run `python -m paper_2102_09878_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "spaqr_analyze": [P, P, P, I64, I64, ctypes.POINTER(Options), ctypes.POINTER(P)],
        "spaqr_get_ordering": [P, P, P],
        "spaqr_set_values": [P, P],
        "spaqr_factorize": [P, D],
        "spaqr_factorize_forced": [P, D, P, I32],
        "spaqr_apply": [P, P, P],
        "spaqr_apply_noalloc": [P, P, P],
        "spaqr_csne": [P, P, D, I32, P, ctypes.POINTER(CglsInfo)],
        "spaqr_apply_op": [P, I32, P, P],
        "spaqr_cgls": [P, P, D, I32, P, ctypes.POINTER(CglsInfo)],
        "spaqr_factor_stats": [P, ctypes.POINTER(Stats)],
        "spaqr_get_ranks": [P, P, I32, ctypes.POINTER(I32)],
        "spaqr_get_op": [P, I32, ctypes.POINTER(OpDesc), P, P, P, P],
        "spaqr_time_kernel": [P, ctypes.c_char_p, ctypes.c_int32],
        "spaqr_adjoint": [P, P, P, P, D, I32, P, P, P, ctypes.POINTER(CglsInfo)],
        "spaqr_batch_analyze": [I32, P, P, P, P, P, P, ctypes.POINTER(P)],
        "spaqr_batch_info": [P, ctypes.POINTER(I32), P, P],
        "spaqr_batch_cgls": [P, P, D, I32, P, P],
        "spaqr_autotune": [P, D, I32, ctypes.c_char_p, ctypes.POINTER(Tune)],
        "spaqr_set_tune": [P, ctypes.POINTER(Tune)],
        "spaqr_get_tune": [P, ctypes.POINTER(Tune)],
        "spaqr_destroy": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.spaqr_last_error.argtypes = [P]
    lib.spaqr_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class SpaqrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"spaqr error {code}: {msg}")
        self.code = code


def _check(lib, h, rc, allow=(OK,)):
    if rc not in allow:
        msg = lib.spaqr_last_error(h)
        raise SpaqrError(rc, msg.decode() if msg else "")
    return rc


def _ptr(a):
    """Device pointer of a torch tensor or host pointer of a numpy array."""
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev_f64(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return t


# ---- functions with the C-ABI names ----------------------------------------

def spaqr_analyze(row_ptr, col_idx, vals, M, N, grid, nd_depth=0, sparsify_skip=-1, sep_width=0,
                  precision=FP64, device=0):
    lib = load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(vals, dtype=np.float64)
    g = [0, 0, 0] if grid is None else list(grid) + [1] * (3 - len(grid))   # no grid: graph partitioning
    opt = Options(nd_depth, sparsify_skip, (ctypes.c_int32 * 3)(*g), sep_width, precision, device, None)
    h = ctypes.c_void_p()
    rc = lib.spaqr_analyze(_ptr(rp), _ptr(ci), _ptr(va), int(M), int(N), ctypes.byref(opt), ctypes.byref(h))
    _check(lib, None, rc)
    return h


def spaqr_get_ordering(h, M, N):
    lib = load()
    cp = np.zeros(N, dtype=np.int32)
    ro = np.zeros(M, dtype=np.int32)
    _check(lib, h, lib.spaqr_get_ordering(h, _ptr(cp), _ptr(ro)))
    return cp, ro


def spaqr_set_values(h, vals_dev):
    lib = load()
    _check(lib, h, lib.spaqr_set_values(h, _ptr(_dev_f64(vals_dev))))


def spaqr_factorize(h, eps):
    lib = load()
    _check(lib, h, lib.spaqr_factorize(h, float(eps)))


def spaqr_factorize_forced(h, eps, ranks):
    lib = load()
    r = np.ascontiguousarray(ranks, dtype=np.int32)
    _check(lib, h, lib.spaqr_factorize_forced(h, float(eps), _ptr(r), int(r.shape[0])))


def spaqr_apply(h, b_dev, x_dev):
    lib = load()
    _check(lib, h, lib.spaqr_apply(h, _ptr(_dev_f64(b_dev)), _ptr(_dev_f64(x_dev))))


def spaqr_apply_noalloc(h, b_dev, x_dev):
    lib = load()
    _check(lib, h, lib.spaqr_apply_noalloc(h, _ptr(_dev_f64(b_dev)), _ptr(_dev_f64(x_dev))))


def spaqr_apply_op(h, op, in_dev, out_dev):
    lib = load()
    _check(lib, h, lib.spaqr_apply_op(h, int(op), _ptr(_dev_f64(in_dev)), _ptr(_dev_f64(out_dev))))


def spaqr_cgls(h, b_dev, x_dev, tol=1e-10, max_iter=200):
    lib = load()
    info = CglsInfo()
    rc = lib.spaqr_cgls(h, _ptr(_dev_f64(b_dev)), float(tol), int(max_iter), _ptr(_dev_f64(x_dev)),
                        ctypes.byref(info))
    _check(lib, h, rc, allow=(OK, NOCONV))
    return dict(iters=info.iters, converged=bool(info.converged), residual=info.residual,
                paper_residual=info.paper_residual, norm_a=info.norm_a, seconds=info.seconds)


def spaqr_csne(h, b_dev, x_dev, tol=1e-10, max_steps=50):
    lib = load()
    info = CglsInfo()
    rc = lib.spaqr_csne(h, _ptr(_dev_f64(b_dev)), float(tol), int(max_steps), _ptr(_dev_f64(x_dev)),
                        ctypes.byref(info))
    _check(lib, h, rc, allow=(OK, NOCONV))
    return dict(steps=info.iters, converged=bool(info.converged), residual=info.residual,
                paper_residual=info.paper_residual, norm_a=info.norm_a, seconds=info.seconds)


def spaqr_adjoint(h, x_dev, b_dev, g_dev, grad_b_dev=None, grad_vals_dev=None, lambda_dev=None, tol=1e-12,
                  max_iter=500):
    lib = load()
    info = CglsInfo()

    def opt(t):
        return None if t is None else _ptr(_dev_f64(t))

    rc = lib.spaqr_adjoint(h, opt(x_dev), opt(b_dev), _ptr(_dev_f64(g_dev)), float(tol), int(max_iter),
                           opt(grad_b_dev), opt(grad_vals_dev), opt(lambda_dev), ctypes.byref(info))
    _check(lib, h, rc, allow=(OK, NOCONV))
    return dict(iters=info.iters, converged=bool(info.converged), residual=info.residual,
                recurrence_residual=info.paper_residual, seconds=info.seconds)


def spaqr_batch_analyze(problems, depths, sparsify_skip=-1, sep_width=0, precision=FP64, device=0):
    """problems: sequence of (row_ptr, col_idx, vals, M, N, grid)."""
    lib = load()
    keep = []
    n = len(problems)
    rps, cis, vas = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
    Ms, Ns = np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64)
    opts = (Options * n)()
    for g, (rp, ci, va, M, N, grid) in enumerate(problems):
        rp = np.ascontiguousarray(rp, dtype=np.int64)
        ci = np.ascontiguousarray(ci, dtype=np.int32)
        va = np.ascontiguousarray(va, dtype=np.float64)
        keep += [rp, ci, va]
        rps[g], cis[g], vas[g] = rp.ctypes.data, ci.ctypes.data, va.ctypes.data
        Ms[g], Ns[g] = M, N
        gr = [0, 0, 0] if grid is None else list(grid) + [1] * (3 - len(grid))
        opts[g] = Options(int(depths[g]), sparsify_skip, (ctypes.c_int32 * 3)(*gr), sep_width, precision, device,
                          None)
    h = ctypes.c_void_p()
    rc = lib.spaqr_batch_analyze(n, ctypes.cast(rps, ctypes.c_void_p), ctypes.cast(cis, ctypes.c_void_p),
                                 ctypes.cast(vas, ctypes.c_void_p), _ptr(Ms), _ptr(Ns),
                                 ctypes.cast(opts, ctypes.c_void_p), ctypes.byref(h))
    _check(lib, None, rc)
    return h


def spaqr_batch_info(h):
    lib = load()
    n = ctypes.c_int32()
    _check(lib, h, lib.spaqr_batch_info(h, ctypes.byref(n), None, None))
    co = np.zeros(n.value + 1, dtype=np.int64)
    ro = np.zeros(n.value + 1, dtype=np.int64)
    _check(lib, h, lib.spaqr_batch_info(h, ctypes.byref(n), _ptr(co), _ptr(ro)))
    return co, ro


def spaqr_batch_cgls(h, b_dev, x_dev, count, tol=1e-10, max_iter=200):
    lib = load()
    infos = (CglsInfo * count)()
    rc = lib.spaqr_batch_cgls(h, _ptr(_dev_f64(b_dev)), float(tol), int(max_iter), _ptr(_dev_f64(x_dev)),
                              ctypes.cast(infos, ctypes.c_void_p))
    _check(lib, h, rc, allow=(OK, NOCONV))
    return [dict(iters=i.iters, converged=bool(i.converged), residual=i.residual,
                 paper_residual=i.paper_residual, norm_a=i.norm_a, seconds=i.seconds) for i in infos]


def spaqr_factor_stats(h):
    lib = load()
    s = Stats()
    _check(lib, h, lib.spaqr_factor_stats(h, ctypes.byref(s)))
    return dict(levels=s.levels, num_ops=s.num_ops, num_ranks=s.num_ranks, top_cols=s.top_cols,
                top_rows=s.top_rows, launches=s.launches, syncs=s.syncs, mem_factor=s.mem_factor,
                device_bytes=s.device_bytes, flops=dict(zip(PHASES, s.flops)),
                bytes=dict(zip(PHASES, s.bytes)), phase_seconds=dict(zip(PHASES, s.phase_seconds)),
                factor_seconds=s.factor_seconds, sync_wait_seconds=s.sync_wait_seconds,
                kernel_span_calls=s.kernel_span_calls, kernel_span_seconds=s.kernel_span_seconds,
                kernel_calls=s.kernel_calls,
                kernel_seconds=s.kernel_seconds, kernel_bytes=s.kernel_bytes, kernel_flops=s.kernel_flops,
                levels_sparsified={m: dict(interfaces=s.level_interfaces[m], aspect=s.level_aspect[m],
                                           cols=s.level_cols[m], rank1=s.level_rank1[m], rank2=s.level_rank2[m])
                                   for m in range(1, min(MAX_LEVELS, s.levels + 1)) if s.level_interfaces[m]})


def spaqr_get_ranks(h):
    lib = load()
    n = ctypes.c_int32()
    _check(lib, h, lib.spaqr_get_ranks(h, None, 0, ctypes.byref(n)))
    out = np.zeros(max(1, n.value), dtype=np.int32)
    _check(lib, h, lib.spaqr_get_ranks(h, _ptr(out), n.value, ctypes.byref(n)))
    return out[:n.value].tolist()


def spaqr_get_op(h, i):
    lib = load()
    d = OpDesc()
    _check(lib, h, lib.spaqr_get_op(h, int(i), ctypes.byref(d), None, None, None, None))
    kind, n1, n2 = d.kind, d.n1, d.n2
    cols = n1 + n2 if kind == 0 else (n1 if kind == 1 else n2)
    mat = np.zeros((n1, cols))
    s1 = np.zeros(n1, dtype=np.int32)
    s2 = np.zeros(max(1, n2 if kind == 0 else 0), dtype=np.int32)
    tau = np.zeros(max(1, n2 if kind == 2 else 0))
    _check(lib, h, lib.spaqr_get_op(h, int(i), ctypes.byref(d), _ptr(mat), _ptr(s1), _ptr(s2), _ptr(tau)))
    out = dict(kind=("elim", "scale", "sparsify")[kind], level=d.level, round=d.round, mat=mat, slots=s1)
    if kind == 0:
        out["nslots"] = s2[:n2]
    if kind == 2:
        out["tau"] = tau[:n2]
    return out


def spaqr_time_kernel(h, family, every=1):
    lib = load()
    _check(lib, h, lib.spaqr_time_kernel(h, family.encode() if family else None, int(every)))


def _tune_dict(t):
    return dict(pqr_poll=t.pqr_poll, pqr_reg_rows=t.pqr_reg_rows, tall_coop=t.tall_coop,
                from_cache=bool(t.from_cache), evaluations=t.evaluations, seconds_default=t.seconds_default,
                seconds_best=t.seconds_best)


def spaqr_autotune(h, eps, reps=2, cache_path=None):
    lib = load()
    t = Tune()
    _check(lib, h, lib.spaqr_autotune(h, float(eps), int(reps), cache_path.encode() if cache_path else None,
                                      ctypes.byref(t)))
    return _tune_dict(t)


def spaqr_set_tune(h, pqr_poll=16, pqr_reg_rows=1024, tall_coop=1):
    lib = load()
    t = Tune(int(pqr_poll), int(pqr_reg_rows), int(tall_coop), 0, 0, 0, 0.0, 0.0)
    _check(lib, h, lib.spaqr_set_tune(h, ctypes.byref(t)))


def spaqr_get_tune(h):
    lib = load()
    t = Tune()
    _check(lib, h, lib.spaqr_get_tune(h, ctypes.byref(t)))
    return _tune_dict(t)


def spaqr_destroy(h):
    lib = load()
    return lib.spaqr_destroy(h)


# ---- convenience wrapper ------------------------------------------------------

class Solver:
    """One least-squares problem: analysis, factor and solves on one GPU."""

    def __init__(self, row_ptr, col_idx, vals, M, N, grid, depth=0, skip=-1, sep_width=0,
                 precision="fp64", device=0):
        self.M, self.N = int(M), int(N)
        self.nnz = int(len(col_idx))
        self.version = 0  # bumped whenever the values or the factor change
        prec = {"fp64": FP64, "fp32": FP32_FACTOR}[precision]
        self.h = spaqr_analyze(row_ptr, col_idx, vals, M, N, grid, depth, skip, sep_width, prec, device)

    @classmethod
    def from_problem(cls, prob, depth=0, skip=-1, precision="fp64"):
        return cls(prob.row_ptr, prob.col_idx, prob.vals, prob.M, prob.N, prob.grid, depth, skip,
                   precision=precision)

    def ordering(self):
        return spaqr_get_ordering(self.h, self.M, self.N)

    def factorize(self, eps, ranks=None):
        self.version += 1
        if ranks is None:
            spaqr_factorize(self.h, eps)
        else:
            spaqr_factorize_forced(self.h, eps, ranks)

    def set_values(self, vals_dev):
        self.version += 1
        spaqr_set_values(self.h, vals_dev)

    def cgls(self, b_dev, tol=1e-10, max_iter=200):
        import torch
        x = torch.empty(self.N, dtype=torch.float64, device=b_dev.device)
        info = spaqr_cgls(self.h, b_dev, x, tol, max_iter)
        return x, info

    def csne(self, b_dev, tol=1e-10, max_steps=50):
        """Corrected seminormal equations with iterative refinement."""
        import torch
        x = torch.empty(self.N, dtype=torch.float64, device=b_dev.device)
        info = spaqr_csne(self.h, b_dev, x, tol, max_steps)
        return x, info

    def adjoint(self, x_dev, b_dev, g_dev, tol=1e-12, max_iter=500):
        """(grad_b, grad_vals, lambda, info) of the least-squares solution x."""
        import torch
        dev = g_dev.device
        gb = torch.empty(self.M, dtype=torch.float64, device=dev)
        gv = torch.empty(self.nnz, dtype=torch.float64, device=dev)
        lam = torch.empty(self.N, dtype=torch.float64, device=dev)
        info = spaqr_adjoint(self.h, x_dev, b_dev, g_dev, gb, gv, lam, tol, max_iter)
        return gb, gv, lam, info

    def apply(self, b_dev):
        import torch
        x = torch.empty(self.N, dtype=torch.float64, device=b_dev.device)
        spaqr_apply(self.h, b_dev, x)
        return x

    def apply_noalloc(self, b_dev, x_dev):
        """spaqr_apply into a caller-provided x_dev, with no device allocation."""
        spaqr_apply_noalloc(self.h, b_dev, x_dev)
        return x_dev

    def apply_op(self, op, v_dev):
        import torch
        out = torch.empty_like(v_dev)
        spaqr_apply_op(self.h, op, v_dev, out)
        return out

    def autotune(self, eps, reps=2, cache_path=None):
        """Tune the launch shapes for this problem (leaves it factorized)."""
        self.version += 1
        return spaqr_autotune(self.h, eps, reps, cache_path)

    def set_tune(self, **kw):
        """Change some launch shapes (pqr_poll, pqr_reg_rows, tall_coop); the rest stay."""
        cur = spaqr_get_tune(self.h)
        spaqr_set_tune(self.h, **{k: kw.get(k, cur[k]) for k in ("pqr_poll", "pqr_reg_rows", "tall_coop")})

    def get_tune(self):
        return spaqr_get_tune(self.h)

    def stats(self):
        return spaqr_factor_stats(self.h)

    def ranks(self):
        return spaqr_get_ranks(self.h)

    def op(self, i):
        return spaqr_get_op(self.h, i)

    def time_kernel(self, family, every=1):
        spaqr_time_kernel(self.h, family, every)

    def close(self):
        if self.h:
            spaqr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver(Solver):
    """Independent problems factorized together (one launch per round for
    all of them) and solved by per-problem CGLS.  Batch vectors hold the
    members back to back (offsets ``col_off`` / ``row_off``)."""

    def __init__(self, problems, depths, skip=-1, sep_width=0, precision="fp64", device=0):
        prec = {"fp64": FP64, "fp32": FP32_FACTOR}[precision]
        self.h = spaqr_batch_analyze(problems, depths, skip, sep_width, prec, device)
        self.col_off, self.row_off = spaqr_batch_info(self.h)
        self.count = len(self.col_off) - 1
        self.M, self.N = int(self.row_off[-1]), int(self.col_off[-1])
        self.nnz = int(sum(len(p[1]) for p in problems))
        self.version = 0

    @classmethod
    def from_problems(cls, probs, depths, skip=-1, precision="fp64"):
        return cls([(p.row_ptr, p.col_idx, p.vals, p.M, p.N, p.grid) for p in probs], depths, skip,
                   precision=precision)

    def cgls_each(self, b_dev, tol=1e-10, max_iter=200):
        """x (batch order) and one info dict per member."""
        import torch
        x = torch.empty(self.N, dtype=torch.float64, device=b_dev.device)
        infos = spaqr_batch_cgls(self.h, b_dev, x, self.count, tol, max_iter)
        return x, infos

    def adjoint(self, *a, **k):
        raise SpaqrError(EARG, "the adjoint solve takes a single-problem Solver")
