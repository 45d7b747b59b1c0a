"""GPU parity of the differentiation form: column scaling on the device,
the adjoint solve and the gradients of x*(A, b), through the C-ABI and the
torch.autograd.Function, against the oracle's plain-definition gradients
(sparse direct normal equations, FP64) and finite differences."""
import numpy as np
import pytest

import paper_2102_09878_amd as pk
from oracle import adjoint as oadj
from synth import config_problem, grid_ls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _oracle_grads(p):
    x = oadj.lstsq_solution(p.row_ptr, p.col_idx, p.vals, p.b, p.M, p.N)
    g = x - p.x_t
    gb, gv, lam = oadj.grads_direct(p.row_ptr, p.col_idx, p.vals, p.b, x, g, p.M, p.N)
    return x, g, gb, gv, lam


def _rel(a, b):
    return float(np.abs(a - b).max() / max(1e-300, np.abs(b).max()))


def test_set_values_scale_invariance():
    """A -> 2A leaves the scaled matrix, hence the factor, unchanged: x halves,
    the ranks and the iteration count stay, ||A|| doubles."""
    p = grid_ls((24, 20), 480, 7)
    s = pk.Solver.from_problem(p, 4, 1)
    s.factorize(1e-2)
    b = dev(p.b)
    x1, i1 = s.cgls(b, tol=1e-12)
    r1 = s.ranks()
    s.set_values(dev(2.0 * p.vals))
    s.factorize(1e-2)
    x2, i2 = s.cgls(b, tol=1e-12)
    assert s.ranks() == r1
    assert i2["iters"] == i1["iters"]
    assert abs(i2["norm_a"] - 2 * i1["norm_a"]) <= 1e-12 * i1["norm_a"]
    assert _rel(2 * host(x2), host(x1)) <= 1e-12
    # back to the original values: bit-identical to the first run
    s.set_values(dev(p.vals))
    s.factorize(1e-2)
    x3, _ = s.cgls(b, tol=1e-12)
    assert np.array_equal(host(x3), host(x1))
    s.close()


def test_set_values_rejects_empty_column():
    p = grid_ls((12, 12), 144, 3)
    s = pk.Solver.from_problem(p, 3, 1)
    v = p.vals.copy()
    v[p.col_idx == 5] = 0.0
    with pytest.raises(pk.SpaqrError) as e:
        s.set_values(dev(v))
    assert e.value.code == -1
    s.close()


@pytest.mark.parametrize("grid,depth,skip,eps", [((24, 20), 4, 1, 1e-2), ((17, 23), 4, 1, 1e-1)])
def test_adjoint_matches_oracle_small(grid, depth, skip, eps):
    n = grid[0] * grid[1]
    p = grid_ls(grid, n, 21, with_target=True)
    x, g, gb, gv, lam = _oracle_grads(p)
    s = pk.Solver.from_problem(p, depth, skip)
    s.factorize(eps)
    gb_d, gv_d, lam_d, info = s.adjoint(dev(x), dev(p.b), dev(g), tol=1e-13)
    print(f"adjoint {grid}: iters {info['iters']} residual {info['residual']:.2e}")
    assert info["converged"] and info["residual"] <= 1e-12
    assert _rel(host(lam_d), lam) <= 1e-10
    assert _rel(host(gb_d), gb) <= 1e-10
    assert _rel(host(gv_d), gv) <= 1e-10
    s.close()


def _gpu_loss(s, p, vals, b, eps):
    s.set_values(dev(vals))
    s.factorize(eps)
    x, info = s.cgls(dev(b), tol=1e-13, max_iter=500)
    assert info["converged"]
    x = host(x)
    return 0.5 * float(np.sum((x - p.x_t) ** 2))


def test_adjoint_matches_finite_differences_small():
    p = grid_ls((24, 20), 480, 22, with_target=True)
    eps = 1e-2
    s = pk.Solver.from_problem(p, 4, 1)
    vals = dev(p.vals).requires_grad_(True)
    b = dev(p.b).requires_grad_(True)
    x = pk.lstsq(s, vals, b, eps, tol=1e-13)
    loss = 0.5 * ((x - dev(p.x_t)) ** 2).sum()
    loss.backward()
    gv, gb = host(vals.grad), host(b.grad)
    scale = max(np.abs(gv).max(), np.abs(gb).max())
    rng = np.random.default_rng(5)
    h = 1e-6
    worst = 0.0
    for e in rng.choice(p.nnz, 20, replace=False):
        vp, vm = p.vals.copy(), p.vals.copy()
        vp[e] += h
        vm[e] -= h
        fd = (_gpu_loss(s, p, vp, p.b, eps) - _gpu_loss(s, p, vm, p.b, eps)) / (2 * h)
        worst = max(worst, abs(fd - gv[e]) / scale)
    for i in rng.choice(p.M, 10, replace=False):
        bp, bm = p.b.copy(), p.b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (_gpu_loss(s, p, p.vals, bp, eps) - _gpu_loss(s, p, p.vals, bm, eps)) / (2 * h)
        worst = max(worst, abs(fd - gb[i]) / scale)
    print(f"FD worst {worst:.2e}")
    assert worst <= 1e-5
    s.close()


def test_config5_gradients_fp32_factor():
    """128 x 128 grid, FP32 factor, FP64 CGLS and adjoint: gradients through
    torch.autograd against the oracle's direct FP64 gradients, and a
    directional finite difference of the loss."""
    p = config_problem(5)
    c = p.meta
    s = pk.Solver.from_problem(p, c["depth"], c["skip"], precision="fp32")
    vals = dev(p.vals).requires_grad_(True)
    b = dev(p.b).requires_grad_(True)
    xt = dev(p.x_t)
    x = pk.lstsq(s, vals, b, c["eps"], tol=1e-12)
    loss = 0.5 * ((x - xt) ** 2).sum()
    loss.backward()
    gv, gb = host(vals.grad), host(b.grad)
    xo, g, gbo, gvo, lam = _oracle_grads(p)
    ex, egb, egv = _rel(host(x), xo), _rel(gb, gbo), _rel(gv, gvo)
    print(f"config5: x err {ex:.2e}  grad_b err {egb:.2e}  grad_vals err {egv:.2e}")
    assert ex <= 1e-8 and egb <= 1e-8 and egv <= 1e-8
    # directional derivative along a random perturbation of (vals, b)
    rng = np.random.default_rng(9)
    dv = rng.standard_normal(p.nnz)
    db = rng.standard_normal(p.M)
    h = 1e-6
    lp = _gpu_loss(s, p, p.vals + h * dv, p.b + h * db, c["eps"])
    lm = _gpu_loss(s, p, p.vals - h * dv, p.b - h * db, c["eps"])
    fd = (lp - lm) / (2 * h)
    an = float(gv @ dv + gb @ db)
    print(f"config5 directional: fd {fd:.10e} adjoint {an:.10e}")
    assert abs(fd - an) <= 1e-5 * abs(an)
    s.close()
