"""torch.autograd.Function of the least-squares solution x*(A, b).

Forward: the nonzero values of A go to the device factorization
(spaqr_set_values, spaqr_factorize) and x = argmin ||A x - b|| comes from
spaQR-preconditioned CGLS.  Backward: spaqr_adjoint solves A^T A lambda = g
with the same factor as preconditioner and returns
    dL/db = A lambda,   dL/dA_ij = r_i lambda_j - (A lambda)_i x_j,  r = b - A x,
for the stored nonzeros.  Every numeric step runs in the library's kernels;
this module only routes tensors.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable


class LstsqFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, solver, eps, tol, max_iter):
        vals_c = vals.detach().contiguous()
        b_c = b.detach().contiguous()
        solver.set_values(vals_c)
        solver.factorize(eps)
        x, info = solver.cgls(b_c, tol, max_iter)
        if not info["converged"]:
            raise RuntimeError(f"CGLS did not reach {tol} in {max_iter} iterations: {info}")
        ctx.solver, ctx.eps, ctx.tol, ctx.max_iter = solver, eps, tol, max_iter
        ctx.version = solver.version
        ctx.save_for_backward(vals_c, b_c, x)
        return x

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        vals, b, x = ctx.saved_tensors
        s = ctx.solver
        if s.version != ctx.version:  # the solver was used for other values meanwhile
            s.set_values(vals)
            s.factorize(ctx.eps)
        gb, gv, _, info = s.adjoint(x, b, g.detach().contiguous(), ctx.tol, ctx.max_iter)
        if not info["converged"]:
            raise RuntimeError(f"adjoint solve did not reach {ctx.tol}: {info}")
        return (gv if ctx.needs_input_grad[0] else None, gb if ctx.needs_input_grad[1] else None,
                None, None, None, None)


def lstsq(solver, vals, b, eps, tol=1e-12, max_iter=500):
    """x*(A, b) for A with the solver's sparsity pattern and values `vals`
    (CSR order, FP64 on the GPU); differentiable in vals and b."""
    return LstsqFunction.apply(vals, b, solver, eps, tol, max_iter)
