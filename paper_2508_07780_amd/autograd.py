"""torch.autograd.Function over the hybrid solver.

forward(eps, sigma) -> traces runs dd_forward with checkpoint saving; backward
takes dJ/dtraces, runs dd_adjoint (checkpointed recompute + adjoint sweep with
FP64 gradient accumulation, eq. adjoint_prob and eq. gradeps of the paper) and
dd_gradient, and returns dJ/deps, dJ/dsigma on the FEM nodes.
"""

import torch


class DDSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, sigma, problem, sources):
        problem.set_coefficients(eps.detach(), sigma.detach())
        traces = problem.forward(sources, save=True)
        ctx.problem = problem
        ctx.dtypes = (eps.dtype, sigma.dtype)
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        p = ctx.problem
        p.adjoint(grad_traces)
        ge, gs = p.gradient()
        return ge.to(ctx.dtypes[0]), gs.to(ctx.dtypes[1]), None, None


def solve(problem, eps, sigma, sources):
    """Traces [n_src, n_steps, n_det, 3] as a differentiable function of eps and sigma."""
    return DDSolve.apply(eps, sigma, problem, sources)
