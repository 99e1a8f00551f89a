"""torch.autograd.Function over the hybrid solver.

forward(eps, sigma) -> traces runs dd_forward with checkpoint saving; backward
takes dJ/dtraces, runs dd_adjoint (checkpointed recompute + adjoint sweep with
FP64 gradient accumulation, eq. adjoint_prob and eq. gradeps of the paper) and
dd_gradient, and returns dJ/deps, dJ/dsigma on the FEM nodes, in the shapes and
dtypes of eps and sigma.

The adjoint reads the forward state the Problem saved.  A Problem keeps one saved
forward, so a node's backward raises if the Problem has run another solve (or changed
its coefficients, div-div form or initial data) since that node's forward: use one
Problem per solve that is differentiated later.
"""

import torch


class DDSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, sigma, problem, sources):
        problem.set_coefficients(eps.detach(), sigma.detach())
        traces = problem.forward(sources, save=True)
        ctx.problem = problem
        ctx.generation = problem.generation
        ctx.meta = ((eps.shape, eps.dtype), (sigma.shape, sigma.dtype))
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        p = ctx.problem
        if p.generation != ctx.generation:
            raise RuntimeError("the Problem ran another solve (or changed its state) after this forward: its saved "
                               "forward no longer belongs to this graph; use one Problem per differentiated solve")
        p.adjoint(grad_traces)
        ge, gs = p.gradient()
        (se, de), (ss, ds) = ctx.meta
        return ge.to(de).reshape(se), gs.to(ds).reshape(ss), None, None


def solve(problem, eps, sigma, sources):
    """Traces [n_src, n_steps, n_det, 3] as a differentiable function of eps and sigma."""
    return DDSolve.apply(eps, sigma, problem, sources)
