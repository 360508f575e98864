"""prot: push-relabel additive epsilon-approximation of the assignment problem
(Lahn, Raghvendra, Zhang, arXiv:2203.03732) on one AMD MI355X.

Python front end of libprot.so (include/prot.h). Typical use:

    import torch, paper_2203_03732_amd as prot
    res = prot.solve_points(X, Y, eps=0.01)     # X, Y: (n, d) float32 on cuda
    res.mate_b        # column matched to each row
    res.y_a, res.y_b  # dual weights in units of eps (before the completion)
    res.stats         # phases, rounds, scanned entries, cost, timings

    prot.solve_points(X, Y, 0.01)               # X: (n_b, d), Y: (n_a, d), n_b <= n_a
                                                # is the unbalanced case (Section 3.3)
    ot = prot.ot_solve(C, nu, mu, eps=0.1)      # transport plan (Section 4)
    ctx = prot.context(); ctx.set_cost_metric("euclidean")  # Section 5's costs
    plan = ctx.batch(ns, d, eps); plan.run(X, Y)             # many instances at once

The library is loaded lazily, so importing this package on a machine without a
GPU works; any solver call then needs the built library and a GPU.
"""
from __future__ import annotations

from ._lib import (Context, OTResult, ProtError, Result, context, load, pitch,  # noqa: F401
                   threshold, EXPORTS)


def solve_cost(C, eps, **kw) -> Result:
    """Cost matrix C (n_b x n_a float32, scaled to [0, 1], n_b <= n_a) ->
    approximate minimum-cost matching of every row (additive error 3 eps n_b;
    eps n_b with eps_mode='strict')."""
    return context().solve_cost(C, eps, **kw)


def solve_points(X, Y, eps, **kw) -> Result:
    """Point sets X (rows, supply, n_b x d) and Y (columns, demand, n_a x d,
    n_b <= n_a) float32, with the context's cost (squared Euclidean by
    default) scaled to max 1."""
    return context().solve_points(X, Y, eps, **kw)


def ot_solve(C, nu, mu, eps, **kw) -> OTResult:
    """Approximate optimal transport plan (Section 4) from supplies nu (rows
    of C) to demands mu (columns); C float32 in [0, 1], nu and mu float64
    probability vectors, all on the device."""
    return context().ot_solve(C, nu, mu, eps, **kw)


def solve_rounded(k, T, n=None, **kw) -> Result:
    """The phase loop alone on an int16 rounded-cost matrix (n x ldk)."""
    return context().solve_rounded(k, T, n, **kw)


def round_costs(C, eps, k=None):
    return context().round_costs(C, eps, k)


def build_costs(X, Y, eps, k=None):
    return context().build_costs(X, Y, eps, k)


def ot_match_loss(X, Y, eps, eps_mode="algorithmic"):
    """Differentiable per-instance loss (1/n) sum ||x_b - y_mate(b)||^2 for
    X, Y of shape (batch, n, d); see paper_2203_03732_amd.autograd."""
    from .autograd import ot_match_loss as f
    return f(X, Y, eps, eps_mode)
