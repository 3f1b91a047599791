"""FP64 reference FISTA solve of the fused-lasso hologram inversion.

TEST INFRASTRUCTURE ONLY.  This is the oracle that the GPU library is checked
against; the product path never imports, calls or links it.

Paper, section "Methodology": the object is the minimiser of Eq. (2),
f(x) + g(x), with f the data misfit (taken here as 1/2 ||A x - b||^2) and g the
fused lasso of Eq. (5); it is found with FISTA, whose shrinkage step (Eq. 7)
applies the proximal operator of Eq. (6) to a gradient step, followed by an
accelerated update built from the previous estimate.  The step is constant,
t = 1 / ||A||^2, with ||A||^2 from the closed form in `optics.lipschitz`; the
gradient is taken at the extrapolated point y_k (standard FISTA):

    x_k     = prox_{t g}( y_k - t A^T (A y_k - b) )
    s_{k+1} = (1 + sqrt(1 + 4 s_k^2)) / 2
    y_{k+1} = x_k + ((s_k - 1) / s_{k+1}) (x_k - x_{k-1})

from x_0 (zero unless given), y_1 = x_0, s_1 = 1.  Optional function-value
restart (reset s to 1 and y to x_k whenever F increases) computes a reference
objective value and is also a solve mode of its own.

Variants of the prox inside (flags, see `prox`): tv_dims=2, the paper's
per-plane 2D TV; dual_warm=True, every prox starts its TV dual from the dual
the previous outer iteration ended with (p = 0 for the first); fgp=True, the
accelerated dual iteration.
"""
from __future__ import annotations

import math

import numpy as np

from . import optics, prox

__all__ = ["objective", "fista", "objective_terms"]


def objective_terms(geom, x, b, l1, tv, tv_dims=3):
    """(1/2||Ax-b||^2, sum|x|, TV(x)) in FP64."""
    r = optics.forward(geom, x) - b
    return 0.5 * float((r * r).sum()), float(np.abs(x).sum()), prox.tv(x, tv_dims)


def objective(geom, x, b, l1, tv, tv_dims=3) -> float:
    """F(x) = 1/2||A x - b||^2 + l1 ||x||_1 + tv TV(x)."""
    d, s, t = objective_terms(geom, x, b, l1, tv, tv_dims)
    return d + l1 * s + tv * t


def fista(geom, b, l1, tv, n_outer, n_inner, x0=None, step=None, nonneg=True,
          restart=False, history=False, tv_dims=3, dual_warm=False, fgp=False, dual_store=None,
          dual_store_every=1, on_iterate=None):
    b = np.asarray(b, dtype=np.float64)
    t = 1.0 / optics.lipschitz(geom) if step is None else float(step)
    x = np.zeros((geom.nz, geom.ny, geom.nx)) if x0 is None else np.array(x0, dtype=np.float64)
    y = x.copy()
    s = 1.0
    p = None
    f_hist = []
    f_prev = objective(geom, x, b, l1, tv, tv_dims) if restart else None
    for _ in range(n_outer):
        g = optics.adjoint(geom, optics.forward(geom, y) - b)
        x_new, p_new = prox.prox_fused_lasso(y - t * g, t, l1, tv, n_inner, nonneg, dims=tv_dims,
                                             p0=p if dual_warm else None, return_dual=True, fast=fgp,
                                             store=dual_store, store_every=dual_store_every)
        if dual_warm:
            # the dual carried to the next outer iteration is stored (rounded, if a store is given)
            p = p_new if dual_store is None else tuple(dual_store(a) for a in p_new)
        s_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * s * s))
        beta = (s - 1.0) / s_new
        if restart or history:
            f = objective(geom, x_new, b, l1, tv, tv_dims)
            f_hist.append(f)
            if restart and f > f_prev:
                s_new, beta = 1.0, 0.0
            f_prev = f
        y = x_new + beta * (x_new - x)
        x, s = x_new, s_new
        if on_iterate is not None:
            on_iterate(x)   # observer of each new iterate (tests); changes nothing
    return (x, f_hist) if history else x
