"""Learned warm start for the FISTA solve.

A 3D U-Net (ri_unet_*, BF16 matrix-core kernels) maps the back-propagated
hologram A^T b, scaled by 1/||A||^2, to a proposed starting volume x_0 >= 0.
Training pairs come from the library's own solver: for each seeded scene the
hologram b and the volume the plain solver reaches from a cold start.  At solve
time the proposal is kept only if its objective is below F(0) (else the solve
starts cold), so the FISTA objective always decides the result.

torch supplies device memory, the RNG for crop positions and tensor slicing
for crops; every computation (A^T, the network, the solve) runs in librihvr.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import rihvr


@dataclass
class Pair:
    b: "object"          # hologram [ny][nx] (cuda float32)
    target: "object"     # solved volume [nz][ny][nx] (cuda float32)


class WarmStart:
    def __init__(self, plan: rihvr.Plan, levels: int = 4, base: int = 16, seed: int = 0):
        import torch
        self.torch = torch
        self.plan = plan
        self.net = rihvr.UNet(levels, base, seed=seed)
        self.levels = levels
        self.scale = 1.0 / plan.lipschitz

    # -- data --------------------------------------------------------------
    def network_input(self, b):
        """A^T b / ||A||^2 (the input the network sees, before its own scale)."""
        return self.plan.adjoint(b)

    def make_pair(self, b, l1, tv, iters, inner):
        x, rep, _ = self.plan.solve(b, l1, tv, iters, inner)
        return Pair(b, x), rep

    # -- training ----------------------------------------------------------
    def train(self, pairs, steps, crop=(32, 64, 64), lr=1e-3, seed=0, log_every=0):
        """Adam on random crops of (A^T b / ||A||^2, solved x) pairs; returns the loss curve."""
        torch = self.torch
        g = torch.Generator().manual_seed(seed)
        nz, ny, nx = self.plan.shape
        cz, cy, cx = (min(c, n) for c, n in zip(crop, (nz, ny, nx)))
        m = 1 << (self.levels - 1)
        cz, cy, cx = cz // m * m, cy // m * m, cx // m * m
        inputs = [self.network_input(p.b) for p in pairs]
        losses = []
        for it in range(steps):
            k = int(torch.randint(len(pairs), (1,), generator=g))
            z0 = int(torch.randint(nz - cz + 1, (1,), generator=g))
            y0 = int(torch.randint(ny - cy + 1, (1,), generator=g))
            x0 = int(torch.randint(nx - cx + 1, (1,), generator=g))
            xi = inputs[k][z0:z0 + cz, y0:y0 + cy, x0:x0 + cx].contiguous()
            ti = pairs[k].target[z0:z0 + cz, y0:y0 + cy, x0:x0 + cx].contiguous()
            loss = self.net.train_step(xi, ti, lr=lr, scale=self.scale)
            if log_every and (it % log_every == 0 or it == steps - 1):
                losses.append((it, float(loss)))
        return losses

    # -- use ---------------------------------------------------------------
    def propose(self, b):
        return self.net.forward(self.network_input(b), scale=self.scale)

    def solve(self, b, l1, tv, max_iters, inner, f_ref=0.0, gap_tol=0.0, check_every=5, flags=0):
        """Warm-started solve with the cold-start fallback.  Returns (x, report, used_warm)."""
        x0 = self.propose(b)
        _, r0, _ = self.plan.solve(b, l1, tv, 0, inner, x=x0.clone())
        f_zero = 0.5 * float((b.double() ** 2).sum())
        warm = r0["objective"] < f_zero and math.isfinite(r0["objective"])
        x, rep, st = self.plan.solve(b, l1, tv, max_iters, inner, x=x0 if warm else None, f_ref=f_ref,
                                     gap_tol=gap_tol, check_every=check_every, flags=flags)
        return x, rep, warm
