"""Learned warm start for the FISTA solve.

A 3D U-Net (ri_unet_*, BF16 matrix-core kernels) maps the back-propagated
hologram A^T b, scaled to unit RMS over the training set, to a proposed
starting volume x_0 >= 0.
Training pairs come from the library's own solver: for each seeded scene the
hologram b and the volume the plain solver reaches from a cold start.

At solve time the proposal x_1 is rescaled to the best multiple s x_1 of
itself: F(s x) is a convex quadratic in s >= 0 (the l1 and TV terms are
positively homogeneous), so F(0), F(x_1) and F(2 x_1) -- three zero-iteration
solves, the last two scaling x_1 inside the solve (x0_scale) -- give
s* = argmin F(s x_1) and F(s* x_1) = F(0) - c^2 / (2a) < F(0) whenever the
proposal helps at all (c > 0); otherwise the solve starts cold.  The FISTA
objective always decides the result.

Normalisation: the network sees A^T b * in_scale (in_scale = 1 / RMS of the
training inputs) and is trained against targets * t_scale (t_scale = 1 / the
largest target value), so that activations and outputs are O(1) in bfloat16;
after training 1/t_scale is folded into the head's weights and bias (the head
is linear before its ReLU), so a proposal is one ri_unet_forward call.

torch supplies device memory, the RNG for crop positions, tensor slicing for
crops and the two normalisation constants of the training data; every
computation on the solve path (A^T, the network, the solve) runs in librihvr.
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
    plan: "object" = None  # geometry of the pair (None: the WarmStart's plan)


class WarmStart:
    def __init__(self, plan: rihvr.Plan, levels: int = 4, base: int = 16, seed: int = 0):
        import torch
        self.torch = torch
        self.plan = plan
        self.net = rihvr.UNet(levels, base, seed=seed)
        self.levels = levels
        self.base = base
        self.scale = None       # in_scale, set by the first train()
        self.t_scale = 1.0      # folded into the head after train()
        self._folded = False

    # -- data --------------------------------------------------------------
    def network_input(self, b, plan=None):
        """A^T b (the network multiplies it by in_scale); plan defaults to the
        training plan (the network is fully convolutional: any geometry with the
        same optics works)."""
        return (plan or self.plan).adjoint(b)

    def _head(self):
        n = self.base + 1  # head weights (one per first-level channel) and bias, last in the vector
        return self.net.params[self.net.n - n:]

    def _fold(self, on: bool):
        if on != self._folded and self.t_scale != 1.0:
            self._head().mul_(1.0 / self.t_scale if on else self.t_scale)
        self._folded = on

    def make_pair(self, b, l1, tv, iters, inner, plan=None):
        x, rep, _ = (plan or self.plan).solve(b, l1, tv, iters, inner)
        return Pair(b, x, plan), rep

    # -- training ----------------------------------------------------------
    def train(self, pairs, steps, crop=(32, 64, 64), lr=1e-3, seed=0, log_every=0, pos_weight=None):
        """Adam on random crops of (A^T b, solved x) pairs; returns the loss curve.

        The solved volumes are sparse (a few percent of voxels non-zero), so the
        loss weights those voxels by pos_weight (default: 0.5 / the non-zero
        fraction, within [1, 50]) to keep the all-zero output from being a
        good minimum."""
        torch = self.torch
        g = torch.Generator().manual_seed(seed)
        m = 1 << (self.levels - 1)
        if self.scale is None:
            # normalisation from (at most) 32 pairs; network inputs are formed
            # per step from the pair's hologram (A^T b by the library), so the
            # training set holds holograms and targets only
            sample = pairs[:32]
            ms = sum(float((self.network_input(p.b, p.plan).double() ** 2).mean()) for p in sample) / len(sample)
            self.scale = 1.0 / math.sqrt(max(ms, 1e-300))
            self.t_scale = 1.0 / max(max(float(p.target.max()) for p in pairs), 1e-30)
        if pos_weight is None:
            rho = sum(float((p.target > 0).double().mean()) for p in pairs) / len(pairs)
            pos_weight = min(50.0, max(1.0, 0.5 / max(rho, 1e-6)))
        self.pos_weight = pos_weight
        self._fold(False)
        losses = []
        for it in range(steps):
            k = int(torch.randint(len(pairs), (1,), generator=g))
            inp = self.network_input(pairs[k].b, pairs[k].plan)
            nz, ny, nx = inp.shape
            cz, cy, cx = (min(c, n) // m * m for c, n in zip(crop, (nz, ny, nx)))
            z0 = int(torch.randint(nz - cz + 1, (1,), generator=g))
            y0 = int(torch.randint(ny - cy + 1, (1,), generator=g))
            x0 = int(torch.randint(nx - cx + 1, (1,), generator=g))
            xi = inp[z0:z0 + cz, y0:y0 + cy, x0:x0 + cx].contiguous()
            ti = (pairs[k].target[z0:z0 + cz, y0:y0 + cy, x0:x0 + cx] * self.t_scale).contiguous()
            loss = self.net.train_step(xi, ti, lr=lr, scale=self.scale, pos_weight=pos_weight)
            if log_every and (it % log_every == 0 or it == steps - 1):
                losses.append((it, float(loss)))
        self._fold(True)
        return losses

    # -- use ---------------------------------------------------------------
    def _forward(self, inp):
        """Network output for a whole volume.  Volumes whose sides are not
        multiples of 2^(levels-1) are zero-padded up to them and the output is
        cropped back (a copy, no arithmetic)."""
        torch = self.torch
        m = 1 << (self.levels - 1)
        shape = tuple(inp.shape)
        padded = tuple((n + m - 1) // m * m for n in shape)
        if padded != shape:
            big = torch.zeros(padded, dtype=inp.dtype, device=inp.device)
            big[:shape[0], :shape[1], :shape[2]] = inp
            inp = big
        out = self.net.forward(inp, scale=self.scale)
        if padded != shape:
            out = out[:shape[0], :shape[1], :shape[2]].contiguous()
        return out

    def _objective(self, b, l1, tv, inner, x=None, plan=None, x0_scale=1.0):
        """F(x0_scale * x) (F(0) when x is None) from a zero-iteration solve
        (launched kernel by kernel: a graph would be captured for one use)."""
        p = plan or self.plan
        return p.solve(b, l1, tv, 0, inner, x=None if x is None else x.clone(), x0_scale=x0_scale,
                       flags=rihvr.RI_SOLVE_NO_GRAPH)[1]["objective"]

    def propose(self, b, l1=None, tv=None, inner=None, plan=None):
        """The network's proposal x_1 for hologram b (of `plan`'s geometry,
        default the training plan).  With the solve's weights, also the scale s*
        that minimises F(s x_1).  Returns (x_1, s*, F(0), F(s* x_1)); x_1 is None
        when no positive multiple of it improves on F(0)."""
        if self.scale is None:
            raise RuntimeError("WarmStart.propose before train()")
        self._fold(True)
        x1 = self._forward(self.network_input(b, plan))
        if l1 is None:
            return x1, 1.0, math.nan, math.nan
        f0 = self._objective(b, l1, tv, inner, plan=plan)
        f1 = self._objective(b, l1, tv, inner, x1, plan=plan)
        f2 = self._objective(b, l1, tv, inner, x1, plan=plan, x0_scale=2.0)
        a = f2 - 2.0 * f1 + f0          # ||A x_1||^2
        c = 0.5 * a - (f1 - f0)         # <A x_1, b> - l1 sum(x_1) - tv TV(x_1)
        if not (math.isfinite(a) and math.isfinite(c) and a > 0.0 and c > 0.0):
            return None, 0.0, f0, math.inf
        return x1, c / a, f0, f0 - c * c / (2.0 * a)

    def solve(self, b, l1, tv, max_iters, inner, f_ref=0.0, gap_tol=0.0, check_every=5, flags=0):
        """Warm-started solve with the cold-start fallback.  Returns (x, report, used_warm)."""
        x1, s, f0, fs = self.propose(b, l1, tv, inner)
        warm = x1 is not None and fs < f0
        x, rep, st = self.plan.solve(b, l1, tv, max_iters, inner, x=x1 if warm else None, f_ref=f_ref,
                                     gap_tol=gap_tol, check_every=check_every, flags=flags,
                                     x0_scale=s if warm else 1.0)
        return x, rep, warm
