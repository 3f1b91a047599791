"""FP64 reference of the fused-lasso proximal operator.

TEST INFRASTRUCTURE ONLY.  This is the oracle that the GPU library is checked
against; the product path never imports, calls or links it.

Paper, section "Methodology":
  * Eq. (3)  l1 regulariser  sum_i |x_i|.
  * Eq. (4)  isotropic TV, extended here to three dimensions (the paper notes the
    norm extends to higher dimensions): sum over voxels of the Euclidean norm of
    the forward differences along x, y and z.  The last difference along each
    axis is zero (Neumann boundary); all axes carry unit weight.
  * Eq. (5)  fused lasso  l1 * ||x||_1 + tv * TV(x).
  * Eq. (6)  prox_t(v) = argmin_x g(x) + 1/(2t) ||x - v||^2.
  * TV prox by the gradient-projection (GP) method of Beck & Teboulle on the dual
    of the TV denoising problem, which stores one dual value per direction and
    voxel.
  * Fused-lasso prox = soft threshold of the TV prox (the separability the paper
    states); Eq. (8) is read as the soft threshold sign(u) (|u| - t l1)_+, which
    becomes max(u - t l1, 0) under the non-negativity constraint.

Variants (each a flag; the defaults are the method above):
  * dims=2: the paper's own regulariser, Eq. (4) applied to every plane on its
    own (differences along x and y only, no coupling between planes).  ||D||^2
    <= 8 in 2D, so the GP step is 1/(8 tau).
  * p0: the dual to start from (a warm start carried over from the previous
    outer iteration) instead of p = 0.
  * fast=True: FGP, the accelerated gradient projection of Beck & Teboulle:
    the projected step is taken at an extrapolated dual r, with the momentum
    sequence of FISTA (t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
    r = p_k + ((t_k - 1)/t_{k+1}) (p_k - p_{k-1})).
  * store: a rounding applied to the dual after every `store_every`-th step
    but the last (a model of a dual stored in a narrower type between passes
    over memory, the last pass keeping it on chip).
"""
from __future__ import annotations

import numpy as np

__all__ = ["grad3", "grad3_adjoint", "tv3", "tv", "prox_tv_gp", "soft_threshold",
           "prox_fused_lasso", "dual_objective"]


def grad3(u: np.ndarray):
    """D u: forward differences along x, y, z of a [nz][ny][nx] volume.

    Returns (dx, dy, dz); the last difference along each axis is 0.
    """
    dx = np.zeros_like(u)
    dy = np.zeros_like(u)
    dz = np.zeros_like(u)
    dx[:, :, :-1] = u[:, :, 1:] - u[:, :, :-1]
    dy[:, :-1, :] = u[:, 1:, :] - u[:, :-1, :]
    dz[:-1, :, :] = u[1:, :, :] - u[:-1, :, :]
    return dx, dy, dz


def grad3_adjoint(px: np.ndarray, py: np.ndarray, pz: np.ndarray) -> np.ndarray:
    """D^T p, the exact transpose of grad3 (so <D u, p> = <u, D^T p>)."""
    out = np.zeros_like(px)
    # d/du of sum_i px[i] (u[i+1] - u[i]) for i < n-1
    out[:, :, :-1] -= px[:, :, :-1]
    out[:, :, 1:] += px[:, :, :-1]
    out[:, :-1, :] -= py[:, :-1, :]
    out[:, 1:, :] += py[:, :-1, :]
    out[:-1, :, :] -= pz[:-1, :, :]
    out[1:, :, :] += pz[:-1, :, :]
    return out


def tv3(u: np.ndarray) -> float:
    """Isotropic 3D total variation, Eq. (4) extended to z."""
    dx, dy, dz = grad3(np.asarray(u, dtype=np.float64))
    return float(np.sqrt(dx * dx + dy * dy + dz * dz).sum())


def tv(u: np.ndarray, dims: int = 3) -> float:
    """Isotropic TV: 3D (dims=3) or the sum over planes of the 2D TV of Eq. (4)
    (dims=2, no z differences)."""
    if dims == 3:
        return tv3(u)
    dx, dy, _ = grad3(np.asarray(u, dtype=np.float64))
    return float(np.sqrt(dx * dx + dy * dy).sum())


def dual_objective(v, tau, px, py, pz) -> float:
    """1/2 ||v - tau D^T p||^2, the dual function that GP decreases."""
    r = v - tau * grad3_adjoint(px, py, pz)
    return 0.5 * float((r * r).sum())


def prox_tv_gp(v: np.ndarray, tau: float, n_iter: int, return_dual: bool = False, dims: int = 3,
               p0=None, fast: bool = False, store=None, store_every: int = 1):
    """argmin_u 1/2||u - v||^2 + tau TV(u), by n_iter gradient-projection steps.

    Dual: min over |p_voxel| <= 1 of 1/2 ||v - tau D^T p||^2, with u = v - tau D^T p.
    The gradient of the dual in p is -tau D u and its Lipschitz constant is
    tau^2 ||D||^2 <= 4 dims tau^2, so each step is
        u = v - tau D^T p
        q = p + D u / (4 dims tau)
        p = q / max(1, |q|)          (projection on the unit ball per voxel)
    starting from p = 0 (or p0).  The primal is recovered once more at the end.
    With dims=2 the z component of the dual stays zero.  fast=True takes each
    step at the FGP extrapolation r instead of p.  store (optional) rounds what
    a step hands on -- the dual, and with fast=True the extrapolated point --
    after every store_every-th step except the last.
    """
    v = np.asarray(v, dtype=np.float64)
    if p0 is None:
        px, py, pz = np.zeros_like(v), np.zeros_like(v), np.zeros_like(v)
    else:
        px, py, pz = (np.array(a, dtype=np.float64) for a in p0)
    if dims == 2:
        pz = np.zeros_like(v)
    if tau == 0.0:
        return (v.copy(), (px, py, pz)) if return_dual else v.copy()
    c = 1.0 / (4.0 * dims * tau)
    rx, ry, rz = px, py, pz          # point the step is taken at (FGP: extrapolated)
    t = 1.0
    for k in range(n_iter):
        u = v - tau * grad3_adjoint(rx, ry, rz)
        gx, gy, gz = grad3(u)
        if dims == 2:
            gz = np.zeros_like(v)
        qx = rx + c * gx
        qy = ry + c * gy
        qz = rz + c * gz
        scale = np.maximum(1.0, np.sqrt(qx * qx + qy * qy + qz * qz))
        nx_, ny_, nz_ = qx / scale, qy / scale, qz / scale
        rounded = store is not None and (k + 1) % store_every == 0 and k + 1 < n_iter
        if fast:
            t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
            w = (t - 1.0) / t_new
            rx, ry, rz = nx_ + w * (nx_ - px), ny_ + w * (ny_ - py), nz_ + w * (nz_ - pz)
            t = t_new
            if rounded:
                rx, ry, rz = store(rx), store(ry), store(rz)
        if rounded:
            nx_, ny_, nz_ = store(nx_), store(ny_), store(nz_)
        if not fast:
            rx, ry, rz = nx_, ny_, nz_
        px, py, pz = nx_, ny_, nz_
    u = v - tau * grad3_adjoint(px, py, pz)
    return (u, (px, py, pz)) if return_dual else u


def soft_threshold(u: np.ndarray, thr: float, nonneg: bool = True) -> np.ndarray:
    """prox of thr*|.|_1 (Eq. 8 as read), optionally restricted to x >= 0."""
    if nonneg:
        return np.maximum(u - thr, 0.0)
    return np.sign(u) * np.maximum(np.abs(u) - thr, 0.0)


def prox_fused_lasso(v: np.ndarray, step: float, l1: float, tv: float, n_iter: int,
                     nonneg: bool = True, dims: int = 3, p0=None, return_dual: bool = False,
                     fast: bool = False, store=None, store_every: int = 1):
    """prox of step * (l1 ||x||_1 + tv TV(x)) [+ x >= 0]: TV prox, then soft threshold."""
    u, p = prox_tv_gp(v, step * tv, n_iter, return_dual=True, dims=dims, p0=p0, fast=fast, store=store,
                      store_every=store_every)
    x = soft_threshold(u, step * l1, nonneg)
    return (x, p) if return_dual else x
