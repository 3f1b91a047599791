"""FP64 reference for a complex-valued object (absorption and phase).

TEST INFRASTRUCTURE ONLY.  This is the oracle that the GPU library's complex
plans are checked against; the product path never imports, calls or links it.

Paper, section "Methodology": the reconstructed volume is held as complex
floating-point values (the paragraph on memory and the sparse storage), and the
soft threshold of Eq. (8) is written with |v| and sign(v).  For a complex value
sign(v) |v| = v, so the threshold is the shrinkage of the modulus with the
phase kept: (1 - t l1 / |v|)_+ v.  Readings used here:
  * the object x is complex [nz][ny][nx]; the hologram model of Eq. (2) keeps
    the form A x = Re( sum_j IFFT2( FFT2(x_j) H_j ) ), which is linear over the
    reals in (Re x, Im x);
  * the adjoint under the real inner product Re<x, y> is complex:
    (A^T r)_j = IFFT2( FFT2(r) conj(H_j) )  (no real part taken);
  * Eq. (3) sums moduli, ||x||_1 = sum_i |x_i|; Eq. (4) takes the modulus of
    the complex differences, TV(x) = sum_voxels sqrt( sum_d |D_d x|^2 )
    (3D, or the per-plane 2D form with dims=2);
  * no sign constraint (x >= 0 has no meaning for a complex field);
  * the TV prox is gradient projection on the dual with one complex dual value
    per direction; real and imaginary parts are projected together on the
    unit ball of C^dims, which is the projection the complex TV's dual needs.
The functions are the definitions written out, one plane at a time.
"""
from __future__ import annotations

import math

import numpy as np

from . import optics

__all__ = ["forward", "adjoint", "lipschitz", "grad", "grad_adjoint", "tv", "shrink",
           "prox_tv_gp", "prox_fused_lasso", "objective", "fista"]


def forward(geom, x: np.ndarray) -> np.ndarray:
    """A x for a complex volume x [nz][ny][nx] -> real hologram [ny][nx]."""
    x = np.asarray(x, dtype=np.complex128)
    assert x.shape == (geom.nz, geom.ny, geom.nx)
    acc = np.zeros((geom.ny, geom.nx), dtype=np.complex128)
    for j, z in enumerate(optics.plane_z(geom)):
        acc += np.fft.ifft2(np.fft.fft2(x[j]) * optics.transfer_function(geom, z))
    return acc.real


def adjoint(geom, y: np.ndarray) -> np.ndarray:
    """A^T y for the real inner product: complex [nz][ny][nx]."""
    y = np.asarray(y, dtype=np.float64)
    assert y.shape == (geom.ny, geom.nx)
    Y = np.fft.fft2(y)
    out = np.empty((geom.nz, geom.ny, geom.nx), dtype=np.complex128)
    for j, z in enumerate(optics.plane_z(geom)):
        out[j] = np.fft.ifft2(Y * np.conj(optics.transfer_function(geom, z)))
    return out


def lipschitz(geom) -> float:
    """||A||^2 = max_f sum_j |H_j(f)|^2: A A^T multiplies the spectrum by
    sum_j (Re H_j)^2 + (Im H_j)^2 (the real part from Re x, the imaginary part
    from Im x), which is nz wherever every frequency propagates."""
    acc = np.zeros((geom.ny, geom.nx), dtype=np.float64)
    for z in optics.plane_z(geom):
        acc += np.abs(optics.transfer_function(geom, z)) ** 2
    return float(acc.max())


def grad(u: np.ndarray, dims: int = 3):
    """Complex forward differences (dx, dy, dz); the last along each axis is 0;
    dz is 0 everywhere for dims=2."""
    dx = np.zeros_like(u)
    dy = np.zeros_like(u)
    dz = np.zeros_like(u)
    dx[:, :, :-1] = u[:, :, 1:] - u[:, :, :-1]
    dy[:, :-1, :] = u[:, 1:, :] - u[:, :-1, :]
    if dims == 3:
        dz[:-1, :, :] = u[1:, :, :] - u[:-1, :, :]
    return dx, dy, dz


def grad_adjoint(px, py, pz) -> np.ndarray:
    """D^T p for complex p, the transpose of grad under Re<.,.>."""
    out = np.zeros_like(px)
    out[:, :, :-1] -= px[:, :, :-1]
    out[:, :, 1:] += px[:, :, :-1]
    out[:, :-1, :] -= py[:, :-1, :]
    out[:, 1:, :] += py[:, :-1, :]
    out[:-1, :, :] -= pz[:-1, :, :]
    out[1:, :, :] += pz[:-1, :, :]
    return out


def tv(u: np.ndarray, dims: int = 3) -> float:
    """sum over voxels of sqrt(|dx|^2 + |dy|^2 (+ |dz|^2))."""
    dx, dy, dz = grad(np.asarray(u, dtype=np.complex128), dims)
    return float(np.sqrt(np.abs(dx) ** 2 + np.abs(dy) ** 2 + np.abs(dz) ** 2).sum())


def shrink(u: np.ndarray, thr: float) -> np.ndarray:
    """Eq. (8) for complex values: (1 - thr/|u|)_+ u (0 where |u| <= thr)."""
    u = np.asarray(u, dtype=np.complex128)
    a = np.abs(u)
    out = np.zeros_like(u)
    keep = a > thr
    out[keep] = (1.0 - thr / a[keep]) * u[keep]
    return out


def prox_tv_gp(v: np.ndarray, tau: float, n_iter: int, dims: int = 3, return_dual: bool = False):
    """argmin_u 1/2 ||u - v||^2 + tau TV(u) for complex v by n_iter GP steps on
    the dual (one complex value per direction, |p_voxel| <= 1 jointly):
        u = v - tau D^T p
        q = p + D u / (4 dims tau)
        p = q / max(1, sqrt(sum_d |q_d|^2))
    from p = 0, and u recovered once more at the end."""
    v = np.asarray(v, dtype=np.complex128)
    px, py, pz = np.zeros_like(v), np.zeros_like(v), np.zeros_like(v)
    if tau == 0.0:
        return (v.copy(), (px, py, pz)) if return_dual else v.copy()
    c = 1.0 / (4.0 * dims * tau)
    for _ in range(n_iter):
        u = v - tau * grad_adjoint(px, py, pz)
        gx, gy, gz = grad(u, dims)
        qx, qy, qz = px + c * gx, py + c * gy, pz + c * gz
        scale = np.maximum(1.0, np.sqrt(np.abs(qx) ** 2 + np.abs(qy) ** 2 + np.abs(qz) ** 2))
        px, py, pz = qx / scale, qy / scale, qz / scale
    u = v - tau * grad_adjoint(px, py, pz)
    return (u, (px, py, pz)) if return_dual else u


def prox_fused_lasso(v, step, l1, tv_w, n_inner, dims: int = 3) -> np.ndarray:
    """prox of step (l1 ||.||_1 + tv TV): the complex shrinkage of the TV prox
    (the separability the paper states for the fused lasso)."""
    u = prox_tv_gp(v, step * tv_w, n_inner, dims) if (tv_w > 0 and n_inner > 0) else \
        np.asarray(v, dtype=np.complex128).copy()
    return shrink(u, step * l1)


def objective(geom, x, b, l1, tv_w, dims: int = 3) -> float:
    """F(x) = 1/2 ||A x - b||^2 + l1 sum |x| + tv TV(x)."""
    r = forward(geom, x) - np.asarray(b, dtype=np.float64)
    return 0.5 * float((r * r).sum()) + l1 * float(np.abs(x).sum()) + tv_w * tv(x, dims)


def fista(geom, b, l1, tv_w, n_outer, n_inner, x0=None, step=None, dims: int = 3, history: bool = False):
    """FISTA on the complex object: x_k = prox(y_k - t A^T (A y_k - b)),
    s_{k+1} = (1 + sqrt(1 + 4 s_k^2)) / 2, y_{k+1} = x_k + ((s_k - 1)/s_{k+1})
    (x_k - x_{k-1}), from x_0 = 0 (or x0), t = 1/||A||^2."""
    b = np.asarray(b, dtype=np.float64)
    t = 1.0 / lipschitz(geom) if step is None else float(step)
    x = np.zeros((geom.nz, geom.ny, geom.nx), dtype=np.complex128) if x0 is None else \
        np.array(x0, dtype=np.complex128)
    y = x.copy()
    s = 1.0
    hist = []
    for _ in range(n_outer):
        g = adjoint(geom, forward(geom, y) - b)
        x_new = prox_fused_lasso(y - t * g, t, l1, tv_w, n_inner, dims)
        s_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * s * s))
        y = x_new + ((s - 1.0) / s_new) * (x_new - x)
        x, s = x_new, s_new
        if history:
            hist.append(objective(geom, x, b, l1, tv_w, dims))
    return (x, hist) if history else x
