"""Seeded synthetic scenes and solver configurations.

This module is shared by the FP64 oracle tests and the GPU path.  It holds
geometry, regularisation settings and random draws only: particle positions,
their rasterisation into a voxel grid, and the per-pixel noise field.  It does
not propagate light, apply a regulariser or touch a GPU; whoever consumes a
scene forms the hologram b = A x_true + noise with its own forward model.

Scene recipes follow the paper's workloads (section "Demonstration Cases"):
tracer particles much smaller than the plane spacing, so each particle is an
in-plane object painted into its nearest reconstruction plane.  Units are
micrometres; volumes are C-contiguous [z][y][x], x fastest.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Geometry", "SolveConfig", "Scene",
    "geometry_c1", "geometry_c2", "config_c1", "config_c2",
    "gaussian_particles", "disk_particles", "burgers_series", "densify",
    "noise_field", "scene_c1", "scene_c2",
]


@dataclass(frozen=True)
class Geometry:
    """Reconstruction grid and optics.

    nx, ny: hologram size in pixels; nz: number of reconstruction planes.
    pixel_um: lateral pixel pitch; wavelength_um: illumination wavelength.
    Plane j sits at z_j = z0_um + j * dz_um from the sensor.
    carrier: keep the exp(i 2 pi z / lambda) carrier in the transfer function.
    tv_dims: 3 for the 3D TV, 2 for the per-plane 2D TV of the paper's Eq. (4).
    tv_fgp, dual_bf16: inner-solver options of the library (accelerated dual
    iteration; dual stored in bfloat16).
    complex_object: the object is complex (absorption and phase); the library
    then holds a volume as [2][nz][ny][nx] (real parts, imaginary parts).
    """
    nx: int
    ny: int
    nz: int
    pixel_um: float
    wavelength_um: float
    z0_um: float
    dz_um: float
    carrier: bool = True
    tv_dims: int = 3
    tv_fgp: bool = False
    dual_bf16: bool = False
    complex_object: bool = False

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def z(self) -> np.ndarray:
        return self.z0_um + self.dz_um * np.arange(self.nz, dtype=np.float64)

    def with_(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


@dataclass(frozen=True)
class SolveConfig:
    """Fused-lasso weights and iteration counts (paper Eq. 5 and the FISTA loop)."""
    l1: float
    tv: float
    outer_iters: int
    inner_iters: int
    noise_sigma: float


@dataclass
class Scene:
    geometry: Geometry
    config: SolveConfig
    # sparse ground truth: integer voxel indices (z, y, x) and values
    idx: np.ndarray
    val: np.ndarray
    noise: np.ndarray            # [ny][nx] float64, already scaled by sigma
    centers: np.ndarray          # [n][3] (z plane, y px, x px) particle centres
    meta: dict = field(default_factory=dict)

    def dense(self, dtype=np.float64) -> np.ndarray:
        return densify(self.geometry.shape, self.idx, self.val, dtype)


# ---------------------------------------------------------------------------
# Configurations.  C1: 128^2 x 32 planes, 632.8 nm, 10 um pixels (the optics of
# the synthetic turbulence case).  C2: 1024^2 x 256 planes, 532 nm, 5 um pixels
# (the optics of the algae case), 50 um plane spacing from 5 mm.
# ---------------------------------------------------------------------------

def geometry_c1() -> Geometry:
    return Geometry(nx=128, ny=128, nz=32, pixel_um=10.0, wavelength_um=0.6328,
                    z0_um=5000.0, dz_um=200.0)


def config_c1() -> SolveConfig:
    return SolveConfig(l1=0.01, tv=0.005, outer_iters=50, inner_iters=10, noise_sigma=0.01)


def geometry_c2() -> Geometry:
    return Geometry(nx=1024, ny=1024, nz=256, pixel_um=5.0, wavelength_um=0.532,
                    z0_um=5000.0, dz_um=50.0)


def config_c2() -> SolveConfig:
    return SolveConfig(l1=0.02, tv=0.01, outer_iters=100, inner_iters=20, noise_sigma=0.02)


# ---------------------------------------------------------------------------
# Rasterisers
# ---------------------------------------------------------------------------

def densify(shape, idx, val, dtype=np.float64) -> np.ndarray:
    out = np.zeros(shape, dtype=dtype)
    if len(val):
        np.maximum.at(out, (idx[:, 0], idx[:, 1], idx[:, 2]), val.astype(dtype))
    return out


def _merge_max(idx: np.ndarray, val: np.ndarray, shape):
    """Collapse duplicate voxels keeping the largest value (opaque overlap)."""
    if len(val) == 0:
        return idx.reshape(0, 3).astype(np.int64), val.astype(np.float64)
    lin = np.ravel_multi_index((idx[:, 0], idx[:, 1], idx[:, 2]), shape)
    order = np.lexsort((-val, lin))
    lin_s, val_s = lin[order], val[order]
    keep = np.ones(len(lin_s), dtype=bool)
    keep[1:] = lin_s[1:] != lin_s[:-1]
    lin_u, val_u = lin_s[keep], val_s[keep]
    z, y, x = np.unravel_index(lin_u, shape)
    return np.stack([z, y, x], axis=1).astype(np.int64), val_u.astype(np.float64)


def gaussian_particles(geom: Geometry, n: int, rng: np.random.Generator,
                       sigma_px: float = 1.0, amp: float = 1.0, radius: int = 4,
                       margin: int = 4):
    """n particles at distinct integer voxels, each an in-plane Gaussian blob.

    Lateral centres are uniform integers in [margin, n - margin); planes are
    uniform integers.  The blob is truncated at `radius` pixels.
    """
    nz, ny, nx = geom.shape
    lin = rng.choice(nz * (ny - 2 * margin) * (nx - 2 * margin), size=n, replace=False)
    z, r = np.divmod(lin, (ny - 2 * margin) * (nx - 2 * margin))
    y, x = np.divmod(r, nx - 2 * margin)
    y = y + margin
    x = x + margin
    offs = np.arange(-radius, radius + 1)
    dy, dx = np.meshgrid(offs, offs, indexing="ij")
    inside = dy ** 2 + dx ** 2 <= radius ** 2
    dy, dx = dy[inside], dx[inside]
    w = amp * np.exp(-(dy ** 2 + dx ** 2) / (2.0 * sigma_px ** 2))
    idx = np.stack([
        np.repeat(z, len(w)),
        (np.repeat(y, len(w)) + np.tile(dy, n)) % ny,
        (np.repeat(x, len(w)) + np.tile(dx, n)) % nx,
    ], axis=1)
    val = np.tile(w, n)
    idx, val = _merge_max(idx, val, geom.shape)
    centers = np.stack([z, y, x], axis=1).astype(np.float64)
    return idx, val, centers


def _paint_disk(cy, cx, d, ny, nx, supersample):
    """Anti-aliased coverage of a disk of diameter d (px) centred at (cy, cx)."""
    r = 0.5 * d
    y0, y1 = int(np.floor(cy - r)), int(np.ceil(cy + r))
    x0, x1 = int(np.floor(cx - r)), int(np.ceil(cx + r))
    ys = np.arange(y0, y1 + 1)
    xs = np.arange(x0, x1 + 1)
    s = (np.arange(supersample) + 0.5) / supersample
    # sample positions inside each pixel: pixel (i) covers [i, i+1)
    sy = (ys[:, None] + s[None, :]).reshape(-1)
    sx = (xs[:, None] + s[None, :]).reshape(-1)
    inside = ((sy[:, None] - cy) ** 2 + (sx[None, :] - cx) ** 2) <= r * r
    cov = inside.reshape(len(ys), supersample, len(xs), supersample).mean(axis=(1, 3))
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    m = cov > 0
    return yy[m] % ny, xx[m] % nx, cov[m]


def disk_particles(geom: Geometry, n: int, rng: np.random.Generator,
                   dmin: float = 2.0, dmax: float = 6.0, amp: float = 1.0,
                   supersample: int = 4, margin: float = 4.0, centers=None, diam=None):
    """Opaque disks (amplitude `amp`) in their nearest plane, 4x4 supersampled.

    Centres are uniform continuous in [margin, n - margin) laterally and in
    [-0.5, nz - 0.5) plane units axially; diameters are uniform in [dmin, dmax].
    """
    nz, ny, nx = geom.shape
    if centers is None:
        cz = rng.uniform(-0.5, nz - 0.5, n)
        cy = rng.uniform(margin, ny - margin, n)
        cx = rng.uniform(margin, nx - margin, n)
        centers = np.stack([cz, cy, cx], axis=1)
    if diam is None:
        diam = rng.uniform(dmin, dmax, len(centers))
    zi_all, yi_all, xi_all, v_all = [], [], [], []
    for (cz, cy, cx), d in zip(centers, diam):
        zi = int(min(nz - 1, max(0, np.floor(cz + 0.5))))
        yy, xx, cov = _paint_disk(cy, cx, d, ny, nx, supersample)
        zi_all.append(np.full(len(yy), zi))
        yi_all.append(yy)
        xi_all.append(xx)
        v_all.append(amp * cov)
    if v_all:
        idx = np.stack([np.concatenate(zi_all), np.concatenate(yi_all), np.concatenate(xi_all)], axis=1)
        val = np.concatenate(v_all)
    else:
        idx, val = np.zeros((0, 3), np.int64), np.zeros(0)
    idx, val = _merge_max(idx, val, geom.shape)
    return idx, val, np.asarray(centers, dtype=np.float64), np.asarray(diam, dtype=np.float64)


def noise_field(geom: Geometry, sigma: float, rng: np.random.Generator) -> np.ndarray:
    return sigma * rng.standard_normal((geom.ny, geom.nx))


def scene_c1(seed: int = 0, geom: Geometry | None = None, n_particles: int = 50,
             config: SolveConfig | None = None) -> Scene:
    """C1: 50 Gaussian blobs (sigma 1 px, amplitude 1) at distinct voxels."""
    geom = geom or geometry_c1()
    config = config or config_c1()
    rng = np.random.default_rng(seed)
    idx, val, centers = gaussian_particles(geom, n_particles, rng)
    noise = noise_field(geom, config.noise_sigma, rng)
    return Scene(geom, config, idx, val, noise, centers, {"seed": seed, "kind": "gaussian"})


def scene_c2(seed: int = 0, geom: Geometry | None = None, n_particles: int = 2000,
             config: SolveConfig | None = None) -> Scene:
    """C2: 2000 opaque disks, diameter U[2, 6] px, uniform in the volume."""
    geom = geom or geometry_c2()
    config = config or config_c2()
    rng = np.random.default_rng(seed)
    idx, val, centers, diam = disk_particles(geom, n_particles, rng)
    noise = noise_field(geom, config.noise_sigma, rng)
    return Scene(geom, config, idx, val, noise, centers,
                 {"seed": seed, "kind": "disk", "diameters": diam})


# ---------------------------------------------------------------------------
# Time series for batched solves: particles advected by a Burgers vortex whose
# axis runs along z through the field centre.
# ---------------------------------------------------------------------------

def burgers_series(n_frames: int, field_px: int, nz_max: int, n_particles: int,
                   rng: np.random.Generator, max_disp_px: float = 3.0,
                   core_frac: float = 0.2):
    """Particle centres (frame, particle, [z, y, x]) in a Burgers vortex.

    u_theta = G / (2 pi r) (1 - exp(-r^2 / rc^2)), u_r = -(a/2) r,
    u_z = a (z - z_mid); a is set so that max |u_r| is 10 % of max u_theta,
    and the time step makes the largest per-frame displacement max_disp_px.
    Positions wrap periodically.
    """
    rc = core_frac * field_px
    c = 0.5 * field_px
    z_mid = 0.5 * nz_max
    G = 1.0
    r_s = np.linspace(1e-3, field_px * 0.75, 4096)
    ut = G / (2 * np.pi * r_s) * (1 - np.exp(-r_s ** 2 / rc ** 2))
    ut_max = ut.max()
    a = 0.1 * ut_max / (0.5 * r_s.max())

    def vel(p):
        z, y, x = p[:, 0], p[:, 1] - c, p[:, 2] - c
        r = np.sqrt(x * x + y * y) + 1e-12
        uth = G / (2 * np.pi * r) * (1 - np.exp(-r * r / rc ** 2))
        ur = -0.5 * a * r
        ux = ur * x / r - uth * y / r
        uy = ur * y / r + uth * x / r
        uz = a * (z - z_mid)
        return np.stack([uz, uy, ux], axis=1)

    p = np.stack([rng.uniform(0, nz_max, n_particles),
                  rng.uniform(0, field_px, n_particles),
                  rng.uniform(0, field_px, n_particles)], axis=1)
    vmax = np.abs(vel(p)).max()
    dt = max_disp_px / max(vmax, 1e-12)
    out = np.empty((n_frames, n_particles, 3))
    for t in range(n_frames):
        out[t] = p
        # midpoint step
        k1 = vel(p)
        k2 = vel(p + 0.5 * dt * k1)
        p = p + dt * k2
        p[:, 0] %= nz_max
        p[:, 1] %= field_px
        p[:, 2] %= field_px
    return out
