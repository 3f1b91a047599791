"""FP64 reference of the hologram forward model and its adjoint.

TEST INFRASTRUCTURE ONLY.  This is the oracle that the GPU library is checked
against; the product path never imports, calls or links it.

The paper poses reconstruction as the inverse problem of Eq. (2) with a
linearised hologram-formation model (section "Methodology", first paragraph):
the hologram b is modelled as a linear function H x of the real object volume
x, twin image and cross-interference being treated as noise.  The paper does
not print the kernel; the one used here is the angular-spectrum
(Rayleigh-Sommerfeld) propagator of the compressive-holography works it
follows:

    A x = Re( sum_j  IFFT2( FFT2(x_j) * H_j ) ),
    H_j(f) = exp(i 2 pi z_j sqrt(1/lambda^2 - fx^2 - fy^2)),

with numpy's unscaled forward / 1/N-scaled inverse FFT pair and the fftfreq
frequency grid.  The square root is the complex principal branch (evanescent
components decay).  With the carrier switched off the transfer function is
taken relative to the reference wave, exp(i 2 pi z (sqrt(.) - 1/lambda)).

Every function here is the definition written out, one plane at a time.
"""
from __future__ import annotations

import numpy as np

__all__ = ["freq_grid", "plane_z", "transfer_function", "forward", "adjoint",
           "lipschitz", "aat_multiplier"]


def freq_grid(ny: int, nx: int, pixel_um: float):
    """Spatial-frequency grid (cycles/um) in numpy FFT order: fy[:, None], fx[None, :]."""
    fy = np.fft.fftfreq(ny, d=pixel_um)
    fx = np.fft.fftfreq(nx, d=pixel_um)
    return fy[:, None], fx[None, :]


def plane_z(geom) -> np.ndarray:
    """z_j = z0 + j dz, j = 0 .. nz-1."""
    return geom.z0_um + geom.dz_um * np.arange(geom.nz, dtype=np.float64)


def transfer_function(geom, z_um: float) -> np.ndarray:
    """H_z on the DFT grid, complex128 [ny][nx]."""
    fy, fx = freq_grid(geom.ny, geom.nx, geom.pixel_um)
    k2 = (1.0 / geom.wavelength_um) ** 2 - fx ** 2 - fy ** 2
    kz = np.sqrt(k2.astype(np.complex128))           # principal branch
    if not getattr(geom, "carrier", True):
        kz = kz - 1.0 / geom.wavelength_um
    return np.exp(1j * 2.0 * np.pi * z_um * kz)


def forward(geom, x: np.ndarray) -> np.ndarray:
    """A x for a real volume x [nz][ny][nx] -> real hologram [ny][nx]."""
    x = np.asarray(x, dtype=np.float64)
    assert x.shape == (geom.nz, geom.ny, geom.nx)
    acc = np.zeros((geom.ny, geom.nx), dtype=np.complex128)
    for j, z in enumerate(plane_z(geom)):
        acc += np.fft.ifft2(np.fft.fft2(x[j]) * transfer_function(geom, z))
    return acc.real


def adjoint(geom, y: np.ndarray) -> np.ndarray:
    """A^T y: back-propagation of a real hologram to every plane with conj(H_j)."""
    y = np.asarray(y, dtype=np.float64)
    assert y.shape == (geom.ny, geom.nx)
    Y = np.fft.fft2(y)
    out = np.empty((geom.nz, geom.ny, geom.nx), dtype=np.float64)
    for j, z in enumerate(plane_z(geom)):
        out[j] = np.fft.ifft2(Y * np.conj(transfer_function(geom, z))).real
    return out


def aat_multiplier(geom) -> np.ndarray:
    """S(f) = sum_j (Re H_j(f))^2, the Fourier multiplier of A A^T for real data.

    A A^T y = ifft2(S * fft2(y)) holds because, on the symmetric fftfreq grid,
    H_j(f) = H_j(-f), so Re(IFFT(H F u)) = IFFT(Re(H) F u) for real u.
    """
    acc = np.zeros((geom.ny, geom.nx), dtype=np.float64)
    for z in plane_z(geom):
        acc += transfer_function(geom, z).real ** 2
    return acc


def lipschitz(geom) -> float:
    """||A||^2 = max_f S(f): Lipschitz constant of the gradient of 1/2||Ax - b||^2."""
    return float(aat_multiplier(geom).max())
