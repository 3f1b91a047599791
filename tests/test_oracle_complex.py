"""Pins of the complex-object oracle (oracle/complex_object.py) against facts
that do not depend on its own code: a single Fourier mode through the
transfer function written out by hand, the adjoint identity under the real
inner product, ||A||^2 = nz, the reductions to the real oracle, the closed
form of the complex shrinkage, the invariance of the complex TV prox under a
global phase, and its duality gap.

Each pin is chosen so that a plausible mistake fails it: a lost conj or a sign
of the imaginary part (plane wave, adjoint identity), real and imaginary parts
projected apart (phase invariance), a wrong GP step (duality gap), the
threshold on the real part instead of the modulus (closed form).
"""
import math

import numpy as np
import pytest

from oracle import complex_object as co, optics, prox, fista
from paper_1904_04884_amd import scenes


def geom(nx=32, ny=24, nz=5, **kw):
    return scenes.geometry_c1().with_(nx=nx, ny=ny, nz=nz, **kw)


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("carrier", [True, False])
def test_forward_of_one_fourier_mode(carrier):
    """x_j = a_j exp(i 2 pi f0 . r) with a complex amplitude per plane: A x is
    Re(sum_j a_j H_j(f0) exp(i 2 pi f0 . r)), H_j(f0) written from its formula."""
    g = geom(carrier=carrier)
    rng = np.random.default_rng(1)
    ky, kx = 3, -5
    fy, fx = ky / (g.ny * g.pixel_um), kx / (g.nx * g.pixel_um)
    yy, xx = np.mgrid[0:g.ny, 0:g.nx]
    wave = np.exp(2j * np.pi * (ky * yy / g.ny + kx * xx / g.nx))
    a = crandn(rng, g.nz)
    x = a[:, None, None] * wave[None]
    want = np.zeros((g.ny, g.nx), dtype=np.complex128)
    for j in range(g.nz):
        z = g.z0_um + j * g.dz_um
        kz = math.sqrt(1.0 / g.wavelength_um ** 2 - fx * fx - fy * fy)
        if not carrier:
            kz -= 1.0 / g.wavelength_um
        want += a[j] * np.exp(2j * np.pi * z * kz) * wave
    np.testing.assert_allclose(co.forward(g, x), want.real, rtol=0, atol=1e-10)


def test_adjoint_identity_real_inner_product():
    g = geom()
    rng = np.random.default_rng(2)
    x = crandn(rng, (g.nz, g.ny, g.nx))
    r = rng.standard_normal((g.ny, g.nx))
    lhs = float((co.forward(g, x) * r).sum())
    rhs = float(np.real(np.conj(x) * co.adjoint(g, r)).sum())
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_norm_is_nz_and_power_iteration_agrees():
    g = geom(nz=7)
    assert co.lipschitz(g) == pytest.approx(7.0, rel=1e-12)
    rng = np.random.default_rng(3)
    x = crandn(rng, (g.nz, g.ny, g.nx))
    lam = 0.0
    for _ in range(60):
        y = co.adjoint(g, co.forward(g, x))
        lam = float(np.real(np.vdot(x, y)) / np.real(np.vdot(x, x)))
        x = y / np.linalg.norm(y)
    assert lam == pytest.approx(7.0, rel=1e-6)


def test_reduces_to_the_real_oracle():
    g = geom()
    rng = np.random.default_rng(4)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    r = rng.standard_normal((g.ny, g.nx))
    np.testing.assert_allclose(co.forward(g, x), optics.forward(g, x), rtol=0, atol=1e-12)
    np.testing.assert_allclose(co.adjoint(g, r).real, optics.adjoint(g, r), rtol=0, atol=1e-12)
    # the imaginary part of the object: A (i x) is A x with every H_j times i
    gi = co.forward(g, 1j * x)
    acc = np.zeros((g.ny, g.nx), dtype=np.complex128)
    for j, z in enumerate(optics.plane_z(g)):
        acc += np.fft.ifft2(np.fft.fft2(x[j]) * optics.transfer_function(g, z) * 1j)
    np.testing.assert_allclose(gi, acc.real, rtol=0, atol=1e-12)


def test_shrink_closed_form():
    u = np.array([3 + 4j, 0.3 - 0.4j, 0.0, -2.0, 1e-3j])
    out = co.shrink(u, 1.0)
    want = np.array([(1 - 1 / 5) * (3 + 4j), 0.0, 0.0, -1.0, 0.0])
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-15)
    # a real argument: the signed soft threshold sign(u) (|u| - t)_+
    r = np.linspace(-3, 3, 61)
    np.testing.assert_allclose(co.shrink(r, 0.7).real, np.sign(r) * np.maximum(np.abs(r) - 0.7, 0), atol=1e-15)
    # the modulus decides, not the real part
    assert co.shrink(np.array([0.1 + 2j]), 1.0)[0] != 0


@pytest.mark.parametrize("dims", [3, 2])
def test_tv_prox_of_a_real_field_is_the_real_prox(dims):
    rng = np.random.default_rng(5)
    v = rng.standard_normal((4, 9, 11))
    got = co.prox_tv_gp(v.astype(np.complex128), 0.3, 25, dims)
    want = prox.prox_tv_gp(v, 0.3, 25, dims=dims)
    np.testing.assert_allclose(got.real, want, rtol=0, atol=1e-12)
    assert np.abs(got.imag).max() == 0.0


@pytest.mark.parametrize("dims", [3, 2])
def test_tv_prox_commutes_with_a_global_phase(dims):
    rng = np.random.default_rng(6)
    v = crandn(rng, (4, 8, 10))
    ph = np.exp(1j * 0.7)
    a = co.prox_tv_gp(ph * v, 0.25, 30, dims)
    b = ph * co.prox_tv_gp(v, 0.25, 30, dims)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
    # projecting the real and imaginary parts apart would break this
    assert np.abs(a - v).max() > 1e-3


@pytest.mark.parametrize("dims", [3, 2])
def test_tv_prox_duality_gap_closes(dims):
    """P(u) = 1/2||u - v||^2 + tau TV(u) and D(p) = 1/2||v||^2 - 1/2||v - tau D^T p||^2
    bound the optimum from both sides; the GP iterates close the gap."""
    rng = np.random.default_rng(7)
    v = crandn(rng, (3, 6, 7))
    tau = 0.2
    gaps = []
    for n in (20, 200, 2000):
        u, (px, py, pz) = co.prox_tv_gp(v, tau, n, dims, return_dual=True)
        P = 0.5 * float(np.abs(u - v).__pow__(2).sum()) + tau * co.tv(u, dims)
        D = 0.5 * float(np.abs(v).__pow__(2).sum()) - 0.5 * float(np.abs(u).__pow__(2).sum())
        assert np.sqrt(np.abs(px) ** 2 + np.abs(py) ** 2 + np.abs(pz) ** 2).max() <= 1 + 1e-12
        gaps.append(P - D)
    assert gaps[0] >= -1e-12 and gaps[-1] >= -1e-12
    assert gaps[-1] < 1e-3 * gaps[0] and gaps[-1] < 1e-6 * max(1.0, abs(P))


def test_fused_lasso_prox_is_shrink_of_tv_prox():
    rng = np.random.default_rng(8)
    v = crandn(rng, (3, 8, 8))
    got = co.prox_fused_lasso(v, 0.5, 0.4, 0.3, 15)
    want = co.shrink(co.prox_tv_gp(v, 0.15, 15), 0.2)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_fista_one_plane_least_squares():
    """nz = 1: |H| = 1 on the grid, so A A^T = I and t = 1; from 0 the first
    iterate is A^T b and it reproduces b exactly."""
    g = geom(nz=1)
    rng = np.random.default_rng(9)
    b = rng.standard_normal((g.ny, g.nx))
    x1 = co.fista(g, b, 0.0, 0.0, 1, 0)
    np.testing.assert_allclose(x1, co.adjoint(g, b), rtol=0, atol=1e-13)
    np.testing.assert_allclose(co.forward(g, x1), b, rtol=0, atol=1e-12)


@pytest.mark.parametrize("tv_w", [0.0, 0.05])
def test_fista_with_identity_optics_is_the_real_fista(tv_w):
    """One plane at z = 0 without the carrier: H = 1, A x = Re x and A^T r = r.
    From a real start the complex iterates stay real and equal the real
    oracle's signed FISTA (whose momentum is pinned by hand elsewhere)."""
    g = geom(nz=1, carrier=False).with_(z0_um=0.0)
    rng = np.random.default_rng(10)
    b = rng.standard_normal((g.ny, g.nx))
    got = co.fista(g, b, 0.3, tv_w, 6, 8, step=0.5)
    want = fista.fista(g, b, 0.3, tv_w, 6, 8, step=0.5, nonneg=False)
    np.testing.assert_allclose(got.real, want, rtol=0, atol=1e-12)
    assert np.abs(got.imag).max() <= 1e-12          # FFT round-off of a real field only


def test_objective_terms():
    g = geom(nz=2)
    rng = np.random.default_rng(11)
    x = crandn(rng, (g.nz, g.ny, g.nx))
    b = rng.standard_normal((g.ny, g.nx))
    F = co.objective(g, x, b, 0.3, 0.2)
    r = co.forward(g, x) - b
    dx = np.diff(x, axis=2, append=x[:, :, -1:])
    dy = np.diff(x, axis=1, append=x[:, -1:, :])
    dz = np.diff(x, axis=0, append=x[-1:, :, :])
    want = 0.5 * (r * r).sum() + 0.3 * np.abs(x).sum() + \
        0.2 * np.sqrt(np.abs(dx) ** 2 + np.abs(dy) ** 2 + np.abs(dz) ** 2).sum()
    assert F == pytest.approx(want, rel=1e-12)
