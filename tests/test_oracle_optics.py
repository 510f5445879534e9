"""Pins for the oracle's Fresnel propagation (oracle/optics.py).

Closed-form Fresnel diffraction of a Gaussian beam (Goodman; Siegman,
Lasers, Gaussian beam propagation), the focus of a conjugate-chirp ("thin
lens") input whose magnitude is a product of Dirichlet kernels, conservation
of energy between the planes, and the exact inverse.
"""
import numpy as np
import pytest

import oracle

LAM = 532e-9
PITCH = 8e-6


def centred(n, pitch):
    return (np.arange(n) - n // 2) * pitch


def gaussian_closed_form(n, pitch, lam, z, w0):
    """Fresnel-propagated field of exp(-r^2/w0^2):
    exp(ikz)/(1 + i z/z_R) * exp(i a b r^2/(a - i b)), a = 1/w0^2, b = pi/(lambda z)."""
    p_out = lam * z / (n * pitch)
    xo = centred(n, p_out)
    r2 = xo[:, None] ** 2 + xo[None, :] ** 2
    a = 1.0 / w0 ** 2
    b = np.pi / (lam * z)
    z_r = np.pi * w0 ** 2 / lam
    kz = 2 * np.pi * np.mod(z / lam, 1.0)
    return np.exp(1j * kz) / (1 + 1j * z / z_r) * np.exp(1j * a * b * r2 / (a - 1j * b))


@pytest.mark.parametrize("n,z,w0", [(256, 0.5, 0.2e-3), (512, 0.45, 0.3e-3)])
def test_gaussian_beam_closed_form(n, z, w0):
    xs = centred(n, PITCH)
    u0 = np.exp(-(xs[:, None] ** 2 + xs[None, :] ** 2) / w0 ** 2)
    uz = oracle.propagate(u0, +1, fresnel=True, wavelength=LAM, pitch=PITCH, distance=z)
    ref = gaussian_closed_form(n, PITCH, LAM, z, w0)
    err = np.linalg.norm(uz - ref) / np.linalg.norm(ref)
    assert err <= 1e-9, err


def test_gaussian_beam_width_law():
    """|U_z|^2 is Gaussian with w(z)^2 = w0^2 (1 + (z/z_R)^2) (second moment)."""
    n, z, w0 = 256, 0.5, 0.2e-3
    xs = centred(n, PITCH)
    u0 = np.exp(-(xs[:, None] ** 2 + xs[None, :] ** 2) / w0 ** 2)
    uz = oracle.propagate(u0, +1, fresnel=True, wavelength=LAM, pitch=PITCH, distance=z)
    p_out = LAM * z / (n * PITCH)
    xo = centred(n, p_out)
    inten = np.abs(uz) ** 2
    # for exp(-2 r^2 / w^2), <x^2> = w^2 / 4
    mx2 = np.sum(inten * xo[None, :] ** 2) / np.sum(inten)
    z_r = np.pi * w0 ** 2 / LAM
    w2 = w0 ** 2 * (1 + (z / z_r) ** 2)
    assert abs(mx2 - w2 / 4) <= 1e-6 * w2


def dirichlet(k, n, m):
    """sum_{j=-(m-1)/2}^{(m-1)/2} exp(-2 pi i j k / n) for odd m (real)."""
    k = np.asarray(k, dtype=np.float64)
    out = np.empty_like(k)
    s = np.sin(np.pi * k / n)
    zero = np.abs(s) < 1e-15
    out[zero] = m
    out[~zero] = np.sin(np.pi * k[~zero] * m / n) / s[~zero]
    return out


def test_conjugate_chirp_focus():
    """U_0 = rect * conj(Q1): the chirp cancels and |U_z| = p^2/(lambda z) |D_y| |D_x|."""
    h, w, z = 96, 128, 0.4
    my, mx = 21, 35
    yy = np.arange(h) - h // 2
    xx = np.arange(w) - w // 2
    rect = (np.abs(yy)[:, None] <= my // 2) & (np.abs(xx)[None, :] <= mx // 2)
    ys = centred(h, PITCH)
    xs = centred(w, PITCH)
    q1 = np.exp(1j * np.pi * (ys[:, None] ** 2 + xs[None, :] ** 2) / (LAM * z))
    u0 = rect * np.conj(q1)
    uz = oracle.propagate(u0, +1, fresnel=True, wavelength=LAM, pitch=PITCH, distance=z)
    ky = np.arange(h) - h // 2
    kx = np.arange(w) - w // 2
    ref = PITCH ** 2 / (LAM * z) * np.abs(dirichlet(ky, h, my))[:, None] * np.abs(dirichlet(kx, w, mx))[None, :]
    assert np.abs(np.abs(uz) - ref).max() <= 1e-12 * ref.max()


@pytest.mark.parametrize("shape,z", [((128, 128), 0.5), ((90, 160), 0.45), ((75, 64), 2.0)])
def test_energy_conservation_and_inverse(shape, z):
    h, w = shape
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    uz = oracle.propagate(u0, +1, fresnel=True, wavelength=LAM, pitch=PITCH, distance=z)
    pyo = LAM * z / (h * PITCH)
    pxo = LAM * z / (w * PITCH)
    e0 = np.sum(np.abs(u0) ** 2) * PITCH ** 2
    ez = np.sum(np.abs(uz) ** 2) * pyo * pxo
    assert abs(ez - e0) <= 1e-12 * e0
    back = oracle.propagate(uz, -1, fresnel=True, wavelength=LAM, pitch=PITCH, distance=z)
    assert np.linalg.norm(back - u0) <= 1e-12 * np.linalg.norm(u0)


def test_fourier_mode_is_raw_transform_pair():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((24, 40)) + 1j * rng.standard_normal((24, 40))
    y = oracle.propagate(x, +1)
    assert np.linalg.norm(y - np.fft.fft2(x)) <= 1e-13 * np.linalg.norm(y)
    assert np.linalg.norm(oracle.propagate(y, -1) - x) <= 1e-13 * np.linalg.norm(x)


# ---------------------------------------------------------------------------
# angular spectrum
# ---------------------------------------------------------------------------
AS = dict(wavelength=532e-9, pitch=8e-6)


def _field(h, w, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(h, w)) + 1j * rng.normal(size=(h, w))


def test_angular_spectrum_zero_distance_is_identity():
    u = _field(24, 40, 1)
    assert np.allclose(oracle.angular_spectrum(u, +1, distance=0.0, **AS), u, rtol=0, atol=1e-12)


def test_angular_spectrum_semigroup_and_inverse():
    u = _field(32, 48, 2)
    a = oracle.angular_spectrum(oracle.angular_spectrum(u, +1, distance=0.03, **AS), +1, distance=0.05, **AS)
    b = oracle.angular_spectrum(u, +1, distance=0.08, **AS)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()
    back = oracle.angular_spectrum(b, -1, distance=0.08, **AS)
    assert np.abs(back - u).max() <= 1e-10 * np.abs(u).max()


def test_angular_spectrum_plane_wave_closed_form():
    h, w, ky, kx, z = 30, 40, 3, -7, 0.11
    yy, xx = np.mgrid[0:h, 0:w]
    u = np.exp(2j * np.pi * (kx * xx / w + ky * yy / h))
    fx, fy = kx / (w * AS["pitch"]), ky / (h * AS["pitch"])
    kz = 2 * np.pi * z * np.sqrt(1 / AS["wavelength"] ** 2 - fx ** 2 - fy ** 2)
    expect = u * np.exp(1j * kz)
    got = oracle.angular_spectrum(u, +1, distance=z, **AS)
    assert np.abs(got - expect).max() <= 1e-9


def test_angular_spectrum_frequencies_follow_fft_order():
    f = oracle.spatial_frequencies(6, 2.0)
    assert np.allclose(f, np.fft.fftfreq(6, 2.0), rtol=0, atol=0)
    f = oracle.spatial_frequencies(5, 0.5)
    assert np.allclose(f, np.fft.fftfreq(5, 0.5), rtol=0, atol=1e-15)


def test_angular_spectrum_gaussian_beam():
    """A paraxial Gaussian beam (waist 10 px) propagated 2 cm: the closed form,
    including exp(i k z), to the sampling accuracy."""
    h = w = 128
    p, lam, w0, z = AS["pitch"], AS["wavelength"], 80e-6, 0.02
    y = (np.arange(h) - h // 2) * p
    x = (np.arange(w) - w // 2) * p
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    u0 = np.exp(-r2 / w0 ** 2)
    zr = np.pi * w0 ** 2 / lam
    wz = w0 * np.sqrt(1 + (z / zr) ** 2)
    inv_r = z / (z ** 2 + zr ** 2)
    k = 2 * np.pi / lam
    kz = 2 * np.pi * np.mod(z / lam, 1.0)
    expect = (w0 / wz) * np.exp(-r2 / wz ** 2) * np.exp(1j * (kz - np.arctan(z / zr) + 0.5 * k * r2 * inv_r))
    got = oracle.angular_spectrum(u0, +1, distance=z, **AS)
    assert np.linalg.norm(got - expect) <= 1e-6 * np.linalg.norm(expect)
