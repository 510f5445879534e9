"""Pins for the oracle's DFT/FFT (oracle/dft.py) against mathematics.

Brute-force double sums in pure Python, Parseval's identity, the closed-form
transforms of a delta and a plane wave, inverse-after-forward identity, and
numpy's FFT as an independent library cross-check (used here only, never in
the oracle).
"""
import cmath
import math

import numpy as np
import pytest

import oracle


def brute_dft2(x):
    """X[k][l] = sum_{m,n} x[m][n] exp(-2 pi i (m k / H + n l / W)), pure Python."""
    h = len(x)
    w = len(x[0])
    out = [[0j] * w for _ in range(h)]
    for k in range(h):
        for l in range(w):
            s = 0j
            for m in range(h):
                for n in range(w):
                    s += x[m][n] * cmath.exp(-2j * math.pi * ((m * k) / h + (n * l) / w))
            out[k][l] = s
    return out


def test_fft2_matches_brute_force_all_shapes_up_to_16():
    rng = np.random.default_rng(123)
    for h in range(1, 17):
        for w in range(1, 17):
            x = rng.standard_normal((h, w)) + 1j * rng.standard_normal((h, w))
            ref = np.array(brute_dft2(x.tolist()))
            got = oracle.fft2(x)
            err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
            assert err <= 1e-13, (h, w, err)


def test_fft1d_matches_brute_force_lengths_to_64():
    rng = np.random.default_rng(7)
    for n in list(range(1, 65)) + [72, 75, 81, 96, 100, 125, 128]:
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        ref = np.array([sum(x[j] * cmath.exp(-2j * math.pi * j * k / n) for j in range(n))
                        for k in range(n)])
        err = np.abs(oracle.fft(x) - ref).max() / np.abs(ref).max()
        assert err <= 1e-13, (n, err)


def test_naive_dft_matches_brute_force():
    rng = np.random.default_rng(8)
    for n in (1, 2, 5, 7, 13, 16):
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        ref = np.array([sum(x[j] * cmath.exp(-2j * math.pi * j * k / n) for j in range(n))
                        for k in range(n)])
        assert np.abs(oracle.dft_naive(x) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("shape", [(256, 256), (1080, 1920), (48, 80), (27, 125)])
def test_parseval(shape):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    X = oracle.fft2(x)
    lhs = np.sum(np.abs(X) ** 2)
    rhs = x.size * np.sum(np.abs(x) ** 2)
    assert abs(lhs - rhs) <= 1e-12 * rhs


@pytest.mark.parametrize("shape,pos", [((64, 64), (3, 17)), ((40, 24), (39, 5)), ((15, 12), (7, 11))])
def test_delta_closed_form(shape, pos):
    h, w = shape
    a, b = pos
    x = np.zeros(shape, dtype=np.complex128)
    x[a, b] = 1.0
    k = np.arange(h)[:, None]
    l = np.arange(w)[None, :]
    ref = np.exp(-2j * np.pi * (a * k / h + b * l / w))
    assert np.abs(oracle.fft2(x) - ref).max() <= 1e-13


@pytest.mark.parametrize("shape,freq", [((64, 32), (5, 30)), ((30, 45), (29, 1)), ((128, 128), (0, 64))])
def test_plane_wave_closed_form(shape, freq):
    h, w = shape
    ky, kx = freq
    m = np.arange(h)[:, None]
    n = np.arange(w)[None, :]
    x = np.exp(2j * np.pi * (np.mod(ky * m, h) / h + np.mod(kx * n, w) / w))
    ref = np.zeros(shape, dtype=np.complex128)
    ref[ky, kx] = h * w
    assert np.abs(oracle.fft2(x) - ref).max() <= 1e-13 * h * w


@pytest.mark.parametrize("shape", [(256, 256), (1080, 1920), (12, 10), (9, 8)])
def test_inverse_after_forward_is_identity(shape):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    back = oracle.ifft2(oracle.fft2(x))
    assert np.linalg.norm(back - x) <= 1e-14 * np.linalg.norm(x) * 10


@pytest.mark.parametrize("shape", [(256, 256), (1024, 1024), (1080, 1920), (512, 512), (33, 50)])
def test_library_cross_check(shape):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = np.fft.fft2(x)
    assert np.linalg.norm(oracle.fft2(x) - ref) <= 1e-13 * np.linalg.norm(ref)
    refi = np.fft.ifft2(x)
    assert np.linalg.norm(oracle.ifft2(x) - refi) <= 1e-13 * np.linalg.norm(refi)


@pytest.mark.parametrize("shape", [(4, 6), (5, 7), (1080, 1920)])
def test_shifts(shape):
    x = np.arange(shape[0] * shape[1]).reshape(shape)
    assert np.array_equal(oracle.fftshift(x), np.fft.fftshift(x))
    assert np.array_equal(oracle.ifftshift(x), np.fft.ifftshift(x))
    assert np.array_equal(oracle.ifftshift(oracle.fftshift(x)), x)
