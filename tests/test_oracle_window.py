"""Pins for the oracle's signal-window GS (oracle/window.py).

* A 2x2 example worked by hand from the definitions: the windowed NMSE as an
  exact rational, the target scale c and the free region in the first step.
* The windowed NMSE against a plain loop over the window's pixels.
* With a window covering the frame the loop is gs_iterate (itself pinned in
  test_oracle_gs.py).
* The target outside the window has no effect.
* Fienup's theorem with a window: the error sum_M (|R| - c T)^2 never increases.
* A target proportional to |R_0| inside the window has zero error at state 0.

Each pin fails for a plausible slip: imposing the target outside the window,
dropping c, or measuring the error over the full frame.
"""
import numpy as np
import pytest

import oracle
from oracle.window import gs_window, window_nmse

TWO_PI = 2 * np.pi
FRESNEL = dict(wavelength=532e-9, pitch=8e-6, distance=0.5)


def dft2x2(a, b, c, d):
    """2x2 DFT of [[a, b], [c, d]] written out: signs (-1)^(mk + nl)."""
    return np.array([[a + b + c + d, a - b + c - d], [a + b - c - d, a - b - c + d]])


def test_worked_2x2_window():
    # T_amp centred [[1, 0], [1, 2]] -> FFT order T_f = [[2, 1], [0, 1]];
    # window centred [[0, 0], [1, 1]] -> FFT order [[1, 1], [0, 0]] (top row)
    t_amp = np.array([[1.0, 0.0], [1.0, 2.0]])
    window = np.array([[0, 0], [1, 1]], dtype=np.uint8)
    phi0 = np.array([[0.0, np.pi / 2], [0.0, np.pi]])          # H0 = [[1, i], [1, -1]]
    out = gs_window(t_amp, window, phi0, 1)
    # R0 = [[1+i, 3-i], [1+i, -1-i]]; inside: I = (2, 10), T^2 = (4, 1)
    # I~ = (1/6, 5/6), T~ = (4/5, 1/5): sum diff^2 = 361/450, sum T~^2 = 17/25
    assert abs(out["nmse"][0] - 361.0 / 306.0) <= 1e-14
    # c^2 = N_px sum A^2 / sum_M T^2 = 16/5; inside R' = c T R/|R|, outside R' = R
    c = 4.0 / np.sqrt(5.0)
    r00 = c * 2.0 * (1 + 1j) / np.sqrt(2.0)
    r01 = c * 1.0 * (3 - 1j) / np.sqrt(10.0)
    g = dft2x2(r00, r01, 1 + 1j, -1 - 1j) / 4.0
    h1 = g / np.abs(g)
    assert np.allclose(out["phase"], np.mod(np.angle(h1), TWO_PI), atol=1e-14, rtol=0)
    r1 = dft2x2(h1[0, 0], h1[0, 1], h1[1, 0], h1[1, 1])
    i1 = np.abs(r1[0]) ** 2
    tn = np.array([4.0, 1.0]) / 5.0
    nm1 = np.sum((i1 / i1.sum() - tn) ** 2) / np.sum(tn ** 2)
    assert abs(out["nmse"][1] - nm1) <= 1e-13


def test_window_nmse_is_the_masked_definition():
    rng = np.random.default_rng(3)
    i = rng.uniform(0, 5, (6, 7))
    t = rng.uniform(0, 2, (6, 7))
    m = rng.uniform(size=(6, 7)) < 0.4
    si = sum(i[y, x] for y in range(6) for x in range(7) if m[y, x])
    st = sum(t[y, x] for y in range(6) for x in range(7) if m[y, x])
    num = sum((i[y, x] / si - t[y, x] / st) ** 2 for y in range(6) for x in range(7) if m[y, x])
    den = sum((t[y, x] / st) ** 2 for y in range(6) for x in range(7) if m[y, x])
    assert abs(window_nmse(i, t, m) - num / den) <= 1e-13 * (num / den)
    assert window_nmse(np.zeros((6, 7)), t, m) == 1.0


def problem(h, w, seed):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 1.0, (h, w))
    phi = rng.uniform(0.0, TWO_PI, (h, w))
    yy, xx = np.mgrid[0:h, 0:w]
    window = ((yy - h / 2) ** 2 + (xx - w / 2) ** 2 <= (0.3 * h) ** 2).astype(np.uint8)
    return t, phi, window


@pytest.mark.parametrize("levels,fresnel", [(0, None), (8, None), (4, FRESNEL)])
def test_full_window_is_gs(levels, fresnel):
    t, phi, _ = problem(24, 32, 5)
    a = gs_window(t, np.ones_like(t, dtype=np.uint8), phi, 6, levels=levels, fresnel=fresnel)
    b = oracle.gs_iterate(t, phi, 6, levels=levels, fresnel=fresnel)
    assert np.allclose(a["nmse"], b["nmse"], rtol=1e-12, atol=0)
    d = np.angle(np.exp(1j * (a["phase"] - b["phase"])))
    assert np.abs(d).max() <= 1e-9
    if levels:
        assert np.array_equal(a["levels"], b["levels"])


@pytest.mark.parametrize("levels", [0, 8])
def test_target_outside_the_window_has_no_effect(levels):
    t, phi, window = problem(32, 32, 7)
    t2 = np.where(window != 0, t, np.random.default_rng(9).uniform(0, 3, t.shape))
    a = gs_window(t, window, phi, 5, levels=levels)
    b = gs_window(t2, window, phi, 5, levels=levels)
    assert a["nmse"] == b["nmse"]
    assert np.array_equal(a["phase"], b["phase"])


@pytest.mark.parametrize("levels,fresnel", [(0, None), (8, None), (4, FRESNEL), (0, FRESNEL)])
def test_fienup_error_never_increases_with_a_window(levels, fresnel):
    t, phi, window = problem(32, 48, 11)
    out = gs_window(t, window, phi, 15, levels=levels, fresnel=fresnel, fienup=True)
    e = np.array(out["fienup"])
    assert np.all(e[1:] <= e[:-1] * (1 + 1e-12)), e
    assert e[-1] < e[0]


def test_consistent_target_inside_the_window_has_zero_error():
    h, w = 16, 16
    rng = np.random.default_rng(2)
    phi = rng.uniform(0, TWO_PI, (h, w))
    r = oracle.fft2(np.exp(1j * phi))
    t_f = 3.0 * np.abs(r)                       # any positive multiple
    t = oracle.fftshift(t_f)
    _, _, window = problem(h, w, 1)
    out = gs_window(t * np.where(window != 0, 1.0, 0.2), window, phi, 0)
    assert out["nmse"][0] <= 1e-26
