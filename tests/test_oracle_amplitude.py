"""Pins for the oracle's amplitude-only GS (oracle/amplitude.py).

* Two 1x2 Fourier holograms worked by hand: exact NMSE values, one that
  reaches its target in one step and one whose back-propagated field has a
  negative real part that the constraint clips to zero.
* A target consistent with some non-negative SLM amplitude is a fixed point.
* The replay-plane distance between the two constraint sets never increases
  (Fienup's error-reduction theorem), Fourier and Fresnel.
* Scaling the starting amplitude changes no later state and no error.

Replacing max(Re G, 0) by |G| or by Re G, or dropping IFFT2's 1/N, fails one
of them.
"""
import numpy as np
import pytest

import oracle
from oracle.amplitude import gs_amplitude, nonnegative_real

FRESNEL = dict(wavelength=532e-9, pitch=8e-6, distance=0.5)


def test_worked_1x2_reaches_the_target():
    # T centred (1, 2) -> FFT order (2, 1); a0 = (1, 1/2): R0 = (3/2, 1/2)
    out = gs_amplitude(np.array([[1.0, 2.0]]), np.array([[1.0, 0.5]]), 1)
    # I~ = (9/10, 1/10), T~ = (4/5, 1/5): sum diff^2 = 1/50, sum T~^2 = 17/25
    assert abs(out["nmse"][0] - 1.0 / 34.0) <= 1e-15
    # R' = (2, 1) -> IFFT2 (3/2, 1/2) -> a1 = (3/2, 1/2), R1 = (2, 1): exact
    assert np.allclose(out["amplitude"], [[1.5, 0.5]], atol=1e-15, rtol=0)
    assert abs(out["nmse"][1]) <= 1e-30


def test_worked_1x2_clips_the_negative_real_part():
    # T centred (3, 1) -> FFT order (1, 3); a0 = (1, 0): R0 = (1, 1)
    out = gs_amplitude(np.array([[3.0, 1.0]]), np.array([[1.0, 0.0]]), 1)
    # I~ = (1/2, 1/2), T~ = (1/10, 9/10): 8/25 over 41/50 = 16/41
    assert abs(out["nmse"][0] - 16.0 / 41.0) <= 1e-15
    # R' = (1, 3) -> IFFT2 (2, -1) -> a1 = (2, 0); R1 = (2, 2): again 16/41
    assert np.allclose(out["amplitude"], [[2.0, 0.0]], atol=1e-15, rtol=0)
    assert abs(out["nmse"][1] - 16.0 / 41.0) <= 1e-15


def test_nonnegative_real_is_the_nearest_nonnegative_value():
    g = np.array([3 + 4j, -2 + 1j, 0.5 - 7j, -0.0 + 0j])
    assert np.array_equal(nonnegative_real(g), [3.0, 0.0, 0.5, 0.0])
    # brute force over a grid of candidates >= 0
    cand = np.linspace(0, 5, 50001)
    for z in g:
        best = cand[np.argmin(np.abs(z - cand))]
        assert abs(best - nonnegative_real(np.array([z]))[0]) <= 1e-4


@pytest.mark.parametrize("fresnel", [None, FRESNEL])
def test_consistent_target_is_a_fixed_point(fresnel):
    h, w = 16, 24
    rng = np.random.default_rng(4)
    a_star = rng.uniform(0.0, 1.0, (h, w))
    if fresnel is None:
        q1 = np.ones((h, w))
    else:
        q1 = np.outer(oracle.fresnel_chirp(h, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]),
                      oracle.fresnel_chirp(w, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]))
    t = oracle.fftshift(np.abs(oracle.fft2(q1 * a_star)))
    out = gs_amplitude(t, a_star, 3, fresnel=fresnel)
    assert max(out["nmse"]) <= 1e-26
    assert np.allclose(out["amplitude"], a_star, atol=1e-12, rtol=0)


@pytest.mark.parametrize("fresnel", [None, FRESNEL])
def test_replay_distance_never_increases(fresnel):
    rng = np.random.default_rng(9)
    t = rng.uniform(0.0, 1.0, (32, 48))
    a0 = rng.uniform(0.0, 1.0, (32, 48))
    out = gs_amplitude(t, a0, 20, fresnel=fresnel, distance_trace=True)
    d = np.array(out["distance"])
    assert np.all(d[1:] <= d[:-1] * (1 + 1e-12)), d
    assert d[-1] < d[0]
    assert (out["amplitude"] >= 0).all()


def test_starting_scale_changes_nothing_after_the_first_step():
    rng = np.random.default_rng(2)
    t = rng.uniform(0.0, 1.0, (20, 20))
    a0 = rng.uniform(-0.5, 1.0, (20, 20))
    a = gs_amplitude(t, a0, 4)
    b = gs_amplitude(t, 7.0 * a0, 4)
    assert np.allclose(a["nmse"], b["nmse"], rtol=1e-12, atol=0)
    assert np.allclose(a["amplitude"], b["amplitude"], rtol=1e-12, atol=1e-15)
