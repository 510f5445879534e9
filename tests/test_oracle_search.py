"""Pins for the oracle's single-pixel search (oracle/search.py).

* The error of every binary 2x2 hologram, from a 2x2 DFT written out by hand.
* Direct binary search never raises the error, accepts exactly the trials
  that lower it, and a sweep without acceptances ends in a state that no
  single-pixel change improves (checked by brute force).
* Annealing at a vanishing temperature decides as direct search; at a huge
  temperature it accepts every trial.
* A trial that keeps a pixel's level changes nothing.
* With Fresnel planes the error is the NMSE of the physical operator.
"""
import itertools

import numpy as np

import oracle

FRESNEL = dict(wavelength=532e-9, pitch=8e-6, distance=0.5)


def hand_error_2x2(bits, t_fft):
    """NMSE of the binary 2x2 hologram bits (0 -> +1, 1 -> -1) against the
    target intensity t_fft given in FFT order, DFT signs (-1)^(mk + nl)."""
    a, b, c, d = [1.0 - 2.0 * v for v in bits]
    r = np.array([[a + b + c + d, a - b + c - d], [a + b - c - d, a - b - c + d]])
    i = r * r
    i_n, t_n = i / i.sum(), t_fft / t_fft.sum()
    return np.sum((i_n - t_n) ** 2) / np.sum(t_n ** 2)


def test_every_binary_2x2_state_against_a_hand_dft():
    t_fft = np.array([[4.0, 1.0], [2.0, 0.5]])
    t_amp_centred = np.sqrt(np.fft.fftshift(t_fft))
    for bits in itertools.product((0, 1), repeat=4):
        lev0 = np.array(bits).reshape(2, 2)
        out = oracle.pixel_search(t_amp_centred, lev0, 2, [])
        assert abs(out["nmse"][0] - hand_error_2x2(bits, t_fft)) <= 1e-14


def problem(h, w, levels, seed, n_trials):
    rng = np.random.default_rng(seed)
    t = np.sqrt(rng.uniform(0, 1, (h, w)))
    lev0 = rng.integers(0, levels, (h, w))
    pix = rng.integers(0, h * w, n_trials)
    cand = (lev0.ravel()[pix] + rng.integers(1, levels, n_trials)) % levels if levels > 2 else None
    return t, lev0, pix, cand, rng


def test_direct_search_is_monotone_and_ends_in_a_local_minimum():
    h, w, levels = 4, 4, 2
    t, lev, _, _, _ = problem(h, w, levels, 1, 0)
    for sweep in range(20):
        # one trial at a time, so that each flip starts from the current level
        accepted_any = False
        for p in range(h * w):
            flip = 1 - lev.ravel()[p]
            o = oracle.pixel_search(t, lev, levels, [(p, flip)])
            assert o["nmse"][1] <= o["nmse"][0]
            assert o["accepted"][0] == (o["dE"][0] < 0)
            lev = o["levels"].astype(np.int64)
            accepted_any |= bool(o["accepted"][0])
        if not accepted_any:
            break
    assert not accepted_any
    base = oracle.pixel_search(t, lev, levels, [])["nmse"][0]
    for p in range(h * w):
        other = lev.copy().ravel()
        other[p] = 1 - other[p]
        assert oracle.pixel_search(t, other.reshape(h, w), levels, [])["nmse"][0] >= base


def test_sequence_monotone_for_direct_search_four_levels():
    t, lev0, pix, cand, _ = problem(8, 6, 4, 2, 120)
    out = oracle.pixel_search(t, lev0, 4, list(zip(pix, cand)))
    e = np.array(out["nmse"])
    assert np.all(e[1:] <= e[:-1])
    assert np.array_equal(out["accepted"], out["dE"] < 0)
    assert e[-1] < e[0]


def test_annealing_limits():
    t, lev0, pix, cand, rng = problem(6, 8, 4, 3, 80)
    trials = list(zip(pix, cand))
    u = rng.uniform(0, 1, len(trials))
    ds = oracle.pixel_search(t, lev0, 4, trials)
    cold = oracle.pixel_search(t, lev0, 4, trials, temperature=[1e-300] * len(trials), uniform=u)
    # a trial whose candidate is already the pixel's level (dE = 0) is accepted
    # by the Metropolis rule and rejected by direct search: both keep the map
    moved = ds["dE"] != 0.0
    assert np.array_equal(cold["accepted"][moved], ds["accepted"][moved])
    assert np.array_equal(cold["levels"], ds["levels"])
    hot = oracle.pixel_search(t, lev0, 4, trials, temperature=[1e300] * len(trials), uniform=u)
    assert hot["accepted"].all()


def test_keeping_a_level_is_a_no_op():
    t, lev0, _, _, _ = problem(4, 4, 2, 4, 0)
    out = oracle.pixel_search(t, lev0, 2, [(5, lev0.ravel()[5])])
    assert out["dE"][0] == 0.0 and not out["accepted"][0]
    assert np.array_equal(out["levels"], lev0)


def test_fresnel_error_is_the_physical_nmse():
    t, lev0, pix, _, _ = problem(12, 10, 2, 5, 30)
    trials = [(p, 1 - lev0.ravel()[p]) for p in pix]
    out = oracle.pixel_search(t, lev0, 2, trials, fresnel=FRESNEL)
    field = np.exp(1j * np.pi * out["levels"])
    replay = oracle.propagate(field, +1, fresnel=True, **FRESNEL)
    assert abs(out["nmse"][-1] - oracle.nmse(np.abs(replay) ** 2, t ** 2)) <= 1e-12
