"""Pins for the oracle's constraints (oracle/constraints.py) and NMSE
(oracle/metrics.py): brute-force nearest level on the circle, the exact
sign/magnitude rule for four levels, idempotence, and closed-form NMSE values.
"""
import numpy as np
import pytest

import oracle

TWO_PI = 2 * np.pi


@pytest.mark.parametrize("levels", [2, 3, 4, 5, 8, 16, 256])
def test_quantiser_is_nearest_level_on_circle(levels):
    rng = np.random.default_rng(levels)
    g = rng.standard_normal(20000) + 1j * rng.standard_normal(20000)
    got = oracle.quantise_level(g, levels)
    theta = np.arctan2(g.imag, g.real)
    cand = np.exp(1j * TWO_PI * np.arange(levels) / levels)
    dist = np.abs(np.exp(1j * theta)[:, None] - cand[None, :])
    best = np.argmin(dist, axis=1)
    srt = np.sort(dist, axis=1)
    clear = srt[:, 1] - srt[:, 0] > 1e-9          # exclude exact ties
    assert np.array_equal(got[clear], best[clear])
    assert got.min() >= 0 and got.max() < levels


def test_quantiser_four_levels_sign_rule():
    rng = np.random.default_rng(44)
    g = rng.standard_normal(50000) + 1j * rng.standard_normal(50000)
    re, im = g.real, g.imag
    # nearest of {1, i, -1, -i}: dominant component and its sign
    rule = np.where(np.abs(re) > np.abs(im), np.where(re > 0, 0, 2), np.where(im > 0, 1, 3))
    clear = np.abs(np.abs(re) - np.abs(im)) > 1e-12
    assert np.array_equal(oracle.quantise_level(g, 4)[clear], rule[clear])


@pytest.mark.parametrize("levels", [2, 4, 8, 7])
def test_quantiser_idempotent_and_zero(levels):
    lv = np.arange(levels)
    on = 3.0 * np.exp(1j * TWO_PI * lv / levels)
    assert np.array_equal(oracle.quantise_level(on, levels), lv)
    assert oracle.quantise_level(np.array([0j]), levels)[0] == 0
    # phase-domain form agrees on and off the circle
    assert np.array_equal(oracle.quantise_phase_level(TWO_PI * lv / levels, levels), lv)
    assert oracle.quantise_phase_level(np.array([TWO_PI]), levels)[0] == 0
    assert oracle.quantise_phase_level(np.array([-TWO_PI / levels]), levels)[0] == levels - 1


def test_quantiser_tie_goes_up():
    # exactly half-way between level 0 and level 1 of L = 4 (angle pi/4)
    assert oracle.quantise_phase_level(np.array([np.pi / 4]), 4)[0] == 1


def test_phase_only_projection():
    rng = np.random.default_rng(9)
    g = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    g[0] = 0
    p = oracle.phase_only(g)
    assert np.allclose(np.abs(p), 1.0, atol=1e-15)
    assert p[0] == 1
    assert np.allclose(np.angle(p[1:]), np.angle(g[1:]), atol=1e-15)
    assert np.allclose(oracle.phase_only(p), p, atol=1e-15)


def test_amplitude_replacement():
    rng = np.random.default_rng(10)
    r = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    t = rng.uniform(0, 2, 1000)
    r[5] = 0
    out = oracle.replace_amplitude(r, t)
    assert np.allclose(np.abs(out), t, atol=1e-15)
    nz = np.arange(1000) != 5
    assert np.allclose(np.angle(out[nz]), np.angle(r[nz]), atol=1e-14)
    assert out[5] == t[5]
    assert np.allclose(oracle.replace_amplitude(out, t), out, atol=1e-15)


def test_binarise_sign_of_real_part():
    g = np.array([1 + 5j, -1e-300 + 0j, 0.0 - 1j, -0.0 + 2j, -3 + 0j])
    assert np.array_equal(oracle.binarise(g), [1, -1, 1, 1, -1])


def test_nmse_closed_forms():
    rng = np.random.default_rng(11)
    t = rng.uniform(0, 1, (32, 32))
    assert oracle.nmse(7.5 * t, t) <= 1e-28
    # constant intensity: 1 - 1 / (N sum T~^2), T~ = T / sum T
    tn = t / t.sum()
    expected = 1.0 - 1.0 / (t.size * np.sum(tn * tn))
    assert abs(oracle.nmse(np.full_like(t, 3.0), t) - expected) <= 1e-14
    # two pixels, worked by hand: I = (1, 3), T = (1, 1)
    # I~ = (1/4, 3/4), T~ = (1/2, 1/2): sum d^2 = 1/8, sum T~^2 = 1/2 -> 1/4
    assert abs(oracle.nmse(np.array([1.0, 3.0]), np.array([1.0, 1.0])) - 0.25) <= 1e-15
