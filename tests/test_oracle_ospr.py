"""Pins for the oracle's One-Step Phase-Retrieval (oracle/ospr.py).

A 2x2 example worked by hand, the centro-symmetry of the replay of a real
(binary) hologram, Parseval's sum sum I = N_px^2 for +-1 holograms, the
single-subframe case against numpy's inverse FFT, and independence of the
subframe order.  Real/imaginary pairs: a pair with phase theta is the plain
method on the two phases theta and theta - pi/2 (Re(-i G) = Im G), and its
replay keeps the centro-symmetry and the energy of plain OSPR.
"""
import numpy as np

import oracle


def test_worked_2x2_two_subframes():
    t_amp = np.array([[1.0, 1.0], [1.0, 2.0]])
    theta = np.zeros((2, 2, 2))
    theta[1, 1, 1] = np.pi
    out = oracle.ospr(t_amp, theta)
    # subframe 0: G = [[1.25, .25], [.25, .25]] -> h = +1 -> I = [[16, 0], [0, 0]]
    # subframe 1: E_f = [[-2, 1], [1, 1]], G = [[.25, -.75], [-.75, -.75]]
    #             h = [[1, -1], [-1, -1]] -> FFT = [[-2, 2], [2, 2]] -> I = 4
    assert out["levels"].tolist() == [[[0, 0], [0, 0]], [[0, 1], [1, 1]]]
    assert np.allclose(out["intensity"], [[2, 2], [2, 10]], atol=1e-13, rtol=0)
    assert abs(out["nmse"] - 3.0 / 304.0) <= 1e-15


def test_symmetry_energy_and_levels():
    rng = np.random.default_rng(31)
    h, w = 48, 64
    t = np.sqrt(rng.uniform(0, 1, (h, w)))
    th = rng.uniform(0, 2 * np.pi, (3, h, w))
    out = oracle.ospr(t, th)
    i_c = out["intensity"]
    mirrored = i_c[(-np.arange(h)) % h][:, (-np.arange(w)) % w]
    assert np.abs(mirrored - i_c).max() <= 1e-9 * i_c.max()
    n_px = h * w
    assert abs(i_c.sum() - n_px ** 2) <= 1e-12 * n_px ** 2
    assert set(np.unique(out["levels"]).tolist()) <= {0, 1}


def test_single_subframe_matches_library_inverse():
    rng = np.random.default_rng(32)
    h, w = 30, 40
    t = np.sqrt(rng.uniform(0, 1, (h, w)))
    th = rng.uniform(0, 2 * np.pi, (1, h, w))
    out = oracle.ospr(t, th)
    g = np.fft.ifft2(np.fft.ifftshift(t * np.exp(1j * th[0])))
    clear = np.abs(g.real) > 1e-12 * np.abs(g).max()
    assert np.array_equal(out["levels"][0][clear], (g.real < 0)[clear].astype(np.uint8))
    hh = np.where(out["levels"][0] == 0, 1.0, -1.0)
    ref = np.fft.fftshift(np.abs(np.fft.fft2(hh)) ** 2)
    assert np.allclose(out["intensity"], ref, rtol=0, atol=1e-9 * ref.max())


def test_subframe_order_independent():
    rng = np.random.default_rng(33)
    t = np.sqrt(rng.uniform(0, 1, (32, 32)))
    th = rng.uniform(0, 2 * np.pi, (4, 32, 32))
    a = oracle.ospr(t, th)
    b = oracle.ospr(t, th[::-1])
    assert np.allclose(a["intensity"], b["intensity"], rtol=1e-12, atol=1e-9)
    assert abs(a["nmse"] - b["nmse"]) <= 1e-12


def test_pairs_equal_plain_ospr_on_quarter_turned_phases():
    rng = np.random.default_rng(34)
    h, w = 24, 40
    t = np.sqrt(rng.uniform(0, 1, (h, w)))
    th = rng.uniform(0, 2 * np.pi, (3, h, w))
    pairs = oracle.ospr_pairs(t, th)
    expanded = np.stack([p for n in range(3) for p in (th[n], th[n] - np.pi / 2)])
    plain = oracle.ospr(t, expanded)
    assert pairs["levels"].shape == (6, h, w)
    # the two routes round differently only at exact ties
    g = [np.fft.ifft2(np.fft.ifftshift(t * np.exp(1j * th[n]))) for n in range(3)]
    parts = np.stack([p for gn in g for p in (gn.real, gn.imag)])
    clear = np.abs(parts) > 1e-12 * np.abs(parts).max()
    assert np.array_equal(pairs["levels"][clear], plain["levels"][clear])
    assert np.allclose(pairs["intensity"], plain["intensity"], rtol=1e-12, atol=1e-9)
    assert abs(pairs["nmse"] - plain["nmse"]) <= 1e-12


def test_pairs_symmetry_and_energy():
    rng = np.random.default_rng(35)
    h, w = 32, 48
    t = np.sqrt(rng.uniform(0, 1, (h, w)))
    out = oracle.ospr_pairs(t, rng.uniform(0, 2 * np.pi, (2, h, w)))
    i_c = out["intensity"]
    mirrored = i_c[(-np.arange(h)) % h][:, (-np.arange(w)) % w]
    assert np.abs(mirrored - i_c).max() <= 1e-9 * i_c.max()
    assert abs(i_c.sum() - (h * w) ** 2) <= 1e-12 * (h * w) ** 2
