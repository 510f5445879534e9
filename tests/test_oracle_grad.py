"""Pins for the oracle's gradient-descent hologram method (oracle/grad.py).

* A 1x2 Fourier hologram worked by hand: the loss and both partial derivatives
  in closed form.
* FP64 central finite differences of the loss at every pixel of small frames,
  for Fourier and Fresnel planes together.
* Global-phase invariance: the gradient sums to zero.
* A target consistent with some phase is a zero of the loss and its gradient.
* The loss built on the Q1-only shortcut equals the NMSE of the physical
  Fresnel operator (optics.propagate: both chirps, prefactor, centring).
* Adam's bias correction: under a constant gradient every step moves each
  pixel by lr * g / (|g| + eps).
"""
import numpy as np
import pytest

import oracle

FRESNEL = dict(wavelength=532e-9, pitch=8e-6, distance=0.5)


def random_problem(h, w, planes, seed):
    rng = np.random.default_rng(seed)
    targets = [np.sqrt(rng.uniform(0.0, 1.0, (h, w))) for _ in planes]
    phi = rng.uniform(0.0, 2 * np.pi, (h, w))
    return phi, targets


def test_worked_1x2_fourier():
    a, b = 0.3, 1.9
    t0, t1 = 0.7, 0.2                      # target intensity in FFT order
    amp_centred = np.sqrt(np.array([[t1, t0]]))   # ifftshift of a length-2 axis swaps
    loss, g, _ = oracle.loss_and_gradient(np.array([[a, b]]), [amp_centred], [None])
    c = np.cos(a - b)
    i_n = np.array([(1 + c) / 2, (1 - c) / 2])     # I = (2 + 2c, 2 - 2c), sum 4
    t_n = np.array([t0, t1]) / (t0 + t1)
    d = np.sum(t_n ** 2)
    assert abs(loss - np.sum((i_n - t_n) ** 2) / d) <= 1e-15
    dl_dc = ((i_n[0] - t_n[0]) - (i_n[1] - t_n[1])) / d
    s = np.sin(a - b)
    assert np.allclose(g, [[-s * dl_dc, s * dl_dc]], rtol=0, atol=1e-15)


@pytest.mark.parametrize("h,w,planes", [
    (12, 16, [None]),
    (16, 12, [FRESNEL]),
    (10, 14, [FRESNEL, dict(FRESNEL, distance=0.4), None]),
])
def test_gradient_matches_central_differences(h, w, planes):
    phi, targets = random_problem(h, w, planes, seed=h * w)
    _, g, _ = oracle.loss_and_gradient(phi, targets, planes)
    step = 1e-5
    fd = np.zeros_like(phi)
    for k in range(phi.size):
        e = np.zeros(phi.size)
        e[k] = step
        e = e.reshape(phi.shape)
        lp = oracle.loss_and_gradient(phi + e, targets, planes, want_grad=False)[0]
        lm = oracle.loss_and_gradient(phi - e, targets, planes, want_grad=False)[0]
        fd.flat[k] = (lp - lm) / (2 * step)
    assert np.abs(fd - g).max() <= 1e-6 * np.abs(g).max()


def test_gradient_sums_to_zero():
    planes = [FRESNEL, None]
    phi, targets = random_problem(24, 20, planes, seed=5)
    _, g, _ = oracle.loss_and_gradient(phi, targets, planes)
    assert abs(g.sum()) <= 1e-12 * np.abs(g).sum()


@pytest.mark.parametrize("planes", [[None], [FRESNEL, FRESNEL]])
def test_consistent_target_is_a_zero(planes):
    h, w = 16, 20
    rng = np.random.default_rng(11)
    phi = rng.uniform(0, 2 * np.pi, (h, w))
    targets = []
    for p in planes:
        q1 = np.ones((h, w)) if p is None else np.outer(
            oracle.fresnel_chirp(h, p["pitch"], p["wavelength"], p["distance"]),
            oracle.fresnel_chirp(w, p["pitch"], p["wavelength"], p["distance"]))
        targets.append(np.fft.fftshift(np.abs(np.fft.fft2(q1 * np.exp(1j * phi)))))
    loss, g, per = oracle.loss_and_gradient(phi, targets, planes)
    assert loss <= 1e-26 and max(per) <= 1e-26
    assert np.abs(g).max() <= 1e-10


def test_loss_equals_physical_fresnel_nmse():
    h, w = 20, 24
    phi, targets = random_problem(h, w, [FRESNEL], seed=3)
    loss, _, _ = oracle.loss_and_gradient(phi, targets, [FRESNEL], want_grad=False)
    replay = oracle.propagate(np.exp(1j * phi), +1, fresnel=True, **FRESNEL)   # centred
    assert abs(loss - oracle.nmse(np.abs(replay) ** 2, targets[0] ** 2)) <= 1e-13


def test_adam_constant_gradient_steps_are_lr_sign():
    rng = np.random.default_rng(2)
    phi = rng.uniform(0, 1, (4, 5))
    g = rng.normal(size=(4, 5))
    m = np.zeros_like(phi)
    v = np.zeros_like(phi)
    lr, eps = 0.05, 1e-8
    for t in range(1, 6):
        new, m, v = oracle.adam_update(phi, m, v, g, t, lr, eps=eps)
        assert np.allclose(phi - new, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
        phi = new


def test_descent_reduces_loss_and_reports_every_state():
    planes = [FRESNEL]
    phi, targets = random_problem(32, 32, planes, seed=9)
    out = oracle.grad_descent(phi, targets, planes, steps=15, lr=0.05)
    assert len(out["loss"]) == 16
    assert out["loss"][-1] < 0.7 * out["loss"][0]
    first = oracle.loss_and_gradient(phi, targets, planes, want_grad=False)[0]
    assert out["loss"][0] == first
    last = oracle.loss_and_gradient(out["phase"], targets, planes, want_grad=False)[0]
    assert out["loss"][-1] == last


def test_gradient_matches_central_differences_at_64x64_three_planes():
    """The gradient workload's own geometry at 64x64: Fresnel planes at 0.40,
    0.45 and 0.50 m (532 nm, 8 um), its seeded synthetic targets (200 + j) and
    starting phase (300); FP64 central differences at every pixel."""
    from paper_2006_10509_amd import workloads as wl
    h = w = 64
    planes = [dict(wavelength=532e-9, pitch=8e-6, distance=z) for z in (0.40, 0.45, 0.50)]
    targets = [wl.target_amplitude(h, w, 200 + j).astype(np.float64) for j in range(3)]
    phi = wl.uniform_phase(h, w, 300).astype(np.float64)
    loss, g, _ = oracle.loss_and_gradient(phi, targets, planes)
    step = 1e-5
    fd = np.zeros_like(phi)
    for k in range(phi.size):
        e = np.zeros(phi.size)
        e[k] = step
        e = e.reshape(phi.shape)
        lp = oracle.loss_and_gradient(phi + e, targets, planes, want_grad=False)[0]
        lm = oracle.loss_and_gradient(phi - e, targets, planes, want_grad=False)[0]
        fd.flat[k] = (lp - lm) / (2 * step)
    assert np.abs(fd - g).max() <= 1e-6 * np.abs(g).max()
    assert np.linalg.norm(fd - g) <= 1e-7 * np.linalg.norm(g)
