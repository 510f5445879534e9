"""Pins for the oracle's Gerchberg-Saxton loop (oracle/gs.py).

* A 2x2 example worked by hand from the definitions (exact rationals).
* Fienup's theorem: the error-reduction error never increases, for the
  continuous and the nearest-level quantised constraint, Fourier and Fresnel.
* A target consistent with some SLM state is a fixed point with zero NMSE.
* Invariance under scaling of the target and of the illumination.
* The loop with only the source chirp equals the loop built on the full
  physical Fresnel operator (oracle/optics.py, itself pinned by the Gaussian
  beam closed form).
* A very distant Fresnel plane reduces to the Fourier hologram.
"""
import numpy as np
import pytest

import oracle

TWO_PI = 2 * np.pi
FRESNEL = dict(wavelength=532e-9, pitch=8e-6, distance=0.5)


def dft2x2(a, b, c, d):
    """2x2 DFT of [[a, b], [c, d]] written out: signs (-1)^(mk + nl)."""
    return np.array([[a + b + c + d, a - b + c - d], [a + b - c - d, a - b - c + d]])


def test_worked_2x2_continuous():
    # T_amp centred [[1, 0], [1, 2]] -> FFT order T_f = [[2, 1], [0, 1]]
    t_amp = np.array([[1.0, 0.0], [1.0, 2.0]])
    phi0 = np.array([[0.0, np.pi / 2], [0.0, np.pi]])     # H0 = [[1, i], [1, -1]]
    out = oracle.gs_iterate(t_amp, phi0, 1)
    # R0 = [[1+i, 3-i], [1+i, -1-i]], I0 = [[2, 10], [2, 2]]
    # I~ = [[1, 5], [1, 1]]/8, T~ = [[4, 1], [0, 1]]/6 -> nmse0 = (300/576)/(1/2) = 25/24
    assert abs(out["nmse"][0] - 25.0 / 24.0) <= 1e-14
    # R' = [[2s, u], [0, -s]], s = (1+i)/sqrt2, u = (3-i)/sqrt10
    s = (1 + 1j) / np.sqrt(2)
    u = (3 - 1j) / np.sqrt(10)
    g = np.array([[s + u, 3 * s - u], [3 * s + u, s - u]]) / 4
    h1 = g / np.abs(g)
    assert np.allclose(out["phase"], np.mod(np.angle(h1), TWO_PI), atol=1e-14, rtol=0)
    r1 = dft2x2(h1[0, 0], h1[0, 1], h1[1, 0], h1[1, 1])
    i1 = np.abs(r1) ** 2
    tn = np.array([[4.0, 1.0], [0.0, 1.0]]) / 6
    nm1 = np.sum((i1 / i1.sum() - tn) ** 2) / np.sum(tn ** 2)
    assert abs(out["nmse"][1] - nm1) <= 1e-14


def test_worked_2x2_four_levels():
    t_amp = np.array([[1.0, 0.0], [1.0, 2.0]])
    phi0 = np.array([[0.0, np.pi / 2], [0.0, np.pi]])
    out = oracle.gs_iterate(t_amp, phi0, 1, levels=4)
    # angles of G: 0.231, 1.122, 0.531, 1.803 rad -> levels 0, 1, 0, 1
    assert out["levels"].tolist() == [[0, 1], [0, 1]]
    # H1 = [[1, i], [1, i]] -> R1 = [[2+2i, 2-2i], [0, 0]], I~ = [[1, 1], [0, 0]]/2
    # diff^2 sum = 1/6, sum T~^2 = 1/2 -> 1/3
    assert abs(out["nmse"][0] - 25.0 / 24.0) <= 1e-14
    assert abs(out["nmse"][1] - 1.0 / 3.0) <= 1e-14
    assert np.allclose(out["phase"], [[0, np.pi / 2], [0, np.pi / 2]], atol=1e-15)


def synthetic(h, w, seed):
    rng = np.random.default_rng(seed)
    t = np.sqrt(rng.uniform(0, 1, (h, w)))
    t[h // 4: h // 2, w // 3: w // 2] = 1.0
    phi = rng.uniform(0, TWO_PI, (h, w))
    return t, phi


@pytest.mark.parametrize("levels", [0, 8, 4, 2])
@pytest.mark.parametrize("fresnel", [None, FRESNEL])
def test_fienup_error_never_increases(levels, fresnel):
    t, phi = synthetic(48, 80, 3 + levels)
    out = oracle.gs_iterate(t, phi, 25, levels=levels, fresnel=fresnel, fienup=True)
    e = np.array(out["fienup"])
    assert np.all(e[1:] <= e[:-1] * (1 + 1e-12)), e
    assert e[-1] < e[0]
    assert len(out["nmse"]) == 26


@pytest.mark.parametrize("levels", [0, 8])
@pytest.mark.parametrize("fresnel", [None, FRESNEL])
def test_consistent_target_is_fixed_point(levels, fresnel):
    h, w = 32, 40
    rng = np.random.default_rng(21)
    if levels:
        lv = rng.integers(0, levels, (h, w))
        phi_star = lv * TWO_PI / levels
    else:
        phi_star = rng.uniform(0, TWO_PI, (h, w))
    q1 = np.ones((h, w))
    if fresnel:
        c = lambda n: np.exp(1j * np.pi * ((np.arange(n) - n // 2) * fresnel["pitch"]) ** 2
                             / (fresnel["wavelength"] * fresnel["distance"]))
        q1 = np.outer(c(h), c(w))
    t_f = np.abs(np.fft.fft2(q1 * np.exp(1j * phi_star)))
    t_amp = np.fft.fftshift(t_f)
    out = oracle.gs_iterate(t_amp, phi_star, 3, levels=levels, fresnel=fresnel)
    assert max(out["nmse"]) <= 1e-24
    d = np.angle(np.exp(1j * (out["phase"] - phi_star)))
    assert np.abs(d).max() <= 1e-10


def test_scale_invariance():
    t, phi = synthetic(40, 40, 5)
    a = oracle.gs_iterate(t, phi, 8, levels=8)
    b = oracle.gs_iterate(3.7 * t, phi, 8, levels=8, illumination=np.full(t.shape, 0.25))
    assert np.array_equal(a["levels"], b["levels"])
    assert np.allclose(a["nmse"], b["nmse"], rtol=1e-12, atol=0)


def test_iterations_zero_returns_constrained_start():
    t, phi = synthetic(16, 24, 6)
    out = oracle.gs_iterate(t, phi, 0, levels=4)
    assert len(out["nmse"]) == 1
    assert np.array_equal(out["levels"], oracle.quantise_phase_level(phi, 4))
    out = oracle.gs_iterate(t, phi, 0)
    assert np.allclose(out["phase"], np.mod(phi, TWO_PI), atol=1e-14)


@pytest.mark.parametrize("levels", [0, 8])
def test_shortcut_equals_physical_fresnel_loop(levels):
    """GS on the full Fresnel operator (both chirps, prefactor, centring)."""
    h, w = 64, 48
    t, phi = synthetic(h, w, 7)
    kw = dict(fresnel=True, **FRESNEL)
    if levels:
        slm = np.exp(1j * oracle.quantise_phase_level(phi, levels) * TWO_PI / levels)
    else:
        slm = np.exp(1j * phi)
    nm = []
    for k in range(6):
        replay = oracle.propagate(slm, +1, **kw)          # centred replay plane
        nm.append(oracle.nmse(np.abs(replay) ** 2, t * t))
        if k == 5:
            break
        back = oracle.propagate(t * replay / np.abs(replay), -1, **kw)
        if levels:
            slm = np.exp(1j * oracle.quantise_level(back, levels) * TWO_PI / levels)
        else:
            slm = back / np.abs(back)
    out = oracle.gs_iterate(t, phi, 5, levels=levels, fresnel=FRESNEL)
    assert np.allclose(out["nmse"], nm, rtol=1e-10, atol=0)
    d = np.angle(slm * np.exp(-1j * out["phase"]))
    assert np.abs(d).max() <= 1e-9


def test_distant_fresnel_plane_is_fourier():
    t, phi = synthetic(32, 32, 8)
    far = dict(wavelength=532e-9, pitch=8e-6, distance=1e9)
    a = oracle.gs_iterate(t, phi, 6)
    b = oracle.gs_iterate(t, phi, 6, fresnel=far)
    assert np.allclose(a["nmse"], b["nmse"], rtol=1e-6, atol=0)


def test_trace_matches_separate_runs():
    t, phi = synthetic(24, 40, 12)
    full = oracle.gs_iterate(t, phi, 4, levels=8, trace=True)
    assert len(full["trace"]) == 5
    for k in (0, 2, 4):
        part = oracle.gs_iterate(t, phi, k, levels=8)
        assert np.array_equal(full["trace"][k]["levels"], part["levels"])
    assert np.array_equal(full["trace"][0]["angle"], phi)


# ---------------------------------------------------------------------------
# multi-plane GS, one plane after another
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("levels", [0, 4])
def test_multiplane_with_one_plane_is_gs(levels):
    t, phi = synthetic(24, 40, 13)
    a = oracle.gs_multiplane([t], phi, 6, [FRESNEL], levels=levels)
    b = oracle.gs_iterate(t, phi, 6, levels=levels, fresnel=FRESNEL)
    assert a["nmse"] == b["nmse"]
    assert np.array_equal(a["phase"], b["phase"])


@pytest.mark.parametrize("levels", [0, 8])
def test_multiplane_with_a_repeated_plane_is_gs_with_twice_the_iterations(levels):
    t, phi = synthetic(32, 24, 14)
    a = oracle.gs_multiplane([t, t], phi, 5, [FRESNEL, FRESNEL], levels=levels)
    b = oracle.gs_iterate(t, phi, 10, levels=levels, fresnel=FRESNEL)
    assert a["nmse"][:10] == b["nmse"][:10]
    assert a["nmse"][10] == a["nmse"][11] == b["nmse"][10]
    assert np.array_equal(a["phase"], b["phase"])


def test_multiplane_consistent_targets_are_a_fixed_point():
    h, w = 20, 24
    rng = np.random.default_rng(15)
    phi = rng.uniform(0, TWO_PI, (h, w))
    planes = [FRESNEL, dict(FRESNEL, distance=0.4), None]
    targets = []
    for p in planes:
        q1 = oracle.source_chirp(h, w, p)
        targets.append(np.fft.fftshift(np.abs(np.fft.fft2(q1 * np.exp(1j * phi)))))
    out = oracle.gs_multiplane(targets, phi, 3, planes)
    assert max(out["nmse"]) <= 1e-24
    assert np.abs(np.angle(np.exp(1j * (out["phase"] - phi)))).max() <= 1e-10


def test_multiplane_final_errors_are_the_physical_ones():
    h, w = 16, 20
    t1, phi = synthetic(h, w, 16)
    t2, _ = synthetic(h, w, 17)
    planes = [FRESNEL, dict(FRESNEL, distance=0.45)]
    out = oracle.gs_multiplane([t1, t2], phi, 4, planes, levels=8)
    slm = np.exp(1j * out["phase"])
    for j, (t, p) in enumerate(zip((t1, t2), planes)):
        replay = oracle.propagate(slm, +1, fresnel=True, **p)
        assert abs(out["nmse"][8 + j] - oracle.nmse(np.abs(replay) ** 2, t * t)) <= 1e-12


ANGULAR = dict(wavelength=532e-9, pitch=8e-6, distance=0.05)


@pytest.mark.parametrize("levels", [0, 8])
def test_angular_spectrum_gs_fienup_error_never_increases(levels):
    t, phi = synthetic(40, 48, 18)
    out = oracle.gs_iterate(t, phi, 20, levels=levels, angular=ANGULAR, fienup=True)
    e = np.array(out["fienup"])
    assert np.all(e[1:] <= e[:-1] * (1 + 1e-12)), e
    assert e[-1] < e[0]


def test_angular_spectrum_gs_consistent_target_is_a_fixed_point():
    h, w = 24, 32
    rng = np.random.default_rng(19)
    phi = rng.uniform(0, TWO_PI, (h, w))
    t = np.abs(oracle.angular_spectrum(np.exp(1j * phi), +1, **ANGULAR))   # natural order, no shift
    out = oracle.gs_iterate(t, phi, 3, angular=ANGULAR)
    assert max(out["nmse"]) <= 1e-24
    assert np.abs(np.angle(np.exp(1j * (out["phase"] - phi)))).max() <= 1e-10


# ---------------------------------------------------------------------------
# non-uniform illumination A (the SLM amplitude the constraint keeps)
# ---------------------------------------------------------------------------
def test_worked_2x2_four_levels_with_illumination():
    """Hand-worked L = 4 case with A = [[2, 1], [1, 1]]; dropping A from the
    constraint or squaring it changes every value below."""
    t_amp = np.array([[1.0, 0.0], [1.0, 2.0]])            # FFT order T_f = [[2, 1], [0, 1]]
    phi0 = np.array([[0.0, np.pi / 2], [np.pi, 0.0]])     # H0 = A exp(i phi0) = [[2, i], [-1, 1]]
    amp = np.array([[2.0, 1.0], [1.0, 1.0]])
    out = oracle.gs_iterate(t_amp, phi0, 1, levels=4, illumination=amp)
    # R0 = [[2+i, -i], [2+i, 4-i]], I0 = [[5, 1], [5, 17]] (sum 28 = 4 sum A^2);
    # against T~ = [[4, 1], [0, 1]]/6: differences (-41, -11, 15, 37)/84
    # -> 3396/7056 / (1/2) = 283/294
    assert abs(out["nmse"][0] - 283.0 / 294.0) <= 1e-14
    # G = IFFT2(T_f R0/|R0|) has angles -0.126, 1.205, 0.166, 0.539 rad
    # -> levels [[0, 1], [0, 0]], H1 = [[2, i], [1, 1]]
    assert out["levels"].tolist() == [[0, 1], [0, 0]]
    # R1 = [[4+i, 2-i], [i, 2-i]], I1 = [[17, 5], [1, 5]]: differences (-5, 1, 3, 1)/84
    # -> 36/7056 / (1/2) = 1/98
    assert abs(out["nmse"][1] - 1.0 / 98.0) <= 1e-14


def gaussian_illumination(h, w, waist=0.35):
    y = (np.arange(h) - h / 2 + 0.5) / (waist * h)
    x = (np.arange(w) - w / 2 + 0.5) / (waist * w)
    return np.exp(-(y[:, None] ** 2 + x[None, :] ** 2))


@pytest.mark.parametrize("levels", [0, 8])
@pytest.mark.parametrize("fresnel", [None, FRESNEL])
def test_consistent_target_with_illumination_is_fixed_point(levels, fresnel):
    """T = |FFT2(Q1 A exp(i phi*))| with a Gaussian A: zero NMSE and phi* kept.
    The loop without A, or with A squared, sees a different replay field."""
    h, w = 32, 40
    rng = np.random.default_rng(22)
    amp = gaussian_illumination(h, w)
    if levels:
        phi_star = rng.integers(0, levels, (h, w)) * TWO_PI / levels
    else:
        phi_star = rng.uniform(0, TWO_PI, (h, w))
    q1 = oracle.source_chirp(h, w, fresnel)
    t_amp = np.fft.fftshift(np.abs(np.fft.fft2(q1 * amp * np.exp(1j * phi_star))))
    out = oracle.gs_iterate(t_amp, phi_star, 3, levels=levels, fresnel=fresnel, illumination=amp)
    assert max(out["nmse"]) <= 1e-24
    assert np.abs(np.angle(np.exp(1j * (out["phase"] - phi_star)))).max() <= 1e-10
    # the same target without the illumination is far from consistent
    plain = oracle.gs_iterate(t_amp, phi_star, 0, levels=levels, fresnel=fresnel)
    assert plain["nmse"][0] > 1e-3


@pytest.mark.parametrize("levels", [0, 8, 2])
@pytest.mark.parametrize("fresnel", [None, FRESNEL])
def test_fienup_error_never_increases_with_illumination(levels, fresnel):
    """Error reduction with A non-uniform: the SLM projection A P(G) is still
    the nearest point of its set, so the Fienup error stays monotone."""
    t, phi = synthetic(40, 48, 31 + levels)
    amp = 0.2 + gaussian_illumination(40, 48)
    out = oracle.gs_iterate(t, phi, 20, levels=levels, fresnel=fresnel, fienup=True, illumination=amp)
    e = np.array(out["fienup"])
    assert np.all(e[1:] <= e[:-1] * (1 + 1e-12)), e
    assert e[-1] < e[0]


def test_multiplane_with_illumination_consistent_targets_are_a_fixed_point():
    h, w = 20, 24
    rng = np.random.default_rng(23)
    phi = rng.uniform(0, TWO_PI, (h, w))
    amp = 0.3 + gaussian_illumination(h, w)
    planes = [FRESNEL, dict(FRESNEL, distance=0.4), None]
    targets = [np.fft.fftshift(np.abs(np.fft.fft2(oracle.source_chirp(h, w, p) * amp * np.exp(1j * phi))))
               for p in planes]
    out = oracle.gs_multiplane(targets, phi, 3, planes, illumination=amp)
    assert max(out["nmse"]) <= 1e-24
    assert np.abs(np.angle(np.exp(1j * (out["phase"] - phi)))).max() <= 1e-10
    bare = oracle.gs_multiplane(targets, phi, 0, planes)
    assert min(bare["nmse"]) > 1e-3


@pytest.mark.parametrize("levels", [0, 4])
def test_multiplane_with_illumination_and_one_plane_is_gs(levels):
    """gs_iterate is pinned with A by the hand-worked case and the fixed point."""
    t, phi = synthetic(24, 32, 24)
    amp = 0.1 + gaussian_illumination(24, 32)
    a = oracle.gs_multiplane([t], phi, 5, [FRESNEL], levels=levels, illumination=amp)
    b = oracle.gs_iterate(t, phi, 5, levels=levels, fresnel=FRESNEL, illumination=amp)
    assert a["nmse"] == b["nmse"]
    assert np.array_equal(a["phase"], b["phase"])
