"""Gerchberg-Saxton error-reduction iteration (FP64).

Test infrastructure only.  The paper's HoloGenAlgGSCuda (Sec. 7.3) runs the
GS iteration in the RunIterations() function of an algorithm object that holds
the target, illumination and starting images (Sec. 4, Algorithm Interface).  The
update rule is the textbook one (Gerchberg & Saxton, Optik 35, 1972; Fienup,
Appl. Opt. 21, 1982, error-reduction form):

  T_f   = ifftshift(T_amp)                 target amplitude in FFT order
  H_0   = A * exp(i C(phi_0))              C = identity, or the quantiser
  for k = 0 .. n:
      R_k  = FFT2(Q1 * H_k)                replay field (Q1 = 1 for Fourier)
      nmse[k] = NMSE(|R_k|^2, T_f^2)
      stop if k == n
      R'_k = T_f * R_k / |R_k|             impose the target amplitude
      G_k  = conj(Q1) * IFFT2(R'_k)        back to the SLM plane
      H_{k+1} = A * P(G_k)                 P = phase-only projection or the
                                           L-level quantiser
  phi_n = mod(arg P(G_{n-1}), 2 pi)        (the constrained phi_0 when n = 0)

Q1 is the source chirp of the single-FFT Fresnel transform.  The output chirp,
the prefactor and the centring permutations of the full Fresnel operator are a
unit-modulus replay-plane factor and a permutation: amplitude replacement keeps
them and the inverse removes them, so the loop above reproduces the physical
Fresnel loop exactly (tests/test_oracle_gs.py checks this against optics.py).

The Fienup error E_k = sum (|R_k| - c T_f)^2, c^2 = N_px sum A^2 / sum T_f^2,
is returned on request; for this nearest-point (error-reduction) iteration it
never increases (Fienup 1982).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .dft import fft2, ifft2, ifftshift
from .optics import fresnel_chirp, angular_spectrum
from .constraints import quantise_level, quantise_phase_level, phase_only, replace_amplitude
from .metrics import nmse as nmse_fn

TWO_PI = 2.0 * np.pi


def gs_iterate(target_amp: np.ndarray, phi0: np.ndarray, iterations: int,
               levels: int = 0, illumination: Optional[np.ndarray] = None,
               fresnel: Optional[dict] = None, fienup: bool = False,
               return_back: bool = False, trace: bool = False,
               angular: Optional[dict] = None) -> dict:
    """Run GS from phi0.

    target_amp, phi0: [H][W] real arrays (target in centred order, phase in SLM
    order).  levels: 0 for a continuous phase-only SLM, else L >= 2.
    fresnel: None for a Fourier hologram, else a dict with keys wavelength,
    pitch, distance (metres).  Returns phase [H][W] in [0, 2pi), levels
    [H][W] int64 (or None), nmse list of length iterations+1 and optionally the
    Fienup errors.  return_back adds the last back-propagated field G_{n-1}
    (None when n = 0), from which a caller can tell how close each quantiser
    decision was to a level boundary.  trace (quantised mode) adds, for every
    state k = 0..n, the levels of H_k and the angle that was quantised to get
    them (phi_0 for k = 0, arg G_{k-1} after that).
    angular: instead of fresnel, a dict (wavelength, pitch, distance) for the
    angular-spectrum model: R_k = AS_z(H_k) and G_k = AS_-z(R'_k) on the SLM's
    own grid, with the target in its centred (natural) order, no shift.
    """
    t_amp = np.asarray(target_amp, dtype=np.float64)
    h, w = t_amp.shape
    t_f = t_amp if angular else ifftshift(t_amp)
    t_int = t_f * t_f
    amp = np.ones((h, w)) if illumination is None else np.asarray(illumination, np.float64)
    if fresnel is None:
        q1 = np.ones((h, w), dtype=np.complex128)
    else:
        q1 = np.outer(fresnel_chirp(h, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]),
                      fresnel_chirp(w, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]))

    phi0 = np.asarray(phi0, dtype=np.float64)
    if levels:
        lev = quantise_phase_level(phi0, levels)
        unit = np.exp(1j * lev * (TWO_PI / levels))
    else:
        lev = None
        unit = np.exp(1j * phi0)
    slm = amp * unit
    states = []
    if trace and levels:
        states.append({"levels": lev.astype(np.uint8), "angle": phi0.copy()})

    # |R|^2 sums to N_px sum A^2 through the unnormalised FFT, to sum A^2 through
    # the (unitary) angular-spectrum operator
    c_scale = np.sqrt((1 if angular else h * w) * np.sum(amp * amp) / np.sum(t_f * t_f))
    errors, fienup_err = [], []
    back = None
    if angular:
        forward = lambda f: angular_spectrum(f, +1, angular["wavelength"], angular["pitch"], angular["distance"])
        backward = lambda f: angular_spectrum(f, -1, angular["wavelength"], angular["pitch"], angular["distance"])
    else:
        forward = lambda f: fft2(q1 * f)
        backward = lambda f: np.conj(q1) * ifft2(f)
    for k in range(iterations + 1):
        replay = forward(slm)
        errors.append(nmse_fn(np.abs(replay) ** 2, t_int))
        if fienup:
            fienup_err.append(float(np.sum((np.abs(replay) - c_scale * t_f) ** 2)))
        if k == iterations:
            break
        back = backward(replace_amplitude(replay, t_f))
        if levels:
            lev = quantise_level(back, levels)
            unit = np.exp(1j * lev * (TWO_PI / levels))
            if trace:
                states.append({"levels": lev.astype(np.uint8), "angle": np.angle(back)})
        else:
            unit = phase_only(back)
        slm = amp * unit

    if levels:
        phase = lev * (TWO_PI / levels)
    else:
        phase = np.mod(np.arctan2(unit.imag, unit.real), TWO_PI)
    out = {"phase": phase, "levels": lev, "nmse": errors}
    if fienup:
        out["fienup"] = fienup_err
    if return_back:
        out["back"] = back
    if trace and levels:
        out["trace"] = states
    return out


def gs_multiplane(target_amps, phi0: np.ndarray, iterations: int, planes, levels: int = 0,
                  illumination: Optional[np.ndarray] = None) -> dict:
    """Multi-plane GS, one plane after another.

    Each iteration runs one GS step per replay plane j = 0..P-1 on the same
    SLM state (plane j: Fresnel dict, or None for a Fourier plane):

      R_j = FFT2(Q1_j H);  record NMSE(|R_j|^2, T_j^2)
      H   = A P(conj(Q1_j) IFFT2(T_j R_j / |R_j|))

    nmse holds the error of every step (iterations * P values, plane j of
    iteration k at k * P + j), then the error of the final state at every
    plane (P values).  With one plane this is gs_iterate.
    """
    t_f = [ifftshift(np.asarray(t, dtype=np.float64)) for t in target_amps]
    h, w = t_f[0].shape
    amp = np.ones((h, w)) if illumination is None else np.asarray(illumination, np.float64)
    q1 = []
    for p in planes:
        if p is None:
            q1.append(np.ones((h, w), dtype=np.complex128))
        else:
            q1.append(np.outer(fresnel_chirp(h, p["pitch"], p["wavelength"], p["distance"]),
                               fresnel_chirp(w, p["pitch"], p["wavelength"], p["distance"])))
    phi0 = np.asarray(phi0, dtype=np.float64)
    if levels:
        lev = quantise_phase_level(phi0, levels)
        unit = np.exp(1j * lev * (TWO_PI / levels))
    else:
        lev = None
        unit = np.exp(1j * phi0)
    slm = amp * unit
    errors = []
    for k in range(iterations):
        for j in range(len(planes)):
            replay = fft2(q1[j] * slm)
            errors.append(nmse_fn(np.abs(replay) ** 2, t_f[j] ** 2))
            back = np.conj(q1[j]) * ifft2(replace_amplitude(replay, t_f[j]))
            if levels:
                lev = quantise_level(back, levels)
                unit = np.exp(1j * lev * (TWO_PI / levels))
            else:
                unit = phase_only(back)
            slm = amp * unit
    for j in range(len(planes)):
        errors.append(nmse_fn(np.abs(fft2(q1[j] * slm)) ** 2, t_f[j] ** 2))
    if levels:
        phase = lev * (TWO_PI / levels)
    else:
        phase = np.mod(np.arctan2(unit.imag, unit.real), TWO_PI)
    return {"phase": phase, "levels": lev, "nmse": errors}
