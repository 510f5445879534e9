"""Gerchberg-Saxton with a signal window in the replay plane (FP64).

Test infrastructure only.  The paper's application lets the user draw masks
over the images it handles (Sec. 7.1, HoloGenUIMask; Sec. 7.2,
HoloGenMaskOptions) but does not say how a mask enters the iteration.  The
reading used here is the signal-window (free-region) form of error reduction
(Fienup, Appl. Opt. 21, 1982, object constraints on a support; Wyrowski &
Bryngdahl, JOSA A 5, 1988, iterative Fourier-transform design with a signal
window): the target amplitude is imposed only inside the window W, the rest
of the replay plane keeps whatever light the hologram sends there, and the
error is measured inside W only.

  T_f  = ifftshift(T_amp),  M = ifftshift(window) != 0          (FFT order)
  c    = sqrt(N_px sum A^2 / sum_M T_f^2)      target at the field's energy
  H_0  = A exp(i C(phi_0))                     as in gs_iterate
  for k = 0 .. n:
      R_k  = FFT2(Q1 H_k)
      nmse[k] = NMSE over M:  sum_M (I/sum_M I - T/sum_M T)^2 / sum_M (T/sum_M T)^2,
                I = |R_k|^2, T = T_f^2
      stop if k == n
      R'_k = c T_f R_k / |R_k| on M (c T_f where R_k = 0),  R_k off M
      H_{k+1} = A P(conj(Q1) IFFT2(R'_k))

The scale c puts the window's target at the energy the SLM field carries
through the unnormalised FFT (sum |R_k|^2 = N_px sum A^2, Parseval), so R'_k
is the nearest point of the set {R : |R| = c T_f on M} and the loop is an
alternation of nearest-point projections: the Fienup error
E_k = sum_M (|R_k| - c T_f)^2 never increases.  Without the window (M = the
whole frame) c only rescales R'_k, which the SLM projection ignores, so the
loop is gs_iterate.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .dft import fft2, ifft2, ifftshift
from .optics import fresnel_chirp
from .constraints import quantise_level, quantise_phase_level, phase_only
from .metrics import nmse as nmse_fn

TWO_PI = 2.0 * np.pi


def window_nmse(intensity: np.ndarray, target_intensity: np.ndarray, inside: np.ndarray) -> float:
    """NMSE of the pixels where `inside` is true (both arrays in one order)."""
    m = np.asarray(inside, dtype=bool)
    i = np.asarray(intensity, dtype=np.float64)[m]
    if i.sum() == 0.0:
        return 1.0   # no light in the window: every normalised difference is -T/sum T
    return nmse_fn(i, np.asarray(target_intensity, dtype=np.float64)[m])


def gs_window(target_amp: np.ndarray, window: np.ndarray, phi0: np.ndarray, iterations: int,
              levels: int = 0, illumination: Optional[np.ndarray] = None,
              fresnel: Optional[dict] = None, fienup: bool = False, trace: bool = False) -> dict:
    """Signal-window GS from phi0.

    target_amp and window are [H][W] in centred replay order (window: nonzero
    inside); phi0 and illumination in SLM order.  levels, fresnel and the
    returned phase / levels / nmse as in gs_iterate; fienup adds the errors
    E_k; trace (quantised mode) adds, for every state, the level map and the
    angle that was quantised to get it.
    """
    t_f = ifftshift(np.asarray(target_amp, dtype=np.float64))
    inside = ifftshift(np.asarray(window) != 0)
    h, w = t_f.shape
    amp = np.ones((h, w)) if illumination is None else np.asarray(illumination, np.float64)
    if fresnel is None:
        q1 = np.ones((h, w), dtype=np.complex128)
    else:
        q1 = np.outer(fresnel_chirp(h, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]),
                      fresnel_chirp(w, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]))
    c = np.sqrt(h * w * np.sum(amp * amp) / np.sum(t_f[inside] ** 2))

    phi0 = np.asarray(phi0, dtype=np.float64)
    if levels:
        lev = quantise_phase_level(phi0, levels)
        unit = np.exp(1j * lev * (TWO_PI / levels))
    else:
        lev = None
        unit = np.exp(1j * phi0)
    slm = amp * unit
    states = [{"levels": lev.astype(np.uint8), "angle": phi0.copy()}] if (trace and levels) else []
    errors, fienup_err = [], []
    for k in range(iterations + 1):
        replay = fft2(q1 * slm)
        errors.append(window_nmse(np.abs(replay) ** 2, t_f * t_f, inside))
        if fienup:
            fienup_err.append(float(np.sum((np.abs(replay[inside]) - c * t_f[inside]) ** 2)))
        if k == iterations:
            break
        imposed = np.where(inside, c * t_f * phase_only(replay), replay)
        back = np.conj(q1) * ifft2(imposed)
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
    if trace and levels:
        out["trace"] = states
    return out
