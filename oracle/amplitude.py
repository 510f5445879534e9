"""Gerchberg-Saxton for an amplitude-only SLM (FP64).

Test infrastructure only.  The paper's SLM options name the SLM type and
multi-amplitude SLMs (Sec. 3.2, SLMTypeOption, MultiAmpSLM) without defining
either.  The reading used here is the continuous amplitude-only modulator
under uniform illumination: the SLM field is a real a >= 0, and the
SLM-plane constraint is the nearest point of that set, the non-negative real
part,

    P(G) = max(Re G, 0)

(the object-domain non-negativity constraint of error reduction; Fienup,
Appl. Opt. 21, 1982).  The loop is that of gs_iterate with P in place of the
phase-only projection:

  T_f  = ifftshift(T_amp)
  a_0  = P(a_in)
  for k = 0 .. n:
      R_k  = FFT2(Q1 a_k);  nmse[k] = NMSE(|R_k|^2, T_f^2) with sum I summed
                            (the SLM field's energy changes from state to
                            state, so there is no Parseval shortcut)
      stop if k == n
      a_{k+1} = P(conj(Q1) IFFT2(T_f R_k / |R_k|))    (IFFT2 with its 1/N_px)
  returns a_n.

With the unnormalised FFT2 forward and the normalised IFFT2 back, P is the
nearest point of {FFT2(Q1 a) : a >= 0} to the replaced replay field, and the
replacement is the nearest point of {|R| = T_f}; both steps are nearest-point
projections, so the replay-plane distance D_k = ||R_k - T_f R_k/|R_k|||
never increases (Fienup 1982).  P is equivariant under positive scaling, so
the iterates after the first do not depend on the scale of a_in.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .dft import fft2, ifft2, ifftshift
from .optics import fresnel_chirp
from .constraints import replace_amplitude
from .metrics import nmse as nmse_fn


def nonnegative_real(g: np.ndarray) -> np.ndarray:
    """Nearest non-negative real value: max(Re G, 0)."""
    return np.maximum(np.asarray(g, dtype=np.complex128).real, 0.0)


def gs_amplitude(target_amp: np.ndarray, a0: np.ndarray, iterations: int,
                 fresnel: Optional[dict] = None, distance_trace: bool = False) -> dict:
    """Amplitude-only GS from the starting amplitude a0 (SLM order).

    target_amp: [H][W] centred; fresnel as in gs_iterate.  Returns the SLM
    amplitude a_n of the last state, the NMSE of every state and, on
    request, the replay-plane distances D_k.
    """
    t_f = ifftshift(np.asarray(target_amp, dtype=np.float64))
    h, w = t_f.shape
    if fresnel is None:
        q1 = np.ones((h, w), dtype=np.complex128)
    else:
        q1 = np.outer(fresnel_chirp(h, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]),
                      fresnel_chirp(w, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]))
    a = nonnegative_real(np.asarray(a0, dtype=np.float64))
    errors, dist = [], []
    for k in range(iterations + 1):
        replay = fft2(q1 * a)
        errors.append(nmse_fn(np.abs(replay) ** 2, t_f * t_f))
        imposed = replace_amplitude(replay, t_f)
        if distance_trace:
            dist.append(float(np.linalg.norm(replay - imposed)))
        if k == iterations:
            break
        a = nonnegative_real(np.conj(q1) * ifft2(imposed))
    out = {"amplitude": a, "nmse": errors}
    if distance_trace:
        out["distance"] = dist
    return out
