"""One-Step Phase-Retrieval, binary phase (FP64).

Test infrastructure only.  The paper's HoloGenAlgOSPRCuda implements
One-Step Phase-Retrieval (Sec. 7.3) and its Randomiser draws random phase
(Sec. 7.3); the steps are those of Cable, Buckley et al. (SID Digest 2004):
for each subframe n

  E_n = T_amp * exp(i theta_n)            target amplitude, random phase
  G_n = IFFT2(ifftshift(E_n))             one inverse transform
  h_n = +1 if Re G_n >= 0 else -1         binary phase 0 / pi (level 0 / 1)
  I_n = |FFT2(h_n)|^2                     replay intensity of the subframe

and the eye sees the time average I_avg = (1/N) sum_n I_n, reported in centred
order as fftshift(I_avg) together with NMSE(fftshift(I_avg), T_amp^2).

Real and imaginary pairs (ospr_pairs): one inverse transform G_n gives two
subframes, h_2n from the sign of Re G_n and h_2n+1 from the sign of Im G_n
(the same >= 0 rule), and the average runs over all 2N subframes.
"""
from __future__ import annotations

import numpy as np

from .dft import fft2, ifft2, fftshift, ifftshift
from .constraints import binarise
from .metrics import nmse as nmse_fn


def ospr(target_amp: np.ndarray, sub_phases: np.ndarray) -> dict:
    """target_amp [H][W] centred; sub_phases [N][H][W] centred.

    Returns levels [N][H][W] (0 for +1, 1 for -1), the centred average
    intensity [H][W] and its NMSE against target_amp^2.
    """
    t_amp = np.asarray(target_amp, dtype=np.float64)
    thetas = np.asarray(sub_phases, dtype=np.float64)
    n_sub = thetas.shape[0]
    acc = np.zeros(t_amp.shape)
    lev = np.empty(thetas.shape, dtype=np.uint8)
    for n in range(n_sub):
        field = t_amp * np.exp(1j * thetas[n])
        g = ifft2(ifftshift(field))
        h = binarise(g)
        lev[n] = (h < 0).astype(np.uint8)
        acc += np.abs(fft2(h)) ** 2
    avg = fftshift(acc / n_sub)
    return {"levels": lev, "intensity": avg, "nmse": nmse_fn(avg, t_amp * t_amp)}


def ospr_pairs(target_amp: np.ndarray, sub_phases: np.ndarray) -> dict:
    """target_amp [H][W] centred; sub_phases [N][H][W] centred, one per pair.

    Returns levels [2N][H][W] (subframe 2n from Re G_n, 2n + 1 from Im G_n),
    the centred average intensity over the 2N subframes and its NMSE.
    """
    t_amp = np.asarray(target_amp, dtype=np.float64)
    thetas = np.asarray(sub_phases, dtype=np.float64)
    n_pairs = thetas.shape[0]
    acc = np.zeros(t_amp.shape)
    lev = np.empty((2 * n_pairs,) + t_amp.shape, dtype=np.uint8)
    for n in range(n_pairs):
        g = ifft2(ifftshift(t_amp * np.exp(1j * thetas[n])))
        for k, part in enumerate((g.real, g.imag)):
            h = np.where(part >= 0.0, 1.0, -1.0)
            lev[2 * n + k] = (h < 0).astype(np.uint8)
            acc += np.abs(fft2(h)) ** 2
    avg = fftshift(acc / (2 * n_pairs))
    return {"levels": lev, "intensity": avg, "nmse": nmse_fn(avg, t_amp * t_amp)}
