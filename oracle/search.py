"""Single-pixel search: direct binary search and simulated annealing (FP64).

Test infrastructure only.  The paper's library holds direct binary search
(HoloGenAlgDSCuda), simulated annealing (HoloGenAlgSACuda) and an updater of
the replay field after a change of one SLM pixel (FFTUpdaterCuda, Sec. 7.3).
It states neither rule; the textbook forms (Seldowitz, Allebach & Sweeney,
Appl. Opt. 26, 1987, for direct binary search; Kirkpatrick et al., Science
220, 1983, for annealing with the Metropolis rule) are written out here,
state by state, with the replay field recomputed from scratch for every
trial (the plain definition; no rank-one update):

  H      = A exp(2 pi i l / L)             L-level phase hologram (A = 1)
  E(H)   = NMSE(|FFT2(Q1 H)|^2, ifftshift(T_amp)^2)
  trial k: pixel p_k, candidate level c_k; H' = H with l[p_k] = c_k
           dE = E(H') - E(H)
           direct search: accept iff dE < 0
           annealing:     accept iff dE < 0 or u_k < exp(-dE / temp_k)
           (u_k uniform in [0, 1) and temp_k > 0 are inputs)
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .dft import fft2, ifftshift
from .metrics import nmse
from .optics import fresnel_chirp

TWO_PI = 2.0 * np.pi


def _replay_error(lev, levels, q1, t_int):
    h = np.exp(1j * lev * (TWO_PI / levels))
    return nmse(np.abs(fft2(q1 * h)) ** 2, t_int)


def pixel_search(target_amp: np.ndarray, levels0: np.ndarray, levels: int,
                 trials: Sequence, temperature: Optional[Sequence[float]] = None,
                 uniform: Optional[Sequence[float]] = None,
                 fresnel: Optional[dict] = None) -> dict:
    """Run the trials in order from the level map levels0.

    trials: (pixel index y * W + x, candidate level) pairs.  temperature None
    means direct binary search; otherwise annealing with uniform[k].
    Returns levels, accepted [n] (bool), nmse [n + 1] (state before trial 0,
    then after each trial) and dE [n] (the error change of each trial)."""
    t_amp = np.asarray(target_amp, dtype=np.float64)
    hh, ww = t_amp.shape
    t_int = ifftshift(t_amp) ** 2
    if fresnel is None:
        q1 = np.ones((hh, ww), dtype=np.complex128)
    else:
        q1 = np.outer(fresnel_chirp(hh, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]),
                      fresnel_chirp(ww, fresnel["pitch"], fresnel["wavelength"], fresnel["distance"]))
    lev = np.array(levels0, dtype=np.int64).copy()
    err = _replay_error(lev, levels, q1, t_int)
    errors, accepted, deltas = [err], [], []
    for k, (p, cand) in enumerate(trials):
        y, x = divmod(int(p), ww)
        trial = lev.copy()
        trial[y, x] = int(cand)
        new_err = _replay_error(trial, levels, q1, t_int)
        d = new_err - err
        if temperature is None:
            ok = d < 0.0
        else:
            ok = d < 0.0 or uniform[k] < np.exp(-d / temperature[k])
        if ok:
            lev, err = trial, new_err
        accepted.append(bool(ok))
        deltas.append(d)
        errors.append(err)
    return {"levels": lev.astype(np.uint8), "accepted": np.array(accepted, dtype=bool),
            "nmse": errors, "dE": np.array(deltas)}
