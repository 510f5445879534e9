"""Energy-normalised mean squared error of a replay intensity (FP64).

Test infrastructure only.  The paper's Normaliser (Sec. 7.3) normalises
vectors on the GPU and its process monitor reports algorithm progress
(Sec. 7.1); the error measure itself is unstated.  Reading used here: both
intensities are normalised to unit total energy over the full frame and

    NMSE(I, T) = sum (I/sum I - T/sum T)^2 / sum (T/sum T)^2 .

It is zero when I is any positive multiple of T and one when I is zero
everywhere except where T is zero.
"""
from __future__ import annotations

import numpy as np


def nmse(intensity: np.ndarray, target_intensity: np.ndarray) -> float:
    i = np.asarray(intensity, dtype=np.float64)
    t = np.asarray(target_intensity, dtype=np.float64)
    i_n = i / i.sum()
    t_n = t / t.sum()
    return float(np.sum((i_n - t_n) ** 2) / np.sum(t_n * t_n))
