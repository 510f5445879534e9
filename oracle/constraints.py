"""SLM-plane and replay-plane constraints of the iterative Fourier loop (FP64).

Test infrastructure only.  The paper names a "base level quantisation
algorithm" (QuantiserCuda, Sec. 7.3) and phase-only SLM types (Sec. 3.2,
SLMTypeOption / MultiAmpSLM) but defines neither; the readings are:

Phase-only projection (continuous SLM): G -> G/|G|, with G = 0 -> 1.  This is
the nearest unit-modulus value (Gerchberg & Saxton 1972; Fienup 1982).

Uniform L-level phase quantiser: levels phi_l = l * Delta, Delta = 2 pi / L,
and the level of a complex value G is
    l = floor(mod(atan2(Im G, Re G), 2 pi) / Delta + 1/2) mod L,
i.e. the nearest level on the circle with ties going up.  G = 0 has angle 0.

Binary-phase binariser (OSPR): Re G >= 0 (including -0.0) -> +1 (level 0,
phase 0), otherwise -1 (level 1, phase pi).

Replay-plane amplitude replacement: R -> T * R/|R|, with R = 0 -> T.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def quantise_phase_level(theta: np.ndarray, levels: int) -> np.ndarray:
    """Level index l in [0, L) of the angle theta (radians, any range)."""
    delta = TWO_PI / levels
    wrapped = np.mod(np.asarray(theta, dtype=np.float64), TWO_PI)
    return (np.floor(wrapped / delta + 0.5).astype(np.int64)) % levels


def quantise_level(g: np.ndarray, levels: int) -> np.ndarray:
    """Level index of a complex field: quantise atan2(Im, Re)."""
    g = np.asarray(g, dtype=np.complex128)
    return quantise_phase_level(np.arctan2(g.imag, g.real), levels)


def phase_only(g: np.ndarray) -> np.ndarray:
    """Unit-modulus projection G/|G| (G = 0 -> 1)."""
    g = np.asarray(g, dtype=np.complex128)
    mag = np.abs(g)
    out = np.ones_like(g)
    nz = mag > 0
    out[nz] = g[nz] / mag[nz]
    return out


def replace_amplitude(r: np.ndarray, target_amp: np.ndarray) -> np.ndarray:
    """Keep the phase of R, impose the amplitude T (R = 0 -> T)."""
    return np.asarray(target_amp, dtype=np.float64) * phase_only(r)


def binarise(g: np.ndarray) -> np.ndarray:
    """Binary-phase hologram h in {+1, -1} from the sign of Re G (>= 0 -> +1)."""
    re = np.asarray(g, dtype=np.complex128).real
    return np.where(re >= 0.0, 1.0, -1.0)
