"""Seeded synthetic workloads shared by the GPU path's tests/bench and the oracle.

This module only *generates inputs*: targets, starting phases and OSPR subframe
phases, plus the named workload descriptions. It contains none of the
hologram-generation arithmetic (no FFT, no constraint, no error metric), so the
oracle and the HIP path can both consume its arrays without sharing any of the
method's code.

The paper evaluates nothing and prints no workload, so every input here is
synthetic.  The target recipe (uniform noise, periodic Gaussian blur of sigma 3
px, twelve filled discs, normalised to a peak of 1, amplitude = sqrt) stands in
for the "target image" that the algorithm object receives (Sec. 4, Algorithm
Interface; Sec. 7.3, AlgorithmCuda).  All draws use numpy's PCG64
``default_rng(seed)`` in float64 and are rounded once to float32, so both sides
see identical bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi

# Fresnel geometry used by the 1024^2 and gradient workloads (metres).
WAVELENGTH_532NM = 532e-9
PITCH_8UM = 8e-6


def _blur_periodic(img: np.ndarray, sigma: float = 3.0) -> np.ndarray:
    """Separable Gaussian blur with wrap-around boundary (axis 0, then axis 1)."""
    radius = int(4.0 * sigma + 0.5)
    taps = np.arange(-radius, radius + 1, dtype=np.float64)
    weights = np.exp(-(taps * taps) / (2.0 * sigma * sigma))
    weights /= weights.sum()
    out = img
    for axis in (0, 1):
        acc = np.zeros_like(out)
        for t, wgt in zip(taps.astype(int), weights):
            acc += wgt * np.roll(out, -t, axis=axis)
        out = acc
    return out


def _target_from_rng(rng: np.random.Generator, height: int, width: int,
                     n_discs: int = 12) -> np.ndarray:
    noise = rng.uniform(0.0, 1.0, (height, width))
    img = _blur_periodic(noise)
    yy = np.arange(height, dtype=np.float64)[:, None] + 0.5
    xx = np.arange(width, dtype=np.float64)[None, :] + 0.5
    for _ in range(n_discs):
        cy = rng.uniform(0.0, height)
        cx = rng.uniform(0.0, width)
        r = rng.uniform(5.0, 30.0)
        inside = (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
        img = img + inside.astype(np.float64)
    img = img / img.max()
    return np.sqrt(img).astype(np.float32)


def target_amplitude(height: int, width: int, seed: int) -> np.ndarray:
    """Synthetic target amplitude [H][W] float32, centred image order."""
    return _target_from_rng(np.random.default_rng(seed), height, width)


def uniform_phase(height: int, width: int, seed: int) -> np.ndarray:
    """Uniform[0, 2pi) phase [H][W] float32 (a value may round up to 2pi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, TWO_PI, (height, width)).astype(np.float32)


def target_and_phase(height: int, width: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """One generator for both: noise, discs, then the starting phase.

    Used for per-instance seeding of batched workloads.
    """
    rng = np.random.default_rng(seed)
    t = _target_from_rng(rng, height, width)
    phi = rng.uniform(0.0, TWO_PI, (height, width)).astype(np.float32)
    return t, phi


def random_field(height: int, width: int, seed: int) -> np.ndarray:
    """Complex64 test field with standard-normal real and imaginary parts."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((height, width))
    im = rng.standard_normal((height, width))
    return (re + 1j * im).astype(np.complex64)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class GSWorkload:
    name: str
    height: int
    width: int
    iterations: int
    levels: int                 # 0 = continuous phase-only SLM
    fresnel: bool
    target_seed: int
    phase_seed: int
    wavelength: float = WAVELENGTH_532NM
    pitch: float = PITCH_8UM
    distance: float = 0.5

    def inputs(self) -> Tuple[np.ndarray, np.ndarray]:
        return (target_amplitude(self.height, self.width, self.target_seed),
                uniform_phase(self.height, self.width, self.phase_seed))


@dataclass(frozen=True)
class OSPRWorkload:
    name: str
    height: int
    width: int
    subframes: int
    target_seed: int
    first_phase_seed: int

    def target(self) -> np.ndarray:
        return target_amplitude(self.height, self.width, self.target_seed)

    def subframe_phase(self, n: int) -> np.ndarray:
        return uniform_phase(self.height, self.width, self.first_phase_seed + n)

    def subframe_phases(self, count: Optional[int] = None) -> np.ndarray:
        count = self.subframes if count is None else count
        return np.stack([self.subframe_phase(n) for n in range(count)])


@dataclass(frozen=True)
class GradWorkload:
    """Gradient-descent hologram problems: one continuous SLM phase per problem,
    one synthetic target per (problem, plane); targets seeded 200 + 3 b + j,
    starting phases 300 + b for problem b and plane j."""
    name: str
    height: int
    width: int
    distances: Tuple[float, ...]
    steps: int
    lr: float
    problems: int
    wavelength: float = WAVELENGTH_532NM
    pitch: float = PITCH_8UM

    def targets(self, b: int = 0) -> np.ndarray:
        return np.stack([target_amplitude(self.height, self.width, 200 + 3 * b + j)
                         for j in range(len(self.distances))])

    def phase0(self, b: int = 0) -> np.ndarray:
        return uniform_phase(self.height, self.width, 300 + b)


# GS Fourier, 256x256, continuous phase, 20 iterations; target seed 0, phase seed 1.
GS_FOURIER_256 = GSWorkload("gs_fourier_256x256_cont_20it", 256, 256, 20, 0, False, 0, 1)
# GS Fresnel, 1024x1024, 8 levels, 100 iterations; lambda 532 nm, 8 um, z 0.5 m;
# target seed 2, phase seed 3.
GS_FRESNEL_1024 = GSWorkload("gs_fresnel_1024x1024_L8_100it", 1024, 1024, 100, 8, True, 2, 3)
# OSPR binary phase, 2048x2048, 24 subframes; target seed 4, subframe seeds 10..33.
OSPR_2048 = OSPRWorkload("ospr_2048x2048_24sub", 2048, 2048, 24, 4, 10)
# Gradient-descent CGH, 1024x1024 phase, Fresnel planes at 0.40 / 0.45 / 0.50 m
# (532 nm, 8 um), summed NMSE loss, Adam lr 0.05, 500 steps, 8 problems.
GRAD_3PLANE_1024 = GradWorkload("grad_fresnel3_1024x1024_adam500", 1024, 1024, (0.40, 0.45, 0.50), 500, 0.05, 8)
# Time-to-NMSE comparison: the 1024x1024 Fresnel geometry of GS_FRESNEL_1024
# (target seed 2, phase seed 3, z 0.5 m) with a continuous phase; the threshold
# is the NMSE continuous GS reaches after 100 iterations.
GS_FRESNEL_1024_CONT = GSWorkload("gs_fresnel_1024x1024_cont_100it", 1024, 1024, 100, 0, True, 2, 3)


def batched_mix() -> List[Tuple[int, int, int]]:
    """(height, width, seed) of the 64-hologram mixed batch, in listed order."""
    shapes = [(512, 512)] * 16 + [(1024, 1024)] * 24 + [(2048, 2048)] * 16 + [(1080, 1920)] * 8
    return [(h, w, 100 + i) for i, (h, w) in enumerate(shapes)]
