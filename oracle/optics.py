"""Fourier and Fresnel propagation between the SLM and replay planes (FP64).

Test infrastructure only.  The paper lists "Fourier" and "Fresnel" holograms
(Abstract keywords) and puts a Fourier transform in its image viewer (Sec. 2,
novel elements) without stating the operators.  Readings used here:

Fourier hologram: the replay field is the forward 2D DFT of the SLM field and
the SLM field is the inverse 2D DFT of the replay field, both in FFT index
order (the raw transform; see dft.py for the convention).

Fresnel hologram: the single-FFT Fresnel transform (Goodman, Introduction to
Fourier Optics, Fresnel diffraction integral evaluated with one Fourier
transform).  With source coordinates xi_n = (n - W//2) p, eta_m = (m - H//2) p,
output pitches p_x' = lambda z / (W p), p_y' = lambda z / (H p) and output
coordinates x_k = (k - W//2) p_x', y_l = (l - H//2) p_y':

  Q1[m][n] = exp(i pi (xi_n^2 + eta_m^2) / (lambda z))        (source chirp)
  Q2[l][k] = exp(i pi (x_k^2 + y_l^2) / (lambda z))            (output chirp)
  c        = exp(i k z) / (i lambda z) * p^2,   k = 2 pi / lambda
  U_z      = c * Q2 * fftshift(FFT2(ifftshift(Q1 * U_0)))

and the backward operator is its exact algebraic inverse

  U_0 = conj(Q1) * fftshift(IFFT2(ifftshift(conj(Q2) * U_z / c))).

Both planes are stored in centred image order (optical axis at (H//2, W//2)).

Angular spectrum (Goodman, propagation of the angular spectrum): the field at
distance z on the same grid (pitch p) is

  U_z = IFFT2(FFT2(U_0) * exp(2 pi i z sqrt(1/lambda^2 - fx^2 - fy^2)))

with fx = kx / (W p) for the FFT index kx (kx - W from kx >= (W + 1) // 2 on),
fy likewise, and zero transfer where the root is imaginary (evanescent
waves).  Backward propagation uses the conjugate transfer function.  Both
planes keep the natural array order (the optical axis at (H//2, W//2) of a
centred image stays there).
"""
from __future__ import annotations

import numpy as np

from .dft import fft2, ifft2, fftshift, ifftshift


def fresnel_chirp(n: int, pitch: float, wavelength: float, distance: float) -> np.ndarray:
    """1D quadratic phase exp(i pi ((j - n//2) pitch)^2 / (lambda z)), j = 0..n-1."""
    c = (np.arange(n, dtype=np.float64) - (n // 2)) * pitch
    return np.exp(1j * np.pi * c * c / (wavelength * distance))


def fresnel_geometry(height: int, width: int, wavelength: float, pitch: float,
                     distance: float) -> dict:
    """Source chirp Q1, output chirp Q2, prefactor c and output pitches."""
    q1 = np.outer(fresnel_chirp(height, pitch, wavelength, distance),
                  fresnel_chirp(width, pitch, wavelength, distance))
    py_out = wavelength * distance / (height * pitch)
    px_out = wavelength * distance / (width * pitch)
    q2 = np.outer(fresnel_chirp(height, py_out, wavelength, distance),
                  fresnel_chirp(width, px_out, wavelength, distance))
    # exp(i k z) with k z = 2 pi z / lambda reduced modulo one wave first
    kz = 2.0 * np.pi * np.mod(distance / wavelength, 1.0)
    pref = np.exp(1j * kz) / (1j * wavelength * distance) * pitch * pitch
    return {"q1": q1, "q2": q2, "prefactor": pref,
            "pitch_out_y": py_out, "pitch_out_x": px_out}


def propagate(u: np.ndarray, direction: int, fresnel: bool = False,
              wavelength: float = 0.0, pitch: float = 0.0,
              distance: float = 0.0) -> np.ndarray:
    """Propagate a complex field; direction +1 = SLM -> replay, -1 = back."""
    u = np.asarray(u, dtype=np.complex128)
    if direction not in (1, -1):
        raise ValueError("direction must be +1 or -1")
    if not fresnel:
        return fft2(u) if direction == 1 else ifft2(u)
    h, w = u.shape[-2:]
    g = fresnel_geometry(h, w, wavelength, pitch, distance)
    if direction == 1:
        return g["prefactor"] * g["q2"] * fftshift(fft2(ifftshift(g["q1"] * u)))
    return np.conj(g["q1"]) * fftshift(ifft2(ifftshift(np.conj(g["q2"]) * u / g["prefactor"])))


def spatial_frequencies(n: int, pitch: float) -> np.ndarray:
    """Frequency (1/m) of FFT index k of an n-point axis with sample pitch p."""
    k = np.arange(n, dtype=np.float64)
    k = np.where(k < (n + 1) // 2, k, k - n)
    return k / (n * pitch)


def angular_transfer(h: int, w: int, wavelength: float, pitch: float, distance: float) -> np.ndarray:
    """exp(2 pi i z sqrt(1/lambda^2 - fx^2 - fy^2)) in FFT order; 0 where evanescent."""
    fy = spatial_frequencies(h, pitch)[:, None]
    fx = spatial_frequencies(w, pitch)[None, :]
    arg = 1.0 / (wavelength * wavelength) - fx * fx - fy * fy
    root = np.sqrt(np.maximum(arg, 0.0))
    return np.where(arg > 0.0, np.exp(2j * np.pi * distance * root), 0.0)


def angular_spectrum(u: np.ndarray, direction: int, wavelength: float, pitch: float,
                     distance: float) -> np.ndarray:
    """Angular-spectrum propagation over `distance` (direction +1) or back (-1)."""
    u = np.asarray(u, dtype=np.complex128)
    if direction not in (1, -1):
        raise ValueError("direction must be +1 or -1")
    h, w = u.shape[-2:]
    tf = angular_transfer(h, w, wavelength, pitch, distance)
    if direction == -1:
        tf = np.conj(tf)
    return ifft2(fft2(u) * tf)
