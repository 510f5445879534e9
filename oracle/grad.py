"""Gradient-descent computer-generated holography (FP64).

Test infrastructure only.  The paper names the algorithms its library holds
and leaves further ones to future work (Sec. 8, Further Research and
Conclusion); this module writes out the gradient method that the GPU library
adds, from its textbook definition, step by step:

Forward, per replay plane j (Fresnel source chirp Q1_j of distance z_j, or
Q1 = 1 for a Fourier plane):

    V_j = Q1_j * exp(i phi)            SLM field seen by plane j
    U_j = FFT2(V_j)                    replay field, FFT index order
    I_j = |U_j|^2

The post-chirp, prefactor and centring of the physical Fresnel operator are
unit-modulus factors and index shifts, so |U_j|^2 equals the physical replay
intensity up to the shift (tests pin this against optics.propagate).

Loss: L = sum_j NMSE(I_j, T_j) with the energy-normalised NMSE of metrics.py
and T_j = |target amplitude|^2 brought into FFT order (ifftshift).

Gradient (Wirtinger calculus; I = U conj(U)):

    dL/dI_j      = 2 (I_j/S_j - T_j/ST_j) / (S_j D_j)
                   S_j = sum I_j, ST_j = sum T_j, D_j = sum (T_j/ST_j)^2
    dL/dconj(U_j) = dL/dI_j * U_j
    G_j          = F^H (dL/dconj(U_j)) = N_px * IFFT2(...)   (adjoint of FFT2)
    dL/dphi      = sum_j 2 Im(conj(V_j) G_j)

S_j does not depend on phi (Parseval: S_j = N_px sum |V_j|^2 = N_px^2), so the
derivative through S_j vanishes and dL/dI_j above is the full derivative.

Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
phi -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = 1, 2, ...
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from .dft import fft2, ifft2, ifftshift
from .metrics import nmse
from .optics import fresnel_chirp


def source_chirp(h: int, w: int, plane: Optional[dict]) -> np.ndarray:
    """Q1 of one plane: ones for a Fourier plane, else the Fresnel source chirp."""
    if plane is None:
        return np.ones((h, w), dtype=np.complex128)
    return np.outer(fresnel_chirp(h, plane["pitch"], plane["wavelength"], plane["distance"]),
                    fresnel_chirp(w, plane["pitch"], plane["wavelength"], plane["distance"]))


def loss_and_gradient(phi: np.ndarray, target_amps: Sequence[np.ndarray],
                      planes: Sequence[Optional[dict]], want_grad: bool = True):
    """(L, dL/dphi, per-plane NMSE) at phase phi for centred target amplitudes."""
    phi = np.asarray(phi, dtype=np.float64)
    h, w = phi.shape
    n_px = h * w
    slm = np.exp(1j * phi)
    total = 0.0
    per_plane = []
    grad = np.zeros((h, w)) if want_grad else None
    for amp, plane in zip(target_amps, planes):
        v = source_chirp(h, w, plane) * slm
        u = fft2(v)
        inten = (u * np.conj(u)).real
        t = ifftshift(np.asarray(amp, dtype=np.float64) ** 2)
        e = nmse(inten, t)
        per_plane.append(e)
        total += e
        if want_grad:
            s = inten.sum()
            st = t.sum()
            d = np.sum((t / st) ** 2)
            dl_di = 2.0 * (inten / s - t / st) / (s * d)
            g = n_px * ifft2(dl_di * u)
            grad += 2.0 * (np.conj(v) * g).imag
    return total, grad, per_plane


def adam_update(phi, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                eps: float = 1e-8):
    """One Adam step t (1-based); returns the new (phi, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return phi - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def grad_descent(phi0: np.ndarray, target_amps: Sequence[np.ndarray],
                 planes: Sequence[Optional[dict]], steps: int, lr: float = 0.05,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> dict:
    """Adam on phi for `steps` steps.

    Returns {"phase": phi after the last step, "loss": [L(phi_0), ..., L(phi_steps)],
    "nmse": per-plane NMSE of every state}."""
    phi = np.asarray(phi0, dtype=np.float64).copy()
    m = np.zeros_like(phi)
    v = np.zeros_like(phi)
    losses: List[float] = []
    per: List[list] = []
    for k in range(steps + 1):
        want = k < steps
        loss, g, pp = loss_and_gradient(phi, target_amps, planes, want_grad=want)
        losses.append(loss)
        per.append(pp)
        if want:
            phi, m, v = adam_update(phi, m, v, g, k + 1, lr, beta1, beta2, eps)
    return {"phase": phi, "loss": losses, "nmse": per}
