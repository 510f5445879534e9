"""Discrete Fourier transforms, written out in FP64 (test infrastructure only).

The paper delegates the FFT to cuFFT behind its FFTHandlerCuda wrapper (Sec. 2
and Sec. 7.3) and never states a convention.  Reading used here:

  forward  X[k] = sum_n x[n] exp(-2 pi i n k / N)          (unnormalised)
  inverse  x[n] = (1/N) sum_k X[k] exp(+2 pi i n k / N)

A 2D transform of an [H][W] array is the 1D transform along every row (the
contiguous axis, length W) followed by the 1D transform along every column.

``fft`` is a recursive decimation-in-time Cooley-Tukey FFT (Cooley & Tukey,
Math. Comp. 19, 1965): split x into r interleaved subsequences x[q::r],
transform each, multiply by the twiddle exp(-2 pi i q k1 / N) and finish with
an r-point DFT across q.  Any length works: the radix is 4, 2, 3 or 5 when it
divides N, otherwise the smallest prime factor, and a prime length is a naive
DFT.  numpy's FFT module is never used here.
"""
from __future__ import annotations

import numpy as np


def _unit_roots(num: np.ndarray, den: int, sign: int) -> np.ndarray:
    """exp(sign * 2 pi i * num / den) with num reduced mod den first (exact ints)."""
    return np.exp(sign * 2j * np.pi * (np.mod(num, den) / den))


def dft_naive(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """O(N^2) DFT along the last axis: X[k] = sum_n x[n] exp(sign 2 pi i n k / N)."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    idx = np.arange(n)
    mat = _unit_roots(np.outer(idx, idx), n, sign)   # mat[k, n]
    return x @ mat.T


def _radix(n: int) -> int:
    for r in (4, 2, 3, 5):
        if n % r == 0:
            return r
    p = 7
    while p * p <= n:
        if n % p == 0:
            return p
        p += 2
    return n


def _fft_last_axis(x: np.ndarray, sign: int) -> np.ndarray:
    n = x.shape[-1]
    if n == 1:
        return x.copy()
    r = _radix(n)
    if r == n:
        return dft_naive(x, sign)
    m = n // r
    lead = x.shape[:-1]
    # sub[..., q, j] = x[..., j*r + q]: the q-th interleaved subsequence
    sub = np.swapaxes(x.reshape(lead + (m, r)), -1, -2)
    spec = _fft_last_axis(np.ascontiguousarray(sub), sign)        # [..., q, k1]
    q = np.arange(r)
    k1 = np.arange(m)
    spec = spec * _unit_roots(np.outer(q, k1), n, sign)         # twiddle W_N^{q k1}
    small = _unit_roots(np.outer(q, q), r, sign)                 # [k2, q]
    out = np.tensordot(small, spec, axes=([1], [-2]))            # [k2, ..., k1]
    out = np.moveaxis(out, 0, -2)                                # [..., k2, k1]
    return out.reshape(lead + (n,))                              # k = k1 + m*k2


def fft(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """Forward unnormalised 1D FFT along ``axis``."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last_axis(np.ascontiguousarray(x), -1), -1, axis)


def ifft(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """Inverse 1D FFT along ``axis`` (exponent +, scaled by 1/N)."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    n = x.shape[-1]
    return np.moveaxis(_fft_last_axis(np.ascontiguousarray(x), +1) / n, -1, axis)


def fft2(x: np.ndarray) -> np.ndarray:
    """Forward 2D FFT of the last two axes: rows (last axis) first, then columns."""
    return fft(fft(x, axis=-1), axis=-2)


def ifft2(x: np.ndarray) -> np.ndarray:
    """Inverse 2D FFT of the last two axes (scaled by 1/(H W))."""
    return ifft(ifft(x, axis=-1), axis=-2)


def fftshift(x: np.ndarray) -> np.ndarray:
    """Move index 0 of each of the last two axes to index N//2 (roll by +N//2)."""
    h, w = x.shape[-2:]
    return np.roll(np.roll(x, h // 2, axis=-2), w // 2, axis=-1)


def ifftshift(x: np.ndarray) -> np.ndarray:
    """Inverse of ``fftshift``: index N//2 goes to index 0 (roll by -(N//2))."""
    h, w = x.shape[-2:]
    return np.roll(np.roll(x, -(h // 2), axis=-2), -(w // 2), axis=-1)
