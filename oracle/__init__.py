"""FP64 CPU oracle for the iterative Fourier-transform hologram path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, tables, constants or helpers) and imports nothing from it.

What it computes, and where it comes from.  The paper (Structure and Design of
HoloGen) names the algorithms and primitives of its CUDA backend -- the cuFFT
wrapper, the quantiser, the normaliser, the randomiser, Gerchberg-Saxton and
One-Step Phase-Retrieval (Sec. 7.3, Algorithm Libraries), Fourier and Fresnel
holograms (Abstract keywords) -- but prints no formula.  Each module therefore
writes out the textbook definition the paper presupposes, in FP64/complex128,
step by step in the order the method performs it:

  dft.py          discrete Fourier transform: a naive O(N^2) DFT and the
                  oracle's own recursive mixed-radix Cooley-Tukey FFT
                  (Cooley & Tukey 1965), 2D as rows then columns.
  optics.py       Fourier, single-FFT Fresnel and angular-spectrum
                  propagation (Goodman, Introduction to Fourier Optics).
  constraints.py  SLM-plane phase-only projection, uniform L-level phase
                  quantiser, binary-phase binariser, replay-plane amplitude
                  replacement.
  metrics.py      energy-normalised NMSE of an intensity against a target.
  gs.py           Gerchberg-Saxton error-reduction iteration (Gerchberg &
                  Saxton 1972; Fienup 1982), and its plane-by-plane
                  multi-plane form.
  ospr.py         One-Step Phase-Retrieval (Cable, Buckley et al. 2004).
  grad.py         gradient-descent hologram optimisation: multi-plane NMSE
                  loss, its Wirtinger gradient and Adam (Kingma & Ba 2015).
  search.py       single-pixel direct binary search and simulated annealing
                  (the paper's HoloGenAlgDSCuda / HoloGenAlgSACuda, Sec. 7.3).
  window.py       GS with a signal window (region of interest) in the replay
                  plane (Fienup 1982; Wyrowski & Bryngdahl 1988).
  amplitude.py    GS for an amplitude-only SLM (non-negativity constraint,
                  Fienup 1982).

Where the paper is silent, each module's docstring states the reading it
takes.  Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
brute-force sums, invariants and independent library routines.
"""
from .dft import dft_naive, fft, ifft, fft2, ifft2, fftshift, ifftshift
from .optics import (fresnel_chirp, fresnel_geometry, propagate, spatial_frequencies,
                     angular_transfer, angular_spectrum)
from .constraints import (quantise_level, quantise_phase_level, phase_only,
                          replace_amplitude, binarise)
from .metrics import nmse
from .gs import gs_iterate, gs_multiplane
from .ospr import ospr, ospr_pairs
from .grad import source_chirp, loss_and_gradient, adam_update, grad_descent
from .search import pixel_search
from .window import gs_window, window_nmse
from .amplitude import gs_amplitude, nonnegative_real

__all__ = [
    "dft_naive", "fft", "ifft", "fft2", "ifft2", "fftshift", "ifftshift",
    "fresnel_chirp", "fresnel_geometry", "propagate", "spatial_frequencies", "angular_transfer",
    "angular_spectrum",
    "quantise_level", "quantise_phase_level", "phase_only", "replace_amplitude",
    "binarise", "nmse", "gs_iterate", "gs_multiplane", "ospr", "ospr_pairs",
    "source_chirp", "loss_and_gradient", "adam_update", "grad_descent", "pixel_search",
    "gs_window", "window_nmse", "gs_amplitude", "nonnegative_real",
]
