"""Helpers shared by the GPU parity tests (tensor plumbing and comparison
metrics only; no hologram arithmetic)."""
import numpy as np

TWO_PI = 2.0 * np.pi


def torch_mod():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible GPU")
    return torch


def dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch_mod().cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(got, ref):
    ref = np.asarray(ref)
    return float(np.linalg.norm(np.asarray(got) - ref) / np.linalg.norm(ref))


def boundary_distance(theta, levels):
    """Angular distance (rad) from theta to the nearest decision boundary of the
    uniform L-level quantiser (boundaries at (l + 1/2) 2 pi / L)."""
    delta = TWO_PI / levels
    f = np.mod(np.mod(theta, TWO_PI) / delta + 0.5, 1.0)
    return np.minimum(f, 1.0 - f) * delta


def level_mismatch(got, ref, theta, levels, band=1e-5):
    """(fraction of pixels whose levels differ outside the boundary band,
    number of differing pixels in total)."""
    diff = np.asarray(got).astype(np.int64) != np.asarray(ref).astype(np.int64)
    outside = diff & (boundary_distance(theta, levels) >= band)
    return outside.sum() / diff.size, int(diff.sum())


def phase_parity(phi_gpu, phi_ref):
    """Continuous-phase parity: relative L2 of the unit phasors and the
    fraction of pixels whose phases differ by more than 1e-3 rad."""
    a = np.exp(1j * np.asarray(phi_gpu, np.float64))
    b = np.exp(1j * np.asarray(phi_ref, np.float64))
    d = np.abs(np.angle(a * np.conj(b)))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b)), float((d > 1e-3).mean())
