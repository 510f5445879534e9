"""GPU parity of hg_propagate (row pass + column pass FFT, Fourier and
Fresnel) against the FP64 oracle on the same FP32 inputs.  Bar: relative L2
error <= 1e-5."""
import numpy as np
import pytest

import oracle
from paper_2006_10509_amd import hologen as hg
from paper_2006_10509_amd import workloads as wl
from gpu_util import dev, host, rel_l2, torch_mod

pytestmark = pytest.mark.gpu
TOL = 1e-5
OPTICS = dict(wavelength=532e-9, pixel_pitch=8e-6, distance=0.5)

SHAPES = [(16, 16), (32, 64), (24, 60), (90, 120), (120, 90), (256, 256), (128, 512),
          (1024, 1024), (2048, 2048), (1080, 1920), (60, 4096), (4096, 24),
          # SLM resolutions 1280 x 1024 / 1536 / 2160 x 3840 and the 8192 transform
          (1024, 1280), (1280, 1536), (1536, 1280), (2160, 3840), (3840, 60), (16, 8192), (8192, 16)]


def run(plan, x, direction, inplace=False):
    torch = torch_mod()
    xin = dev(x)
    out = xin if inplace else torch.empty_like(xin)
    hg.hg_propagate(plan, xin, out, direction, plan.workspace())
    return host(out)


@pytest.mark.parametrize("shape", SHAPES)
def test_fourier_forward_and_inverse(shape):
    h, w = shape
    print(f"fourier propagate {h}x{w}", flush=True)
    plan = hg.Plan(w, h)
    x = wl.random_field(h, w, seed=h * 7 + w)
    fx = run(plan, x, hg.HG_FORWARD)
    ref = oracle.fft2(x.astype(np.complex128))
    assert rel_l2(fx, ref) <= TOL
    ix = run(plan, x, hg.HG_INVERSE)
    ref_i = oracle.ifft2(x.astype(np.complex128))
    assert rel_l2(ix, ref_i) <= TOL


@pytest.mark.parametrize("shape", [(256, 256), (90, 120), (1080, 1920), (1024, 1024)])
def test_fresnel_forward_and_inverse(shape):
    h, w = shape
    print(f"fresnel propagate {h}x{w}", flush=True)
    plan = hg.Plan(w, h, hg.HG_FRESNEL, **OPTICS)
    x = wl.random_field(h, w, seed=11)
    kw = dict(fresnel=True, wavelength=OPTICS["wavelength"], pitch=OPTICS["pixel_pitch"],
              distance=OPTICS["distance"])
    fx = run(plan, x, hg.HG_FORWARD)
    ref = oracle.propagate(x.astype(np.complex128), +1, **kw)
    assert rel_l2(fx, ref) <= TOL
    bx = run(plan, x, hg.HG_INVERSE)
    ref_b = oracle.propagate(x.astype(np.complex128), -1, **kw)
    assert rel_l2(bx, ref_b) <= TOL


@pytest.mark.parametrize("fresnel", [False, True])
def test_in_place(fresnel):
    h, w = 120, 90
    plan = hg.Plan(w, h, hg.HG_FRESNEL, **OPTICS) if fresnel else hg.Plan(w, h)
    x = wl.random_field(h, w, seed=5)
    a = run(plan, x, hg.HG_FORWARD)
    b = run(plan, x, hg.HG_FORWARD, inplace=True)
    assert np.array_equal(a, b)


def test_delta_and_plane_wave_closed_forms():
    h, w = 256, 1024
    plan = hg.Plan(w, h)
    x = np.zeros((h, w), np.complex64)
    x[3, 17] = 1.0
    k = np.arange(h)[:, None]
    l = np.arange(w)[None, :]
    ref = np.exp(-2j * np.pi * (3 * k / h + 17 * l / w))
    assert np.abs(run(plan, x, hg.HG_FORWARD) - ref).max() <= 1e-5
    m = np.arange(h)[:, None]
    n = np.arange(w)[None, :]
    pw = np.exp(2j * np.pi * (np.mod(5 * m, h) / h + np.mod(300 * n, w) / w)).astype(np.complex64)
    ref = np.zeros((h, w))
    ref[5, 300] = h * w
    assert np.abs(run(plan, pw, hg.HG_FORWARD) - ref).max() <= 1e-5 * h * w


def test_gaussian_beam_closed_form_on_gpu():
    """Fresnel propagation of exp(-r^2/w0^2) against the closed form."""
    n, z, w0 = 256, 0.5, 0.2e-3
    lam, p = OPTICS["wavelength"], OPTICS["pixel_pitch"]
    plan = hg.Plan(n, n, hg.HG_FRESNEL, lam, p, z)
    xs = (np.arange(n) - n // 2) * p
    u0 = np.exp(-(xs[:, None] ** 2 + xs[None, :] ** 2) / w0 ** 2).astype(np.complex64)
    uz = run(plan, u0, hg.HG_FORWARD)
    xo = (np.arange(n) - n // 2) * lam * z / (n * p)
    r2 = xo[:, None] ** 2 + xo[None, :] ** 2
    a, b = 1 / w0 ** 2, np.pi / (lam * z)
    zr = np.pi * w0 ** 2 / lam
    ref = np.exp(2j * np.pi * np.mod(z / lam, 1.0)) / (1 + 1j * z / zr) * np.exp(1j * a * b * r2 / (a - 1j * b))
    assert rel_l2(uz, ref) <= TOL


def test_8192_full_size_closed_forms():
    """8192 x 8192, past the 256 MiB last-level cache: the forward transform
    of a delta on sampled rows against its closed form, of a plane wave
    (one bin of height H W, zero elsewhere) everywhere, and the inverse of the
    plane wave's spectrum back to the plane wave."""
    torch = torch_mod()
    h = w = 8192
    print("fourier propagate 8192x8192 closed forms", flush=True)
    plan = hg.Plan(w, h)
    ws = plan.workspace()
    x = torch.zeros((h, w), dtype=torch.complex64, device="cuda")
    x[3, 17] = 1.0
    out = torch.empty_like(x)
    hg.hg_propagate(plan, x, out, hg.HG_FORWARD, ws)
    rows = np.array([0, 1, 2, 3, 4095, 4096, 8191] + list(np.random.default_rng(8).integers(0, h, 9)))
    got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    l = np.arange(w)[None, :]
    ref = np.exp(-2j * np.pi * (np.mod(3 * rows[:, None], h) / h + np.mod(17 * l, w) / w))
    assert np.abs(got - ref).max() <= 1e-5
    m = torch.arange(h, device="cuda", dtype=torch.float64)[:, None]
    n = torch.arange(w, device="cuda", dtype=torch.float64)[None, :]
    ang = 2 * np.pi * (torch.remainder(5 * m, h) / h + torch.remainder(300 * n, w) / w)
    pw = torch.polar(torch.ones_like(ang), ang).to(torch.complex64)
    del ang
    hg.hg_propagate(plan, pw, out, hg.HG_FORWARD, ws)
    err = out.clone()
    err[5, 300] -= h * w
    assert float(err.abs().max()) <= 1e-5 * h * w
    back = torch.empty_like(out)
    hg.hg_propagate(plan, out, back, hg.HG_INVERSE, ws)
    rel = float(torch.linalg.vector_norm(back - pw) / torch.linalg.vector_norm(pw))
    assert rel <= TOL, rel
