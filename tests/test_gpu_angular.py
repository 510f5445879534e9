"""GPU angular-spectrum propagation and Gerchberg-Saxton on it (HG_ANGULAR)
against the FP64 oracle (oracle.angular_spectrum, oracle.gs_iterate with
`angular`), plus a closed form that does not go through the oracle: a sampled
plane wave is an eigenfunction of the operator, so it comes out multiplied by
the transfer function at its own frequency.

Bars: propagation relative L2 <= 1e-5 (as for the other transforms); GS NMSE
per iteration within 1e-4 relative; continuous phase as in the other GS
tests; quantised levels state by state up to the first in-band tie."""
import numpy as np
import pytest

import oracle
from paper_2006_10509_amd import hologen as hg
from paper_2006_10509_amd import workloads as wl
from gpu_util import boundary_distance, dev, host, phase_parity, rel_l2, torch_mod

pytestmark = pytest.mark.gpu
TOL = 1e-5
NMSE_TOL = 1e-4
LAMBDA, PITCH = 532e-9, 8e-6


def as_plan(h, w, z, levels=0, pitch=PITCH):
    mod = hg.HG_PHASE_QUANTISED if levels else hg.HG_PHASE
    return hg.Plan(w, h, hg.HG_ANGULAR, LAMBDA, pitch, z, mod, levels)


def propagate(plan, x, direction, inplace=False):
    torch = torch_mod()
    xin = dev(x)
    out = xin if inplace else torch.empty_like(xin)
    hg.hg_propagate(plan, xin, out, direction, plan.workspace())
    return host(out)


@pytest.mark.parametrize("h,w,z", [(64, 64, 0.01), (128, 120, 0.05), (90, 120, -0.02), (256, 256, 0.2),
                                   (1024, 1024, 0.05), (1080, 1920, 0.1)])
def test_propagate_matches_oracle(h, w, z):
    print(f"angular propagate {h}x{w} z={z}", flush=True)
    plan = as_plan(h, w, z)
    x = wl.random_field(h, w, seed=h + 3 * w)
    x64 = x.astype(np.complex128)
    for direction in (hg.HG_FORWARD, hg.HG_INVERSE):
        got = propagate(plan, x, direction, inplace=direction == hg.HG_INVERSE)
        ref = oracle.angular_spectrum(x64, direction, LAMBDA, PITCH, z)
        assert rel_l2(got, ref) <= TOL, direction


@pytest.mark.parametrize("ky,kx", [(0, 0), (3, 5), (-7, 11), (31, -30), (-32, -32)])
def test_plane_wave_is_scaled_by_the_transfer_function(ky, kx):
    h = w = 64
    z = 0.03
    y, x = np.mgrid[0:h, 0:w]
    wave = np.exp(2j * np.pi * (ky * y / h + kx * x / w))
    fy, fx = ky / (h * PITCH), kx / (w * PITCH)
    kz = 2 * np.pi * np.sqrt(1.0 / LAMBDA ** 2 - fx * fx - fy * fy)
    plan = as_plan(h, w, z)
    got = propagate(plan, wave.astype(np.complex64), hg.HG_FORWARD)
    assert rel_l2(got, wave * np.exp(1j * kz * z)) <= TOL
    back = propagate(plan, wave.astype(np.complex64), hg.HG_INVERSE)
    assert rel_l2(back, wave * np.exp(-1j * kz * z)) <= TOL


def test_forward_then_inverse_is_the_identity():
    h, w = 256, 120
    plan = as_plan(h, w, 0.1)
    x = wl.random_field(h, w, seed=3)
    y = propagate(plan, propagate(plan, x, hg.HG_FORWARD), hg.HG_INVERSE)
    assert rel_l2(y, x) <= 2 * TOL


def test_zero_distance_is_the_identity_and_pitch_limit_is_checked():
    x = wl.random_field(32, 32, seed=4)
    assert rel_l2(propagate(as_plan(32, 32, 0.0), x, hg.HG_FORWARD), x) <= TOL
    with pytest.raises(hg.HologenError, match="wavelength"):
        as_plan(32, 32, 0.01, pitch=LAMBDA / np.sqrt(2) * 0.99)


def run_gs(plan, target, phi0, iters, illum=None):
    torch = torch_mod()
    ph = dev(phi0.copy())
    lv = torch.zeros(target.shape, dtype=torch.uint8, device="cuda")
    nm = torch.zeros(iters + 1, dtype=torch.float32, device="cuda")
    hg.hg_gs_iterate(plan, dev(target), ph, iters, plan.workspace(),
                     illumination=None if illum is None else dev(illum), levels=lv, nmse=nm)
    return host(ph), host(lv), host(nm)


@pytest.mark.parametrize("h,w,levels,z,iters,illum", [
    (128, 128, 0, 0.05, 10, False),
    (120, 128, 0, 0.02, 8, True),
    (256, 256, 8, 0.05, 6, False),
    (64, 90, 2, 0.01, 6, False),
    (1024, 1024, 0, 0.05, 3, False),
])
def test_gs_matches_oracle(h, w, levels, z, iters, illum):
    print(f"angular GS {h}x{w} L={levels} z={z} iters={iters} illum={illum}", flush=True)
    target, phi0 = wl.target_and_phase(h, w, seed=h + w + levels)
    yy, xx = np.mgrid[0:h, 0:w]
    a = np.exp(-((yy - h / 2) ** 2 + (xx - w / 2) ** 2) / (2 * 40.0 ** 2)).astype(np.float32) if illum else None
    plan = as_plan(h, w, z, levels)
    phase, lev, nm = run_gs(plan, target, phi0, iters, a)
    ref = oracle.gs_iterate(target, phi0, iters, levels=levels, illumination=a, trace=bool(levels),
                            angular=dict(wavelength=LAMBDA, pitch=PITCH, distance=z))
    rel = np.abs(nm - np.array(ref["nmse"])) / np.array(ref["nmse"])
    assert rel.max() <= NMSE_TOL, (rel.max(), int(rel.argmax()))
    if levels:
        # one iteration per call, state by state, up to the first in-band tie
        torch = torch_mod()
        ph = dev(phi0.copy())
        lv = torch.zeros((h, w), dtype=torch.uint8, device="cuda")
        ws, t = plan.workspace(), dev(target)
        for k in range(iters + 1):
            hg.hg_gs_iterate(plan, t, ph, 0 if k == 0 else 1, ws, levels=lv)
            g, r = host(lv), ref["trace"][k]
            diff = g != r["levels"]
            if diff.any():
                band = boundary_distance(r["angle"], levels) < 1e-5
                assert not (diff & ~band).any(), f"state {k}"
                break
        else:
            assert np.array_equal(lev, ref["levels"])
    else:
        l2, frac = phase_parity(phase, ref["phase"])
        assert l2 <= 1e-4 and frac <= 1e-4, (l2, frac)


def test_gs_replay_is_the_angular_propagation_of_the_hologram():
    """The NMSE the loop reports for its final state equals the NMSE of
    hg_propagate applied to that state's hologram, against the unshifted target."""
    h, w, z, iters = 128, 128, 0.05, 5
    target, phi0 = wl.target_and_phase(h, w, seed=11)
    plan = as_plan(h, w, z)
    phase, _, nm = run_gs(plan, target, phi0, iters)
    replay = propagate(plan, np.exp(1j * phase.astype(np.float64)).astype(np.complex64), hg.HG_FORWARD)
    e = oracle.nmse(np.abs(replay.astype(np.complex128)) ** 2, target.astype(np.float64) ** 2)
    assert abs(nm[-1] - e) <= 1e-4 * e


def test_angular_plans_are_rejected_where_unsupported():
    torch = torch_mod()
    h = w = 64
    plan = as_plan(h, w, 0.05, levels=2)
    t = dev(wl.target_amplitude(h, w, seed=1))
    ph = torch.zeros((2, h, w), dtype=torch.float32, device="cuda")
    ws = torch.empty(hg.workspace_bytes_batched(plan, 2), dtype=torch.uint8, device="cuda")
    with pytest.raises(hg.HologenError, match="HG_FOURIER or HG_FRESNEL"):
        hg.hg_gs_iterate_batched(plan, torch.stack([t, t]), ph, 1, ws)
    with pytest.raises(hg.HologenError, match="HG_FOURIER or HG_FRESNEL"):
        hg.hg_grad([plan], t.reshape(1, h, w), ph[0], hg.grad_workspace([plan]),
                   grad=torch.empty((h, w), dtype=torch.float32, device="cuda"))
    lv = torch.zeros((h, w), dtype=torch.uint8, device="cuda")
    trials = torch.zeros((1, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(hg.HologenError, match="HG_FOURIER or HG_FRESNEL"):
        hg.hg_pixel_search(plan, t, lv, trials, hg.search_workspace(plan))
