"""Batched GS (hg_gs_iterate_batched): one launch per pass over a stack of
same-shape holograms.  Bar: bitwise equal to hg_gs_iterate on each item
(same kernels, one more grid dimension), which the single-hologram parity
tests tie to the oracle; one item of a batch is also checked against the
oracle directly."""
import numpy as np
import pytest

import oracle
from paper_2006_10509_amd import hologen as hg
from paper_2006_10509_amd import workloads as wl
from gpu_util import dev, host, torch_mod

pytestmark = pytest.mark.gpu


def stack(h, w, batch, seed0):
    ts, ps = zip(*[wl.target_and_phase(h, w, seed0 + i) for i in range(batch)])
    return np.stack(ts), np.stack(ps)


def make_plan(h, w, levels, fresnel):
    mod = hg.HG_PHASE_QUANTISED if levels else hg.HG_PHASE
    if fresnel:
        return hg.Plan(w, h, hg.HG_FRESNEL, 532e-9, 8e-6, 0.5, mod, levels)
    return hg.Plan(w, h, hg.HG_FOURIER, 0.0, 0.0, 0.0, mod, levels)


def run_batched(plan, targets, phases, iters, illum=None):
    torch = torch_mod()
    b = targets.shape[0]
    ph = dev(phases.copy())
    lv = torch.zeros(targets.shape, dtype=torch.uint8, device="cuda")
    nm = torch.zeros((b, iters + 1), dtype=torch.float32, device="cuda")
    ws = torch.empty(hg.workspace_bytes_batched(plan, b), dtype=torch.uint8, device="cuda")
    hg.hg_gs_iterate_batched(plan, dev(targets), ph, iters, ws, illumination=None if illum is None else dev(illum),
                             levels=lv, nmse=nm)
    return host(ph), host(lv), host(nm)


def run_single(plan, target, phase, iters, illum=None):
    torch = torch_mod()
    ph = dev(phase.copy())
    lv = torch.zeros(target.shape, dtype=torch.uint8, device="cuda")
    nm = torch.zeros(iters + 1, dtype=torch.float32, device="cuda")
    hg.hg_gs_iterate(plan, dev(target), ph, iters, plan.workspace(),
                     illumination=None if illum is None else dev(illum), levels=lv, nmse=nm)
    return host(ph), host(lv), host(nm)


@pytest.mark.parametrize("h,w,batch,levels,fresnel,iters", [
    (256, 256, 5, 8, True, 12),
    (512, 512, 3, 4, False, 6),
    (1080, 1920, 2, 4, False, 3),
    (120, 90, 4, 0, True, 7),
    (2048, 2048, 2, 4, False, 2),
    (1024, 1024, 3, 8, True, 3),
    (1080, 1024, 2, 4, False, 2),
])
def test_batched_equals_single_calls_bitwise(h, w, batch, levels, fresnel, iters):
    print(f"batched {batch} x {h}x{w} L={levels} fresnel={fresnel} it={iters}", flush=True)
    plan = make_plan(h, w, levels, fresnel)
    targets, phases = stack(h, w, batch, 100 + h)
    bp, bl, bn = run_batched(plan, targets, phases, iters)
    for i in range(batch):
        sp, sl, sn = run_single(plan, targets[i], phases[i], iters)
        assert np.array_equal(bp[i], sp) and np.array_equal(bl[i], sl) and np.array_equal(bn[i], sn), i


def test_batched_shared_illumination_and_zero_iterations():
    h, w, batch = 128, 128, 3
    plan = make_plan(h, w, 8, True)
    targets, phases = stack(h, w, batch, 7)
    yy, xx = np.mgrid[0:h, 0:w]
    illum = np.exp(-((yy - h / 2) ** 2 + (xx - w / 2) ** 2) / (2 * 40.0 ** 2)).astype(np.float32)
    for iters in (0, 4):
        bp, bl, bn = run_batched(plan, targets, phases, iters, illum)
        for i in range(batch):
            sp, sl, sn = run_single(plan, targets[i], phases[i], iters, illum)
            assert np.array_equal(bp[i], sp) and np.array_equal(bl[i], sl) and np.array_equal(bn[i], sn)


def test_batch_item_against_oracle():
    h, w, batch, iters = 512, 512, 4, 5
    plan = make_plan(h, w, 4, False)
    targets, phases = stack(h, w, batch, 40)
    _, _, bn = run_batched(plan, targets, phases, iters)
    i = batch - 1
    ref = oracle.gs_iterate(targets[i], phases[i], iters, levels=4)
    rel = np.abs(bn[i] - np.array(ref["nmse"])) / np.array(ref["nmse"])
    assert rel.max() <= 1e-4


def test_batched_argument_checks():
    torch = torch_mod()
    plan = make_plan(64, 64, 4, False)
    targets, phases = stack(64, 64, 2, 1)
    ws = torch.empty(hg.workspace_bytes_batched(plan, 1), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):   # workspace sized for one item
        hg.hg_gs_iterate_batched(plan, dev(targets), dev(phases), 2, ws)
    assert hg.workspace_bytes_batched(plan, 1) == plan.workspace_bytes()
    assert hg.workspace_bytes_batched(plan, 0) == 0


def batched_level_states(plan, targets, phases, iters):
    """Level maps of every state 0..iters of every item, one batched iteration
    per call (bitwise the same as one long call), plus the NMSE of one long call."""
    torch = torch_mod()
    b = targets.shape[0]
    t = dev(targets)
    ws = torch.empty(hg.workspace_bytes_batched(plan, b), dtype=torch.uint8, device="cuda")
    ph = dev(phases.copy())
    lv = torch.zeros(targets.shape, dtype=torch.uint8, device="cuda")
    hg.hg_gs_iterate_batched(plan, t, ph, 0, ws, levels=lv)
    states = [host(lv).copy()]
    for _ in range(iters):
        hg.hg_gs_iterate_batched(plan, t, ph, 1, ws, levels=lv)
        states.append(host(lv).copy())
    full_ph, full_lv, nm = run_batched(plan, targets, phases, iters)
    assert np.array_equal(full_lv, states[-1])
    return [[s[i] for s in states] for i in range(b)], nm


# (height, width, iterations) per shape class of the 64-hologram mix, Fourier, L = 4
MIX_CLASSES = [(512, 512, 10), (1024, 1024, 6), (2048, 2048, 3), (1080, 1920, 4)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("h,w,iters", MIX_CLASSES)
def test_mix_shape_class_item_against_oracle(h, w, iters):
    """One item of each shape class of the mixed batch (its own seed from the
    mix, run in a batch of two of that class as the mix runs it) against the
    oracle: levels of every state outside the boundary band and the NMSE of
    every state, the oracle restarted from the GPU's state at an in-band tie."""
    from test_gpu_gs import check_quantised_segments
    mix = [(hh, ww, seed) for hh, ww, seed in wl.batched_mix() if (hh, ww) == (h, w)]
    seeds = [mix[0][2], mix[-1][2]]
    print(f"mix class {h}x{w}: seeds {seeds}, {iters} iterations", flush=True)
    ts, ps = zip(*[wl.target_and_phase(h, w, s) for s in seeds])
    targets, phases = np.stack(ts), np.stack(ps)
    plan = make_plan(h, w, 4, False)
    states, nm = batched_level_states(plan, targets, phases, iters)
    i = 1            # the class's last item: the second of its batch
    restarts = check_quantised_segments(targets[i], phases[i], iters, 4, None, None, nm[i], states[i])
    print(f"oracle restarted at states {restarts}")


# ---------------------------------------------------------------------------
# batched multi-plane GS (hg_gs_multiplane_batched)
# ---------------------------------------------------------------------------
def mp_planes(h, w, specs, levels):
    mod = hg.HG_PHASE_QUANTISED if levels else hg.HG_PHASE
    return [hg.Plan(w, h, hg.HG_FOURIER, 0.0, 0.0, 0.0, mod, levels) if z is None else
            hg.Plan(w, h, hg.HG_FRESNEL, 532e-9, 8e-6, z, mod, levels) for z in specs]


def mp_problems(h, w, P, batch, seed0):
    t = np.stack([np.stack([wl.target_amplitude(h, w, seed=seed0 + 10 * b + j) for j in range(P)])
                  for b in range(batch)])
    ph = np.stack([wl.uniform_phase(h, w, seed=seed0 + 10 * b + 9) for b in range(batch)])
    return t, ph


@pytest.mark.parametrize("h,w,specs,levels,batch,iters", [
    (256, 256, [0.40, 0.45, 0.50], 8, 3, 4),
    (90, 120, [0.5, None], 0, 4, 5),
    (1024, 1024, [0.45, 0.50], 4, 2, 2),     # four-column workgroups for the batch
    (64, 64, [None, 0.5, None], 3, 5, 3),
])
def test_batched_multiplane_equals_single_calls_bitwise(h, w, specs, levels, batch, iters):
    """Every problem of one batched multi-plane call (phase, level map, the
    error of every step and of the final state at every plane) is bitwise
    the single-problem hg_gs_multiplane call."""
    print(f"batched multiplane {h}x{w} planes={specs} L={levels} batch={batch} it={iters}", flush=True)
    torch = torch_mod()
    planes = mp_planes(h, w, specs, levels)
    P = len(planes)
    t, ph0 = mp_problems(h, w, P, batch, 40)
    ph = dev(ph0.copy())
    lv = torch.zeros((batch, h, w), dtype=torch.uint8, device="cuda")
    nm = torch.zeros((batch, iters * P + P), dtype=torch.float32, device="cuda")
    hg.hg_gs_multiplane_batched(planes, dev(t), ph, iters, hg.multiplane_workspace_batched(planes, batch),
                                levels=lv, nmse=nm)
    ph, lv, nm = host(ph), host(lv), host(nm)
    for b in range(batch):
        p1 = dev(ph0[b].copy())
        l1 = torch.zeros((h, w), dtype=torch.uint8, device="cuda")
        n1 = torch.zeros(iters * P + P, dtype=torch.float32, device="cuda")
        hg.hg_gs_multiplane(planes, dev(t[b]), p1, iters, hg.multiplane_workspace(planes), levels=l1, nmse=n1)
        assert np.array_equal(ph[b].view(np.uint32), host(p1).view(np.uint32)), b
        assert np.array_equal(lv[b], host(l1)), b
        assert np.array_equal(nm[b].view(np.uint32), host(n1).view(np.uint32)), b


def test_batched_multiplane_item_against_oracle():
    """One problem of a batch against the FP64 oracle: the error of every step
    within 1e-4 relative and the continuous phase at the continuous-phase bar."""
    from gpu_util import phase_parity
    torch = torch_mod()
    h = w = 128
    zs = (0.40, 0.45, 0.50)
    planes = mp_planes(h, w, list(zs), 0)
    batch, iters = 3, 2
    t, ph0 = mp_problems(h, w, 3, batch, 70)
    ph = dev(ph0.copy())
    nm = torch.zeros((batch, iters * 3 + 3), dtype=torch.float32, device="cuda")
    hg.hg_gs_multiplane_batched(planes, dev(t), ph, iters, hg.multiplane_workspace_batched(planes, batch), nmse=nm)
    b = 2
    ref = oracle.gs_multiplane(list(t[b]), ph0[b], iters,
                               [dict(wavelength=532e-9, pitch=8e-6, distance=z) for z in zs])
    rel = np.abs(host(nm)[b] - np.array(ref["nmse"])) / np.array(ref["nmse"])
    assert rel.max() <= 1e-4, (rel.max(), int(rel.argmax()))
    l2, frac = phase_parity(host(ph)[b], ref["phase"])
    assert l2 <= 1e-4 and frac <= 1e-4, (l2, frac)


def test_batched_multiplane_argument_checks():
    torch = torch_mod()
    h = w = 64
    planes = mp_planes(h, w, [0.5, None], 4)
    t = torch.ones((2, 2, h, w), dtype=torch.float32, device="cuda")
    ph = torch.zeros((2, h, w), dtype=torch.float32, device="cuda")
    assert hg.library().hg_multiplane_workspace_bytes_batched(planes[0].handle, 2, 0) == 0
    assert hg.library().hg_multiplane_workspace_bytes_batched(planes[0].handle, 2, 65536) == 0
    assert (hg.library().hg_multiplane_workspace_bytes_batched(planes[0].handle, 2, 1) ==
            hg.library().hg_multiplane_workspace_bytes(planes[0].handle, 2))
    with pytest.raises(ValueError):   # workspace for one problem, two in the call
        hg.hg_gs_multiplane_batched(planes, t, ph, 1, hg.multiplane_workspace(planes))
    amp = [hg.Plan(w, h, hg.HG_FOURIER, 0.0, 0.0, 0.0, hg.HG_AMPLITUDE, 0)]
    with pytest.raises(hg.HologenError):
        hg.hg_gs_multiplane_batched(amp, t[:, :1].contiguous(), ph, 1, hg.multiplane_workspace_batched(amp, 2))
