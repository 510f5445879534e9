"""HIP graph capture of library calls: a call enqueues kernels only (no host
synchronisation, allocation, copy or memset), so it can be captured into a
graph and replayed.  Every replay is checked against the eager result, with
eager work and synchronisation between replays."""
import numpy as np
import pytest

from paper_2006_10509_amd import hologen as hg
from paper_2006_10509_amd import workloads as wl
from gpu_util import dev, host, torch_mod

pytestmark = pytest.mark.gpu


def test_captured_batched_gs_replays_match_eager():
    torch = torch_mod()
    h, w, batch, iters = 256, 256, 3, 10
    plan = hg.Plan(w, h, hg.HG_FRESNEL, 532e-9, 8e-6, 0.5, hg.HG_PHASE_QUANTISED, 8)
    ts, ps = zip(*[wl.target_and_phase(h, w, 60 + i) for i in range(batch)])
    target = dev(np.stack(ts))
    phase0 = dev(np.stack(ps))
    ws = torch.empty(hg.workspace_bytes_batched(plan, batch), dtype=torch.uint8, device="cuda")
    phase = phase0.clone()
    nmse = torch.zeros((batch, iters + 1), dtype=torch.float32, device="cuda")
    hg.hg_gs_iterate_batched(plan, target, phase, iters, ws, nmse=nmse)
    eager_phase, eager_nmse = host(phase).copy(), host(nmse).copy()

    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        phase.copy_(phase0)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            hg.hg_gs_iterate_batched(plan, target, phase, iters, ws, nmse=nmse)
    torch.cuda.current_stream().wait_stream(side)
    for replay in range(4):
        phase.copy_(phase0)                  # eager work between replays
        nmse.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(phase), eager_phase), replay
        assert np.array_equal(host(nmse), eager_nmse), replay


def test_captured_gradient_steps_replay_like_successive_calls():
    torch = torch_mod()
    h, w, steps = 128, 128, 5
    planes = [hg.Plan(w, h, hg.HG_FRESNEL, 532e-9, 8e-6, z) for z in (0.45, 0.5)]
    rng = np.random.default_rng(3)
    target = dev(np.stack([wl.target_amplitude(h, w, 70 + j) for j in range(2)]))
    phi0 = dev(rng.uniform(0, 2 * np.pi, (h, w)).astype(np.float32))
    gws = hg.grad_workspace(planes)

    def eager(first):
        ph, m, v = phi0.clone(), torch.zeros_like(phi0), torch.zeros_like(phi0)
        loss = torch.empty(steps + 1, device="cuda")
        hg.hg_grad_adam(planes, target, ph, m, v, steps, gws, first_step=1, loss=loss)
        return host(ph).copy(), host(loss).copy()

    ref_phase, ref_loss = eager(1)
    ph, m, v = phi0.clone(), torch.zeros_like(phi0), torch.zeros_like(phi0)
    loss = torch.empty(steps + 1, device="cuda")
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            hg.hg_grad_adam(planes, target, ph, m, v, steps, gws, first_step=1, loss=loss)
    torch.cuda.current_stream().wait_stream(side)
    for replay in range(3):
        ph.copy_(phi0)
        m.zero_()
        v.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(ph), ref_phase), replay
        assert np.array_equal(host(loss), ref_loss), replay


def test_captured_ospr_replays_match_eager():
    """Plain OSPR (half-spectrum column pass, row pairs) and the real/imaginary
    pairs, each captured once; the inputs are unchanged by a call, so every
    replay must reproduce the eager outputs."""
    torch = torch_mod()
    h, w, n_sub = 256, 256, 4
    t = dev(wl.target_amplitude(h, w, seed=5))
    th = dev(np.stack([wl.uniform_phase(h, w, seed=70 + n) for n in range(n_sub)]))
    plan = hg.Plan(w, h, hg.HG_FOURIER, 0, 0, 0, hg.HG_BINARY_PHASE, 2)
    ws = plan.workspace()
    for pairs in (False, True):
        call = hg.hg_ospr_pairs if pairs else hg.hg_ospr
        inten = torch.empty((h, w), dtype=torch.float32, device="cuda")
        holo = torch.empty((n_sub, h, w), dtype=torch.uint8, device="cuda")   # pairs: 2 per phase
        nm = torch.empty(1, dtype=torch.float32, device="cuda")
        phases = th[: n_sub // 2] if pairs else th
        call(plan, t, phases, inten, ws, holograms=holo, nmse=nm)
        eager = [host(x).copy() for x in (inten, holo, nm)]
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            torch.cuda.synchronize()
            with torch.cuda.graph(graph, stream=side):
                call(plan, t, phases, inten, ws, holograms=holo, nmse=nm)
        torch.cuda.current_stream().wait_stream(side)
        for replay in range(3):
            inten.zero_()                    # eager work between replays
            holo.zero_()
            nm.zero_()
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            for name, e, g in zip(("intensity", "holograms", "nmse"), eager, (inten, holo, nm)):
                assert np.array_equal(host(g), e), (pairs, replay, name)


def test_captured_pixel_search_replays_match_eager():
    """Direct search captured once (one launch per two trials); each replay
    starts from the same level map and must reproduce the eager decisions,
    level map and error trace."""
    torch = torch_mod()
    h = w = 128
    n_trials = 301
    rng = np.random.default_rng(21)
    t = dev(wl.target_amplitude(h, w, seed=6))
    plan = hg.Plan(w, h, hg.HG_FOURIER, 0, 0, 0, hg.HG_BINARY_PHASE, 2)
    lev0 = dev(rng.integers(0, 2, (h, w)).astype(np.uint8))
    trials = dev(np.stack([rng.integers(0, h * w, n_trials), rng.integers(0, 2, n_trials)],
                          axis=1).astype(np.int32))
    ws = hg.search_workspace(plan)
    lev = lev0.clone()
    acc = torch.empty(n_trials, dtype=torch.uint8, device="cuda")
    nm = torch.empty(n_trials + 1, dtype=torch.float32, device="cuda")
    hg.hg_pixel_search(plan, t, lev, trials, ws, accepted=acc, nmse=nm)
    eager = [host(x).copy() for x in (lev, acc, nm)]
    assert 0 < eager[1].sum() < n_trials
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        lev.copy_(lev0)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            hg.hg_pixel_search(plan, t, lev, trials, ws, accepted=acc, nmse=nm)
    torch.cuda.current_stream().wait_stream(side)
    for replay in range(3):
        lev.copy_(lev0)                      # eager work between replays
        acc.zero_()
        nm.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for name, e, g in zip(("levels", "accepted", "nmse"), eager, (lev, acc, nm)):
            assert np.array_equal(host(g), e), (replay, name)
