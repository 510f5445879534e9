"""Throughput of the Gerchberg-Saxton hot path on one MI355X.

Workload: Fresnel GS hologram, 1024x1024 complex FP32 field, 8-level phase
quantisation, 100 iterations per step (lambda 532 nm, 8 um pitch, z 0.5 m;
synthetic target seed 2, starting phase seed 3).  One step = one
hg_gs_iterate call: per-call statistics, the start row pass, 100 x (replay
column pass + SLM row pass), the final NMSE pass and the NMSE reduction.
Successive steps continue from the SLM state the previous step left, which
is the same work per step.

Output: one JSON line with iterations/s, the roofline position of the
dominant kernel (HIP events on the launch stream) and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GS iterations/s at 1024² (HBM GB/s, % peak); grad-CGH vs GS time to NMSE"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per pixel of one launch: field read + target read + field write
BYTES_PER_PX = {"gs_replay_column_pass": 8 + 4 + 8, "gs_slm_row_pass": 8 + 8}
# back-to-back executions per timed launch (hg_timing_begin): one event pair
# around each group, nothing attached to the kernel launches themselves
TIMING_REPEATS = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2006_10509_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    entry = data.get(kernel)
    if not entry or entry.get("source_hash") != source_hash():
        return None
    return entry.get("bytes_per_launch")


def host_identity() -> dict:
    """The host the CPU baseline ran on: logical CPUs, the CPUs this process
    may use, the CPU model and the NumPy version."""
    import platform
    import numpy as np
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "cpu_model": model, "numpy": np.__version__}


def cpu_baseline(workload, target, phi0, sample_iters: int):
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    fres = dict(wavelength=workload.wavelength, pitch=workload.pitch, distance=workload.distance)
    t0 = time.perf_counter()
    oracle.gs_iterate(target, phi0, sample_iters, levels=workload.levels, fresnel=fres)
    dt = time.perf_counter() - t0
    return {"value": sample_iters / dt, "unit": "iterations/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{sample_iters} of the {workload.iterations} iterations of the same "
                      f"{workload.height}x{workload.width} workload and inputs, FP64, "
                      f"including its one extra NMSE transform ({dt:.1f} s)",
            "threads": "one Python process; its FFT's batched small-DFT products run on the BLAS "
                       f"thread pool ({threads} threads), the rest of NumPy on one thread",
            "host": host_identity()}


def time_to_nmse(hg, wl, torch, stream) -> dict:
    """Wall-clock time for gradient-descent CGH (Adam, lr 0.05, one Fresnel
    plane, continuous phase) to reach the NMSE that continuous GS reaches after
    100 iterations, on the same 1024x1024 target, starting phase and geometry;
    both timed with HIP events on the launch stream, inputs resident."""
    w = wl.GS_FRESNEL_1024_CONT
    target, phi0 = w.inputs()
    t = torch.from_numpy(target).cuda()
    plan = hg.Plan(w.width, w.height, hg.HG_FRESNEL, w.wavelength, w.pitch, w.distance, hg.HG_PHASE, 0)
    ws = plan.workspace()
    nm = torch.empty(w.iterations + 1, dtype=torch.float32, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run_gs():
        ph = torch.from_numpy(phi0.copy()).cuda()
        torch.cuda.synchronize()
        a.record(stream)
        hg.hg_gs_iterate(plan, t, ph, w.iterations, ws, nmse=nm, stream=stream)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b)

    run_gs()
    gs_ms = run_gs()
    threshold = float(nm[-1].item())
    planes = [plan]
    gws = hg.grad_workspace(planes)
    tt = t[None].contiguous()
    max_steps = 500

    def run_grad(steps):
        ph = torch.from_numpy(phi0.copy()).cuda()
        m = torch.zeros_like(ph)
        v = torch.zeros_like(ph)
        loss = torch.empty(steps + 1, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        a.record(stream)
        hg.hg_grad_adam(planes, tt, ph, m, v, steps, gws, lr=0.05, loss=loss, stream=stream)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b), loss.cpu().numpy()

    run_grad(10)
    full_ms, losses = run_grad(max_steps)
    hit = [k for k, x in enumerate(losses) if x <= threshold]
    steps = hit[0] if hit else None
    grad_ms = run_grad(steps)[0] if steps else None
    return {"workload": w.name, "threshold_nmse": threshold, "gs_iterations": w.iterations,
            "gs_ms": round(gs_ms, 3), "grad_steps_to_threshold": steps,
            "grad_ms_to_threshold": None if grad_ms is None else round(grad_ms, 3),
            "grad_ms_per_step": round(full_ms / max_steps, 4), "grad_nmse_after_500": float(losses[-1]),
            "optimizer": "adam lr 0.05, one Fresnel plane z 0.5 m, continuous phase"}


def grad_batch(hg, wl, torch, stream, problems: int) -> dict:
    """The 3-plane gradient workload: `problems` problems of 500 Adam steps
    each, all in one hg_grad_adam_batched call (problems on grid.y), against
    one hg_grad_adam call per problem; problem-steps/s, results compared
    bitwise."""
    w = wl.GRAD_3PLANE_1024
    planes = [hg.Plan(w.width, w.height, hg.HG_FRESNEL, w.wavelength, w.pitch, z, hg.HG_PHASE, 0)
              for z in w.distances]
    gws = hg.grad_workspace(planes)
    data = [(torch.from_numpy(w.targets(bi)).cuda(), torch.from_numpy(w.phase0(bi)).cuda())
            for bi in range(problems)]
    seq_losses = torch.empty((problems, w.steps + 1), dtype=torch.float32, device="cuda")
    seq_phase = []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for bi, (tg, p0) in enumerate(data):
        ph = p0.clone()
        m = torch.zeros_like(ph)
        v = torch.zeros_like(ph)
        hg.hg_grad_adam(planes, tg, ph, m, v, w.steps, gws, lr=w.lr, loss=seq_losses[bi], stream=stream)
        seq_phase.append(ph)
    b.record(stream)
    b.synchronize()
    seq_ms = a.elapsed_time(b)
    tb = torch.stack([tg for tg, _ in data])
    pb0 = torch.stack([p0 for _, p0 in data])
    bws = hg.grad_workspace_batched(planes, problems)
    losses = torch.empty((problems, w.steps + 1), dtype=torch.float32, device="cuda")

    def run_batched():
        ph = pb0.clone()
        m = torch.zeros_like(ph)
        v = torch.zeros_like(ph)
        torch.cuda.synchronize()
        a.record(stream)
        hg.hg_grad_adam_batched(planes, tb, ph, m, v, w.steps, bws, lr=w.lr, loss=losses, stream=stream)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b), ph

    run_batched()
    ms, bph = run_batched()
    same = bool(torch.equal(losses, seq_losses) and all(torch.equal(bph[i], seq_phase[i]) for i in range(problems)))
    fin = losses[:, -1].cpu().numpy()
    # the same problems with plane-by-plane multi-plane GS (continuous phase),
    # 100 iterations of 3 steps each: summed final NMSE over the planes
    # (all problems in one hg_gs_multiplane_batched call, and one call each)
    mws = hg.multiplane_workspace(planes)
    iters = 100
    n_mp = iters * len(planes) + len(planes)
    mnm = torch.empty((problems, n_mp), dtype=torch.float32, device="cuda")
    seq_ph = torch.stack([p0 for _, p0 in data])
    torch.cuda.synchronize()
    a.record(stream)
    for bi, (tg, _) in enumerate(data):
        hg.hg_gs_multiplane(planes, tg, seq_ph[bi], iters, mws, nmse=mnm[bi], stream=stream)
    b.record(stream)
    b.synchronize()
    mp_seq_ms = a.elapsed_time(b)
    bws = hg.multiplane_workspace_batched(planes, problems)
    all_t = torch.stack([tg for tg, _ in data])
    bnm = torch.empty((problems, n_mp), dtype=torch.float32, device="cuda")

    def run_mp_batched():
        ph = torch.stack([p0 for _, p0 in data])
        torch.cuda.synchronize()
        a.record(stream)
        hg.hg_gs_multiplane_batched(planes, all_t, ph, iters, bws, nmse=bnm, stream=stream)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b), ph

    run_mp_batched()
    mp_ms, mp_ph = run_mp_batched()
    mp_same = bool(torch.equal(bnm, mnm) and torch.equal(mp_ph, seq_ph))
    mp_final = bnm[:, -len(planes):].sum(dim=1).cpu().numpy()
    return {"workload": w.name, "problems": problems, "steps": w.steps, "planes": len(w.distances),
            "multiplane_gs": {"iterations": iters, "ms": round(mp_ms, 2), "sequential_ms": round(mp_seq_ms, 2),
                              "launch": "one hg_gs_multiplane_batched call for all problems",
                              "batched_equals_sequential_bitwise": mp_same,
                              "final_loss_mean": float(mp_final.mean())},
            "launch": "one hg_grad_adam_batched call for all problems",
            "ms": round(ms, 2), "problem_steps_per_s": round(problems * w.steps / (ms * 1e-3), 1),
            "ms_per_step": round(ms / (problems * w.steps), 4),
            "sequential_ms": round(seq_ms, 2),
            "sequential_problem_steps_per_s": round(problems * w.steps / (seq_ms * 1e-3), 1),
            "batched_equals_sequential_bitwise": same,
            "final_loss_mean": float(fin.mean()), "initial_loss_mean": float(losses[:, 0].mean().item())}


def grad_batched_only(hg, wl, torch, stream, problems: int, steps: int = 50) -> dict:
    """The 3-plane gradient workload's batched call alone, `steps` Adam steps
    of every problem in one hg_grad_adam_batched call, timed twice (profiler
    runs: one column launch and one row launch per step)."""
    w = wl.GRAD_3PLANE_1024
    planes = [hg.Plan(w.width, w.height, hg.HG_FRESNEL, w.wavelength, w.pitch, z, hg.HG_PHASE, 0)
              for z in w.distances]
    tb = torch.stack([torch.from_numpy(w.targets(bi)) for bi in range(problems)]).cuda()
    pb0 = torch.stack([torch.from_numpy(w.phase0(bi)) for bi in range(problems)]).cuda()
    bws = hg.grad_workspace_batched(planes, problems)
    loss = torch.empty((problems, steps + 1), dtype=torch.float32, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(2):
        ph = pb0.clone()
        m = torch.zeros_like(ph)
        v = torch.zeros_like(ph)
        torch.cuda.synchronize()
        a.record(stream)
        hg.hg_grad_adam_batched(planes, tb, ph, m, v, steps, bws, lr=w.lr, loss=loss, stream=stream)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return {"workload": w.name, "problems": problems, "steps": steps, "ms": round(ms[-1], 3),
            "problem_steps_per_s": round(problems * steps / (ms[-1] * 1e-3), 1)}


def _mix_inputs(item):
    from paper_2006_10509_amd import workloads as wl
    h, w, seed = item
    return wl.target_and_phase(h, w, seed)


def mix_inputs(wl):
    """Inputs of the mixed batch, generated in worker processes.  Called before
    this process touches the GPU, so the workers start from a GPU-free state."""
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return list(ex.map(_mix_inputs, wl.batched_mix()))


def batched_1024(hg, wl, torch, stream, batch: int = 8, iterations: int = 50) -> dict:
    """The headline workload's kernels with the GPU full: `batch` copies of
    the 1024^2 Fresnel L = 8 problem in one hg_gs_iterate_batched call (NMSE
    of every state), time per hologram-iteration and algorithmic GB/s at
    36 B/px.  Context for the single-hologram roofline, not the metric."""
    w = wl.GS_FRESNEL_1024
    t, p = w.inputs()
    plan = hg.Plan(w.width, w.height, hg.HG_FRESNEL, w.wavelength, w.pitch, w.distance, hg.HG_PHASE_QUANTISED,
                   w.levels)
    tb = torch.from_numpy(t).cuda().expand(batch, w.height, w.width).contiguous()
    pb0 = torch.from_numpy(p).cuda().expand(batch, w.height, w.width).contiguous()
    pb = pb0.clone()
    nm = torch.empty((batch, iterations + 1), dtype=torch.float32, device="cuda")
    ws = torch.empty(hg.workspace_bytes_batched(plan, batch), dtype=torch.uint8, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run():
        pb.copy_(pb0)
        torch.cuda.synchronize()
        a.record(stream)
        hg.hg_gs_iterate_batched(plan, tb, pb, iterations, ws, nmse=nm, stream=stream)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b)

    run()
    ms = min(run() for _ in range(3))
    us = ms * 1e3 / (iterations * batch)
    gbs = sum(BYTES_PER_PX.values()) * w.height * w.width / (us * 1e-6) / 1e9
    return {"workload": w.name, "holograms": batch, "iterations": iterations,
            "us_per_hologram_iteration": round(us, 3), "iteration_gbs": round(gbs, 1),
            "iteration_frac": round(gbs / HBM_PEAK_GBS, 4)}


def batched_mix(hg, wl, torch, stream, inputs, iterations: int = 50) -> dict:
    """The 64-hologram mixed batch (16 x 512^2, 24 x 1024^2, 16 x 2048^2,
    8 x 1080x1920; Fourier GS, 4 levels, 50 iterations, NMSE of every state):
    one hg_gs_iterate_batched call per shape against 64 hg_gs_iterate calls,
    both on one stream with inputs resident, holograms/s."""
    items = wl.batched_mix()
    shapes = sorted({(h, w) for h, w, _ in items})
    plans = {sh: hg.Plan(sh[1], sh[0], hg.HG_FOURIER, 0.0, 0.0, 0.0, hg.HG_PHASE_QUANTISED, 4) for sh in shapes}
    groups = {sh: [i for i, (h, w, _) in enumerate(items) if (h, w) == sh] for sh in shapes}
    targets = [torch.from_numpy(t).cuda() for t, _ in inputs]
    phase0 = [torch.from_numpy(p).cuda() for _, p in inputs]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    single_ws = {sh: plans[sh].workspace() for sh in shapes}
    seq_phase = [p.clone() for p in phase0]
    seq_nmse = [torch.empty(iterations + 1, dtype=torch.float32, device="cuda") for _ in items]

    def run_sequential():
        for i, (h, w, _) in enumerate(items):
            seq_phase[i].copy_(phase0[i])
        torch.cuda.synchronize()
        a.record(stream)
        for i, (h, w, _) in enumerate(items):
            hg.hg_gs_iterate(plans[(h, w)], targets[i], seq_phase[i], iterations, single_ws[(h, w)],
                             nmse=seq_nmse[i], stream=stream)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b)

    bt = {sh: torch.stack([targets[i] for i in groups[sh]]) for sh in shapes}
    bp0 = {sh: torch.stack([phase0[i] for i in groups[sh]]) for sh in shapes}
    bp = {sh: bp0[sh].clone() for sh in shapes}
    bn = {sh: torch.empty((len(groups[sh]), iterations + 1), dtype=torch.float32, device="cuda") for sh in shapes}
    bws = {sh: torch.empty(hg.workspace_bytes_batched(plans[sh], len(groups[sh])), dtype=torch.uint8,
                           device="cuda") for sh in shapes}

    def run_batched():
        for sh in shapes:
            bp[sh].copy_(bp0[sh])
        torch.cuda.synchronize()
        a.record(stream)
        for sh in shapes:
            hg.hg_gs_iterate_batched(plans[sh], bt[sh], bp[sh], iterations, bws[sh], nmse=bn[sh], stream=stream)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b)

    run_sequential()
    run_batched()
    seq_ms = min(run_sequential() for _ in range(3))
    bat_ms = min(run_batched() for _ in range(3))

    # the four batched calls captured once into a HIP graph and replayed
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            for sh in shapes:
                hg.hg_gs_iterate_batched(plans[sh], bt[sh], bp[sh], iterations, bws[sh], nmse=bn[sh])
    stream.wait_stream(side)

    def run_graph():
        for sh in shapes:
            bp[sh].copy_(bp0[sh])
        torch.cuda.synchronize()
        a.record(stream)
        graph.replay()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b)

    run_graph()
    graph_ms = min(run_graph() for _ in range(3))
    same = all(torch.equal(bp[sh][k], seq_phase[i]) and torch.equal(bn[sh][k], seq_nmse[i])
               for sh in shapes for k, i in enumerate(groups[sh]))

    # the four batched calls on four streams of default priority, so that the
    # shapes' passes can run side by side on the GPU
    side_streams = [torch.cuda.Stream() for _ in shapes]

    def run_streams():
        for sh in shapes:
            bp[sh].copy_(bp0[sh])
        torch.cuda.synchronize()
        a.record(stream)
        for sh, ss in zip(shapes, side_streams):
            ss.wait_stream(stream)
            hg.hg_gs_iterate_batched(plans[sh], bt[sh], bp[sh], iterations, bws[sh], nmse=bn[sh], stream=ss)
        for ss in side_streams:
            stream.wait_stream(ss)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b)

    run_streams()
    streams_ms = min(run_streams() for _ in range(3))
    same = same and all(torch.equal(bp[sh][k], seq_phase[i]) and torch.equal(bn[sh][k], seq_nmse[i])
                        for sh in shapes for k, i in enumerate(groups[sh]))
    n = len(items)
    return {"workload": "gs_fourier_L4_50it_mixed64", "holograms": n, "iterations": iterations,
            "sequential_ms": round(seq_ms, 2), "batched_ms": round(bat_ms, 2),
            "sequential_holograms_per_s": round(n / (seq_ms * 1e-3), 1),
            "batched_holograms_per_s": round(n / (bat_ms * 1e-3), 1),
            "speedup": round(seq_ms / bat_ms, 3), "identical_results": bool(same),
            "graph_ms": round(graph_ms, 2), "graph_holograms_per_s": round(n / (graph_ms * 1e-3), 1),
            "four_streams_ms": round(streams_ms, 2),
            "four_streams_holograms_per_s": round(n / (streams_ms * 1e-3), 1),
            "launches": f"{len(shapes)} batched calls vs {n} single calls"}


def ospr_2048(hg, wl, torch, stream) -> dict:
    """The 2048x2048 binary OSPR workload (24 subframes): plain OSPR (one
    inverse transform per subframe) against real/imaginary pairs (two
    subframes per inverse transform, 12 pairs), subframes/s."""
    w = wl.OSPR_2048
    t = torch.from_numpy(w.target()).cuda()
    th = torch.from_numpy(w.subframe_phases()).cuda()
    plan = hg.Plan(w.width, w.height, hg.HG_FOURIER, 0.0, 0.0, 0.0, hg.HG_BINARY_PHASE, 2)
    ws = plan.workspace()
    inten = torch.empty((w.height, w.width), dtype=torch.float32, device="cuda")
    nm = torch.empty(1, dtype=torch.float32, device="cuda")
    # every call writes its binary holograms (level maps) too
    holo = torch.empty((w.subframes, w.height, w.width), dtype=torch.uint8, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(f):
        f()
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(5):
            f()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / 5

    plain_ms = timed(lambda: hg.hg_ospr(plan, t, th, inten, ws, holograms=holo, nmse=nm, stream=stream))
    plain_nmse = float(nm.item())
    eager_out = (inten.clone(), nm.clone(), holo.clone())
    # the plain call captured once into a HIP graph and replayed (its inputs
    # are unchanged by a call, so every replay must equal the eager call)
    inten_g = torch.empty_like(inten)
    nm_g = torch.empty_like(nm)
    holo_g = torch.empty_like(holo)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            hg.hg_ospr(plan, t, th, inten_g, ws, holograms=holo_g, nmse=nm_g)
    stream.wait_stream(side)
    graph.replay()
    torch.cuda.synchronize()
    graph_same = all(torch.equal(x, y) for x, y in zip((inten_g, nm_g, holo_g), eager_out))
    graph_ms = timed(lambda: graph.replay())
    graph_same = graph_same and all(torch.equal(x, y) for x, y in zip((inten_g, nm_g, holo_g), eager_out))
    pair_ms = timed(lambda: hg.hg_ospr_pairs(plan, t, th[:w.subframes // 2], inten, ws, holograms=holo, nmse=nm,
                                             stream=stream))
    pair_nmse = float(nm.item())
    # per-pass durations of the plain run (every launch executed TIMING_REPEATS
    # times back to back).  The hologram is real, so pass B stores only the
    # rows y <= H/2 of its column transform: it reads 8 B/px, writes the level
    # (1 B/px) and half the field (4 B/px), 13 B/px.  Pass C, which after the
    # first subframe also runs the next subframe's pass A, reads that half
    # (4), reads and writes the running intensity of the same rows (the
    # intensity is centro-symmetric; 2 + 2), reads the target and the next
    # phase (8) and writes the field (8): 24 B/px
    npx = w.width * w.height
    passes = {}
    for name, kid, bpp in (("pass_b", hg.HG_KERNEL_OSPR_B, 13), ("pass_c", hg.HG_KERNEL_OSPR_C, 24)):
        hg.hg_timing_begin(plan, kid, TIMING_REPEATS)
        hg.hg_ospr(plan, t, th, inten, ws, holograms=holo, nmse=nm, stream=stream)
        total_ms, count = hg.hg_timing_end(plan)
        us = total_ms * 1e3 / count
        gbs = bpp * npx / (us * 1e-6) / 1e9
        passes[name] = {"us_per_launch": round(us, 3), "algorithmic_bytes_per_px": bpp,
                        "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return {"workload": w.name, "subframes": w.subframes, "plain_ms": round(plain_ms, 3),
            "plain_subframes_per_s": round(w.subframes / (plain_ms * 1e-3), 1), "plain_nmse": plain_nmse,
            "plain_graph": {"ms": round(graph_ms, 3), "subframes_per_s": round(w.subframes / (graph_ms * 1e-3), 1),
                            "bitwise_equal_to_eager": graph_same},
            "pairs_ms": round(pair_ms, 3), "pairs_subframes_per_s": round(w.subframes / (pair_ms * 1e-3), 1),
            "pairs_nmse": pair_nmse, "passes": passes}


def pixel_search_1024(hg, wl, torch, stream, n_trials: int = 2000) -> dict:
    """Direct binary search on a 1024x1024 binary Fourier hologram (target of
    the 1024^2 workload, random start and trial list from seed 12): trials/s.
    Each launch is one pass over the replay field (rank-one updates) that
    decides the previous two trials and evaluates the next two."""
    import numpy as np
    w = wl.GS_FRESNEL_1024
    t = torch.from_numpy(w.inputs()[0]).cuda()
    plan = hg.Plan(w.width, w.height, hg.HG_FOURIER, 0.0, 0.0, 0.0, hg.HG_BINARY_PHASE, 2)
    rng = np.random.default_rng(12)
    lev0 = torch.from_numpy(rng.integers(0, 2, (w.height, w.width)).astype(np.uint8)).cuda()
    trials = torch.from_numpy(np.stack([rng.integers(0, w.height * w.width, n_trials),
                                        rng.integers(0, 2, n_trials)], axis=1).astype(np.int32)).cuda()
    ws = hg.search_workspace(plan)
    acc = torch.empty(n_trials, dtype=torch.uint8, device="cuda")
    nm = torch.empty(n_trials + 1, dtype=torch.float32, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lev = lev0.clone()
    hg.hg_pixel_search(plan, t, lev, trials[:50], ws, accepted=acc[:50], nmse=nm[:51], stream=stream)
    lev = lev0.clone()
    torch.cuda.synchronize()
    a.record(stream)
    hg.hg_pixel_search(plan, t, lev, trials, ws, accepted=acc, nmse=nm, stream=stream)
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b)
    eager_out = (lev.clone(), acc.clone(), nm.clone())
    # the same call captured once into a HIP graph (its 1000 launches), replayed
    # from the same starting level map; every replay must equal the eager call
    lev_g = lev0.clone()
    acc_g = torch.empty_like(acc)
    nm_g = torch.empty_like(nm)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            hg.hg_pixel_search(plan, t, lev_g, trials, ws, accepted=acc_g, nmse=nm_g)
    stream.wait_stream(side)
    graph_ms, graph_same = [], True
    for _ in range(3):
        lev_g.copy_(lev0)
        torch.cuda.synchronize()
        a.record(stream)
        graph.replay()
        b.record(stream)
        b.synchronize()
        graph_ms.append(a.elapsed_time(b))
        graph_same = graph_same and all(torch.equal(x, y) for x, y in zip((lev_g, acc_g, nm_g), eager_out))
    g_ms = min(graph_ms)
    rate = float(acc.float().mean().item())
    # one pass over R per two trials: it reads R and T^2 and writes R back when
    # either trial of the previous pair was accepted
    launches = (n_trials + 1) // 2
    pairs_written = float(acc[: n_trials // 2 * 2].view(-1, 2).amax(dim=1).float().mean().item())
    npx = w.height * w.width
    # (a binary Fourier hologram is real: the pass keeps the rows y <= H/2 of
    # R, reads T^2 at every pixel and its mirror)
    kept = (w.height // 2 + 1) * w.width
    pass_bytes = kept * (8 + 8 * pairs_written) + npx * 4
    us_launch = ms * 1e3 / launches
    gbs = pass_bytes / (us_launch * 1e-6) / 1e9
    return {"workload": "dbs_fourier_binary_1024x1024", "trials": n_trials, "ms": round(ms, 2),
            "trials_per_s": round(n_trials / (ms * 1e-3), 1), "us_per_trial": round(ms * 1e3 / n_trials, 2),
            "trials_per_launch": 2, "us_per_launch": round(us_launch, 2),
            "accept_rate": round(rate, 4), "nmse_start": float(nm[0].item()), "nmse_end": float(nm[-1].item()),
            "pass_gbs": round(gbs, 1), "pass_frac": round(gbs / HBM_PEAK_GBS, 4),
            "graph": {"ms": round(g_ms, 2), "trials_per_s": round(n_trials / (g_ms * 1e-3), 1),
                      "us_per_launch": round(g_ms * 1e3 / launches, 2), "bitwise_equal_to_eager": graph_same}}


SWEEP_SIZES = (256, 512, 1024, 2048, 4096, 8192)


def size_sweep(hg, wl, torch, stream, sizes=SWEEP_SIZES, iterations: int = 20) -> list:
    """The headline's GS (Fresnel, 532 nm, 8 um, 0.5 m, 8 levels, NMSE of every
    state) on square frames from 256^2 to 8192^2, whose working set (field,
    target, phase: 20 B/px) passes the 256 MiB last-level cache above 4096^2.
    The target is the 1024^2 workload's target repeated periodically (cropped
    below 1024), the starting phase uniform from seed 3.  us per iteration,
    algorithmic GB/s at 36 B/px and its fraction of 8 TB/s."""
    w = wl.GS_FRESNEL_1024
    base_t, _ = w.inputs()
    base = torch.from_numpy(base_t).cuda()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = []
    for n in sizes:
        reps = (n + 1023) // 1024
        t = base.repeat(reps, reps)[:n, :n].contiguous()
        g = torch.Generator(device="cuda").manual_seed(3)
        ph0 = torch.rand((n, n), generator=g, device="cuda", dtype=torch.float32) * (2 * 3.141592653589793)
        plan = hg.Plan(n, n, hg.HG_FRESNEL, w.wavelength, w.pitch, w.distance, hg.HG_PHASE_QUANTISED, w.levels)
        ws = plan.workspace()
        nm = torch.empty(iterations + 1, dtype=torch.float32, device="cuda")
        ph = ph0.clone()
        hg.hg_gs_iterate(plan, t, ph, iterations, ws, nmse=nm, stream=stream)
        times = []
        for _ in range(3):
            ph.copy_(ph0)
            torch.cuda.synchronize()
            a.record(stream)
            hg.hg_gs_iterate(plan, t, ph, iterations, ws, nmse=nm, stream=stream)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        us = min(times) * 1e3 / iterations
        gbs = sum(BYTES_PER_PX.values()) * n * n / (us * 1e-6) / 1e9
        out.append({"n": n, "us_per_iteration": round(us, 2), "iterations_per_s": round(1e6 / us, 1),
                    "algorithmic_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "working_set_mib": round(20 * n * n / 2 ** 20, 1), "final_nmse": float(nm[-1].item())})
        log(f"  sweep {n}^2: {out[-1]}")
        del ws, t, ph, ph0, plan
        torch.cuda.empty_cache()
    return out


def rocfft_reference(torch, stream, n: int = 1024, reps: int = 200) -> dict:
    """torch.fft (rocFFT) forward + inverse 2D transform of one n x n complex64
    field, back to back: a vendor-library reference point, not part of the path."""
    x = torch.randn((n, n), dtype=torch.complex64, device="cuda")
    for _ in range(5):
        x = torch.fft.ifft2(torch.fft.fft2(x))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        x = torch.fft.ifft2(torch.fft.fft2(x))
    b.record(stream)
    b.synchronize()
    return {"what": f"torch.fft.fft2 + ifft2 of a {n}x{n} complex64 field (rocFFT)",
            "us_per_pair": round(a.elapsed_time(b) / reps * 1e3, 3)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample-iters", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient-CGH measurements")
    ap.add_argument("--grad-problems", type=int, default=8)
    ap.add_argument("--no-batched", action="store_true", help="skip the mixed-batch measurement")
    ap.add_argument("--driver", choices=("graph", "eager"), default="graph",
                    help="how the timed steps are issued: one captured HIP graph replayed per step "
                         "(default), or the library call per step; both are measured and reported")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload and its kernel timings (for profiler runs)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 256^2 to 8192^2 size sweep")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the size sweep (for profiler runs), printed as one JSON line")
    ap.add_argument("--grad-only", action="store_true",
                    help="only the 3-plane gradient workload, all problems in one call (for profiler runs)")
    ap.add_argument("--ospr-only", action="store_true",
                    help="only the 2048^2 OSPR workload (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 20 device copies of an 8 MiB buffer (rocprofv3 counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2006_10509_amd import hologen as hg
    from paper_2006_10509_amd import workloads as wl

    if args.headline_only or args.sweep_only or args.grad_only or args.ospr_only:
        args.no_grad = args.no_batched = args.no_cpu_baseline = True
    mixed = None
    if not (args.no_batched or args.calibrate_copy):
        log("generating the mixed-batch inputs")
        mixed = mix_inputs(wl)
    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        return 1
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1024 * 1024, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_dispatch": src.numel() * 8,
                          "bytes_written_per_dispatch": dst.numel() * 8, "dispatches": 20}))
        return 0
    if args.sweep_only:
        print(json.dumps({"size_sweep": size_sweep(hg, wl, torch, torch.cuda.current_stream())}), flush=True)
        return 0
    if args.grad_only:
        print(json.dumps({"grad_batched": grad_batched_only(hg, wl, torch, torch.cuda.current_stream(),
                                                            args.grad_problems)}), flush=True)
        return 0
    if args.ospr_only:
        print(json.dumps({"ospr": ospr_2048(hg, wl, torch, torch.cuda.current_stream())}), flush=True)
        return 0
    w = wl.GS_FRESNEL_1024
    target, phi0 = w.inputs()
    plan = hg.Plan(w.width, w.height, hg.HG_FRESNEL, w.wavelength, w.pitch, w.distance,
                   hg.HG_PHASE_QUANTISED, w.levels)
    t = torch.from_numpy(target).cuda()
    phase = torch.from_numpy(phi0.copy()).cuda()
    levels = torch.empty((w.height, w.width), dtype=torch.uint8, device="cuda")
    nmse = torch.empty(w.iterations + 1, dtype=torch.float32, device="cuda")
    ws = plan.workspace()
    stream = torch.cuda.current_stream()

    def step():
        hg.hg_gs_iterate(plan, t, phase, w.iterations, ws, levels=levels, nmse=nmse, stream=stream)

    # The step captured once into a HIP graph: replaying it enqueues the same
    # launches with the same arguments.  One eager step and one replay from
    # the same SLM state must give bitwise the same results.
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            hg.hg_gs_iterate(plan, t, phase, w.iterations, ws, levels=levels, nmse=nmse)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    snap = phase.clone()
    step()
    torch.cuda.synchronize()
    eager_out = (phase.clone(), levels.clone(), nmse.clone())
    phase.copy_(snap)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    graph_same = all(torch.equal(a_, b_) for a_, b_ in zip((phase, levels, nmse), eager_out))
    if not graph_same:
        log("graph replay differs from the eager call: timing the eager driver only")
    phase.copy_(snap)

    def timed_steps(run, label):
        log(f"warmup {args.warmup} steps of {w.name} ({label})")
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        log(f"timed {args.steps} steps ({label}): {el / args.steps * 1e3:.3f} ms/step, "
            f"{w.iterations * args.steps / el:.0f} iterations/s, final NMSE {float(nmse[-1].item()):.6f}")
        return el

    eager_el = timed_steps(step, "eager calls")
    graph_el = timed_steps(graph.replay, "graph replay") if graph_same else None
    use_graph = args.driver == "graph" and graph_same
    elapsed = graph_el if use_graph else eager_el
    ms_per_step = elapsed / args.steps * 1e3
    value = w.iterations * args.steps / elapsed
    drivers = {"eager": {"ms_per_step": round(eager_el / args.steps * 1e3, 4),
                         "iterations_per_s": round(w.iterations * args.steps / eager_el, 1)},
               "graph": None if graph_el is None else
               {"ms_per_step": round(graph_el / args.steps * 1e3, 4),
                "iterations_per_s": round(w.iterations * args.steps / graph_el, 1),
                "bitwise_equal_to_eager": graph_same}}

    # per-kernel durations with HIP events on the launch stream, after the
    # timed region: every launch of the kernel runs TIMING_REPEATS times back
    # to back between two events (the state these calls leave is not used)
    kstats = {}
    for name, kid in (("gs_replay_column_pass", hg.HG_KERNEL_GS_REPLAY), ("gs_slm_row_pass", hg.HG_KERNEL_GS_SLM)):
        hg.hg_timing_begin(plan, kid, TIMING_REPEATS)
        for _ in range(max(3, args.steps // 5)):
            step()
        total_ms, count = hg.hg_timing_end(plan)
        kstats[name] = total_ms / max(count, 1)
        log(f"{name}: {kstats[name] * 1e3:.2f} us/launch over {count} executions")
    dominant = max(kstats, key=kstats.get)
    npx = w.height * w.width
    alg_bytes = BYTES_PER_PX[dominant] * npx
    achieved = alg_bytes / (kstats[dominant] * 1e-3) / 1e9
    iter_gbs = sum(BYTES_PER_PX.values()) * npx * value / 1e9
    per_kernel = {}
    for name, ms in kstats.items():
        gbs = BYTES_PER_PX[name] * npx / (ms * 1e-3) / 1e9
        per_kernel[name] = {"us_per_launch": round(ms * 1e3, 3), "algorithmic_bytes_per_launch": BYTES_PER_PX[name] * npx,
                            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                            "traffic": measured_traffic(name)}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dominant),
                "kernel": dominant, "us_per_launch": round(kstats[dominant] * 1e3, 3),
                "timing": f"HIP events around groups of {TIMING_REPEATS} back-to-back launches",
                "algorithmic_bytes_per_launch": alg_bytes,
                "kernels": per_kernel,
                "iteration_gbs": round(iter_gbs, 1), "iteration_frac": round(iter_gbs / HBM_PEAK_GBS, 4)}

    ttn = gb = None
    if not args.no_grad:
        log("time to NMSE: continuous GS vs gradient CGH")
        ttn = time_to_nmse(hg, wl, torch, stream)
        log(f"  {ttn}")
        log(f"gradient CGH: {args.grad_problems} problems x 500 steps, 3 Fresnel planes")
        gb = grad_batch(hg, wl, torch, stream, args.grad_problems)
        log(f"  {gb}")

    mix = b1024 = None
    if not args.no_batched:
        log("mixed batch: 64 holograms, batched vs sequential")
        mix = batched_mix(hg, wl, torch, stream, mixed)
        log(f"  {mix}")
        b1024 = batched_1024(hg, wl, torch, stream)
        log(f"batched 1024^2: {b1024}")

    srch = osp = rf = None
    if not args.headline_only:
        srch = pixel_search_1024(hg, wl, torch, stream)
        log(f"pixel search: {srch}")
        osp = ospr_2048(hg, wl, torch, stream)
        log(f"OSPR 2048: {osp}")
        rf = rocfft_reference(torch, stream)
        log(f"rocFFT reference: {rf}")

    sweep = None
    if not (args.headline_only or args.no_sweep):
        log("size sweep 256^2 .. 8192^2")
        sweep = size_sweep(hg, wl, torch, stream)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_sample_iters} iterations")
        cpu = cpu_baseline(w, target, phi0, args.cpu_sample_iters)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "iterations/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": w.name, "height": w.height, "width": w.width,
                      "iterations_per_step": w.iterations, "levels": w.levels, "propagation": "fresnel",
                      "wavelength_m": w.wavelength, "pitch_m": w.pitch, "distance_m": w.distance,
                      "target_seed": w.target_seed, "phase_seed": w.phase_seed,
                      "driver": "hip_graph_replay" if use_graph else "eager_calls"},
           "drivers": drivers,
           "roofline": roofline, "cpu_baseline": cpu, "time_to_nmse": ttn, "grad_cgh": gb,
           "batched_mix": mix, "batched_1024": b1024, "ospr": osp, "pixel_search": srch,
           "rocfft_reference": rf, "size_sweep": sweep}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
