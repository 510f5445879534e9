"""Offline autotuner of the compiled launch shapes (csrc/sizes.hpp).

For a frame shape H x W it times the Gerchberg-Saxton loop (Fourier, four
levels: the shape's two passes and nothing else) of variant builds of the
library that differ in one group of launch parameters at a time, and keeps
the fastest of each group (coordinate descent):

  1. the row shape of length W: rows per workgroup and threads per row;
  2. its radix order (the current radices reordered, and other radix
     multisets with few stages);
  3. its tile width FT of the tiled field layout (0, the column tile width
     or twice it);
  4. the column shape of length H: columns per workgroup and threads per
     column;
  5. its radix order.

A candidate that does not compile (a kernel's static checks) or whose plan
cannot be created (more LDS than a workgroup may use) is skipped, and so is
one whose results differ from the current build's: each timing run also
returns the NMSE of three continuous-phase GS iterations, which must match
the current configuration's within 1e-4 relative.  Every measurement is
cached in a JSON file keyed by the GPU, the frame shape and the two
configurations, so a rerun only builds and times what is new.
--apply writes the winners into csrc/sizes.hpp; rebuild afterwards with
`python -m paper_2006_10509_amd.build`.  Launch shapes stay compile-time
constants of the kernels (template arguments), so the tuner works ahead of
time rather than inside the library.

    python -m paper_2006_10509_amd.autotune --shape 1080x1920 [--shape ...]
        [--batch B] [--max-candidates 6] [--cache PATH] [--apply]

--batch B times B same-shape holograms per launch (hg_gs_iterate_batched)
and ranks by time per hologram-iteration: small frames that run in batches
tune differently from a single hologram, which is latency-bound.

Needs hipcc for the variant builds and a GPU for the timing, which runs in a
child process per candidate (`--measure LIB HxW`).
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import re
import shutil
import subprocess
import sys
import tempfile
import time
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Tuple

from . import build as hb

RADICES = (16, 8, 5, 4, 3, 2)
ROW_RE = re.compile(r"HG_ROW_CFG\(\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*([\d,\s]+)\)")
COL_RE = re.compile(r"HG_COL_CFG\(\s*(\d+),\s*(\d+),\s*(\d+),\s*([\d,\s]+)\)")

RowCfg = Tuple[int, int, int, Tuple[int, ...]]   # teams, threads per row, FT, radices
ColCfg = Tuple[int, int, Tuple[int, ...]]        # columns per workgroup, threads per column, radices


def _radices(text: str) -> Tuple[int, ...]:
    return tuple(int(v) for v in text.replace(" ", "").split(",") if v)


def read_configs(sizes_text: str) -> Tuple[Dict[int, RowCfg], Dict[int, ColCfg]]:
    rows = {int(m[0]): (int(m[1]), int(m[2]), int(m[3]), _radices(m[4])) for m in ROW_RE.findall(sizes_text)}
    cols = {int(m[0]): (int(m[1]), int(m[2]), _radices(m[3])) for m in COL_RE.findall(sizes_text)}
    return rows, cols


def row_line(n: int, c: RowCfg) -> str:
    return f"HG_ROW_CFG({n}, {c[0]}, {c[1]}, {c[2]}, {', '.join(map(str, c[3]))})"


def col_line(n: int, c: ColCfg) -> str:
    return f"HG_COL_CFG({n}, {c[0]}, {c[1]}, {', '.join(map(str, c[2]))})"


def with_configs(sizes_text: str, rows: Dict[int, RowCfg], cols: Dict[int, ColCfg],
                 only_lengths: Optional[List[int]] = None) -> str:
    """sizes.hpp text with the given lines replaced and, when only_lengths is
    given, the compiled length list restricted to those lengths."""
    def sub_row(m):
        n = int(m.group(1))
        return row_line(n, rows[n]) if n in rows else m.group(0)

    def sub_col(m):
        n = int(m.group(1))
        return col_line(n, cols[n]) if n in cols else m.group(0)

    text = ROW_RE.sub(sub_row, sizes_text)
    text = COL_RE.sub(sub_col, text)
    if only_lengths:
        start = text.index("#define HG_FOR_EACH_LENGTH")
        end = text.index("\n\n", start)
        text = (text[:start] + "#define HG_FOR_EACH_LENGTH(X) " + " ".join(f"X({n})" for n in only_lengths)
                + text[end:])
    return text


def radix_orders(n: int, current: Tuple[int, ...], limit: int) -> List[Tuple[int, ...]]:
    """Radix lists for length n: the current one, its reorderings, then other
    multisets of supported radices with at most one stage more."""
    out: List[Tuple[int, ...]] = []

    def add(r):
        r = tuple(r)
        if r not in out:
            out.append(r)

    add(current)
    for perm in sorted(set(itertools.permutations(current)), key=lambda p: p != tuple(sorted(p, reverse=True))):
        add(perm)
    multisets = []

    def split(rem, smallest_allowed, acc):
        if rem == 1:
            if 2 <= len(acc) <= len(current) + 1:
                multisets.append(tuple(acc))
            return
        for r in RADICES:
            if r <= smallest_allowed and rem % r == 0:
                split(rem // r, r, acc + [r])

    split(n, max(RADICES), [])
    for m in sorted(multisets, key=len):
        add(m)
    return out[:limit]


def row_shapes(n: int, cur: RowCfg, limit: int) -> List[RowCfg]:
    out = [cur]
    for teams, t in itertools.product((1, 2, 4, 8), (64, 128, 256, 512)):
        threads = teams * t
        if threads % 64 or threads > 1024 or t > n:
            continue
        # a tiled field needs teams that exchange through s_barrier (more than 64 threads)
        ft = cur[2] if (t > 64 and t % max(cur[2], 1) == 0) else 0
        c = (teams, t, ft, cur[3])
        if c not in out:
            out.append(c)
    return out[:limit]


def col_shapes(n: int, cur: ColCfg, limit: int) -> List[ColCfg]:
    out = [cur]
    for cols, t in itertools.product((1, 2, 4, 8, 16), (64, 128, 256, 512)):
        threads = cols * t
        if threads % 64 or threads > 1024 or t > n:
            continue
        c = (cols, t, cur[2])
        if c not in out:
            out.append(c)
    return out[:limit]


# ---------------------------------------------------------------------------
# measurement (child process)
# ---------------------------------------------------------------------------
def measure(lib: str, h: int, w: int, batch: int = 1) -> dict:
    sys.path.insert(0, hb.ROOT)
    from paper_2006_10509_amd import hologen as hg
    hg.LIB_PATH = os.path.abspath(lib)
    import torch
    from paper_2006_10509_amd import workloads as wl
    t, p = wl.target_and_phase(h, w, 5)
    plan = hg.Plan(w, h, hg.HG_FOURIER, 0.0, 0.0, 0.0, hg.HG_PHASE_QUANTISED, 4)
    target = torch.from_numpy(t).cuda()
    phase = torch.from_numpy(p).cuda()
    ws = plan.workspace()
    iters, calls = 50, 5
    if batch > 1:
        target_b = target.expand(batch, h, w).contiguous()
        phase_b = phase.expand(batch, h, w).contiguous()
        ws_b = torch.empty(hg.workspace_bytes_batched(plan, batch), dtype=torch.uint8, device="cuda")
        run = lambda: hg.hg_gs_iterate_batched(plan, target_b, phase_b, iters, ws_b)  # noqa: E731
    else:
        run = lambda: hg.hg_gs_iterate(plan, target, phase, iters, ws)  # noqa: E731
    run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(calls):
        run()
    b.record()
    b.synchronize()
    us = a.elapsed_time(b) * 1e3 / (iters * calls * batch)
    # results check: three continuous-phase iterations from the same start
    cplan = hg.Plan(w, h, hg.HG_FOURIER, 0.0, 0.0, 0.0, hg.HG_PHASE, 0)
    nm = torch.zeros(4, dtype=torch.float32, device="cuda")
    hg.hg_gs_iterate(cplan, target, torch.from_numpy(p).cuda(), 3, cplan.workspace(), nmse=nm)
    return {"us_per_iteration": us, "gpu": torch.cuda.get_device_name(0), "check": nm.cpu().tolist()}


# ---------------------------------------------------------------------------
# tuner (parent process: builds on the CPU, one child per timing)
# ---------------------------------------------------------------------------
class Tuner:
    def __init__(self, cache_path: str, jobs: int, batch: int = 1, verbose: bool = True):
        self.batch = batch
        self.cache_path = cache_path
        self.cache = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        self.jobs = jobs
        self.verbose = verbose
        self.sizes_text = open(os.path.join(hb.CSRC, "sizes.hpp")).read()
        self.gpu: Optional[str] = self.cache.get("_gpu")
        self.reference: Optional[List[float]] = None

    def log(self, *a):
        if self.verbose:
            print(*a, flush=True)

    def key(self, h, w, row: RowCfg, col: ColCfg) -> str:
        return f"{self.gpu}|{h}x{w}x{self.batch}|{row_line(w, row)}|{col_line(h, col)}"

    def _build(self, tmp: str, h: int, w: int, row: RowCfg, col: ColCfg) -> Optional[str]:
        src = os.path.join(tmp, "csrc")
        shutil.copytree(hb.CSRC, src)
        lens = sorted({h, w})
        text = with_configs(self.sizes_text, {w: row}, {h: col}, lens)
        open(os.path.join(src, "sizes.hpp"), "w").write(text)
        out = os.path.join(tmp, "libhologen.so")
        try:
            hb.build_library(src, out, jobs=4)
        except RuntimeError:
            return None
        return out

    def _time(self, lib: str, h: int, w: int) -> Optional[dict]:
        cmd = [sys.executable, "-m", "paper_2006_10509_amd.autotune", "--measure", lib, f"{h}x{w}",
               "--batch", str(self.batch)]
        try:
            proc = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=hb.ROOT)
        except subprocess.TimeoutExpired:
            return None
        if proc.returncode != 0:
            return None
        return json.loads(proc.stdout.strip().splitlines()[-1])

    def consistent(self, check: List[float]) -> bool:
        ref = self.reference
        return ref is None or all(abs(a - b) <= 1e-4 * abs(b) for a, b in zip(check, ref))

    def evaluate(self, h: int, w: int, cands: List[Tuple[RowCfg, ColCfg]],
                 force: bool = False) -> List[Tuple[float, RowCfg, ColCfg]]:
        # the current configuration is always run (it supplies the results check)
        todo = [(r, c) for r, c in cands
                if force or self.gpu is None or self.key(h, w, r, c) not in self.cache]
        if todo:
            self.log(f"  building {len(todo)} variant(s)")
        with tempfile.TemporaryDirectory(prefix="hg_tune_") as tmp:
            dirs = [os.path.join(tmp, str(i)) for i in range(len(todo))]
            for d in dirs:
                os.makedirs(d)
            with ThreadPoolExecutor(max_workers=self.jobs) as ex:
                libs = list(ex.map(lambda a: self._build(*a), [(d, h, w, r, c) for d, (r, c) in zip(dirs, todo)]))
            for (r, c), lib in zip(todo, libs):
                res = self._time(lib, h, w) if lib else None
                if res and self.gpu is None:
                    self.gpu = res["gpu"]
                    self.cache["_gpu"] = self.gpu
                us = res["us_per_iteration"] if res else None
                note = "skipped (build or plan failed)"
                if res and self.reference is None:
                    self.reference = res["check"]
                if res and not self.consistent(res["check"]):
                    us, note = None, "rejected (results differ from the current build)"
                self.cache[self.key(h, w, r, c)] = us
                self.log(f"  {row_line(w, r):44s} {col_line(h, c):40s} "
                         f"{'%.2f us/hologram-iteration' % us if us else note}")
                json.dump(self.cache, open(self.cache_path, "w"), indent=1, sort_keys=True)
        out = []
        for r, c in cands:
            us = self.cache.get(self.key(h, w, r, c))
            if us:
                out.append((us, r, c))
        return sorted(out, key=lambda x: x[0])

    def tune(self, h: int, w: int, limit: int) -> Tuple[RowCfg, ColCfg, float, float]:
        rows, cols = read_configs(self.sizes_text)
        row, col = rows[w], cols[h]
        self.reference = None
        base = self.evaluate(h, w, [(row, col)], force=True)
        if not base:
            raise RuntimeError(f"the current shapes of {h}x{w} do not run")
        start = base[0][0]
        best = start
        rounds = [
            ("row shape", lambda r, c: [(x, c) for x in row_shapes(w, r, limit)]),
            ("row radices", lambda r, c: [((r[0], r[1], r[2], rad), c) for rad in radix_orders(w, r[3], limit)]),
            ("row tile width", lambda r, c: [((r[0], r[1], ft, r[3]), c) for ft in sorted({0, c[0], 2 * c[0], r[2]})
                                             if ft == 0 or (r[0] > 1 and r[1] > 64 and r[1] % ft == 0)]),
            ("column shape", lambda r, c: [(r, x) for x in col_shapes(h, c, limit)]),
            ("column radices", lambda r, c: [(r, (c[0], c[1], rad)) for rad in radix_orders(h, c[2], limit)]),
        ]
        for name, gen in rounds:
            self.log(f"{h}x{w}: {name}")
            res = self.evaluate(h, w, gen(row, col))
            if res and res[0][0] < best:
                best, row, col = res[0]
        return row, col, start, best


def apply(rows: Dict[int, RowCfg], cols: Dict[int, ColCfg]) -> None:
    path = os.path.join(hb.CSRC, "sizes.hpp")
    text = open(path).read()
    open(path, "w").write(with_configs(text, rows, cols))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--shape", action="append", default=[], help="frame shape HxW (repeatable)")
    ap.add_argument("--max-candidates", type=int, default=6, help="candidates per round")
    ap.add_argument("--batch", type=int, default=1, help="holograms per launch while timing")
    ap.add_argument("--cache", default=os.path.join(os.path.expanduser("~"), ".cache", "hologen_tune.json"))
    ap.add_argument("--jobs", type=int, default=4, help="variant builds in parallel")
    ap.add_argument("--apply", action="store_true", help="write the winners into csrc/sizes.hpp")
    ap.add_argument("--measure", nargs=2, metavar=("LIB", "HxW"), help=argparse.SUPPRESS)
    a = ap.parse_args(argv)
    if a.measure:
        h, w = (int(v) for v in a.measure[1].split("x"))
        print(json.dumps(measure(a.measure[0], h, w, a.batch)))
        return 0
    if not a.shape:
        ap.error("give at least one --shape HxW")
    os.makedirs(os.path.dirname(os.path.abspath(a.cache)), exist_ok=True)
    tuner = Tuner(a.cache, a.jobs, a.batch)
    rows, cols = {}, {}
    for s in a.shape:
        h, w = (int(v) for v in s.split("x"))
        t0 = time.time()
        row, col, start, best = tuner.tune(h, w, a.max_candidates)
        print(f"{h}x{w} (batch {a.batch}): {start:.2f} -> {best:.2f} us per hologram-iteration "
              f"({time.time() - t0:.0f} s)")
        print("  " + row_line(w, row))
        print("  " + col_line(h, col))
        rows[w], cols[h] = row, col
    if a.apply:
        apply(rows, cols)
        print("written to csrc/sizes.hpp; rebuild with python -m paper_2006_10509_amd.build")
    return 0


if __name__ == "__main__":
    sys.exit(main())
