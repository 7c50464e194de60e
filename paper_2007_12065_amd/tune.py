"""Autotuner for tile shapes and sweep fusion.

For each stage (Laplacian, bilateral) and window size, candidate
(tile_rows, tile_cols, fuse) shapes are timed with HIP events on a
representative frame through the single-frame entry points, the fastest is
installed with pl_tune_set, and the choice is cached in a JSON file keyed by
the GPU architecture, stage, window size and frame size.  The batched path
has table entries of its own (PL_STAGE_BATCH_*), tuned by timing graph
replays of a whole batch plan per candidate.  float32 results do not depend
on the choice (the arithmetic of every output is the same for every tiling),
so tuning only moves time.
"""
from __future__ import annotations

import json
import os

import torch

import paper_2007_12065_amd as pl

LAP_CANDIDATES = {
    3: [(16, 32, 4), (16, 64, 4), (32, 32, 4), (16, 16, 4), (8, 64, 2), (16, 32, 2), (32, 32, 2),
        (32, 16, 2), (16, 16, 2), (8, 32, 1), (4, 64, 1), (32, 32, 1), (8, 16, 4), (8, 32, 4)],
    5: [(8, 32, 1), (4, 64, 1), (16, 32, 1), (8, 64, 2), (16, 32, 2), (16, 16, 2), (32, 32, 2),
        (16, 16, 4), (32, 32, 1), (8, 16, 2), (8, 16, 1), (4, 32, 1)],
}
BIL_CANDIDATES = {
    3: [(8, 32, 1), (4, 64, 1), (16, 16, 1), (16, 32, 1), (8, 32, 2), (4, 32, 1), (8, 64, 1),
        (2, 128, 1), (4, 16, 1), (8, 16, 2), (4, 32, 2), (4, 16, 2), (16, 16, 2), (8, 8, 2)],
    5: [(8, 32, 1), (4, 64, 1), (16, 16, 1), (16, 32, 1), (4, 32, 1), (8, 64, 1), (4, 16, 1),
        (8, 8, 1), (2, 32, 1), (4, 16, 3), (8, 8, 3), (2, 32, 3), (4, 16, 2), (8, 8, 2)],
}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pl_tune.json")


STAGE_NAMES = {pl.PL_STAGE_LAPLACIAN: "laplacian", pl.PL_STAGE_BILATERAL: "bilateral",
               pl.PL_STAGE_BATCH_LAPLACIAN: "batch_laplacian",
               pl.PL_STAGE_BATCH_BILATERAL: "batch_bilateral",
               pl.PL_STAGE_LAPLACIAN_SMALL: "laplacian_small",
               pl.PL_STAGE_BILATERAL_SMALL: "bilateral_small"}


def frame_stages(M: int, N: int) -> tuple[int, int]:
    """The (Laplacian, bilateral) table entries a single M x N frame reads."""
    if M * N <= pl.SMALL_FRAME_POINTS:
        return pl.PL_STAGE_LAPLACIAN_SMALL, pl.PL_STAGE_BILATERAL_SMALL
    return pl.PL_STAGE_LAPLACIAN, pl.PL_STAGE_BILATERAL


def arch_name(device=None) -> str:
    p = torch.cuda.get_device_properties(device or 0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _time(fn, reps: int) -> float:
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps * 1e3      # microseconds per call


def tune_stage(stage: int, kernel: int, pts: torch.Tensor, iterations: int, reps: int = 30,
               candidates=None) -> dict:
    """Time each candidate shape for one stage and window size on `pts`
    (a [M, N, 3] device frame); install and return the fastest."""
    bilateral = stage in (pl.PL_STAGE_BILATERAL, pl.PL_STAGE_BILATERAL_SMALL)
    cands = candidates or (BIL_CANDIDATES if bilateral else LAP_CANDIDATES).get(kernel, [(8, 32, 1)])
    before = pl.pl_tune_get(stage, kernel)
    if bilateral:
        n, c = pl.pl_tri_normals(pts)
        out = torch.empty_like(n)
        call = lambda: pl.pl_bilateral(n, c, kernel, 0.1, 0.1, iterations, out=out)
    else:
        out = torch.empty_like(pts)
        call = lambda: pl.pl_laplacian(pts, kernel, 1.0, iterations, out=out)
    times = {}
    for cfg in cands:
        try:
            pl.pl_tune_set(stage, kernel, *cfg)
        except pl.PLError:
            continue
        times[cfg] = _time(call, reps)
    if not times:
        pl.pl_tune_set(stage, kernel, *before)
        return {"best": before, "times_us": {}}
    best = min(times, key=times.get)
    pl.pl_tune_set(stage, kernel, *best)
    return {"best": best, "times_us": {f"{a}x{b}/{f}": round(t, 2) for (a, b, f), t in times.items()},
            "previous": before}


def autotune(workloads, cache_path: str | None = DEFAULT_CACHE, reps: int = 30) -> dict:
    """Tune every (stage, window size) the workloads use.  `workloads` is a
    list of (pts device tensor, kernel_lap, iters_lap, kernel_bil, iters_bil);
    the largest frame of each window size is the representative.  Results
    are installed and, with a cache path, merged into the JSON cache."""
    arch = arch_name()
    reps_by = {}
    for pts, kl, il, kb, ib in workloads:
        ls, bs = frame_stages(int(pts.shape[0]), int(pts.shape[1]))
        for stage, k, it in ((ls, kl, il), (bs, kb, ib)):
            key = (stage, k)
            size = int(pts.shape[0]) * int(pts.shape[1])
            if key not in reps_by or size > reps_by[key][1]:
                reps_by[key] = (pts, size, max(it, 1))
    report = {}
    for (stage, k), (pts, size, it) in sorted(reps_by.items(), key=lambda x: x[0]):
        r = tune_stage(stage, k, pts, it, reps)
        name = STAGE_NAMES[stage] + f"_k{k}"
        report[name] = dict(r, frame=list(pts.shape[:2]))
    if cache_path:
        save_cache(cache_path, arch, report)
    return report


def tune_frame(workloads, cache_path: str | None = None, reps: int = 40) -> dict:
    """Tune the single-frame table entries on the fused entry point: for each
    window size, every pair of (Laplacian shape, bilateral shape) candidates
    is timed on pl_smooth_frame (FramePlan.run_fused, preallocated buffers,
    HIP events, frames rotating over `sets` buffer sets) and the fastest pair
    is installed.  `workloads` is a list of (frames: list of [M, N, 3] device
    tensors, kernel_lap, lam, iters_lap, kernel_bil, sigma_length,
    sigma_angle, iters_bil) with kernel_lap == kernel_bil; the frames of one
    window size should be its most important workload.  Cached like
    autotune() (entries laplacian_k*, bilateral_k*)."""
    arch = arch_name()
    report = {}
    for frames, kl, lam, il, kb, sl, sa, ib in workloads:
        M, N = int(frames[0].shape[0]), int(frames[0].shape[1])
        sl_stage, sb_stage = frame_stages(M, N)
        dev = frames[0].device
        plans = [pl.FramePlan(M, N, kl, lam, il, kb, sl, sa, ib, torch.float32, dev)
                 for _ in frames]
        stream = pl._stream(dev)
        before = (pl.pl_tune_get(sl_stage, kl), pl.pl_tune_get(sb_stage, kb))
        times = {}
        for lc in LAP_CANDIDATES.get(kl, [(8, 32, 1)]):
            for bc in BIL_CANDIDATES.get(kb, [(8, 32, 1)]):
                try:
                    pl.pl_tune_set(sl_stage, kl, *lc)
                    pl.pl_tune_set(sb_stage, kb, *bc)
                except pl.PLError:
                    continue
                for p in plans:          # the workspace size depends on the shapes
                    p._frame = None
                k = [0]

                def call():
                    i = k[0] % len(plans)
                    plans[i].run_fused(frames[i], stream)
                    k[0] += 1
                times[(lc, bc)] = _time(call, reps)
        if not times:
            pl.pl_tune_set(sl_stage, kl, *before[0])
            pl.pl_tune_set(sb_stage, kb, *before[1])
            continue
        lc, bc = min(times, key=times.get)
        pl.pl_tune_set(sl_stage, kl, *lc)
        pl.pl_tune_set(sb_stage, kb, *bc)
        ranked = sorted(times.items(), key=lambda x: x[1])[:8]
        common = {"frame": [M, N], "objective": "pl_smooth_frame",
                  "frame_us": round(times[(lc, bc)], 2),
                  "fastest_pairs_us": {f"{a[0]}x{a[1]}/{a[2]} + {b[0]}x{b[1]}/{b[2]}": round(t, 2)
                                       for (a, b), t in ranked}}
        report[STAGE_NAMES[sl_stage] + f"_k{kl}"] = dict(common, best=lc)
        report[STAGE_NAMES[sb_stage] + f"_k{kb}"] = dict(common, best=bc)
    if cache_path:
        save_cache(cache_path, arch, report)
    return report


def tune_batch_stage(stage: int, kernel: int, frames: list, reps: int = 10,
                     normal_dtype=None) -> dict:
    """Time each candidate shape for a batched stage (PL_STAGE_BATCH_*) by
    graph replays of a plan over `frames` (Batch frame dicts); install and
    return the fastest.  Plans read the table when created, so each
    candidate gets its own plan."""
    normal_dtype = normal_dtype or torch.float32
    lap = stage == pl.PL_STAGE_BATCH_LAPLACIAN
    cands = (LAP_CANDIDATES if lap else BIL_CANDIDATES).get(kernel, [(8, 32, 1)])
    before = pl.pl_tune_get(stage, kernel)
    times = {}
    for cfg in cands:
        try:
            pl.pl_tune_set(stage, kernel, *cfg)
        except pl.PLError:
            continue
        b = pl.Batch(frames, normal_dtype)
        try:
            b.run()
            b.capture()
            times[cfg] = _time(b.replay, reps)
        finally:
            b.close()
    if not times:
        pl.pl_tune_set(stage, kernel, *before)
        return {"best": before, "times_us": {}}
    best = min(times, key=times.get)
    pl.pl_tune_set(stage, kernel, *best)
    return {"best": best, "times_us": {f"{a}x{b}/{f}": round(t, 2) for (a, b, f), t in times.items()},
            "previous": before}


def autotune_batch(frames: list, cache_path: str | None = DEFAULT_CACHE, reps: int = 10) -> dict:
    """Tune the batched path's entries for every window size `frames` use
    (Batch frame dicts), on the whole batch; cached like autotune()."""
    arch = arch_name()
    report = {}
    for stage, key in ((pl.PL_STAGE_BATCH_LAPLACIAN, "kernel_lap"), (pl.PL_STAGE_BATCH_BILATERAL, "kernel_bil")):
        for k in sorted({int(f[key]) for f in frames}):
            r = tune_batch_stage(stage, k, frames, reps)
            report[STAGE_NAMES[stage] + f"_k{k}"] = dict(r, frame=[len(frames)])
    if cache_path:
        save_cache(cache_path, arch, report)
    return report


def save_cache(path: str, arch: str, report: dict) -> None:
    data = {}
    if os.path.exists(path):
        try:
            data = json.load(open(path))
        except (OSError, ValueError):
            data = {}
    data.setdefault(arch, {})
    for name, r in report.items():
        data[arch][name] = {k: (list(v) if k == "best" else v) for k, v in r.items()
                            if k in ("best", "frame", "objective", "frame_us", "fastest_pairs_us")}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load_cache(path: str = DEFAULT_CACHE) -> int:
    """Install cached shapes for the current architecture; returns how many."""
    if not os.path.exists(path):
        return 0
    try:
        data = json.load(open(path)).get(arch_name(), {})
    except (OSError, ValueError):
        return 0
    n = 0
    by_name = {v: k for k, v in STAGE_NAMES.items()}
    for name, entry in data.items():
        stage_name, k = name.rsplit("_k", 1)
        if stage_name not in by_name:
            continue
        stage = by_name[stage_name]
        try:
            pl.pl_tune_set(stage, int(k), *entry["best"])
            n += 1
        except (pl.PLError, ValueError, TypeError):
            continue
    return n
