"""Benchmark of the whole OPC meshing + smoothing path on one MI355X.

One step = one pass of the single-frame path (pl_smooth_frame, three
launches) over one 480x640 synthetic RGBD frame (floor, two walls, six boxes,
8% NaN holes): mesh extraction (Alg. 1-2), 4 Laplacian sweeps (3x3,
lambda = 1), triangle normals and centroids, 2 bilateral sweeps (3x3 quads,
sigma_length = sigma_angle = 0.1) and the gather onto T, all in float32.
Inputs are resident in HBM before the timed region; 16 frames with separate
input and output buffers rotate so the working set (~1.1 GB) exceeds the
256 MB last-level cache.  The same frames also go through the four separate
single-frame calls (pl_mesh_opc, pl_laplacian, pl_tri_normals, pl_bilateral),
the baseline of the batched and served comparisons.

Tile shapes and fusion come from the committed tuning file
(profiles/tune.json) unless --retune is given.  The timed steps run the path
alone on the stream; a separate pass with HIP events between the launches
(pl_smooth_frame_events) gives each launch's duration, from which the
roofline of the dominant launch is computed: algorithmic bytes against the
8 TB/s HBM peak and algorithmic VALU lane-operations against the 3.93e13/s
non-packed FP32 issue rate (256 CUs x 64 lanes x 2.4 GHz; transcendental
operations count four slots), the larger of the two fractions naming the
bound.

Prints one JSON line (the contract fields plus the roofline, per-workload
records, the auxiliary kernels, the batched and served comparisons and the
FP64 oracle's CPU throughput).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "smoothed triangles/s (Laplacian+bilateral) & %HBM peak; p99 frame latency batched vs plain"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9   # non-packed FP32 issue: 3.93e13 lane-operations/s
TUNE_FILE = os.path.join(ROOT, "profiles", "tune.json")

# Algorithmic VALU lane-slots per unit of work (each floating-point operation
# of the formulas one slot, a transcendental -- rsqrt, exp2, rcp -- four).
#  Laplacian, per updated point and sweep, per neighbour: difference 3,
#  squared distance 3, rsqrt 4, weight sum 1, weighted sum 3; then 1/W 4 and
#  the update 4.
#  Bilateral, per triangle and sweep, per neighbour: two squared differences
#  12, exponent 2, exp2 4, weighted sum 3 (Eq. 6 renormalises, so the sum of
#  the weights is not needed); then renormalisation 10.
#  Centroid and normal of a triangle: 31.


def lap_lane_ops(kernel):
    return (kernel * kernel - 1) * 14 + 8


def bil_lane_ops(kernel):
    return 2 * (kernel * kernel - 1) * 21 + 10


GEOM_LANE_OPS = 31


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--sets", type=int, default=16, help="rotating frame buffer sets")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="bound on the oracle's CPU-baseline sample (0 = skip)")
    ap.add_argument("--batched", type=int, default=1,
                    help="also measure the 64-frame mixed batch (0 = skip)")
    ap.add_argument("--per-config", type=int, default=1,
                    help="also measure the 120x160, 64x1024 and 128x2048 workloads (0 = skip)")
    ap.add_argument("--aux", type=int, default=1,
                    help="also measure group assignment, the accumulator, user half-edges "
                         "and the vertex update (0 = skip)")
    ap.add_argument("--tune-file", default=TUNE_FILE,
                    help="tuning file to load (default: the committed profiles/tune.json)")
    ap.add_argument("--retune", default=None, metavar="PATH",
                    help="tune in-process instead of loading a file, and write the result to PATH")
    ap.add_argument("--serving-seconds", type=float, default=10.0,
                    help="measured seconds of the Poisson serving run after 1 s warm-up (0 = skip)")
    ap.add_argument("--pool", type=int, default=64, help="served frames pre-generated per size class")
    return ap.parse_args()


def frame_counts(M, N, k, n_tri, pts_np=None):
    """Units of work of one frame: points P, quads Q, T_FC triangles T, valid
    triangles |T|, and the points a Laplacian sweep updates (valid pixels
    outside the border band)."""
    P, Q = M * N, (M - 1) * (N - 1)
    r = k.kernel_lap // 2
    if pts_np is not None:
        import numpy as np
        inner = pts_np[r:M - r, r:N - r]
        upd = float(np.mean([int((~np.isnan(inner).any(-1)).sum())]))
    else:
        upd = float((M - 2 * r) * (N - 2 * r))
    return {"P": P, "Q": Q, "T": 2 * Q, "n_tri": float(n_tri), "lap_points": upd}


def launch_model(kind, c, k):
    """Algorithmic bytes and VALU lane-slots of one launch of the fused path,
    from the work its kind bits say it carries (each input read once, each
    output written once; see the lane-slot counts above)."""
    import paper_2007_12065_amd as pl
    F = (kind >> 8) & 0xff
    P, Q, T, nt = c["P"], c["Q"], c["T"], c["n_tri"]
    nbytes = 0.0
    ops = 0.0
    parts = []
    reads_pts = False
    if kind & pl.PL_LAUNCH_LAPLACIAN:
        nbytes += 24 * P
        reads_pts = True
        ops += F * c["lap_points"] * lap_lane_ops(k.kernel_lap)
        parts.append(f"laplacian x{F}")
    if kind & pl.PL_LAUNCH_MESH_COUNT:
        nbytes += (0 if reads_pts else 12 * P) + Q + T
        parts.append("mesh count")
    if kind & pl.PL_LAUNCH_MESH_EMIT:
        nbytes += Q + 4 * T + 24 * nt
        parts.append("mesh emit")
    if kind & pl.PL_LAUNCH_BILATERAL:
        if kind & pl.PL_LAUNCH_NORMALS:
            nbytes += 12 * P + 24 * T          # smoothed points in; centroids, normals out
            ops += nt * GEOM_LANE_OPS
            parts.append("normals")
        else:
            nbytes += 36 * T
        ops += F * nt * bil_lane_ops(k.kernel_bil)
        parts.append(f"bilateral x{F}")
    if kind & pl.PL_LAUNCH_GATHER:
        nbytes += 4 * T + 12 * nt
        parts.append("gather")
    return {"work": " + ".join(parts), "bytes": nbytes, "lane_ops": ops}


def staged_bytes(c, k):
    """The staged algorithmic bytes of the whole path (each call reading its
    inputs and writing its outputs once, 24P per Laplacian sweep, 36T per
    bilateral sweep): mesh 12P + T/8 + 4T + 24|T|, Laplacian, normals
    12P + 24T, bilateral, gather 4T + 24|T|."""
    P, T, nt = c["P"], c["T"], c["n_tri"]
    return (12 * P + T / 8 + 4 * T + 24 * nt) + 24 * P * k.iters_lap + (12 * P + 24 * T) \
        + 36 * T * k.iters_bil + (4 * T + 24 * nt)


def roofline(nbytes, ops, seconds):
    gbs = nbytes / seconds / 1e9
    lanes = ops / seconds
    hf, vf = gbs / HBM_PEAK_GBS, lanes / VALU_PEAK_LANE_OPS
    if hf >= vf:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(hf, 4)}
    else:
        r = {"bound": "alu", "achieved": round(lanes / 1e12, 3),
             "peak": round(VALU_PEAK_LANE_OPS / 1e12, 3), "unit": "Tlane-op/s",
             "frac": round(vf, 4)}
    r.update({"hbm_frac": round(hf, 4), "valu_frac": round(vf, 4)})
    return r


FRAME_SOURCES = ("paper_2007_12065_amd/csrc/tiles.h", "paper_2007_12065_amd/csrc/common.h",
                 "paper_2007_12065_amd/csrc/frame.hip")
GROUP_SOURCES = ("paper_2007_12065_amd/csrc/common.h", "paper_2007_12065_amd/csrc/groups.h",
                 "paper_2007_12065_amd/csrc/groups.hip")


def kernel_source_digest(files=FRAME_SOURCES):
    """SHA-256 over the sources a kernel is built from (default: the fused
    single-frame path's kernels)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(key, files=FRAME_SOURCES):
    """The committed counter summary of launch `key` (profiles/traffic.json:
    FETCH_SIZE and WRITE_SIZE runs calibrated on a copy of known size, and
    SQ_INSTS_VALU), or None when there is none or the kernel's sources
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    r = rec.get(key)
    if not r or r.get("source_digest") != kernel_source_digest(files):
        return None
    return r


def measured_traffic(key, files=FRAME_SOURCES):
    """HBM bytes per launch for `key` from the committed counters, or None."""
    r = measured_counters(key, files)
    return r.get("bytes_per_launch") if r else None


def frame_kernel_name(kind, k):
    """The kernel template a launch of the fused path runs (as the profiler
    names it), from its kind bits."""
    import paper_2007_12065_amd as pl
    mesh = 1 if kind & pl.PL_LAUNCH_MESH_COUNT else 2 if kind & pl.PL_LAUNCH_MESH_EMIT else 0
    if kind & pl.PL_LAUNCH_BILATERAL:
        from_pts = "true" if kind & pl.PL_LAUNCH_NORMALS else "false"
        # the gathering pass beside the emit ranks the triangles from the codes
        by_codes = "true" if (kind & pl.PL_LAUNCH_GATHER and kind & pl.PL_LAUNCH_MESH_EMIT) else "false"
        return f"void k_frame_bilateral<{k.kernel_bil // 2}, float, {from_pts}, {mesh}, {by_codes}>"
    return f"void k_frame_laplacian<{k.kernel_lap // 2}, {mesh}>"


def cpu_baseline(frames_np, k, seconds, threads=None):
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    if threads is None:
        threads = max(1, min(cores, int(os.environ.get("OMP_NUM_THREADS", cores))))
    oracle.build(force=False)
    T = 2 * (k.M - 1) * (k.N - 1)
    done = 0
    t0 = time.perf_counter()
    while True:
        oracle.pipeline(frames_np[done % len(frames_np)], k.kernel_lap, k.lam, k.iters_lap,
                        k.kernel_bil, k.sigma_length, k.sigma_angle, k.iters_bil, threads)
        done += 1
        el = time.perf_counter() - t0
        if el >= seconds or done >= 1000:
            break
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": T * done / el, "unit": "triangles/s", "cores": threads, "kind": "oracle",
            "host_cpus": cores, "cpu_model": model,
            "sample": f"{done} frames of the 480x640 workload (whole path, FP64 C oracle, "
                      f"{threads} OpenMP threads), {el:.1f} s"}


def graph_us(calls, replays=20):
    """Average device time of one call: the calls (one per frame set) are
    captured into a HIP graph on a side stream, and the graph is replayed
    `replays` times between two events, so host issue cost does not enter.
    Every call writes preallocated buffers only."""
    import torch
    for c in calls:
        c()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for c in calls:
            c()
    g.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(replays):
        g.replay()
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) * 1e3 / (replays * len(calls))


def groups_bench(plans, k, stream, s, reps=300):
    """Group assignment (Alg. 4) over the frame sets after the timed path:
    per-launch device time of k_group_assign (graph replays) on float32 normals with each frame's
    three scene planes as dominant normals, its roofline (HBM bound: T, the
    normals and the labels streamed once, every point read once), and the
    oracle's time for the same labels on one frame."""
    import numpy as np
    import torch

    import oracle
    from synth import scene_planes
    sets = len(plans)
    doms = [torch.from_numpy(scene_planes("rgbd", 1000 + i)).to(plans[0].device) for i in range(sets)]
    us = graph_us([lambda i=i: plans[i].run_groups(doms[i], k.l_max, k.ang_min) for i in range(sets)])
    n_tri = float(np.mean([int(p.n_tri.item()) for p in plans]))
    P = plans[0].M * plans[0].N
    nbytes = 12 * n_tri + 12 * n_tri + n_tri + 12 * P
    gbs = nbytes / (us * 1e-6) / 1e9
    labels = plans[0].groups[: int(plans[0].n_tri.item())].cpu().numpy()
    # the oracle on the same float32 inputs (the GPU frame's own T, points and
    # normals: a timing of the CPU code, not a parity check)
    p0 = plans[0]
    n0 = int(p0.n_tri.item())
    args = (p0.points.cpu().numpy(), p0.triangles[:n0].cpu().numpy(),
            p0.normals_T[:n0].cpu().numpy(), doms[0].cpu().numpy(), k.l_max, k.ang_min)
    oracle.build(force=False)
    t0 = time.perf_counter()
    r = 0
    while time.perf_counter() - t0 < 1.0:
        oracle.group_assign(*args)
        r += 1
    cpu_s = (time.perf_counter() - t0) / r
    return {"kernel": "k_group_assign", "launch_us": round(us, 2),
            "labels_per_s": round(n_tri / (us * 1e-6), 1),
            "bytes_per_launch": int(nbytes), "achieved_gbs": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("k_group_assign:rgbd", GROUP_SOURCES),
            "assigned_frac": round(float(np.mean(labels != 255)), 4),
            "l_max": k.l_max, "ang_min": k.ang_min, "dominant_normals": 3,
            "cpu_oracle_labels_per_s": round(n_tri / cpu_s, 1), "cpu_oracle_threads": 1}


def ga_bench(plans, stream, reps=200, level=4, stride=1):
    """Gaussian accumulator integration (Alg. 3) of each frame's filtered
    normals (all |T| rows, float32) into a level-4 accumulator: per-launch
    time of k_ga_integrate, normals per second, algorithmic HBM bytes (the
    normals read once; cells, bin tables and counts stay in cache), and the
    oracle's brute-force rate on one thread for the same normals."""
    import numpy as np
    import torch

    import oracle
    import paper_2007_12065_amd as pl
    sets = len(plans)
    ga = pl.GaussianAccumulator(level, device=plans[0].device)
    counts = torch.zeros(ga.n_cells, dtype=torch.uint32, device=plans[0].device)
    us = graph_us([lambda i=i: ga.integrate(plans[i].normals_T, n=plans[i].n_tri, stride=stride,
                                            counts=counts) for i in range(sets)])
    n_tri = float(np.mean([int(p.n_tri.item()) for p in plans]))
    rows = n_tri / stride
    nbytes = 12 * rows
    p0 = plans[0]
    n0 = int(p0.n_tri.item())
    normals = p0.normals_T[:n0].cpu().numpy()
    from oracle import ga_icosahedron
    _, _, cells = ga_icosahedron(level)
    sample = normals[: max(1, len(normals) // 50)]
    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.ga_integrate(cells, sample)
    cpu_s = time.perf_counter() - t0
    ga.close()
    return {"kernel": "k_ga_integrate", "level": level, "cells": 20 * 4 ** level, "stride": stride,
            "launch_us": round(us, 2), "normals_per_s": round(rows / (us * 1e-6), 1),
            "bytes_per_launch": int(nbytes), "achieved_gbs": round(nbytes / (us * 1e-6) / 1e9, 1),
            "hbm_frac": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "cpu_oracle_normals_per_s": round(len(sample) / cpu_s, 1), "cpu_oracle_threads": 1,
            "cpu_oracle_sample": f"{len(sample)} normals of one frame, brute force over all cells"}


def user_halfedges_bench(plans, stream, reps=100):
    """Half-edges of a user mesh (Sec. 4.3) on each frame's T taken as a
    user-provided triangle list: per-call device time (graph replays) of the
    partitioned way's five launches (bucket counts, their scan, the scatter
    into bucket regions, the per-bucket LDS tables, the fallback check),
    half-edges per second, and the oracle's rate (sort and binary searches,
    one thread) on the same triangles."""
    import numpy as np
    import torch

    import oracle
    import paper_2007_12065_amd as pl
    sets = len(plans)
    outs = [torch.empty(3 * p.T, dtype=torch.int32, device=p.device) for p in plans]
    cap = plans[0].T
    ws_n = pl._lib.pl_user_halfedges_workspace(cap)
    ws = torch.empty(ws_n, dtype=torch.uint8, device=plans[0].device)
    def call(i):
        p = plans[i % sets]
        pl._check(pl._lib.pl_user_halfedges(pl._ptr(p.triangles), pl._ptr(p.n_tri), p.T,
                                            pl._ptr(outs[i % sets]), pl._ptr(ws), ws_n,
                                            pl._stream(p.device)), "pl_user_halfedges")
    us = graph_us([lambda i=i: call(i) for i in range(sets)], replays=5)
    n_tri = float(np.mean([int(p.n_tri.item()) for p in plans]))
    n0 = int(plans[0].n_tri.item())
    same = bool(torch.equal(outs[0][:3 * n0], plans[0].halfedges[:3 * n0]))
    T = plans[0].triangles[:n0].cpu().numpy()
    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.user_halfedges(T)
    cpu_s = time.perf_counter() - t0
    return {"kernels": ["k_he_count", "k_he_offsets", "k_he_scatter", "k_he_solve", "k_he_fallback"],
            "call_us": round(us, 2),
            "halfedges_per_s": round(3 * n_tri / (us * 1e-6), 1), "workspace_bytes": int(ws_n),
            "equals_alg2_he": same,
            "cpu_oracle_halfedges_per_s": round(3 * n0 / cpu_s, 1), "cpu_oracle_threads": 1}


def vertex_update_bench(plans, stream, reps=100, iterations=1):
    """Vertex update from the filtered normals (one sweep per call) on each
    frame: per-launch device time (graph replays) of k_vertex_update, its algorithmic bytes (points
    read and written once, the T_FC normals read once) and HBM fraction."""
    import numpy as np
    import torch

    import paper_2007_12065_amd as pl
    sets = len(plans)
    outs = [torch.empty_like(p.points) for p in plans]
    M, N = plans[0].M, plans[0].N

    def call(i):
        p = plans[i % sets]
        pl._check(pl._lib.pl_vertex_update(pl._ptr(p.points), pl._ptr(outs[i % sets]), M, N,
                                           pl._ptr(p.filtered), p.ndt, iterations, None, 0,
                                           pl._stream(p.device)), "pl_vertex_update")
    us = graph_us([lambda i=i: call(i) for i in range(sets)])
    nbytes = 24 * M * N + 12 * 2 * (M - 1) * (N - 1)
    return {"kernel": "k_vertex_update", "sweeps": iterations, "launch_us": round(us, 2),
            "parity": "unpinned: the paper cites this update (Sec. 2.3, Sec. 5.2) but prints no "
                      "formula; the oracle restates it and the kernel matches the oracle within "
                      "1e-5 relative",
            "points_per_s": round(M * N / (us * 1e-6), 1), "bytes_per_launch": int(nbytes),
            "achieved_gbs": round(nbytes / (us * 1e-6) / 1e9, 1),
            "hbm_frac": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}


def angle_stats(got, ref):
    import numpy as np
    g = np.asarray(got, dtype=np.float64).reshape(-1, 3)
    r = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    ok = ~np.isnan(r).any(-1)
    a = np.arctan2(np.linalg.norm(np.cross(g[ok], r[ok]), axis=-1), np.sum(g[ok] * r[ok], axis=-1))
    return {"p50": float(np.median(a)), "p99": float(np.percentile(a, 99)), "max": float(a.max())}


def batched_bench(tuning, reps=20):
    """The 64-frame mix (16x 120x160, 24x 480x640, 16x 64x1024, 8x 128x2048):
    the plain per-frame float32 path (the four single-frame calls per frame,
    and the fused single-frame entry) vs one batch plan (graph replay),
    float32 and float16 normals.  The batched path's tile shapes come from
    `tuning` (the tuning file's batch_* entries) or are tuned on this mix.
    Angular error against the FP64 oracle for one frame of each size."""
    import numpy as np
    import torch

    import oracle
    import paper_2007_12065_amd as pl
    from synth import KINDS, batch_mix, make_frame
    dev = torch.device("cuda:0")
    host, specs = [], []
    for kind, seed in batch_mix():
        k = KINDS[kind]
        f = make_frame(kind, seed)
        host.append((f, k))
        specs.append(dict(pts=torch.from_numpy(f).to(dev), kernel_lap=k.kernel_lap, lam=k.lam,
                          iters_lap=k.iters_lap, kernel_bil=k.kernel_bil, sigma_length=k.sigma_length,
                          sigma_angle=k.sigma_angle, iters_bil=k.iters_bil))
    T = sum(2 * (f.shape[0] - 1) * (f.shape[1] - 1) for f, _ in host)
    from paper_2007_12065_amd import tune
    batch_tuning = {k: v for k, v in tuning.items() if k.startswith("batch_")}
    if not batch_tuning:
        batch_tuning = tune.autotune_batch(specs, cache_path=None, reps=10)
    plans = [pl.FramePlan(f.shape[0], f.shape[1], k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                          k.sigma_length, k.sigma_angle, k.iters_bil, torch.float32, dev)
             for f, k in host]

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize(dev)
        return (time.perf_counter() - t0) / reps

    def plain():
        for p, sp in zip(plans, specs):
            p.run(sp["pts"])

    def plain_fused():
        for p, sp in zip(plans, specs):
            p.run_fused(sp["pts"])
    t_plain = timed(plain)
    t_fused = timed(plain_fused)
    out = {"frames": len(specs), "triangles": T,
           "tuning": {name: {"tile": list(r["best"][:2]), "fuse": r["best"][2]}
                      for name, r in batch_tuning.items()},
           "plain_f32": {"ms": round(t_plain * 1e3, 3), "triangles_per_s": T / t_plain,
                         "path": "four single-frame calls per frame"},
           "plain_fused_f32": {"ms": round(t_fused * 1e3, 3), "triangles_per_s": T / t_fused,
                               "path": "pl_smooth_frame per frame"}}
    sample = {"rgbd_small": 0, "rgbd": 16, "lidar": 40, "lidar128": 56}
    refs = {}
    for kind, i in sample.items():
        f, k = host[i]
        refs[kind] = oracle.pipeline(f, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                                     k.sigma_length, k.sigma_angle, k.iters_bil,
                                     threads=min(16, os.cpu_count() or 1))["normals_T"]
    for name, dt in (("batched_f32", torch.float32), ("batched_f16", torch.float16)):
        b = pl.Batch(specs, dt)
        b.run()
        b.capture()
        t = timed(b.replay)
        errs = {}
        for kind, i in sample.items():
            n = int(b.outputs[i]["n_tri"].item())
            errs[kind] = angle_stats(b.outputs[i]["normals_T"][:n].float().cpu().numpy(), refs[kind])
        out[name] = {"ms": round(t * 1e3, 3), "triangles_per_s": T / t, "vs_plain_f32": t_plain / t,
                     "vs_plain_fused_f32": t_fused / t, "angle_err_rad_vs_fp64": errs}
        b.close()
    return out


def serving_pool(pool_per_kind):
    """The served frames: `pool_per_kind` seeded frames per size class,
    generated in worker processes (call before the GPU is initialised)."""
    from concurrent.futures import ProcessPoolExecutor

    from synth import KINDS, make_frame
    jobs = [(k, 4000 + 100 * j + i) for j, k in enumerate(KINDS) for i in range(pool_per_kind)]
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        made = list(ex.map(make_frame, [a for a, _ in jobs], [b for _, b in jobs], chunksize=4))
    host = {k: [] for k in KINDS}
    for (k, _), f in zip(jobs, made):
        host[k].append(f)
    return host


def serving_bench(seconds, host):
    """Poisson arrivals at 1500 frames/s, sizes 40% 480x640, 30% 64x1024,
    20% 128x2048, 10% 120x160, 16 GB budget, float16 normals, graph replay;
    the same stream through the plain per-frame float32 path.  `host` holds
    the pre-generated frames of each class (serving_pool)."""
    import torch

    from paper_2007_12065_amd.serve import FrameClass, PlainServer, Server
    from synth import KINDS, poisson_arrivals
    classes = {k: FrameClass(k, v.M, v.N, v.kernel_lap, v.lam, v.iters_lap, v.kernel_bil,
                             v.sigma_length, v.sigma_angle, v.iters_bil)
               for k, v in KINDS.items()}
    pool_per_kind = min(len(v) for v in host.values())
    warm = 1.0
    times, kinds = poisson_arrivals(1500.0, warm + seconds, seed=4000)
    srv = Server(classes, host, 16 << 30, torch.float16)
    srv.presize({"rgbd": 16, "lidar": 12, "lidar128": 8, "rgbd_small": 4})
    batched = srv.serve(times, kinds, warmup_s=warm)
    plain_srv = PlainServer(classes, host)
    plain = plain_srv.serve(times, kinds, warmup_s=warm)
    batched["steps_per_frame"] = round(batched.get("steps", 0) / max(len(times), 1), 4)
    out = {"rate_hz": 1500.0, "measured_s": seconds, "pool_per_kind": pool_per_kind,
           "continuous_batching_f16": batched,
           "plain_f32": plain,
           "throughput_ratio": batched.get("triangles_per_s", 0) / max(plain.get("triangles_per_s", 1), 1)}
    # capacity: the same size mix offered far above what either server
    # sustains; completed triangles per second over the measured window.
    # Frames from pinned host memory (each copy crosses PCIe), then from
    # device memory (frames already resident, as for the headline value).
    sat_rate, sat_s = 30000.0, 1.0
    st, sk = poisson_arrivals(sat_rate, 0.25 + sat_s, seed=4100)
    keep = ("frames", "rejected", "triangles_per_s", "frames_per_s", "steps", "max_step", "plan_rebuilds")
    dev_frames = {k: [torch.from_numpy(f).to("cuda:0") for f in v] for k, v in host.items()}
    del srv
    torch.cuda.empty_cache()
    for mode, frames in (("saturated_host_inputs", host), ("saturated_device_inputs", dev_frames)):
        # 80 slots (2.3 GB), frozen: no re-plan while saturated
        bsrv = Server(classes, frames, 16 << 30, torch.float16)
        bsrv.presize({"rgbd": 32, "lidar": 24, "lidar128": 16, "rgbd_small": 8}, freeze=True)
        psrv = PlainServer(classes, frames)
        sb = bsrv.serve(st, sk, warmup_s=0.25)
        sp = psrv.serve(st, sk, warmup_s=0.25)
        del bsrv
        torch.cuda.empty_cache()
        out[mode] = {"offered_hz": sat_rate, "offered_s": sat_s, "slots": 80,
                     "continuous_batching_f16": {k: sb.get(k) for k in keep},
                     "plain_f32": {k: sp.get(k) for k in keep},
                     "throughput_ratio": sb.get("triangles_per_s", 0) / max(sp.get("triangles_per_s", 1), 1)}
    return out


def fused_pass(plans, frames, k, steps, warmup, stream):
    """Time `steps` fused single-frame calls (frames rotating over the plans),
    then a separate pass with events between the launches.  Returns the
    frame time (s), the mean duration of each launch (s) and their kinds."""
    import numpy as np
    import torch
    sets = len(plans)
    for i in range(warmup):
        plans[i % sets].run_fused(frames[i % sets], stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        plans[i % sets].run_fused(frames[i % sets], stream)
    torch.cuda.synchronize()
    frame_s = (time.perf_counter() - t0) / steps
    kinds = plans[0].run_fused_events(frames[0], [torch.cuda.Event(enable_timing=True)
                                                  for _ in range(17)], stream)
    nl = len(kinds)
    reps = max(20, min(steps, 200))
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nl + 1)] for _ in range(reps)]
    for i in range(reps):
        plans[i % sets].run_fused_events(frames[i % sets], evs[i], stream)
    torch.cuda.synchronize()
    dur = np.array([[evs[i][j].elapsed_time(evs[i][j + 1]) * 1e-3 for j in range(nl)]
                    for i in range(reps)])
    lat = np.array([evs[i][0].elapsed_time(evs[i][nl]) * 1e-3 for i in range(reps)])
    return frame_s, dur.mean(axis=0), kinds, lat


def path_record(kind_name, k, M, N, frame_s, launch_s, kinds, n_tri, pts_np, traffic_key=None):
    """Throughput, effective bandwidth and the per-launch roofline of one
    workload on the fused single-frame path."""
    import paper_2007_12065_amd as pl
    c = frame_counts(M, N, k, n_tri, pts_np)
    # Each launch's duration: the uninstrumented frame time shared out in the
    # proportions the event-bracketed pass measured (an event between two
    # launches delays the next one by a few microseconds, so the bracketed
    # durations are upper bounds; they are reported beside).
    share = frame_s / float(sum(launch_s))
    launches = []
    for j, (kind, t) in enumerate(zip(kinds, launch_s)):
        m = launch_model(kind, c, k)
        r = roofline(m["bytes"], m["lane_ops"], t * share)
        launches.append({"launch": j + 1, "work": m["work"], "kind_bits": kind,
                         "us": round(t * share * 1e6, 2), "us_bracketed": round(t * 1e6, 2),
                         "bytes": int(m["bytes"]),
                         "lane_ops": int(m["lane_ops"]), "bound": r["bound"],
                         "hbm_frac": r["hbm_frac"], "valu_frac": r["valu_frac"]})
    dom = max(range(len(kinds)), key=lambda j: launch_s[j])
    m = launch_model(kinds[dom], c, k)
    roof = roofline(m["bytes"], m["lane_ops"], launch_s[dom] * share)
    roof.update({"kernel": "k_frame_bilateral" if kinds[dom] & pl.PL_LAUNCH_BILATERAL
                 else "k_frame_laplacian", "launch": dom + 1, "work": m["work"],
                 "launch_us": round(launch_s[dom] * share * 1e6, 2),
                 "launch_us_bracketed": round(launch_s[dom] * 1e6, 2),
                 "bytes_per_launch": int(m["bytes"]),
                 "lane_ops_per_launch": int(m["lane_ops"]),
                 "timing": "uninstrumented frame time apportioned by the launches' shares in a "
                           "pass with HIP events around each launch on its stream"})
    # counters of the same launch (workload and kernel template), if the
    # committed summary has them
    cnt = measured_counters(f"{traffic_key}:{frame_kernel_name(kinds[dom], k)}") if traffic_key else None
    roof["traffic"] = cnt.get("bytes_per_launch") if cnt else None
    if cnt and cnt.get("valu_insts"):
        # issued VALU lane-slots (SQ_INSTS_VALU x 64) over the launch time: the
        # hardware's own VALU occupancy, beside the algorithmic valu_frac
        roof["valu_issue_frac"] = round(cnt["valu_insts"] * 64 / (launch_s[dom] * share)
                                        / VALU_PEAK_LANE_OPS, 4)
    staged = staged_bytes(c, k)
    T = c["T"]
    return {"workload": kind_name, "frame": [M, N], "triangles_per_frame": T,
            "valid_triangles_mean": c["n_tri"], "ms_per_frame": round(frame_s * 1e3, 5),
            "triangles_per_s": round(T / frame_s, 1),
            "hbm_effective_gbs": round(staged / frame_s / 1e9, 1),
            "hbm_effective_frac": round(staged / frame_s / 1e9 / HBM_PEAK_GBS, 4),
            "staged_bytes_per_frame": int(staged),
            "frame_valu_frac": round(sum(launch_model(kd, c, k)["lane_ops"] for kd in kinds)
                                     / frame_s / VALU_PEAK_LANE_OPS, 4),
            "launches": launches, "roofline": roof}


def angle_records(kind, k, pts_np, plans_by_dtype, stream, threads):
    """End-to-end normal angle error (p50/p99/max) of the fused path in
    float32 and float16 normal storage against the FP64 oracle on one frame,
    beside the yardstick: the FP64 pipeline restarted from its own smoothed
    vertices rounded to float32 (the spread exact arithmetic shows for a
    float32-sized perturbation)."""
    import numpy as np
    import torch

    import oracle
    ref = oracle.pipeline(pts_np, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
                          k.sigma_angle, k.iters_bil, threads)
    n = len(ref["triangles"])
    n32, c32 = oracle.tri_normals(ref["points"].astype(np.float32), threads)
    f32 = oracle.bilateral(n32, c32, k.kernel_bil, k.sigma_length, k.sigma_angle, k.iters_bil,
                           threads)
    yard = angle_stats(oracle.gather(f32, ref["tri_map"], n), ref["normals_T"])
    out = {"yardstick_fp64_on_f32_vertices": yard}
    x = torch.from_numpy(pts_np).to(plans_by_dtype["f32"].device)
    for name, p in plans_by_dtype.items():
        p.run_fused(x, stream)
        torch.cuda.synchronize()
        assert int(p.n_tri.item()) == n
        out[name] = angle_stats(p.normals_T[:n].float().cpu().numpy(), ref["normals_T"])
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the path shards by frame with no exchange between "
              "GPUs, and multi-GPU runs are not part of this build (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from synth import KINDS, make_frame

    # host inputs first (worker processes, before the GPU is initialised)
    serve_host = serving_pool(args.pool) if args.serving_seconds > 0 else None
    k = KINDS["rgbd"]
    M, N = k.M, k.N
    sets = args.sets
    frames_np = [make_frame("rgbd", 1000 + i) for i in range(sets)]
    print("[bench] inputs ready", file=sys.stderr, flush=True)

    import torch

    import paper_2007_12065_amd as pl
    from paper_2007_12065_amd import tune
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    threads = min(16, os.cpu_count() or 1)
    frames = [torch.from_numpy(f).to(dev) for f in frames_np]
    mk = lambda kk, dt=torch.float32: pl.FramePlan(kk.M, kk.N, kk.kernel_lap, kk.lam, kk.iters_lap,
                                                   kk.kernel_bil, kk.sigma_length, kk.sigma_angle,
                                                   kk.iters_bil, dt, dev)
    plans = [mk(k) for _ in range(sets)]
    stream = pl._stream(dev)

    # tile shapes and sweep fusion: the committed tuning file, or tuned here
    if args.retune:
        per = {}
        # one workload per table entry: large frames (480x640 3x3, 128x2048
        # 5x5) and small ones (120x160 3x3, 64x1024 5x5)
        for kind in ("rgbd", "lidar128", "rgbd_small", "lidar"):
            kk = KINDS[kind]
            fr = frames if kind == "rgbd" else [torch.from_numpy(make_frame(kind, 7 + i)).to(dev)
                                                for i in range(8)]
            per[kind] = (fr, kk.kernel_lap, kk.lam, kk.iters_lap, kk.kernel_bil, kk.sigma_length,
                         kk.sigma_angle, kk.iters_bil)
        tune.tune_frame(list(per.values()), cache_path=args.retune)
        from synth import batch_mix
        specs = [dict(pts=torch.from_numpy(make_frame(kd, sd)).to(dev), kernel_lap=KINDS[kd].kernel_lap,
                      lam=KINDS[kd].lam, iters_lap=KINDS[kd].iters_lap, kernel_bil=KINDS[kd].kernel_bil,
                      sigma_length=KINDS[kd].sigma_length, sigma_angle=KINDS[kd].sigma_angle,
                      iters_bil=KINDS[kd].iters_bil) for kd, sd in batch_mix()]
        tune.autotune_batch(specs, cache_path=args.retune, reps=10)
        del specs
        tune_path = args.retune
    else:
        tune_path = args.tune_file
        if tune.load_cache(tune_path) == 0:
            print(f"bench.py: no tuning for {tune.arch_name()} in {tune_path}; run with --retune PATH",
                  file=sys.stderr)
            sys.exit(3)
    tuning = json.load(open(tune_path)).get(tune.arch_name(), {})
    print(f"[bench] {sets} frame sets ready; warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)

    # the headline: the fused single-frame path, timed alone on the stream
    K = args.steps
    frame_s, launch_s, kinds, lat = fused_pass(plans, frames, k, K, args.warmup, stream)
    n_tri = [int(p.n_tri.item()) for p in plans]
    rec = path_record("rgbd", k, M, N, frame_s, launch_s, kinds, float(np.mean(n_tri)),
                      frames_np[0], traffic_key="rgbd")
    T = rec["triangles_per_frame"]

    # the four single-frame calls (the plain baseline of the batched and
    # served comparisons), uninstrumented, then with events between calls
    calls = ["pl_mesh_opc", "pl_laplacian", "pl_tri_normals", "pl_bilateral"]

    def four(i, ev=None):
        p, x = plans[i % sets], frames[i % sets]
        for j, fn in enumerate((lambda: p.run_mesh(x, stream), lambda: p.run_laplacian(x, stream),
                                lambda: p.run_normals(stream), lambda: p.run_bilateral(stream))):
            if ev is not None:
                ev[j].record()
            fn()
        if ev is not None:
            ev[4].record()
    for i in range(args.warmup):
        four(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        four(i)
    torch.cuda.synchronize()
    four_s = (time.perf_counter() - t0) / K
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        p, x = plans[i % sets], frames[i % sets]
        p.run_laplacian(x, stream)
        p.run_normals(stream)
        p.run_bilateral(stream)
    torch.cuda.synchronize()
    smooth_s = (time.perf_counter() - t0) / K
    reps = min(K, 200)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(reps)]
    for i in range(reps):
        four(i, evs[i])
    torch.cuda.synchronize()
    per_call = {c: float(np.median([evs[i][j].elapsed_time(evs[i][j + 1]) * 1e3 for i in range(reps)]))
                for j, c in enumerate(calls)}

    # measured HBM ceiling: a 256 MiB device-to-device copy (read + write)
    ca = torch.empty(64 << 20, dtype=torch.float32, device=dev)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        cb.copy_(ca)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * ca.numel() * 4 * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del ca, cb

    out = {
        "metric": METRIC, "value": round(T / frame_s, 1), "unit": "triangles/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(frame_s * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rgbd 480x640 single-frame path (pl_smooth_frame: mesh + Laplacian "
                               "3x3 x4 + normals + bilateral 3x3 x2 + gather), float32 normals",
                   "frame": [M, N], "triangles_per_frame": T,
                   "valid_triangles_mean": float(np.mean(n_tri)), "frame_sets": sets,
                   "tuning_file": os.path.relpath(tune_path, ROOT)},
        "roofline": rec["roofline"],
        "launches": rec["launches"],
        "hbm_effective_gbs": rec["hbm_effective_gbs"],
        "hbm_effective_frac": rec["hbm_effective_frac"],
        "staged_bytes_per_frame": rec["staged_bytes_per_frame"],
        "frame_valu_frac": rec["frame_valu_frac"],
        "hbm_copy_ceiling_gbs": round(copy_gbs, 1),
        "instrumented_frame_us": {"p50": round(float(np.median(lat)) * 1e6, 2),
                                  "p99": round(float(np.percentile(lat, 99)) * 1e6, 2)},
        "four_call_path": {"ms_per_frame": round(four_s * 1e3, 5),
                           "triangles_per_s": round(T / four_s, 1),
                           "smoothing_only_triangles_per_s": round(T / smooth_s, 1),
                           "call_us_instrumented": {c: round(v, 2) for c, v in per_call.items()},
                           "note": "medians per call from a separate event-instrumented pass"},
        "tuning": {name: {"tile": list(r["best"][:2]), "fuse": r["best"][2]}
                   for name, r in tuning.items()},
    }
    print(f"[bench] fused frame {frame_s * 1e6:.2f} us, four calls {four_s * 1e6:.2f} us",
          file=sys.stderr, flush=True)

    # the same frames with float16 normal storage (m1): the fused path's time
    # beside the float32 headline
    plans16 = [mk(k, torch.float16) for _ in range(sets)]
    f16_s, f16_launch, f16_kinds, _ = fused_pass(plans16, frames, k, K, args.warmup, stream)
    out["fused_f16"] = {"ms_per_frame": round(f16_s * 1e3, 5),
                        "triangles_per_s": round(T / f16_s, 1),
                        "vs_f32": round(frame_s / f16_s, 4),
                        "launch_us_bracketed": [round(t * 1e6, 2) for t in f16_launch],
                        "note": "float16 normals (raw, intermediate and filtered), float32 "
                                "arithmetic and points"}
    del plans16

    if args.per_config:
        print("[bench] per-workload records", file=sys.stderr, flush=True)
        per = {}
        for name, kind in (("c0_rgbd_120x160", "rgbd_small"), ("c1_rgbd_480x640", "rgbd"),
                           ("c2_lidar_64x1024", "lidar"), ("lidar_128x2048", "lidar128")):
            kk = KINDS[kind]
            if kind == "rgbd":
                r = {kk2: v for kk2, v in rec.items() if kk2 != "launches"}
                fnp = frames_np[0]
            else:
                fr_np = [make_frame(kind, 1000 * {"rgbd_small": 0, "lidar": 2}.get(kind, 5) + i)
                         for i in range(sets)]
                fr = [torch.from_numpy(f).to(dev) for f in fr_np]
                pp = [mk(kk) for _ in range(sets)]
                fs, ls, kd, _ = fused_pass(pp, fr, kk, K, args.warmup, stream)
                nt = float(np.mean([int(p.n_tri.item()) for p in pp]))
                r = path_record(kind, kk, kk.M, kk.N, fs, ls, kd, nt, fr_np[0],
                                traffic_key=kind)
                fnp = fr_np[0]
                del fr, pp
            r["angle_err_rad_vs_fp64"] = angle_records(kind, kk, fnp,
                                                       {"f32": mk(kk), "f16": mk(kk, torch.float16)},
                                                       stream, threads)
            per[name] = r
        out["per_config"] = per
    if args.aux:
        print("[bench] group assignment", file=sys.stderr, flush=True)
        for p, x in zip(plans, frames):
            p.run(x)          # T_FC normals for the vertex update
        torch.cuda.synchronize()
        out["groups"] = groups_bench(plans, k, stream, stream)
        print("[bench] gaussian accumulator", file=sys.stderr, flush=True)
        out["gaussian_accumulator"] = ga_bench(plans, stream)
        # the paper integrates a sample of about 12% of the normals (sample_pct)
        out["gaussian_accumulator_sampled"] = ga_bench(plans, stream, stride=8)
        print("[bench] user-mesh half-edges", file=sys.stderr, flush=True)
        out["user_halfedges"] = user_halfedges_bench(plans, stream)
        print("[bench] vertex update", file=sys.stderr, flush=True)
        out["vertex_update"] = vertex_update_bench(plans, stream)
    if args.batched:
        print("[bench] batched 64-frame mix", file=sys.stderr, flush=True)
        out["batched"] = batched_bench(tuning)
    if args.serving_seconds > 0:
        print("[bench] serving stream", file=sys.stderr, flush=True)
        del plans, frames
        torch.cuda.empty_cache()
        out["serving"] = serving_bench(args.serving_seconds, serve_host)
    if args.cpu_seconds > 0:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(frames_np, k, args.cpu_seconds)
        out["cpu_baseline_1thread"] = cpu_baseline(frames_np, k, max(2.0, args.cpu_seconds / 2),
                                                   threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
