"""Benchmark of the whole OPC meshing + smoothing path on one MI355X.

One step = one pass of the plain per-frame path over one 480x640 synthetic
RGBD frame (floor, two walls, six boxes, 8% NaN holes): mesh extraction
(Alg. 1-2), 4 Laplacian sweeps (3x3, lambda = 1), triangle normals and
centroids, 2 bilateral sweeps (3x3 quads, sigma_length = sigma_angle = 0.1)
and the gather onto T, all in float32.  Inputs are resident in HBM before the
timed region; 16 frames with separate input and output buffers rotate so the
working set (~1.1 GB) exceeds the 256 MB last-level cache.

Prints one JSON line (the contract fields plus the dominant kernel's
roofline and the FP64 oracle's CPU throughput).
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
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--sets", type=int, default=16, help="rotating frame buffer sets")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="bound on the oracle's CPU-baseline sample (0 = skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain copy kernel of known size (counter calibration)")
    return ap.parse_args()


def kernel_specs(k, M, N, n_tri_mean):
    """Per-call launch counts and algorithmic traffic / arithmetic per launch.

    Bytes are the minimal HBM traffic of one launch (each input read once,
    each output written once).  Flops count the arithmetic of the paper's
    formulas per output: Laplacian 17 per neighbour (difference 3, squared
    norm 5, inverse root 1, weight sum 1, weighted sum 6, + update), bilateral
    26 per neighbour pair (two squared differences 16, exponent 3, exp 1,
    weighted sum 6)."""
    P = M * N
    T = 2 * (M - 1) * (N - 1)
    nb_lap = k.kernel_lap ** 2 - 1
    nb_bil = 2 * (k.kernel_bil ** 2 - 1)
    from paper_2007_12065_amd import lap_fused_sweeps
    F = lap_fused_sweeps(k.kernel_lap)
    lap_launches = -(-k.iters_lap // F)
    return {
        "pl_laplacian": dict(kernel="k_laplacian", launches=lap_launches,
                             bytes=24 * P, flops=P * (k.iters_lap / lap_launches) * (17 * nb_lap + 7)),
        "pl_tri_normals": dict(kernel="k_tri_normals", launches=1, bytes=12 * P + 24 * T,
                               flops=T * 30),
        "pl_bilateral": dict(kernel="k_bilateral", launches=k.iters_bil,
                             bytes=36 * T + (4 * T + 12 * n_tri_mean) / k.iters_bil,
                             flops=T * (26 * nb_bil + 10)),
        "pl_mesh_opc": dict(kernel="k_mesh_*", launches=3,
                            bytes=(12 * P + T // 2 + 4 * T + 24 * n_tri_mean) / 3, flops=0),
    }


def cpu_baseline(frames_np, k, seconds):
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
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
    return {"value": T * done / el, "unit": "triangles/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} frames of the 480x640 workload (whole path, FP64 C oracle, "
                      f"{threads} OpenMP threads), {el:.1f} s"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the path shards by frame with no exchange between "
              "GPUs, and multi-GPU runs are not part of this build (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2007_12065_amd as pl
    from synth import KINDS, make_frame

    k = KINDS["rgbd"]
    M, N = k.M, k.N
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sets = args.sets
    frames_np = [make_frame("rgbd", 1000 + i) for i in range(sets)]
    frames = [torch.from_numpy(f).to(dev) for f in frames_np]
    plans = [pl.FramePlan(M, N, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                          k.sigma_length, k.sigma_angle, k.iters_bil, torch.float32, dev)
             for _ in range(sets)]
    stream = torch.cuda.current_stream(dev)
    s = pl._stream(dev)
    print(f"[bench] {sets} frame sets ready; warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)

    calls = ["pl_mesh_opc", "pl_laplacian", "pl_tri_normals", "pl_bilateral"]

    def step(i, ev=None):
        p, x = plans[i % sets], frames[i % sets]
        if ev is not None:
            ev[0].record(stream)
        p.run_mesh(x, s)
        if ev is not None:
            ev[1].record(stream)
        p.run_laplacian(x, s)
        if ev is not None:
            ev[2].record(stream)
        p.run_normals(s)
        if ev is not None:
            ev[3].record(stream)
        p.run_bilateral(s)
        if ev is not None:
            ev[4].record(stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize(dev)

    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for i in range(K):
        step(i, evs[i])
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - t0

    per_call = {c: np.array([evs[i][j].elapsed_time(evs[i][j + 1]) * 1e3 for i in range(K)])
                for j, c in enumerate(calls)}
    lat = np.array([evs[i][0].elapsed_time(evs[i][4]) * 1e3 for i in range(K)])
    n_tri = [int(p.n_tri.item()) for p in plans]
    T = 2 * (M - 1) * (N - 1)
    ms = elapsed / K * 1e3
    value = T / (elapsed / K)

    specs = kernel_specs(k, M, N, float(np.mean(n_tri)))
    launch_us = {c: float(per_call[c].mean() / specs[c]["launches"]) for c in calls}
    dom = max(("pl_laplacian", "pl_tri_normals", "pl_bilateral"), key=lambda c: per_call[c].mean())
    sp = specs[dom]
    t_launch = launch_us[dom] * 1e-6
    gbs = sp["bytes"] / t_launch / 1e9
    tflops = sp["flops"] / t_launch / 1e12
    byte_frac = gbs / HBM_PEAK_GBS
    alu_frac = tflops / FP32_VECTOR_PEAK_TFLOPS
    if byte_frac >= alu_frac:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(byte_frac, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(tflops, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(alu_frac, 4)}
    roof.update({"kernel": sp["kernel"], "launch_us": round(launch_us[dom], 2),
                 "bytes_per_launch": int(sp["bytes"]), "flops_per_launch": int(sp["flops"]),
                 "hbm_frac": round(byte_frac, 4), "traffic": None})

    if args.copy_probe:
        # plain copy kernel of known size for counter calibration: 12 P bytes
        # read and written (pl_laplacian with zero sweeps is a copy)
        for p, x in zip(plans[:4], frames[:4]):
            pl.pl_laplacian(x, k.kernel_lap, k.lam, 0, out=p.points)
        torch.cuda.synchronize(dev)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "triangles/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rgbd 480x640 plain per-frame path (mesh + Laplacian 3x3 x4 + "
                               "normals + bilateral 3x3 x2 + gather), float32 normals",
                   "frame": [M, N], "triangles_per_frame": T, "valid_triangles_mean": float(np.mean(n_tri)),
                   "frame_sets": sets},
        "stage_us": {c: round(float(np.median(per_call[c])), 2) for c in calls},
        "frame_latency_us": {"p50": round(float(np.median(lat)), 2),
                             "p99": round(float(np.percentile(lat, 99)), 2)},
        "hbm_effective_gbs": round(sum(specs[c]["bytes"] * specs[c]["launches"] for c in calls)
                                   / (elapsed / K) / 1e9, 1),
        "roofline": roof,
    }
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(frames_np, k, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
