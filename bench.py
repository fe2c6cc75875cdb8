#!/usr/bin/env python3
"""Benchmark of the Yee/UPML hot path on one MI355X.

One benchmark "step" is one full leapfrog step (B/H then D/E with UPML, the PEC
planes, 8 current sources and 64 probes fused in the field kernel) over the
large-board workload: 1048 x 792 x 88 cells (1024 x 768 x 64 interior + a
12-cell PML on every face), the running FP64 DFT of every probe at 256
frequencies folded in once per timed call.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
  python bench.py --copy-calibration      # plain device copy for PMC scaling
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "field_step_config3_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1008_2602_amd", "csrc", f)
                  for f in ("fdtd_kernels.hip", "fdtd_internal.h")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per field-kernel launch from the committed PMC summary, or None
    when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def copy_calibration(nbytes=1 << 30, reps=5):
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": nbytes, "reps": reps}), flush=True)


def cpu_baseline(board, budget_s=20.0):
    """The FP64 oracle, as it stands, on this host's cores: a bounded number of
    steps of the same board (one untimed step touches the memory, two more
    calibrate the per-step time), in Gcell-updates/s."""
    import oracle
    st = oracle.new_state(board)
    oracle.run(board, nsteps=1, state=st)
    t0 = time.perf_counter()
    oracle.run(board, nsteps=2, state=st)
    per = (time.perf_counter() - t0) / 2
    n = int(max(2, min(400, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(board, nsteps=n, state=st)
    dt = time.perf_counter() - t0
    return {"value": round(board.cells * n / dt / 1e9, 4), "unit": "Gcell-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} steps of the full {board.nx}x{board.ny}x{board.nz} board after 3 "
                      f"calibration steps ({dt:.1f} s; FP64, unified D/B storage)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--tile", default="")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X: this build has no multi-GPU path "
              "(boards shard whole across GPUs by design; see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return

    import boardgen
    from paper_1008_2602_amd import fdtd as F

    board = boardgen.config3()
    K, W = int(args.steps), int(args.warmup)
    tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else (64, 16)
    stream = torch.cuda.current_stream().cuda_stream
    g, ids = F.grid_from_board(board, max_steps=W + K, hip_stream=stream, tile=tile)
    info = F.fdtd_get_info(g)
    F.fdtd_step_n(g, W)
    F.fdtd_synchronize(g)

    F.fdtd_set_timing(g, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fdtd_step_n(g, K)
    F.fdtd_synchronize(g)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = F.fdtd_get_timing(g)
    info = F.fdtd_get_info(g)
    probe0 = F.fdtd_get_probe(g, ids[0], W + K)
    F.fdtd_destroy_grid(g)
    assert np.all(np.isfinite(probe0))

    cells = board.cells
    value = cells * K / wall / 1e9
    per_launch_s = kern_ms / 1e3 / launches
    achieved = info.step_bytes / per_launch_s / 1e9
    traffic = measured_traffic()
    out = {
        "metric": "Gcell-updates/s + % HBM roofline (1 GPU); served solves p50/p99 latency",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(wall / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "large-board HBM stress: 1048x792x88 cells (1024x768x64 interior "
                        "+ 12-cell UPML per face), eps_r 4.2 slab, two PEC power islands, "
                        "8 Gaussian Jz sources, 64 probes, FP64 DFT at 256 frequencies",
            "cells": cells,
            "tile": f"{tile[0]}x{tile[1]}",
            "dt_s": info.dt,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "field_step",
            "algorithmic_bytes_per_launch": info.step_bytes,
            "avg_launch_ms": round(per_launch_s * 1e3, 4),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(board)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
