#!/usr/bin/env python3
"""Benchmark of the Yee/UPML hot path on one MI355X.

One benchmark "step" is one full leapfrog step (B/H then D/E with UPML, the PEC
planes, 8 current sources and 64 probes fused in the field kernel) over the
large-board workload: 1048 x 792 x 88 cells (1024 x 768 x 64 interior + a
12-cell PML on every face), the running FP64 DFT of every probe at 256
frequencies folded in once per timed call.  Prints one JSON line.

Beside it, the same line carries
  * "batched": 64 uneven board variants advanced together by fdtd_step_many
    (one field launch per step over all boards), Gcell-updates/s and the HBM
    fraction on algorithmic bytes;
  * "served": 512 seeded Poisson arrivals of board variants (5 % large
    800x800x64 boards) offered at 0.7x the measured batched capacity for the
    stream's mean board, admitted by device footprint into 85 % of free HBM,
    advanced in 500-step chunks in the tuned batched shape, each finished solve
    read back with its probe spectra; p50/p99 latency over all solves,
    throughput and the GPU-busy fraction.  Each solve is 8000 steps; the arrivals
    span about 7 minutes, most of the default run (--serve-requests cuts it).
    Unless --no-cpu-baseline, the oracle re-runs the smallest served solve and
    the largest probe relative L2 is reported beside the latencies;
  * "plane_dft": the large board with a 16-frequency DFT of its ground-plane Ez
    over the whole plane, against the plain step;
  * "node_passes": boards in the node passes' arithmetic: the large board run
    into the PML with Eq. 2's eps_rw (material two-step kernel and node passes
    alone), the large board lossy with copper planes, the paper's Fig. 3 board
    and a lossy Table 1 run;
  * "zconv": the z-convergence study (1..15 cells across the dielectric) as
    one batched call;
  * "shard": the large board cut into 8 y-slabs of 1048x99x88 cells (one
    rank's share of a slab decomposition, halo stubbed), every slab timed on
    its own;
  * "realistic", "small": the 444x364x60 realistic board's full 20000-step
    solve with its 16 probe spectra, and the 80x72x37 small board's 3000-step
    solve (beside the oracle's whole run of it), one board at a time;
  * "table1": the paper's own Table 1 run (resistive source, 30000 steps) as
    one solve, and a 64-board sweep of its source resistance, with the oracle's
    time for the same whole run beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                  [--only single|batch|serve|table1|plane|zconv|eps|eps_large|shard|realistic]
  python bench.py --copy-calibration      # plain device copy for PMC scaling
"""
import argparse
import dataclasses
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "field_step2_1048x792x88_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1008_2602_amd", "csrc", f)
                  for f in ("fdtd_kernels.hip", "fdtd_kernels2.hip", "fdtd_device.h",
                            "fdtd_internal.h", "fdtd_host.cpp")]


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace runs collapsed: what the
    compiler sees, so that editing a comment does not void the counters."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash(read=None) -> str:
    """Hash of the field-kernel sources' code (comments and layout ignored).
    read(path) -> text, default: the working tree."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        if read is None:
            with open(p, encoding="utf-8") as f:
                text = f.read()
        else:
            text = read(p)
        h.update(_code_only(text).encode())
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


def host_cpu():
    """CPU model and logical core count of this host (the oracle's machine)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" in line:
                    k, v = (x.strip() for x in line.split(":", 1))
                    if k in ("model name", "cpu family", "model") and k not in info:
                        info[k] = v
    except OSError:
        pass
    model = info.get("model name", "unknown")
    if "cpu family" in info:
        model += f" (family {info['cpu family']}, model {info.get('model', '?')})"
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def _oracle_rate(board, threads, budget_s, max_steps=400):
    """Gcell-updates/s of the oracle on ``board`` with ``threads`` threads: one
    untimed step touches the memory, two more calibrate the per-step time, then
    about budget_s seconds of steps are timed.  Returns (rate, steps, seconds)."""
    import oracle
    oracle.set_threads(threads)
    st = oracle.new_state(board)
    oracle.run(board, nsteps=1, state=st)
    t0 = time.perf_counter()
    oracle.run(board, nsteps=2, state=st)
    per = (time.perf_counter() - t0) / 2
    n = int(max(2, min(max_steps, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(board, nsteps=n, state=st)
    dt = time.perf_counter() - t0
    return board.cells * n / dt / 1e9, n, dt


def cpu_baseline(board, budget_s=20.0, single_budget_s=8.0):
    """The FP64 oracle, as it stands, on this host's cores: a bounded number of
    steps of the same board, in Gcell-updates/s, with all host threads and with
    one thread."""
    import oracle
    threads = oracle.num_threads()        # OpenMP's default: every host thread it may use
    rate, n, dt = _oracle_rate(board, threads, budget_s)
    cores = oracle.num_threads()
    rate1, n1, dt1 = _oracle_rate(board, 1, single_budget_s)
    oracle.set_threads(threads)
    out = {"value": round(rate, 4), "unit": "Gcell-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} steps of the full {board.nx}x{board.ny}x{board.nz} board after 3 "
                     f"calibration steps ({dt:.1f} s; FP64, unified D/B storage)",
           "single_thread": {"value": round(rate1, 5), "unit": "Gcell-updates/s", "cores": 1,
                             "sample": f"{n1} steps of the same board ({dt1:.1f} s)"}}
    out.update(host_cpu())
    return out


def sec8d_step_bytes(info):
    """Algorithmic bytes of one step, counted as two separate passes per step in
    the split layout (D/B kept only where a PML loss acts):
    per cell 72 B (separate H and E passes: E, H read and H written, then H, E
    read and E written, FP32) plus the class index, plus 8 B (read and write) for
    every kept D/B component.  The kept D/B bytes are the library's own count
    (its step_bytes minus the 48 B of E and H and the class per cell)."""
    cls = 2 if info.n_classes > 256 else 1
    aux = info.step_bytes - info.cells * (48 + cls)
    return info.cells * (72 + cls) + aux


def run_single(F, torch, K, W, tile):
    import numpy as np
    import boardgen
    board = boardgen.large_board()
    stream = torch.cuda.current_stream().cuda_stream
    if tile is None:
        from paper_1008_2602_amd import tune
        tile = tune.tune_board(board)
    g, ids = F.grid_from_board(board, max_steps=W + K, hip_stream=stream, tile=tile)
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
    return board, tile, info, wall, kern_ms, launches


def run_plane_dft(F, torch, K, W, plain_ms_per_step):
    """The large board with the plane DFT of its ground-plane Ez (the row above
    the ground sheet) at 16 frequencies, 0.5-8 GHz: ms per step against the plain
    path, and the fold kernel's algorithmic bytes (each fold reads 32 FP32 samples
    and reads and writes an FP64 complex accumulator per frequency, per padded
    plane node; the field kernel adds one 4-byte ring store per plane node and
    step)."""
    import numpy as np
    import boardgen
    from paper_1008_2602_amd import tune
    board = boardgen.large_board()
    nf = 16
    board.plane_dft = (board.meta["layout"]["kg"], np.linspace(0.5e9, 8e9, nf))
    tile = tune.tune_board(board)
    g, _ = F.grid_from_board(board, max_steps=W + K, tile=tile)
    F.fdtd_step_n(g, W)
    F.fdtd_synchronize(g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fdtd_step_n(g, K)
    F.fdtd_synchronize(g)
    wall = time.perf_counter() - t0
    plane = F.fdtd_get_plane_dft(g, board.ny, board.nx)
    F.fdtd_destroy_grid(g)
    assert np.all(np.isfinite(plane))
    pitch = (board.nx + 1 + 31) // 32 * 32
    plane_nodes = pitch * (board.ny + 1)
    ms = wall / K * 1e3
    return {
        "workload": f"large board {board.nx}x{board.ny}x{board.nz} with the plane DFT of Ez at "
                    f"k={board.plane_dft[0]} (above the ground sheet), {nf} frequencies 0.5-8 GHz",
        "tile": "x".join(str(v) for v in tile),
        "steps": K,
        "ms_per_step": round(ms, 4),
        "overhead_vs_plain": round(ms / plain_ms_per_step - 1.0, 4),
        "gcell_updates_per_s": round(board.cells * K / wall / 1e9, 3),
        "fold_launches": -(-K // 32),
        "fold_bytes_per_launch": int(plane_nodes * (32 * 4 + nf * 32)),
        "ring_store_bytes_per_step": int(plane_nodes * 4),
    }


def run_eps(F, torch, K=200, W=10, large_only=False, only=None):
    """Boards in the node passes' arithmetic (Eq. 2's eps_rw, lossy dielectrics,
    resistive sheets).  (1) The large board with its eps_r 4.2 slab run through
    the x/y PML to the outer wall (1048x792x88), eps_rw on: pairs of steps on the
    two-step kernels (the plain one and its material variant, the default), and
    every step on the node passes,
    against the fused kernels on the same board with eps_rw = 1; (2) the large
    board with a lossy dielectric (loss tangent 0.02 at 5 GHz) and copper planes
    (resistive sheets, 18.4 milliohm per square); (3) the paper's Fig. 3 board
    (100x60x0.8 mm running into the UPML), 1000 steps of 1 ps; (4) the Table 1 run
    with a lossy dielectric.  large_only: (1) and (2) alone; only: the one case
    of (1) and (2) so named (for a profiler run)."""
    import boardgen
    from paper_1008_2602_amd import tune
    b = boardgen.large_board(steps=W + K)
    kg, kt = b.meta["layout"]["kg"], b.meta["layout"]["kt"]
    b.eps_r_cell[kg:kt, :, :] = 4.2
    b.sources, b.probes, b.dft_freqs = b.sources, b.probes[:4], None
    lossy = boardgen.conductor_loss(boardgen.lossy_dielectric(boardgen.large_board(steps=W + K), 0.02))
    lossy.probes, lossy.dft_freqs = lossy.probes[:4], None
    out = {}
    cases = (("eps_rw", dataclasses.replace(b, pml_eps_rw=True), None, 1),
             ("eps_rw_node_passes", dataclasses.replace(b, pml_eps_rw=True), (64, 8, 1), 0),
             ("fused_eps_rw_1", b, "tune", -1),
             ("lossy_copper", lossy, None, 1))
    for name, bb, tile, mat in cases:
        if only is not None and name != only:
            continue
        if tile == "tune":
            tile = tune.tune_board(bb)
        g, _ = F.grid_from_board(bb, max_steps=W + K, tile=tile)
        F.fdtd_step_n(g, W)
        F.fdtd_synchronize(g)
        t0 = time.perf_counter()
        F.fdtd_step_n(g, K)
        F.fdtd_synchronize(g)
        wall = time.perf_counter() - t0
        info = F.fdtd_get_info(g)
        F.fdtd_destroy_grid(g)
        assert info.node_passes == (1 if mat >= 0 else 0) and info.material_two_step == max(mat, 0)
        split = {0: "no tile plane needs the material variant",
                 1: f"material variant per tile, 64x14x2, on {info.material_permille / 10:.1f} % of "
                    f"the tile planes",
                 2: f"material variant per plane, 64x10x2, on {info.material_permille / 10:.1f} % of "
                    f"the tile planes"}
        out[name] = {
            "kernel": (f"plain 64x14x2 and its variants ({split[info.material_split]}; "
                       f"conduction-only flavour, 64x14x2, on {info.conduct_permille / 10:.1f} %), "
                       f"odd steps on the node passes" if mat == 1 else
                       "node passes" if mat == 0 else f"fused {info.tile_x}x{info.tile_y}x{info.tile_steps}"),
            "ms_per_step": round(wall / K * 1e3, 4),
            "gcell_updates_per_s": round(bb.cells * K / wall / 1e9, 3),
            # the algorithmic bytes of a step of this board (sec8d_step_bytes)
            "hbm_frac_algorithmic": round(sec8d_step_bytes(info) * K / wall / 1e9 / HBM_PEAK_GBS, 4),
        }
    if large_only or only is not None:
        return out
    f3 = boardgen.fig3_board(steps=1000)
    g, _ = F.grid_from_board(f3, max_steps=f3.steps)
    F.fdtd_step_n(g, 0)
    F.fdtd_synchronize(g)
    t0 = time.perf_counter()
    F.fdtd_step_n(g, f3.steps)
    F.fdtd_synchronize(g)
    wall = time.perf_counter() - t0
    F.fdtd_destroy_grid(g)
    out["fig3"] = {"cells": f3.cells, "steps": f3.steps, "wall_s": round(wall, 4),
                   "gcell_updates_per_s": round(f3.cells * f3.steps / wall / 1e9, 3)}
    # the Table 1 run with a lossy dielectric (loss tangent 0.02 at 5 GHz)
    t1 = boardgen.lossy_dielectric(boardgen.table1_board(steps=30000, source="resistive"), 0.02)
    g, _ = F.grid_from_board(t1, max_steps=t1.steps)
    F.fdtd_step_n(g, 0)
    F.fdtd_synchronize(g)
    t0 = time.perf_counter()
    F.fdtd_step_n(g, t1.steps)
    F.fdtd_synchronize(g)
    wall = time.perf_counter() - t0
    assert F.fdtd_get_info(g).node_passes == 1
    F.fdtd_destroy_grid(g)
    out["lossy_table1"] = {"cells": t1.cells, "steps": t1.steps, "wall_s": round(wall, 4),
                           "gcell_updates_per_s": round(t1.cells * t1.steps / wall / 1e9, 3)}
    out["workload"] = ("material boards: large board 1048x792x88 with its eps_r 4.2 slab through the "
                       "x/y PML (eps_rw on: the material two-step kernel and the node passes, vs "
                       "the fused kernels at eps_rw = 1); the large board lossy (tan d 0.02) with "
                       "copper planes; Fig. 3 board "
                       f"{f3.nx}x{f3.ny}x{f3.nz} running into the UPML, 1000 steps; the Table 1 "
                       "run with a loss tangent of 0.02, 30000 steps")
    return out


def run_zconv(F, torch, steps=4000):
    """The z-convergence study of the Results section: the Table 1 footprint with
    the 0.8 mm dielectric cut into 1..15 z cells (15 boards, 48x43x21 .. 48x43x91),
    all advanced together by one fdtd_step_many call.  Reports the wall time and
    how far 2 cells sit from 15 (ground-plane Ez, relative L2 over the series and
    the far-corner peak)."""
    import numpy as np
    import boardgen
    boards = [boardgen.zconv_board(n, steps=steps) for n in range(1, 16)]
    hs = [F.grid_from_board(b, max_steps=steps) for b in boards]
    gs = [g for g, _ in hs]
    for g in gs:
        F.fdtd_step_n(g, 0)
    F.fdtd_synchronize(gs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fdtd_step_many(gs, [steps] * len(gs))
    F.fdtd_synchronize(gs[0])
    wall = time.perf_counter() - t0
    series = [np.stack([F.fdtd_get_probe(g, p, steps) for p in ids]).astype(np.float64)
              for g, ids in hs]
    for g in gs:
        F.fdtd_destroy_grid(g)
    ref, two = series[-1], series[1]
    rel = max(float(np.linalg.norm(two[p] - ref[p]) / np.linalg.norm(ref[p])) for p in range(3))
    corner = float(abs(np.abs(two[2]).max() - np.abs(ref[2]).max()) / np.abs(ref[2]).max())
    cells = sum(b.cells for b in boards)
    return {
        "workload": "z-convergence family: 40x30x0.8 mm board, 1..15 cells across the dielectric "
                    f"(15 boards, {cells} cells in all), {steps} steps, one batched call",
        "wall_s": round(wall, 3),
        "gcell_updates_per_s": round(cells * steps / wall / 1e9, 3),
        "two_vs_fifteen_rel_l2": round(rel, 5),
        "two_vs_fifteen_corner_peak": round(corner, 6),
    }


def run_shard(F, torch, K=400, W=20, nranks=8):
    """The field kernel at one rank's share of the large board slab-decomposed
    along y (8 slabs of 1048x99x88 cells; the cut faces carry no PML and, with no
    exchange, act as PEC walls: the halo is stubbed).  Each slab is timed on its
    own; a decomposed step would take the slowest slab's time plus the exchange,
    which is not built.  Reports per-slab ms per step and the HBM fraction of the
    slowest slab's launches on their algorithmic bytes."""
    import numpy as np
    import boardgen
    from paper_1008_2602_amd import tune
    per = []
    for rank in range(nranks):
        board = boardgen.large_board_shard(rank, nranks)
        tile = tune.tune_board(board)
        g, ids = F.grid_from_board(board, max_steps=W + K, tile=tile)
        F.fdtd_step_n(g, W)
        F.fdtd_synchronize(g)
        F.fdtd_set_timing(g, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.fdtd_step_n(g, K)
        F.fdtd_synchronize(g)
        wall = time.perf_counter() - t0
        kern_ms, launches = F.fdtd_get_timing(g)
        info = F.fdtd_get_info(g)
        probe = F.fdtd_get_probe(g, ids[0], W + K) if ids else np.zeros(1)
        F.fdtd_destroy_grid(g)
        assert np.all(np.isfinite(probe))
        launch_s = kern_ms / 1e3 / launches
        per.append({"rank": rank, "tile": "x".join(str(v) for v in tile),
                    "ms_per_step": wall / K * 1e3, "launch_s": launch_s,
                    "launch_bytes": sec8d_step_bytes(info) * K / launches, "cells": board.cells})
    slow = max(per, key=lambda r: r["ms_per_step"])
    achieved = slow["launch_bytes"] / slow["launch_s"] / 1e9
    return {
        "workload": f"large board split into {nranks} y-slabs of 1048x{792 // nranks}x88 cells "
                    "(cut faces without PML, halo stubbed), each slab stepped alone",
        "cells_per_slab": slow["cells"],
        "steps": K,
        "tiles": sorted({r["tile"] for r in per}),
        "ms_per_step": [round(r["ms_per_step"], 4) for r in per],
        "ms_per_step_slowest": round(slow["ms_per_step"], 4),
        "gcell_updates_per_s_slowest": round(slow["cells"] / slow["ms_per_step"] / 1e6, 3),
        "frac_effective_slowest": round(achieved / HBM_PEAK_GBS, 4),
        "avg_launch_ms_slowest": round(slow["launch_s"] * 1e3, 4),
    }


def run_realistic(F, torch, which="realistic"):
    """The realistic board (444x364x60 cells, 16 probes) as one plain solve: its
    full 20000 steps and the 16 probe spectra, one board at a time; with
    which="small", the small board (80x72x37, 3000 steps, 4 probes) likewise."""
    import numpy as np
    import boardgen
    from paper_1008_2602_amd import tune
    b = boardgen.realistic_board() if which == "realistic" else boardgen.small_board()
    tile = tune.tune_board(b)
    g, ids = F.grid_from_board(b, max_steps=b.steps, tile=tile)
    F.fdtd_step_n(g, 0)                  # set-up (tables, work lists) outside the timing
    F.fdtd_synchronize(g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fdtd_step_n(g, b.steps)
    n_fft = 1
    while n_fft < b.steps:
        n_fft *= 2
    spec = [F.fdtd_probe_fft(g, p, n_fft) for p in ids]
    wall = time.perf_counter() - t0
    F.fdtd_destroy_grid(g)
    assert all(np.all(np.isfinite(x)) for x in spec)
    return {
        "workload": f"{which} board {b.nx}x{b.ny}x{b.nz} cells, "
                    f"{b.steps} steps, {len(ids)} probe spectra, one plain solve",
        "tile": "x".join(str(v) for v in tile),
        "wall_s": round(wall, 3),
        "gcell_updates_per_s": round(b.cells * b.steps / wall / 1e9, 3),
    }, b


def run_batch(F, torch, K, W):
    """The 64-board variant batch, all boards advanced by K steps together."""
    import boardgen
    from paper_1008_2602_amd import tune
    boards = boardgen.variant_batch(steps=W + K)
    tile = tune.tune_batch(boards)
    handles = [F.grid_from_board(b, max_steps=W + K) for b in boards]
    gs = [h for h, _ in handles]
    F.fdtd_set_tile(gs[0], *tile)
    F.fdtd_step_many(gs, [W] * len(gs))
    F.fdtd_synchronize(gs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fdtd_step_many(gs, [K] * len(gs))
    F.fdtd_synchronize(gs[0])
    wall = time.perf_counter() - t0
    infos = [F.fdtd_get_info(g) for g in gs]
    step_bytes = sum(sec8d_step_bytes(i) for i in infos)
    fused_bytes = sum(i.step_bytes for i in infos)
    for g in gs:
        F.fdtd_destroy_grid(g)
    cells = sum(b.cells for b in boards)
    return {
        "workload": f"{len(boards)} board variants (in-plane 100-600 cells, z 24-64, eps_r "
                    f"3.5-4.8, 8-cell PML), {cells} cells in all, one launch per "
                    f"{tile[2] if len(tile) > 2 else 1} step(s) over every board",
        "value": round(cells * K / wall / 1e9, 3),
        "unit": "Gcell-updates/s",
        "steps": K,
        "ms_per_step": round(wall / K * 1e3, 4),
        "tile": "x".join(str(v) for v in tile),
        # on the algorithmic bytes (sec8d_step_bytes); effective (two steps per pass)
        "frac_effective": round(step_bytes * K / wall / 1e9 / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_step": int(step_bytes),
        "frac_on_fused_bytes": round(fused_bytes * K / wall / 1e9 / HBM_PEAK_GBS, 4),
    }, cells / len(boards)


def run_table1(F, torch, n_sweep=64, kernel_steps=200):
    """The paper's Table 1 run (40 x 30 x 0.8 mm board, 5 V / 10 ohm DGAUSS
    resistive corner source, opposite-corner ground-plane Ez probe and the plane
    voltage there, 30000 steps of 1 ps) as one solve, with its probe spectrum;
    then the source-resistance sweep the paper proposes (n_sweep copies, R from
    1 ohm to 1 kohm) advanced together by fdtd_step_many.  The board is small
    (62k cells), so one solve is bound by launch latency, not HBM; the kernel's
    own duration is timed apart over kernel_steps further steps."""
    import numpy as np
    import boardgen
    from paper_1008_2602_amd import tune
    b = boardgen.table1_board(steps=30000, source="resistive")
    N = b.steps
    lay = b.meta["layout"]
    pi, pj, _ = b.probes[0]
    tile = tune.tune_board(b)
    g, ids = F.grid_from_board(b, max_steps=N + kernel_steps, tile=tile)
    vid = F.fdtd_add_voltage_probe(g, pi, pj, lay["kg"], lay["kt"])
    F.fdtd_step_n(g, 0)                  # set-up (tables, work lists) outside the timing
    F.fdtd_synchronize(g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fdtd_step_n(g, N)
    n_fft = 1
    while n_fft < N:
        n_fft *= 2
    spec = F.fdtd_probe_fft(g, ids[0], n_fft)
    volt = F.fdtd_get_voltage(g, vid, N)
    wall = time.perf_counter() - t0
    assert np.all(np.isfinite(spec)) and np.all(np.isfinite(volt))
    F.fdtd_set_timing(g, True)
    F.fdtd_step_n(g, kernel_steps)
    kern_ms, launches = F.fdtd_get_timing(g)
    info = F.fdtd_get_info(g)
    F.fdtd_destroy_grid(g)
    per_launch_s = kern_ms / 1e3 / launches
    launch_bytes = sec8d_step_bytes(info) * kernel_steps / launches

    boards = []
    for r in np.geomspace(1.0, 1000.0, n_sweep):
        bb = boardgen.table1_board(steps=N, source="resistive")
        bb.sources[0].R = float(r)
        boards.append(bb)
    stile = tune.tune_batch(boards)
    gs = [F.grid_from_board(bb, max_steps=N)[0] for bb in boards]
    F.fdtd_set_tile(gs[0], *stile)
    for h in gs:
        F.fdtd_step_n(h, 0)
    F.fdtd_synchronize(gs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fdtd_step_many(gs, [N] * len(gs))
    F.fdtd_synchronize(gs[0])
    sweep_wall = time.perf_counter() - t0
    for h in gs:
        F.fdtd_destroy_grid(h)
    return {
        "workload": f"Table 1 run: {b.nx}x{b.ny}x{b.nz} cells (40x30x0.8 mm board, 2/2/0.4 mm "
                    f"cells, eps_r 4.0, 6 air + 8 PML cells), 5 V / 10 ohm DGAUSS resistive "
                    f"corner source, {N} steps of 1 ps, probe FFT ({n_fft} points) and plane "
                    f"voltage read back",
        "tile": "x".join(str(v) for v in tile),
        "wall_s": round(wall, 4),
        "ms_per_step": round(wall / N * 1e3, 5),
        "gcell_updates_per_s": round(b.cells * N / wall / 1e9, 3),
        "kernel_avg_launch_us": round(per_launch_s * 1e6, 2),
        "kernel_frac_effective": round(launch_bytes / per_launch_s / 1e9 / HBM_PEAK_GBS, 4),
        "r_sweep": {
            "boards": len(boards),
            "R_ohm": [1.0, 1000.0],
            "tile": "x".join(str(v) for v in stile),
            "wall_s": round(sweep_wall, 3),
            "gcell_updates_per_s": round(b.cells * N * len(boards) / sweep_wall / 1e9, 3),
        },
    }, b


def table1_cpu(board):
    """The oracle's whole run of a board small enough to run in full (the Table 1
    board, the small board)."""
    import oracle
    t0 = time.perf_counter()
    oracle.run(board, threads=None)
    dt = time.perf_counter() - t0
    return {"value": round(board.cells * board.steps / dt / 1e9, 4),
            "unit": "Gcell-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"the whole {board.steps}-step run ({dt:.1f} s; FP64)"}


def oracle_full_realistic(F, torch, chunk=1000):
    """The oracle's whole run of the realistic board (444x364x60 cells, 20000
    steps, 16 probes) on all host threads, in chunks that carry the state and the
    DFT accumulators over (progress on stderr), timed; then the GPU's plain solve
    of the same board, whose probe series are compared with it (largest relative
    L2 over the probes)."""
    import numpy as np
    import boardgen
    import oracle
    from paper_1008_2602_amd import tune
    b = boardgen.realistic_board()
    st, dft, series = oracle.new_state(b), None, []
    t0 = time.perf_counter()
    for s0 in range(0, b.steps, chunk):
        r = oracle.run(b, nsteps=min(chunk, b.steps - s0), state=st, dft=dft, threads=None)
        st, dft = r.state, r.dft
        series.append(r.probes)
        print(f"[oracle] {s0 + r.probes.shape[1]} of {b.steps} steps at "
              f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    cpu_s = time.perf_counter() - t0
    ref = np.concatenate(series, axis=1)
    g, ids = F.grid_from_board(b, max_steps=b.steps, tile=tune.tune_board(b))
    try:
        F.fdtd_step_n(g, b.steps)
        got = np.stack([F.fdtd_get_probe(g, p, b.steps) for p in ids]).astype(np.float64)
    finally:
        F.fdtd_destroy_grid(g)
    errs = [float(np.linalg.norm(got[p] - ref[p]) / np.linalg.norm(ref[p])) for p in range(len(ids))]
    return {"workload": f"realistic board {b.nx}x{b.ny}x{b.nz} cells, {b.steps} steps, "
                        f"{len(ids)} probes: the oracle's whole run",
            "value": round(b.cells * b.steps / cpu_s / 1e9, 4), "unit": "Gcell-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle", "wall_s": round(cpu_s, 1),
            "gpu_max_probe_rel_l2": float(f"{max(errs):.3g}")}


def sampled_cpu(board, budget_s=15.0):
    """The oracle on a bounded sample of a board's steps (all host threads), with
    the whole run's time extrapolated from it."""
    import oracle
    rate, n, dt = _oracle_rate(board, oracle.num_threads(), budget_s)
    return {"value": round(rate, 4), "unit": "Gcell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} of the {board.steps} steps ({dt:.1f} s; FP64); the whole run "
                      f"would take about {board.cells * board.steps / rate / 1e9:.0f} s "
                      f"(extrapolated)"}


def run_serve(F, torch, capacity_gcells, n_requests, steps):
    import numpy as np
    import boardgen
    from paper_1008_2602_amd.serve import GpuExecutor, Server, summarize
    # the request stream at unit rate (arrival times scale with 1/rate; the boards
    # do not depend on it), then the rate that offers 0.7x the measured batched
    # capacity for this stream's own mean board (the large boards included)
    reqs = boardgen.served_requests(1.0, n_requests=n_requests, steps=steps)
    mean_cells = float(np.mean([r.board.cells for r in reqs]))
    capacity = capacity_gcells * 1e9 / (mean_cells * steps)           # boards per second
    rate = 0.7 * capacity
    from paper_1008_2602_amd.serve import SolveRequest
    requests = [SolveRequest(r.rid, r.arrival_s / rate, r.board) for r in reqs]
    free, _total = torch.cuda.mem_get_info()
    budget = int(0.85 * free)

    class FftExecutor(GpuExecutor):
        def finish(self, handle, probe_ids, req):
            n_fft = 1
            while n_fft < req.n_steps:
                n_fft *= 2
            spectra = [self.F.fdtd_probe_fft(handle, p, n_fft) for p in probe_ids]
            assert all(np.all(np.isfinite(x)) for x in spectra)
            return super().finish(handle, probe_ids, req)

    # the batched shape tuned on the first 64 requests' boards (the mix the
    # chunks will hold), then used by every served handle
    from paper_1008_2602_amd import tune
    tile = tune.tune_batch([r.board for r in requests[:64]])
    ex = FftExecutor(allocator=F.TorchAllocator(), tile=tile)

    def progress(d):
        # progress on stderr (stdout carries only the JSON line)
        if d["chunk"] % 50 == 0:
            print(f"[served] chunk {d['chunk']} at {d['t']:.0f} s: {d['resident']} resident, "
                  f"{d['waiting']} waiting", file=sys.stderr, flush=True)

    srv = Server(ex, budget, chunk=500, workers=2, depth=2, log=progress)
    t0 = time.perf_counter()
    res = srv.run(requests)
    wall = time.perf_counter() - t0
    s = summarize(res, wall_s=wall)
    busy = ex.busy_fraction()
    ex.close()
    large = {r.rid for r in requests if (r.board.nx, r.board.ny) == (800, 800)}
    lat_large = np.array([r.latency_s for r in res if r.rid in large])
    lat_var = np.array([r.latency_s for r in res if r.rid not in large])
    wait = np.array([r.wait_s for r in res])
    out = {
        "workload": f"{n_requests} seeded Poisson arrivals at {rate:.3f}/s (0.7x the measured "
                    f"batched capacity for the stream's mean board of {mean_cells / 1e6:.2f} M "
                    f"cells) of board variants, 5% 800x800x64, {steps} steps each, "
                    f"500-step chunks (up to two in flight, set-up and read-back on two "
                    f"worker threads), probe FFT per solve",
        "p50_latency_s": round(s["p50_latency_s"], 4),
        "p99_latency_s": round(s["p99_latency_s"], 4),
        "solves_per_s": round(s["solves_per_s"], 4),
        "gcell_updates_per_s": round(s["gcell_updates_per_s"], 3),
        "requests": n_requests,
        "large_boards": len(large),
        "latency_samples": s["completed"],
        "completed": s["completed"],
        "gpu_busy_frac": round(busy, 4) if busy is not None else None,
        # the two kinds of solve apart (arrival to result), and the wait for
        # admission (arrival to the first chunk that holds the solve)
        "variant_p50_p99_latency_s": [round(float(np.percentile(lat_var, q)), 4) for q in (50, 99)]
                                     if lat_var.size else None,
        "large_p50_max_latency_s": [round(float(np.percentile(lat_large, 50)), 4),
                                    round(float(lat_large.max()), 4)] if lat_large.size else None,
        "wait_p50_p99_s": [round(float(np.percentile(wait, q)), 4) for q in (50, 99)],
        "chunks": srv.chunks,
        "tile": "x".join(str(v) for v in tile),
        "peak_resident": srv.peak_resident,
        "budget_gb": round(budget / 1e9, 1),
    }
    return out, res, requests


def served_oracle_check(results, requests):
    """The CPU leg beside the served numbers: the oracle re-runs the smallest
    served solve, and the served probe series are compared with it (largest
    relative L2 over the solve's probes)."""
    import numpy as np
    import oracle
    by_rid = {r.rid: r for r in requests}
    pick = min(results, key=lambda r: r.cells)
    req = by_rid[pick.rid]
    t0 = time.perf_counter()
    ref = oracle.run(req.board, nsteps=req.n_steps, threads=None)
    cpu_s = time.perf_counter() - t0
    errs = [float(np.linalg.norm(pick.probes[p].astype(np.float64) - ref.probes[p])
                  / np.linalg.norm(ref.probes[p])) for p in range(len(ref.probes))]
    return {"rid": pick.rid, "cells": pick.cells, "steps": req.n_steps,
            "max_probe_rel_l2": float(f"{max(errs):.3g}"), "oracle_s": round(cpu_s, 2),
            "cores": oracle.num_threads()}


def main():
    import faulthandler
    faulthandler.enable()            # a native crash prints every thread's Python stack
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--tile", default="",
                    help="field-kernel shape tile_x x tile_y x steps per pass, e.g. 64x15x1 or "
                         "64x10x2 (default: autotuned)")
    ap.add_argument("--only", choices=["single", "batch", "serve", "table1", "plane", "zconv",
                                       "eps", "eps_large", "eps_rw", "lossy_copper", "shard",
                                       "realistic"], default=None)
    ap.add_argument("--batch-steps", type=int, default=50)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-steps", type=int, default=8000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--oracle-full", action="store_true",
                    help="time the oracle's whole realistic-board run (several minutes) "
                         "and compare the GPU's probes with it; prints that alone")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X: the library has no multi-GPU path "
              "(boards shard whole across GPUs by design).", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return

    from paper_1008_2602_amd import fdtd as F
    if args.oracle_full:
        print(json.dumps({"oracle_full_run": oracle_full_realistic(F, torch)}), flush=True)
        return

    K, W = int(args.steps), int(args.warmup)
    tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else None
    out = {}
    clock = [time.perf_counter()]

    def section(name):
        # progress and the time of each part on stderr (stdout carries only the JSON line)
        now = time.perf_counter()
        print(f"[bench] {name}: {now - clock[0]:.1f} s", file=sys.stderr, flush=True)
        clock[0] = now
    if args.only in (None, "single"):
        board, tile, info, wall, kern_ms, launches = run_single(F, torch, K, W, tile)
        cells = board.cells
        per_launch_s = kern_ms / 1e3 / launches
        steps_per_launch = K / launches          # 2 for a two-step shape (K even)
        traffic = measured_traffic()
        sec8d_step = sec8d_step_bytes(info)
        launch_bytes = sec8d_step * steps_per_launch
        achieved = launch_bytes / per_launch_s / 1e9
        fused_launch_bytes = info.step_bytes * steps_per_launch
        out.update({
            "metric": "Gcell-updates/s + % HBM roofline (1 GPU); served solves p50/p99 latency",
            "value": round(cells * K / wall / 1e9, 3),
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
                "tile": "x".join(str(v) for v in tile),
                "dt_s": info.dt,
            },
            "roofline": {
                "bound": "hbm",
                # algorithmic bytes: the per cell-update count of two separate passes
                # in the layout used (D/B kept only where a PML loss acts): 72 B of E and H
                # for separate H and E passes, the class byte(s), 8 B per kept D/B
                # component, times the steps one launch advances
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS,
                "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                # above 1 is possible: the kernel keeps step n+1 on chip, so it moves
                # fewer bytes than two separate steps of that count
                "frac_kind": "effective (temporally blocked: two steps per pass)",
                "traffic": traffic,
                # HBM bytes actually moved (PMC) over the launch time, against the peak
                "measured_hbm_gbs": (round(traffic / per_launch_s / 1e9, 1)
                                     if traffic is not None else None),
                "hbm_frac_measured": (round(traffic / per_launch_s / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic is not None else None),
                "kernel": "field_step2" if info.tile_steps == 2 else "field_step",
                "steps_per_launch": steps_per_launch,
                "bytes_per_cell_update": round(sec8d_step / cells, 2),
                "algorithmic_bytes_per_launch": int(launch_bytes),
                "avg_launch_ms": round(per_launch_s * 1e3, 4),
                # the library's own count (one fused pass per step: E and H read and
                # written once, class, kept D/B), and the fraction on it
                "fused_bytes_per_cell_update": round(info.step_bytes / cells, 2),
                "frac_on_fused_bytes": round(fused_launch_bytes / per_launch_s / 1e9 / HBM_PEAK_GBS, 4),
            },
        })
        section("single")
    def guarded(key, fn):
        # a secondary part that fails leaves its error in the line (traceback on
        # stderr) instead of ending the run without one
        try:
            fn()
        except Exception as e:                     # noqa: BLE001 (reported, not hidden)
            import traceback
            traceback.print_exc(file=sys.stderr)
            part = out.get(key)
            if not isinstance(part, dict):
                part = out[key] = {}
            part["error"] = f"{type(e).__name__}: {e}"
        section(key)

    if args.only in (None, "batch", "serve"):
        def batched():
            out["batched"], _ = run_batch(F, torch, args.batch_steps, 5)
        guarded("batched", batched)
        if args.only == "serve":
            batch = out.pop("batched", {})
        else:
            batch = out.get("batched", {})
        if args.only in (None, "serve") and "value" in batch:
            def served():
                out["served"], served_res, served_req = run_serve(F, torch, batch["value"],
                                                                  args.serve_requests,
                                                                  args.serve_steps)
                if not args.no_cpu_baseline:
                    out["served"]["oracle_check"] = served_oracle_check(served_res, served_req)
            guarded("served", served)
    if args.only in (None, "plane"):
        def plane():
            plain = out.get("ms_per_step")
            if plain is None:
                _, _, _, wall0, _, _ = run_single(F, torch, K, W, tile)
                plain = wall0 / K * 1e3
            out["plane_dft"] = run_plane_dft(F, torch, K, W, plain)
        guarded("plane_dft", plane)
    if args.only in (None, "eps", "eps_large", "eps_rw", "lossy_copper"):
        def material():
            out["node_passes"] = run_eps(F, torch, large_only=args.only == "eps_large",
                                         only=args.only if args.only in ("eps_rw", "lossy_copper")
                                         else None)
        guarded("node_passes", material)
    if args.only in (None, "zconv"):
        def zconv():
            out["zconv"] = run_zconv(F, torch)
        guarded("zconv", zconv)
    if args.only in (None, "shard"):
        def shard():
            out["shard"] = run_shard(F, torch)
        guarded("shard", shard)
    if args.only in (None, "realistic"):
        def realistic():
            out["realistic"], real_board = run_realistic(F, torch)
            if not args.no_cpu_baseline:
                out["realistic"]["cpu_baseline"] = sampled_cpu(real_board)
        guarded("realistic", realistic)

        def small():
            out["small"], small_board = run_realistic(F, torch, "small")
            if not args.no_cpu_baseline:
                out["small"]["cpu_baseline"] = table1_cpu(small_board)
        guarded("small", small)
    if args.only in (None, "table1"):
        def table1():
            out["table1"], t1_board = run_table1(F, torch)
            if not args.no_cpu_baseline:
                out["table1"]["cpu_baseline"] = table1_cpu(t1_board)
        guarded("table1", table1)
    if args.only in (None, "single") and not args.no_cpu_baseline:
        def cpu():
            import boardgen
            out["cpu_baseline"] = cpu_baseline(boardgen.large_board())
        guarded("cpu_baseline", cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
