"""Tile-shape autotuner for the field kernel.

The field kernel's results do not depend on its tile shape (bitwise), only its
speed does.  A shape is (tile_x, tile_y, steps per pass); timings are per step.  ``tune_board`` / ``tune_batch`` time every supported shape on
scratch handles with the same geometry and materials (zero fields, no sources),
keep the fastest, and cache the choice in a JSON file keyed by the geometry, so
the live solve never runs a timing step.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

Shape = Tuple[int, ...]   # (tile_x, tile_y, steps per pass)


def cache_path() -> str:
    """FDTD_TUNE_CACHE, else the package's tile_cache.json (shipped with the
    choices measured on MI355X for the standard workloads)."""
    p = os.environ.get("FDTD_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_cache.json")


def _load(path: str) -> Dict[str, list]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: Dict[str, list]) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def board_key(board) -> str:
    """Grid size and PML; a plane DFT selects other kernel variants, so it is part
    of the key."""
    key = f"{board.nx}x{board.ny}x{board.nz}/pml{'-'.join(str(v) for v in board.npml)}"
    if getattr(board, "plane_dft", None) is not None:
        key += "/plane"
    return key


def batch_key(boards: Sequence) -> str:
    return "batch:" + ";".join(sorted(board_key(b) for b in boards))


def cached(key: str, shapes: Sequence[Shape], path: Optional[str] = None) -> Optional[Shape]:
    """The cached choice for ``key`` if it is one of ``shapes``, else None."""
    data = _load(path or cache_path())
    if key not in data:
        return None
    best = tuple(data[key][0])
    return best if best in {tuple(s) for s in shapes} else None


def pick(timings: Dict[Shape, float]) -> Shape:
    """Fastest shape; ties go to the first listed (the default ordering)."""
    best = None
    for shape, t in timings.items():
        if best is None or t < timings[best]:
            best = shape
    return best


def tune(key: str, time_shape: Callable[[Shape], float], shapes: Iterable[Shape],
         path: Optional[str] = None, refresh: bool = False) -> Tuple[Shape, Dict[Shape, float]]:
    """Return the cached shape for ``key`` or time every shape and cache the best.
    A cached shape that is no longer among ``shapes`` is timed again."""
    path = path or cache_path()
    shapes = [tuple(s) for s in shapes]
    hit = cached(key, shapes, path)
    if hit is not None and not refresh:
        return hit, {}
    data = _load(path)
    timings = {s: float(time_shape(s)) for s in shapes}
    best = pick(timings)
    data[key] = [list(best), {"x".join(str(v) for v in s): t for s, t in timings.items()}]
    _store(path, data)
    return best, timings


# ---------------------------------------------------------------------------
# GPU timing through the C-ABI

def _scratch(F, board, steps):
    import dataclasses
    b = dataclasses.replace(board, sources=[], probes=[], dft_freqs=None)
    g, _ = F.grid_from_board(b, max_steps=steps)
    return g


def tune_board(board, steps: int = 6, warm: int = 2, path: Optional[str] = None,
               refresh: bool = False) -> Shape:
    from . import fdtd as F
    shapes = F.fdtd_tile_shapes()
    total = len(shapes) * (steps + warm) + 1

    def run() -> Shape:
        g = _scratch(F, board, total)
        try:
            def time_shape(shape):
                F.fdtd_set_tile(g, *shape)
                F.fdtd_step_n(g, warm)
                F.fdtd_set_timing(g, True)
                F.fdtd_get_timing(g)          # clears
                F.fdtd_step_n(g, steps)
                ms, _ = F.fdtd_get_timing(g)
                F.fdtd_set_timing(g, False)
                return ms / steps        # per step: a two-step shape makes half the launches
            best, _ = tune(board_key(board), time_shape, shapes, path, refresh)
            return best
        finally:
            F.fdtd_destroy_grid(g)

    hit = cached(board_key(board), shapes, path)
    if hit is not None and not refresh:
        return hit
    return run()


def tune_batch(boards: Sequence, steps: int = 4, warm: int = 1, path: Optional[str] = None,
               refresh: bool = False) -> Shape:
    from . import fdtd as F
    key = batch_key(boards)
    shapes = F.fdtd_tile_shapes()
    hit = cached(key, shapes, path)
    if hit is not None and not refresh:
        return hit
    total = len(shapes) * (steps + warm) + 1
    gs = [_scratch(F, b, total) for b in boards]
    try:
        def time_shape(shape):
            F.fdtd_set_tile(gs[0], *shape)
            F.fdtd_step_many(gs, [warm] * len(gs))
            F.fdtd_synchronize(gs[0])
            t0 = time.perf_counter()
            F.fdtd_step_many(gs, [steps] * len(gs))
            F.fdtd_synchronize(gs[0])
            return (time.perf_counter() - t0) * 1e3 / steps
        best, _ = tune(key, time_shape, shapes, path, refresh)
        return best
    finally:
        for g in gs:
            F.fdtd_destroy_grid(g)
