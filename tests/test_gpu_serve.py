"""Served and tuned solves on the GPU: every result equals the same board run
alone (bitwise) and the FP64 oracle (probe relative L2 <= 1e-4)."""
import sys

import numpy as np
import pytest

import boardgen
from _util import rel_l2

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def _boards(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        b = boardgen.variant_board(rng, i, steps=int(rng.integers(500, 900)),
                                   n_xy=(int(rng.integers(40, 110)), int(rng.integers(40, 110))),
                                   nz=int(rng.integers(24, 36)))
        for s in b.sources:
            s.t0, s.sigma = 40e-12, 10e-12
        out.append(b)
    return out


def test_served_results_equal_alone_and_oracle(F, oracle_mod):
    from paper_1008_2602_amd.serve import GpuExecutor, Server, SolveRequest, summarize
    boards = _boards(21, 6)
    reqs = [SolveRequest(i, 0.002 * i, b) for i, b in enumerate(boards)]
    alloc = F.TorchAllocator()
    ex = GpuExecutor(allocator=alloc)
    budget = sum(F.board_bytes(b) for b in boards[:3])     # at most ~3 resident at once
    announce(f"serving {len(reqs)} boards, budget {budget/1e6:.0f} MB, chunk 37")
    srv = Server(ex, budget, chunk=37)
    res = srv.run(reqs)
    assert [r.rid for r in res] == list(range(len(boards)))
    assert srv.peak_bytes <= budget and srv.peak_resident >= 2
    assert alloc.live_bytes == 0
    s = summarize(res)
    assert s["completed"] == len(boards) and s["p99_latency_s"] >= s["p50_latency_s"]
    for r, b in zip(res, boards):
        g, ids = F.grid_from_board(b)
        F.fdtd_step_n(g, b.steps)
        alone = np.stack([F.fdtd_get_probe(g, p, b.steps) for p in ids])
        F.fdtd_destroy_grid(g)
        assert np.array_equal(r.probes, alone), b.name
        ref = oracle_mod.run(b, threads=16).probes
        top = max(np.linalg.norm(ref[p]) for p in range(len(ids)))
        for p in range(len(ids)):
            e = rel_l2(r.probes[p], ref[p])
            print(f"{b.name} probe {p}: norm/top {np.linalg.norm(ref[p]) / top:.3e} rel_l2 {e:.3e}")
            assert e <= 1e-4, (b.name, p)


def test_autotuned_tile_keeps_results(F, tmp_path):
    from paper_1008_2602_amd import tune
    b = boardgen.small_board(steps=64)
    path = str(tmp_path / "tiles.json")
    shape = tune.tune_board(b, path=path)
    assert shape in F.fdtd_tile_shapes()
    assert tune.tune_board(b, path=path) == shape          # cached
    out = []
    for tile in (shape, (64, 8, 1)):
        g, ids = F.grid_from_board(b, tile=tile)
        F.fdtd_step_n(g, b.steps)
        out.append(F.fdtd_get_probe(g, ids[0], b.steps))
        F.fdtd_destroy_grid(g)
    assert np.array_equal(out[0], out[1])
    batch = _boards(5, 3)
    bshape = tune.tune_batch(batch, path=path)
    assert bshape in F.fdtd_tile_shapes()
