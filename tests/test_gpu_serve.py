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


def _material(b, kind):
    """A variant board in the node passes' arithmetic: "lossy" a lossy dielectric
    (tan d 0.02) between copper planes; "eps_rw" its dielectric run through the
    x/y PML to the outer wall, with Eq. 2's eps_rw."""
    if kind == "lossy":
        return boardgen.conductor_loss(boardgen.lossy_dielectric(b, 0.02))
    ks = np.nonzero((b.eps_r_cell > 1.0).any(axis=(1, 2)))[0]
    b.eps_r_cell[ks.min():ks.max() + 1] = b.eps_r_cell.max()
    b.pml_eps_rw = True
    return b


def test_served_material_and_plain_boards_equal_alone(F):
    """The pipelined loop (two workers, two chunks in flight) serving plain and
    material boards together in odd-sized chunks: every probe series bitwise
    equal to the board run alone, and every material board on the two-step
    kernels."""
    from paper_1008_2602_amd.serve import GpuExecutor, Server, SolveRequest
    boards = _boards(33, 6)
    boards[1] = _material(boards[1], "lossy")
    boards[2] = _material(boards[2], "eps_rw")
    boards[4] = _material(boards[4], "lossy")
    reqs = [SolveRequest(i, 0.001 * i, b) for i, b in enumerate(boards)]
    ex = GpuExecutor(allocator=F.TorchAllocator())
    budget = sum(F.board_bytes(b) for b in boards)
    announce(f"serving {len(reqs)} boards (3 material), chunk 37, pipelined")
    srv = Server(ex, budget, chunk=37, workers=2, depth=2)
    try:
        res = srv.run(reqs)
    finally:
        ex.close()
    assert [r.rid for r in res] == list(range(len(boards)))
    assert srv.peak_resident >= 2
    for r, b in zip(res, boards):
        g, ids = F.grid_from_board(b)
        try:
            info = F.fdtd_get_info(g)
            F.fdtd_step_n(g, b.steps)
            F.fdtd_synchronize(g)
            info = F.fdtd_get_info(g)
            alone = np.stack([F.fdtd_get_probe(g, p, b.steps) for p in ids])
        finally:
            F.fdtd_destroy_grid(g)
        assert info.material_two_step == (1 if b.pml_eps_rw or b.sigma_cell is not None else 0), b.name
        assert np.abs(alone).max() > 0, b.name
        assert np.array_equal(r.probes, alone), b.name
