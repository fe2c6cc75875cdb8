"""The batched and served workloads at their full sizes, through the C-ABI.

* The 64-board variant batch (the benchmark's batched workload, 293.7 M cells in
  the benchmark's tile): every board advanced 5 to 7 steps from an arbitrary E
  and H by one fdtd_step_many call, bitwise equal (the whole state image: all 12
  arrays and the probe series) to the same board stepped alone; the smallest
  board also against the FP64 oracle.
* A served mix holding one 800 x 800 x 64 board (the large boards of the served
  workload) beside three variant boards, in 100-step chunks (the large board's
  run without the variants, as the benchmark serves): each result (probe series
  and the final Ez and Hx arrays) bitwise equal to the board run alone, and the
  large board's probes within 1e-4 of the oracle.
"""
import numpy as np
import pytest

import boardgen
from _compare import FIELDS, compare_fields
from _util import rel_l2
from test_gpu_parity import announce

pytestmark = pytest.mark.gpu

_C0 = 299792458.0
_MU0 = 4e-7 * np.pi
_ETA0 = _MU0 * _C0


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def _pool(seed=7, n=1 << 24):
    """A pool of uniform values in [-0.5, 0.5) that arbitrary states are cut
    from (E in V/m, and the same scaled by 1/eta0 for H, so that both are O(1)
    in the library's units)."""
    rng = np.random.default_rng(seed)
    e = rng.random(n, dtype=np.float32) - np.float32(0.5)
    return e, (e.astype(np.float64) / _ETA0).astype(np.float32)


def set_arbitrary_eh(F, g, board, q, pool):
    """Arbitrary E and H (D and B start at zero): each array a run of the pool
    from an offset of its own.  The library keeps only the entries the state
    holds (it stores zero elsewhere), so no masks are needed."""
    shp = (board.nz + 1, board.ny + 1, board.nx + 1)
    size = int(np.prod(shp))
    for c in range(6):
        src = pool[0] if c < 3 else pool[1]
        start = (7919 * (6 * q + c)) % (src.size - 1)
        out = np.empty(size, np.float32)
        pos = 0
        while pos < size:                 # the pool from `start` on, wrapped around
            n = min(size - pos, src.size - start)
            out[pos:pos + n] = src[start:start + n]
            pos += n
            start = 0
        F.fdtd_set_field(g, c, out.reshape(shp))


@pytest.mark.timeout(900)
def test_variant_batch_full_size_bitwise_and_oracle(F, oracle_mod):
    from paper_1008_2602_amd import tune
    boards = boardgen.variant_batch(steps=16)
    tile = tune.tune_batch(boards)
    ns = [5 + (q % 3) for q in range(len(boards))]        # uneven; odd counts end on one single step
    cells = sum(b.cells for b in boards)
    pool = _pool()
    announce(f"variant batch: {len(boards)} boards, {cells} cells, tile {tile}, steps 5-7: alone")
    alone = []
    for q, (b, n) in enumerate(zip(boards, ns)):
        if q % 8 == 0:
            announce(f"alone {q}: {b.name}")
        g, _ = F.grid_from_board(b, max_steps=b.steps, tile=tile)
        try:
            set_arbitrary_eh(F, g, b, q, pool)
            F.fdtd_step_n(g, n)
            alone.append(F.fdtd_save_state(g))      # all 12 arrays and the probe series
        finally:
            F.fdtd_destroy_grid(g)
    announce("variant batch: batched")
    hs = []
    try:
        for q, b in enumerate(boards):
            if q % 8 == 0:
                announce(f"batched: set-up of board {q}")
            hs.append(F.grid_from_board(b, max_steps=b.steps, tile=tile))
            set_arbitrary_eh(F, hs[-1][0], b, q, pool)
        F.fdtd_step_many([g for g, _ in hs], ns)
        F.fdtd_synchronize(hs[0][0])
        assert F.fdtd_get_info(hs[0][0]).tile_steps == tile[2]
        for q, ((g, _), b) in enumerate(zip(hs, boards)):
            assert F.fdtd_save_state(g) == alone[q], b.name
        alone = None
        # the smallest board against the oracle, from the same state
        q = min(range(len(boards)), key=lambda t: boards[t].cells)
        b, (g, _) = boards[q], hs[q]
        announce(f"variant batch: {b.name} against the oracle")
        shp = (b.nz + 1, b.ny + 1, b.nx + 1)
        g0, _ = F.grid_from_board(b, max_steps=b.steps)
        try:
            set_arbitrary_eh(F, g0, b, q, pool)      # the state as the library keeps it
            init = {name: F.fdtd_get_field(g0, c, shp) for c, name in enumerate(FIELDS)}
        finally:
            F.fdtd_destroy_grid(g0)
        ref_state = oracle_mod.new_state(b)
        for name in FIELDS:
            ref_state[name][...] = init[name]
        ref = oracle_mod.run(b, nsteps=ns[q], state=ref_state, threads=16)
        got = {name: F.fdtd_get_field(g, c, shp).astype(np.float64) for c, name in enumerate(FIELDS)}
        compare_fields(ref.state, got, b, 2e-5, elem_tol=1e-5)
    finally:
        for g, _ in hs:
            F.fdtd_destroy_grid(g)


def _served_mix(steps):
    rng = np.random.default_rng(77)
    boards = [boardgen.variant_board(rng, 0, steps, n_xy=(800, 800), nz=64)]
    boards += [boardgen.variant_board(rng, q, steps) for q in (1, 2, 3)]
    for b in boards:
        lay = b.meta["layout"]
        s = b.sources[0]
        s.t0, s.sigma = 40e-12, 10e-12
        # probes near the source, so that the pulse reaches them in the run
        b.probes = [(s.i + di, s.j + dj, lay["kg"]) for di, dj in ((6, 0), (0, -9), (-12, 5), (3, 14))]
    return boards


@pytest.mark.timeout(900)
def test_served_mix_with_large_board_equals_alone(F, oracle_mod):
    from paper_1008_2602_amd.serve import GpuExecutor, Server, SolveRequest

    steps = 300
    boards = _served_mix(steps)
    assert (boards[0].nx, boards[0].ny, boards[0].nz) == (800, 800, 64)

    class Keep(GpuExecutor):
        """Keeps the final Ez and Hx of every solve beside its probe series."""
        kept = {}

        def finish(self, handle, probe_ids, req):
            b = req.board
            shp = (b.nz + 1, b.ny + 1, b.nx + 1)
            self.kept[req.rid] = (self.F.fdtd_get_field(handle, self.F.FDTD_EZ, shp),
                                  self.F.fdtd_get_field(handle, self.F.FDTD_HX, shp))
            return super().finish(handle, probe_ids, req)

    reqs = [SolveRequest(q, 0.0005 * q, b) for q, b in enumerate(boards)]
    budget = sum(F.board_bytes(b, max_steps=steps) for b in boards)
    announce(f"served mix: {[f'{b.nx}x{b.ny}x{b.nz}' for b in boards]}, chunk 100")
    ex = Keep(allocator=F.TorchAllocator())
    srv = Server(ex, budget, chunk=100, solo_cells=30_000_000)   # as the benchmark serves
    res = srv.run(reqs)
    assert [r.rid for r in res] == list(range(len(boards)))
    assert srv.peak_resident >= 2
    for r, b in zip(res, boards):
        announce(f"served mix: {b.name} alone")
        g, ids = F.grid_from_board(b, max_steps=steps)
        try:
            F.fdtd_step_n(g, steps)
            alone = np.stack([F.fdtd_get_probe(g, p, steps) for p in ids])
            shp = (b.nz + 1, b.ny + 1, b.nx + 1)
            ez, hx = F.fdtd_get_field(g, F.FDTD_EZ, shp), F.fdtd_get_field(g, F.FDTD_HX, shp)
        finally:
            F.fdtd_destroy_grid(g)
        assert np.abs(alone).max() > 0, b.name
        assert np.array_equal(r.probes, alone), b.name
        assert np.array_equal(ex.kept[r.rid][0], ez), b.name
        assert np.array_equal(ex.kept[r.rid][1], hx), b.name
    announce("served mix: the 800x800x64 board on the oracle")
    ref = oracle_mod.run(boards[0], threads=16).probes
    for p in range(len(boards[0].probes)):
        e = rel_l2(res[0].probes[p], ref[p])
        print(f"large board probe {p}: rel_l2 {e:.3e}")
        assert e <= 1e-4, (p, e)
