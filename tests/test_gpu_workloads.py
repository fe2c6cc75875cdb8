"""The batched and served workloads at their full sizes, through the C-ABI.

* The 64-board variant batch (the benchmark's batched workload, 293.7 M cells in
  the benchmark's tile): every board advanced a few steps from an arbitrary
  state by one fdtd_step_many call, bitwise equal (all 12 arrays and the probe
  series) to the same board stepped alone; the smallest board also against the
  FP64 oracle.
* A served mix holding one 800 x 800 x 64 board (the large boards of the served
  workload) beside three variant boards, in 100-step chunks: each result (probe
  series and the final Ez and Hx arrays) bitwise equal to the board run alone,
  and the large board's probes within 1e-4 of the oracle.
"""
import hashlib

import numpy as np
import pytest

import boardgen
from _compare import FIELDS, aux_masks, compare_fields
from _util import live_masks, rel_l2
from test_gpu_parity import announce

pytestmark = pytest.mark.gpu

_C0 = 299792458.0
_MU0 = 4e-7 * np.pi
_EPS0 = 1.0 / (_MU0 * _C0 * _C0)
_ETA0 = _MU0 * _C0
_SI = {"e": 1.0, "h": 1.0 / _ETA0, "d": _EPS0, "b": 1.0 / _C0}


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def state32(board, seed):
    """An arbitrary state in SI units (FP32): uniform values of O(1) in the
    library's scaled units on every entry the state holds (live E and H, D/B
    where a PML loss keeps them), zero elsewhere."""
    rng = np.random.default_rng(seed)
    m, am = live_masks(board), aux_masks(board)
    shp = (board.nz + 1, board.ny + 1, board.nx + 1)
    out = {}
    for n in FIELDS:
        v = rng.random(shp, dtype=np.float32)
        v -= np.float32(0.5)
        v *= m[n] & am[n[-1]] if n[0] in "db" else m[n]
        out[n] = (v.astype(np.float64) * _SI[n[0]]).astype(np.float32)
    return out


def digests(F, g, board, ids, steps):
    shp = (board.nz + 1, board.ny + 1, board.nx + 1)
    out = [hashlib.sha256(F.fdtd_get_field(g, c, shp).tobytes()).hexdigest()
           for c in range(len(FIELDS))]
    if ids:
        out.append(hashlib.sha256(np.stack([F.fdtd_get_probe(g, p, steps) for p in ids])
                                  .tobytes()).hexdigest())
    return out


@pytest.mark.timeout(900)
def test_variant_batch_full_size_bitwise_and_oracle(F, oracle_mod):
    from paper_1008_2602_amd import tune
    boards = boardgen.variant_batch(steps=16)
    tile = tune.tune_batch(boards)
    ns = [5 + (q % 3) for q in range(len(boards))]        # uneven; odd counts end on one single step
    cells = sum(b.cells for b in boards)
    announce(f"variant batch: {len(boards)} boards, {cells} cells, tile {tile}, steps 5-7: alone")
    alone = []
    for q, (b, n) in enumerate(zip(boards, ns)):
        st = state32(b, 100 + q)
        g, ids = F.grid_from_board(b, max_steps=b.steps, tile=tile)
        try:
            for c, name in enumerate(FIELDS):
                F.fdtd_set_field(g, c, st[name])
            F.fdtd_step_n(g, n)
            alone.append(digests(F, g, b, ids, n))
        finally:
            F.fdtd_destroy_grid(g)
    announce("variant batch: batched")
    hs = []
    try:
        for q, b in enumerate(boards):
            hs.append(F.grid_from_board(b, max_steps=b.steps, tile=tile))
            st = state32(b, 100 + q)
            for c, name in enumerate(FIELDS):
                F.fdtd_set_field(hs[-1][0], c, st[name])
        F.fdtd_step_many([g for g, _ in hs], ns)
        F.fdtd_synchronize(hs[0][0])
        assert F.fdtd_get_info(hs[0][0]).tile_steps == tile[2]
        for q, ((g, ids), b, n) in enumerate(zip(hs, boards, ns)):
            assert digests(F, g, b, ids, n) == alone[q], b.name
        # the smallest board against the oracle, from the same state
        q = min(range(len(boards)), key=lambda t: boards[t].cells)
        b, (g, _) = boards[q], hs[q]
        announce(f"variant batch: {b.name} against the oracle")
        st = state32(b, 100 + q)
        ref_state = oracle_mod.new_state(b)
        for name in FIELDS:
            ref_state[name][...] = st[name]
        ref = oracle_mod.run(b, nsteps=ns[q], state=ref_state, threads=16)
        shp = (b.nz + 1, b.ny + 1, b.nx + 1)
        got = {name: F.fdtd_get_field(g, c, shp).astype(np.float64) for c, name in enumerate(FIELDS)}
        compare_fields(ref.state, got, b, 2e-5)
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
    srv = Server(ex, budget, chunk=100)
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
