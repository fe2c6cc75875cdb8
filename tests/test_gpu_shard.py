"""The field kernel at one rank's share of a slab decomposition of the large
board along y (1048x99x88 cells per slab, halo stubbed: the cut faces carry no
PML and act as PEC walls), on the HIP path.

* Against the FP64 oracle from an arbitrary state, in the benchmark's tile:
  whole-array relative L2 <= 2e-5 (FP32 arithmetic over three steps), as for
  the whole large board.
* Against the whole large board on the GPU: away from its cut faces a slab
  evolves bitwise like the same rows of the whole board (fields and the probe
  series), which is the locality a decomposition with exchanged halos relies on.
"""
import numpy as np
import pytest

import boardgen
from _util import live_masks
from test_gpu_parity import (FIELDS, announce, aux_masks, compare_fields, gpu_run,
                             random_state)

pytestmark = pytest.mark.gpu

STEPS = 3


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def _tile(board):
    from paper_1008_2602_amd import tune
    return tune.tune_board(board)


@pytest.mark.parametrize("rank", [0, 1, 7])
def test_shard_random_state_vs_oracle(F, oracle_mod, rank):
    b = boardgen.large_board_shard(rank, steps=STEPS)
    b.dft_freqs = None
    tile = _tile(b)
    announce(f"shard rank {rank} {b.nx}x{b.ny}x{b.nz} pml={b.npml} tile={tile}: setup")
    st = random_state(oracle_mod, b, seed=40 + rank)
    init = {n: st[n].copy() for n in FIELDS}
    announce(f"shard rank {rank}: oracle")
    ref = oracle_mod.run(b, state=st, threads=16)
    announce(f"shard rank {rank}: gpu")
    _, fields, _, _ = gpu_run(F, b, init=init, tile=tile)
    compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)


def test_shard_matches_whole_board_interior(F):
    """Slab 1 of 8 (rows 99..198, three of the eight sources, ten probes) and the
    whole board, both from the same arbitrary state, each in its own benchmark
    tile: rows more than STEPS + 1 cells from a cut face agree bitwise."""
    rank, nranks = 1, 8
    whole = boardgen.large_board(steps=STEPS)
    whole.dft_freqs = None
    rng = np.random.default_rng(77)
    m, am = live_masks(whole), aux_masks(whole)
    axis = {"ddx": "x", "ddy": "y", "ddz": "z", "bbx": "x", "bby": "y", "bbz": "z"}
    scale = {"h": 1.0 / 376.73, "d": 8.854187817620389e-12, "b": 4e-7 * np.pi / 376.73}
    init = {}
    for n in FIELDS:
        mask = m[n] & am[axis[n]] if n in axis else m[n]
        v = rng.standard_normal(mask.shape, dtype=np.float32)
        v *= np.float32(scale.get(n[0], 1.0))
        v *= mask
        init[n] = v
    announce(f"whole large board tile={_tile(whole)}: gpu")
    wp, wf, _, _ = gpu_run(F, whole, init=init, tile=_tile(whole))

    h = whole.ny // nranks
    j0, j1 = rank * h, (rank + 1) * h
    sl = boardgen.large_board_shard(rank, nranks, steps=STEPS)
    sl.dft_freqs = None
    ms, ams = live_masks(sl), aux_masks(sl)
    sinit = {}
    for n in FIELDS:
        mask = ms[n] & ams[axis[n]] if n in axis else ms[n]
        sinit[n] = np.ascontiguousarray(init[n][:, j0:j1 + 1, :] * mask)
    del init
    announce(f"slab {rank} tile={_tile(sl)}: gpu")
    sp, sf, _, _ = gpu_run(F, sl, init=sinit, tile=_tile(sl))

    margin = STEPS + 2
    lo, hi = margin, (j1 - j0) - margin
    for n in FIELDS:
        a = sf[n][:, lo:hi + 1, :]
        w = wf[n][:, j0 + lo:j0 + hi + 1, :]
        assert np.array_equal(a, w), n
    assert np.abs(sf["ez"][:, lo:hi + 1, :]).max() > 0
    # probes of the slab that lie in the compared rows, against the same probes of the whole board
    checked = 0
    for q, (i, j, k) in enumerate(sl.probes):
        if lo <= j <= hi:
            p = whole.probes.index((i, j + j0, k))
            assert np.array_equal(sp[q], wp[p]), q
            checked += 1
    assert checked >= 5
