"""The plane-wide DFT of Ez and plane snapshots on the HIP path (the ground-plane
field of the Results section, Figs. 3-5), against the FP64 oracle.

Tolerance: per frequency, the relative L2 over the plane <= 1e-4 (FP32 samples,
FP64 accumulators), as for the probe DFT.  Each sample is folded into the
accumulators on its own, so tile shapes, call splits, graphs, the batched launch
and checkpoints give bitwise equal accumulators, and turning the plane DFT on
changes no field bit.
"""
import dataclasses

import numpy as np
import pytest

import boardgen
from _util import rel_l2
from test_gpu_parity import FIELDS, TWO_STEP, announce, gpu_fields

pytestmark = pytest.mark.gpu

ONE_STEP = (64, 8, 1)
TALL = (64, 14, 2)        # the plane variant of the tallest two-step shape


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def plane_board(seed, steps, nx=70, ny=19, nz=10):
    """random_tiny with the plane DFT on the Ez row above its PEC sheet, at the
    board's four probe-DFT frequencies plus 0 Hz."""
    b = boardgen.random_tiny(seed, nx=nx, ny=ny, nz=nz, npml=2, steps=steps)
    k = int(np.nonzero((b.pec_edge_mask & 3).any(axis=(1, 2)))[0][0])
    b.plane_dft = (k, np.concatenate([[0.0], b.dft_freqs]))
    return b


def run_plane(F, b, tile=None, chunks=None, timing=False, plane=True):
    bb = b if plane else dataclasses.replace(b, plane_dft=None)
    g, ids = F.grid_from_board(bb, max_steps=b.steps, tile=tile)
    try:
        if timing:
            F.fdtd_set_timing(g, True)
        for n in (chunks or [b.steps]):
            F.fdtd_step_n(g, n)
        F.fdtd_synchronize(g)
        pd = F.fdtd_get_plane_dft(g, b.ny, b.nx) if plane else None
        probes = np.stack([F.fdtd_get_probe(g, p, b.steps) for p in ids])
        dft = (np.stack([F.fdtd_get_dft(g, p) for p in ids])
               if b.dft_freqs is not None and ids else None)
        fields = gpu_fields(F, g, b)
    finally:
        F.fdtd_destroy_grid(g)
    return pd, probes, dft, fields


def check_against_oracle(pd, ref):
    peak = max(np.linalg.norm(ref[f]) for f in range(len(ref)))
    for f in range(len(ref)):
        if np.linalg.norm(ref[f]) > 1e-6 * peak:
            e = rel_l2(pd[f], ref[f])
            assert e <= 1e-4, (f, e)
        else:
            assert np.abs(pd[f] - ref[f]).max() <= 1e-4 * peak, f


@pytest.mark.parametrize("tile", [ONE_STEP, None, TWO_STEP, TALL])
def test_plane_dft_matches_oracle(F, oracle_mod, tile):
    b = plane_board(2, steps=77)
    announce(f"plane dft {b.nx}x{b.ny}x{b.nz} k={b.plane_dft[0]} tile={tile}")
    ref = oracle_mod.run(b)
    pd, probes, _, fields = run_plane(F, b, tile=tile)
    assert pd.shape == ref.plane_dft.shape
    check_against_oracle(pd, ref.plane_dft)
    # the plane DFT changes no field or probe bit
    _, probes0, _, fields0 = run_plane(F, b, tile=tile, plane=False)
    assert np.array_equal(probes, probes0)
    for n in FIELDS:
        assert np.array_equal(fields[n], fields0[n]), n


def test_plane_dft_bitwise_across_shapes_calls_and_graphs(F):
    b = plane_board(4, steps=101)
    outs = []
    for tile in F.fdtd_tile_shapes():
        announce(f"plane dft bitwise tile {tile}")
        outs.append(run_plane(F, b, tile=tile)[0])
    outs.append(run_plane(F, b, chunks=[7, 40, 33, 1, 20])[0])   # graphs and eager folds
    outs.append(run_plane(F, b, timing=True)[0])                  # all eager (timed launches)
    for pd in outs[1:]:
        assert np.array_equal(pd, outs[0])


def test_plane_dft_at_probe_nodes_equals_probe_dft(F):
    b = plane_board(6, steps=90)
    k = b.plane_dft[0]
    b.probes = [(3, 4, k), (b.nx // 2, b.ny // 2, k), (b.nx - 2, b.ny - 3, k)]
    pd, _, dft, _ = run_plane(F, b)
    for q, (i, j, _k) in enumerate(b.probes):
        got = pd[1:, j, i]          # plane frequencies 1.. are the probe frequencies
        assert np.abs(got - dft[q]).max() <= 1e-12 * max(np.abs(dft[q]).max(), 1e-300), q


def test_plane_dft_checkpoint_resume_bitwise(F):
    b = plane_board(8, steps=90)
    full = run_plane(F, b)[0]
    g, _ = F.grid_from_board(b, max_steps=b.steps)
    g2, _ = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, 45)
        img = F.fdtd_save_state(g)
        F.fdtd_load_state(g2, img)
        F.fdtd_step_n(g2, 45)
        F.fdtd_synchronize(g2)
        assert np.array_equal(F.fdtd_get_plane_dft(g2, b.ny, b.nx), full)
    finally:
        F.fdtd_destroy_grid(g)
        F.fdtd_destroy_grid(g2)


def test_plane_dft_batched_equals_alone(F):
    boards = [plane_board(10, steps=70), plane_board(11, steps=45, nx=40, ny=30, nz=12),
              boardgen.random_tiny(12, nx=50, ny=22, nz=9, npml=2, steps=33)]
    alone = [run_plane(F, b, plane=b.plane_dft is not None) for b in boards]
    hs = [F.grid_from_board(b, max_steps=b.steps) for b in boards]
    gs = [h for h, _ in hs]
    try:
        F.fdtd_step_many(gs, [b.steps for b in boards])
        F.fdtd_synchronize(gs[0])
        for b, g, ref in zip(boards, gs, alone):
            if b.plane_dft is not None:
                assert np.array_equal(F.fdtd_get_plane_dft(g, b.ny, b.nx), ref[0])
            fields = gpu_fields(F, g, b)
            for n in FIELDS:
                assert np.array_equal(fields[n], ref[3][n]), n
    finally:
        for g in gs:
            F.fdtd_destroy_grid(g)


def test_plane_snapshot_equals_field_slice(F):
    b = plane_board(14, steps=23)
    g, _ = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, b.steps)
        shp = (b.nz + 1, b.ny + 1, b.nx + 1)
        for comp in (2, 0, 4):
            full = F.fdtd_get_field(g, comp, shp)
            for k in (0, b.plane_dft[0], b.nz):
                snap = F.fdtd_get_plane(g, comp, k, b.ny, b.nx)
                assert np.array_equal(snap, full[k]), (comp, k)
    finally:
        F.fdtd_destroy_grid(g)


def test_plane_dft_argument_errors(F):
    b = boardgen.random_tiny(16, nx=20, ny=12, nz=8, npml=2, steps=5)
    g, _ = F.grid_from_board(b, max_steps=5)
    try:
        with pytest.raises(F.FdtdError) as ei:
            F.fdtd_get_plane_dft(g, b.ny, b.nx)
        assert ei.value.code == F.FDTD_ESTATE
        for k, fr in ((-1, [1e9]), (b.nz, [1e9]), (2, []), (2, [-1.0]), (2, [float("nan")]),
                      (2, np.ones(257))):
            with pytest.raises(F.FdtdError) as ei:
                F.fdtd_set_plane_dft(g, k, fr)
            assert ei.value.code == F.FDTD_EINVAL, (k, fr)
        for comp, k in ((12, 0), (-1, 0), (0, -1), (0, b.nz + 1)):
            with pytest.raises(F.FdtdError):
                F.fdtd_get_plane(g, comp, k, b.ny, b.nx)
        F.fdtd_set_plane_dft(g, 2, [1e9, 2e9])
        F.fdtd_step_n(g, 5)
        assert F.fdtd_get_info(g).plane_k == 2 and F.fdtd_get_info(g).plane_nf == 2
        with pytest.raises(F.FdtdError) as ei:
            F.fdtd_set_plane_dft(g, 3, [1e9])
        assert ei.value.code == F.FDTD_ESTATE
    finally:
        F.fdtd_destroy_grid(g)


def test_large_board_plane_dft_full_size(F, oracle_mod):
    """The large board at full size (1048 x 792 x 88) with the plane DFT of Ez on
    the row above the ground sheet at 4 frequencies, 200 steps with the sources
    firing early, in the tile the tuner picks for it: every node of the plane
    against the oracle."""
    from paper_1008_2602_amd import tune
    b = boardgen.large_board(steps=200)
    dt = oracle_mod.time_step(b)
    for s_idx, s in enumerate(b.sources):
        s.t0, s.sigma = (24 + 4 * s_idx) * dt, 6 * dt
    b.probes, b.dft_freqs = b.probes[:4], None
    b.plane_dft = (b.meta["layout"]["kg"], np.array([1e9, 5e9, 20e9, 80e9]))
    tile = tune.tune_board(b)
    announce(f"large board plane dft tile={tile}: oracle")
    ref = oracle_mod.run(b, threads=16)
    announce("large board plane dft: gpu")
    pd, _, _, _ = run_plane(F, b, tile=tile)
    announce("large board plane dft: compare")
    check_against_oracle(pd, ref.plane_dft)
