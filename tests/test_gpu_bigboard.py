"""A board past the tiled kernels' 4 GiB offset window: 2047 x 1023 x 190 cells
(4.0e8 padded nodes, 1.6 GB per field array, 38 GB of fields) creates, steps on
the node passes from per-component bases moved to each z chunk, and matches the
FP64 oracle.  The arbitrary start state is held to a band of rows; three steps
later the fields have spread at most three rows, so a y-slab of the board ten
rows wider than the band on each side (its cut faces, which the slab treats as
PEC walls, stay out of the band's reach) computes exactly what the whole board
computes there.  The slab runs on the oracle: every array, element and region
within the fused kernels' bounds, and every row outside the slab still zero on
the GPU."""
import numpy as np
import pytest

import boardgen
from _compare import FIELDS, compare_fields
from test_gpu_parity import announce, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


@pytest.mark.timeout(900)
def test_board_past_the_32bit_window(F, oracle_mod):
    nx, ny, nz = 2047, 1023, 190
    steps = 3
    eps, mask = boardgen.air(nx, ny, nz)
    eps[80:110] = 4.2
    eps[90:100, 500:520, 900:1000] = 2.2
    boardgen.pec_sheet(mask, 80, 20, nx - 20, 20, ny - 20)
    boardgen.pec_sheet(mask, 110, 600, 1500, 505, 700)
    J0, J1 = 500, 530           # band of rows holding the start state
    j0, j1 = J0 - 10, J1 + 10   # the slab run on the oracle
    b = boardgen.Board("big2047", nx, ny, nz, 0.3e-3, 0.3e-3, 0.05e-3, eps, mask,
                       npml=(8, 8, 8, 8, 8, 8), steps=steps)
    b.sources = [boardgen.Source(1200, 512, 95, boardgen.GAUSS, 1e6, 0.0, 0.2e-12)]
    b.probes = [(1203, 515, 95), (700, 520, 105)]
    slab = boardgen.y_slab(b, j0, j1)
    st = random_state(oracle_mod, slab, seed=77)
    band = np.zeros(slab.ny + 1, bool)
    band[J0 - j0:J1 - j0] = True
    for n in FIELDS:
        st[n][:, ~band, :] = 0.0
    init = {n: st[n].astype(np.float32) for n in FIELDS}
    announce(f"big board {nx}x{ny}x{nz}: oracle on the slab {slab.nx}x{slab.ny}x{slab.nz}")
    ref = oracle_mod.run(slab, state=st, threads=16)
    announce("big board: create and set the state")
    shp = (nz + 1, ny + 1, nx + 1)
    g, ids = F.grid_from_board(b, max_steps=steps)
    try:
        for c, n in enumerate(FIELDS):
            full = np.zeros(shp, np.float32)
            full[:, j0:j1 + 1, :] = init[n]
            F.fdtd_set_field(g, c, full)
            del full
        announce("big board: step")
        F.fdtd_step_n(g, steps)
        F.fdtd_synchronize(g)
        info = F.fdtd_get_info(g)
        assert info.node_passes == 1 and info.step == steps
        announce("big board: read back")
        got = {}
        for c, n in enumerate(FIELDS):
            full = F.fdtd_get_field(g, c, shp)
            outside = np.abs(full[:, :j0, :]).max(initial=0.0) + np.abs(full[:, j1 + 1:, :]).max(initial=0.0)
            assert outside == 0.0, n
            got[n] = full[:, j0:j1 + 1, :].astype(np.float64)
            del full
        probes = np.stack([F.fdtd_get_probe(g, p, steps) for p in ids])
    finally:
        F.fdtd_destroy_grid(g)
    announce("big board: compare")
    rep = compare_fields(ref.state, got, slab, 2e-5, elem_tol=1e-5)
    for n, (whole, elem, reg, where) in rep.items():
        print(f"{n}: whole {whole:.2e} element {elem:.2e} worst region {reg:.2e} ({where})")
    np.testing.assert_allclose(probes, ref.probes, rtol=0, atol=2e-5 * np.abs(ref.probes).max())
