"""Lossy dielectrics and resistive sheets (conductor loss) on the HIP path (the
material two-step kernel and the node passes), against the FP64 oracle: probes
within 1e-4 (relative L2), all 12 arrays within 2e-5 after a few steps from
arbitrary states, a resistive source on a lossy edge (the two conductances
add), sheet edges on lossy cells, the two-step kernel bitwise equal to the node
passes across call splits, graphs and checkpoints, and the argument checks."""
import dataclasses

import numpy as np
import pytest

import boardgen
from _util import rel_l2
from test_gpu_eps import NODE_ONLY, run, two_step_equals_node_passes
from test_gpu_parity import FIELDS, announce, compare_fields, gpu_fields, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def lossy_board(seed, steps, nx=28, ny=20, nz=13):
    b = boardgen.random_tiny(seed, nx=nx, ny=ny, nz=nz, npml=3, steps=steps)
    rng = np.random.default_rng(seed + 11)
    p = b.npml
    sig = np.zeros(b.eps_r_cell.shape, np.float32)
    inner = (slice(p[4], nz - p[5]), slice(p[2], ny - p[3]), slice(p[0], nx - p[1]))
    sig[inner] = rng.choice([0.0, 0.02, 0.5, 3.0], size=sig[inner].shape).astype(np.float32)
    b.sigma_cell = sig
    i, j, k = (p[0] + nx - p[1]) // 2, (p[2] + ny - p[3]) // 2, (p[4] + nz - p[5]) // 2
    while b.pec_edge_mask[k, j, i] & 4 or any((s.i, s.j, s.k) == (i, j, k) for s in b.sources):
        i += 1
    b.sources.append(boardgen.Source(i, j, k, boardgen.GAUSS, 3.0, 12e-12, 4e-12, R=15.0))
    b.probes.append((i, j, k))
    return b


@pytest.mark.parametrize("seed", [0, 1])
def test_lossy_from_zero_against_oracle(F, oracle_mod, seed):
    b = lossy_board(seed, steps=71)
    announce(f"lossy board seed={seed}")
    ref = oracle_mod.run(b)
    g, ids = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, b.steps)
        F.fdtd_synchronize(g)
        assert F.fdtd_get_info(g).node_passes == 1
        probes = np.stack([F.fdtd_get_probe(g, p, b.steps) for p in ids])
        fields = gpu_fields(F, g, b)
    finally:
        F.fdtd_destroy_grid(g)
    for p in range(len(b.probes)):
        if np.abs(ref.probes[p]).max() > 0:
            assert rel_l2(probes[p], ref.probes[p]) <= 1e-4, p
    compare_fields(ref.state, fields, b, 2e-5)
    # the loss matters here
    ref0 = oracle_mod.run(dataclasses.replace(b, sigma_cell=None))
    assert rel_l2(ref0.probes[-1], ref.probes[-1]) > 1e-2


@pytest.mark.parametrize("eps_rw", [False, True])
def test_lossy_random_state_few_steps(F, oracle_mod, eps_rw):
    b = lossy_board(3, steps=5)
    b.sources = []
    b.pml_eps_rw = eps_rw
    st = random_state(oracle_mod, b, seed=9)
    init = {n: st[n].copy() for n in FIELDS}
    announce(f"lossy random state eps_rw={eps_rw}")
    ref = oracle_mod.run(b, state=st)
    fields = two_step_equals_node_passes(F, b, init)
    compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)


def test_lossy_table1_board_against_oracle(F, oracle_mod):
    """The Table 1 board with a loss tangent of 0.02 at 5 GHz in its dielectric,
    10000 steps: probe and the faster decay against the oracle."""
    b = boardgen.lossy_dielectric(boardgen.table1_board(steps=10000, source="resistive"), 0.02)
    announce("lossy table1: oracle")
    ref = oracle_mod.run(b, threads=16).probes[0]
    g, ids = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, b.steps)
        F.fdtd_synchronize(g)
        e = F.fdtd_get_probe(g, ids[0], b.steps).astype(np.float64)
    finally:
        F.fdtd_destroy_grid(g)
    assert rel_l2(e, ref) <= 1e-4
    assert np.sqrt(np.mean(e[8000:] ** 2)) < 0.1 * np.sqrt(np.mean(e[:2000] ** 2))


def test_conductivity_argument_errors(F):
    b = boardgen.random_tiny(5, nx=16, ny=14, nz=12, npml=2, steps=3)
    g, _ = F.grid_from_board(b, max_steps=3)
    try:
        sig = np.zeros(b.eps_r_cell.shape, np.float32)
        bad_pml = sig.copy()
        bad_pml[0, 5, 5] = 1.0
        with pytest.raises(F.FdtdError) as ei:
            F.fdtd_set_conductivity(g, bad_pml)
        assert ei.value.code == F.FDTD_EINVAL and "PML" in str(ei.value)
        for v in (-1.0, np.nan, np.inf):
            x = sig.copy()
            x[6, 6, 6] = v
            with pytest.raises(F.FdtdError) as ei:
                F.fdtd_set_conductivity(g, x)
            assert ei.value.code == F.FDTD_EINVAL
        F.fdtd_set_conductivity(g, sig)          # all zero: lossless, fused kernels
        F.fdtd_step_n(g, 1)
        assert F.fdtd_get_info(g).node_passes == 0
        with pytest.raises(F.FdtdError) as ei:
            F.fdtd_set_conductivity(g, sig)
        assert ei.value.code == F.FDTD_ESTATE
    finally:
        F.fdtd_destroy_grid(g)


# ---------------------------------------------------------------------------
# conductor loss: the PEC sheets as resistive sheets of surface resistance R_s
# ---------------------------------------------------------------------------

def sheet_board(seed, steps):
    """lossy_board with its PEC sheet kept inside the PML's inner region and
    given a surface resistance (the sheet edges then add to the cells' loss)."""
    b = lossy_board(seed, steps)
    p = b.npml
    mask = b.pec_edge_mask
    mask[:] &= 4
    k = (p[4] + b.nz - p[5]) // 2
    boardgen.pec_sheet(mask, k, p[0] + 2, b.nx - p[1] - 3, p[2] + 2, b.ny - p[3] - 3)
    b.sheet_R = 0.35
    return b


@pytest.mark.parametrize("seed", [0, 1])
def test_sheet_from_zero_against_oracle(F, oracle_mod, seed):
    b = sheet_board(seed, steps=73)
    b.sources.append(boardgen.Source(b.nx // 2, b.ny // 2, b.nz // 2 - 2, boardgen.GAUSS, 2e6,
                                     10e-12, 3e-12))
    b.probes.append((b.nx // 2 + 2, b.ny // 2, b.nz // 2 + 1))
    announce(f"resistive-sheet board seed={seed}")
    ref = oracle_mod.run(b)
    g, ids = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, b.steps)
        F.fdtd_synchronize(g)
        assert F.fdtd_get_info(g).node_passes == 1
        probes = np.stack([F.fdtd_get_probe(g, p, b.steps) for p in ids])
        fields = gpu_fields(F, g, b)
    finally:
        F.fdtd_destroy_grid(g)
    for p in range(len(b.probes)):
        if np.abs(ref.probes[p]).max() > 0:
            assert rel_l2(probes[p], ref.probes[p]) <= 1e-4, p
    compare_fields(ref.state, fields, b, 2e-5)
    # the sheet matters: perfect conductors give another field
    ref0 = oracle_mod.run(dataclasses.replace(b, sheet_R=0.0))
    assert rel_l2(ref0.state["ex"], ref.state["ex"]) > 1e-3


@pytest.mark.parametrize("eps_rw", [False, True])
def test_sheet_random_state_few_steps(F, oracle_mod, eps_rw):
    b = sheet_board(4, steps=5)
    b.pml_eps_rw = eps_rw
    b.sheet_R = 2.0
    st = random_state(oracle_mod, b, seed=19)
    # the sheet edges are state too once they are resistive
    rng = np.random.default_rng(3)
    for n, bit in (("ex", 1), ("ey", 2)):
        on = (b.pec_edge_mask & bit) != 0
        st[n][on] = rng.standard_normal(int(on.sum()))
    init = {n: st[n].copy() for n in FIELDS}
    announce(f"resistive sheet random state eps_rw={eps_rw}")
    ref = oracle_mod.run(b, state=st)
    fields = two_step_equals_node_passes(F, b, init)
    compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)


@pytest.mark.parametrize("wide", [False, True])
def test_lossy_sheet_bitwise_across_calls_graphs_and_checkpoints(F, wide):
    """A lossy board with a resistive sheet and a resistive source, 75 steps
    (two 32-step graph chunks and an odd tail): odd call splits, timed launches
    and the node passes alone give the same bits, and so does a checkpoint at
    step 41 (an odd step count on each side).  wide: per-cell eps_r as well, so
    that the board has more than 256 material classes (16-bit class map)."""
    b = sheet_board(5, steps=75)
    b.probes.append((b.nx // 2 + 2, b.ny // 2, b.nz // 2 + 1))
    if wide:
        rng = np.random.default_rng(12)
        b.eps_r_cell[:] = rng.choice([1.0, 2.2, 3.3, 4.4], size=b.eps_r_cell.shape).astype(np.float32)
        b.pml_eps_rw = True
    else:     # one conductivity over the inner region: few classes (8-bit class map)
        p = b.npml
        b.sigma_cell[:] = 0.0
        b.sigma_cell[p[4]:b.nz - p[5], p[2]:b.ny - p[3], p[0]:b.nx - p[1]] = 0.5
    ref = run(F, b)
    assert ref[0].material_two_step == 1 and (ref[0].n_classes > 256) == wide
    assert np.abs(ref[1]).max() > 0
    for out in (run(F, b, chunks=[7, 1, 33, 34]), run(F, b, timing=True), run(F, b, tile=NODE_ONLY)):
        assert np.array_equal(out[1], ref[1])
        for n in FIELDS:
            assert np.array_equal(out[3][n], ref[3][n]), n
    g, _ = F.grid_from_board(b, max_steps=b.steps)
    g2, _ = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, 41)
        F.fdtd_load_state(g2, F.fdtd_save_state(g))
        F.fdtd_step_n(g2, 34)
        F.fdtd_synchronize(g2)
        fields = gpu_fields(F, g2, b)
        for n in FIELDS:
            assert np.array_equal(fields[n], ref[3][n]), n
    finally:
        F.fdtd_destroy_grid(g)
        F.fdtd_destroy_grid(g2)


def test_conductor_loss_table1_board_against_oracle(F, oracle_mod):
    """The Table 1 board with copper planes (surface resistance at 5 GHz, 18.4
    milliohms per square) and a lossless dielectric, 10000 steps: the probe
    against the oracle, and the planes' loss shortens the ringing against the
    perfect conductors."""
    b = boardgen.conductor_loss(boardgen.table1_board(steps=10000, source="resistive"))
    announce(f"conductor-loss table1 (R_s {b.sheet_R:.4g} ohm): oracle")
    ref = oracle_mod.run(b, threads=16).probes[0]
    g, ids = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, b.steps)
        F.fdtd_synchronize(g)
        assert F.fdtd_get_info(g).node_passes == 1
        e = F.fdtd_get_probe(g, ids[0], b.steps).astype(np.float64)
    finally:
        F.fdtd_destroy_grid(g)
    assert rel_l2(e, ref) <= 1e-4
    pec = oracle_mod.run(dataclasses.replace(b, sheet_R=0.0), threads=16).probes[0]
    late = slice(6000, None)
    assert np.sqrt(np.mean(e[late] ** 2)) < 0.95 * np.sqrt(np.mean(pec[late] ** 2))


def test_sheet_argument_errors(F):
    b = boardgen.random_tiny(6, nx=16, ny=14, nz=12, npml=2, steps=3)
    g, _ = F.grid_from_board(b, max_steps=3)
    try:
        for v in (-1.0, np.nan, np.inf):
            with pytest.raises(F.FdtdError) as ei:
                F.fdtd_set_sheet_resistance(g, v)
            assert ei.value.code == F.FDTD_EINVAL
    finally:
        F.fdtd_destroy_grid(g)
    # a sheet running into a PML slab is refused at the first step
    b2 = boardgen.random_tiny(6, nx=16, ny=14, nz=12, npml=2, steps=3)
    b2.pec_edge_mask[:] &= 4
    boardgen.pec_sheet(b2.pec_edge_mask, 6, 0, 16, 0, 14)
    b2.sheet_R = 1.0
    g, _ = F.grid_from_board(b2, max_steps=3)
    try:
        with pytest.raises(F.FdtdError) as ei:
            F.fdtd_step_n(g, 1)
        assert ei.value.code == F.FDTD_EINVAL and "PML" in str(ei.value)
    finally:
        F.fdtd_destroy_grid(g)
    g, _ = F.grid_from_board(b, max_steps=3)
    try:
        F.fdtd_step_n(g, 1)
        with pytest.raises(F.FdtdError) as ei:
            F.fdtd_set_sheet_resistance(g, 1.0)
        assert ei.value.code == F.FDTD_ESTATE
    finally:
        F.fdtd_destroy_grid(g)


def test_material_boards_batched_bitwise(F):
    """Material boards join fdtd_step_many with their own split of tile planes:
    an eps_rw board (with a plane DFT; the material variant per plane), a lossy
    board with a resistive sheet and one with per-cell eps_r as well (more than
    256 classes), the wide slab board (the material variant per tile) and a
    lossy slab board without eps_rw (the conduction-only flavour) beside two
    plain boards, uneven step counts (odd ones end on the node passes), in two
    calls; every array, probe series and plane DFT bitwise equal to the board
    stepped alone, and the second call replays the first call's plan (one
    graph)."""
    from test_gpu_eps import eps_board
    wide = sheet_board(6, steps=60)
    rng = np.random.default_rng(21)
    wide.eps_r_cell[:] = rng.choice([1.0, 2.2, 3.3, 4.4], size=wide.eps_r_cell.shape).astype(np.float32)
    wide.pml_eps_rw = True
    boards = [boardgen.random_tiny(4, nx=40, ny=20, nz=10, npml=2, steps=60), eps_board(3, steps=60),
              sheet_board(5, steps=60), wide, boardgen.random_tiny(7, nx=33, ny=25, nz=9, npml=3, steps=60),
              slab_board(60, False, 512, 132, 30), slab_board(60, True, 70, 40, 44, eps_rw=False)]
    call = [17, 21, 9, 16, 20, 13, 19]
    totals = [2 * n for n in call]
    alone = [run(F, dataclasses.replace(b, steps=t)) for b, t in zip(boards, totals)]
    hs = [F.grid_from_board(b, max_steps=60) for b in boards]
    try:
        for _ in range(2):
            F.fdtd_step_many([g for g, _ in hs], call)
        F.fdtd_synchronize(hs[0][0])
        infos = [F.fdtd_get_info(g) for g, _ in hs]
        assert [i.material_two_step for i in infos] == [0, 1, 1, 1, 0, 1, 1]
        assert infos[3].n_classes > 256
        assert infos[5].material_split == 1 and infos[6].conduct_permille > 0
        assert infos[0].batch_plans == 1 and infos[0].batch_graphs == 1
        for q, ((g, ids), b) in enumerate(zip(hs, boards)):
            if ids:
                probes = np.stack([F.fdtd_get_probe(g, p, totals[q]) for p in ids])
                assert np.array_equal(probes, alone[q][1]), b.name
            if b.plane_dft is not None:
                assert np.array_equal(F.fdtd_get_plane_dft(g, b.ny, b.nx), alone[q][2]), b.name
            fields = gpu_fields(F, g, b)
            for n in FIELDS:
                assert np.array_equal(fields[n], alone[q][3][n]), (b.name, n)
    finally:
        for g, _ in hs:
            F.fdtd_destroy_grid(g)


def slab_board(steps, lossy=True, nx=70, ny=40, nz=44, eps_rw=True):
    """A board whose material sits in a few planes: an eps_r 4.2 slab (6 planes
    from nz // 2 - 6) through the x/y PML with eps_rw on between two PEC sheets,
    a resistive source and probes in it.  lossy: the slab is lossy inside the
    PML's inner region and the sheets resistive, so every tile holds material
    nodes near the slab (split per plane); else only tiles at the x/y PML do
    (split per tile on a board this wide).  Without eps_rw only the lossy
    layer's conducting edges need more than the plain kernel (its
    conduction-only flavour)."""
    eps, mask = boardgen.air(nx, ny, nz)
    k0 = nz // 2 - 6
    eps[k0:k0 + 6] = 4.2
    boardgen.pec_sheet(mask, k0, 6, nx - 7, 6, ny - 7)
    boardgen.pec_sheet(mask, k0 + 6, 6, nx - 7, 6, ny - 7)
    p = 4
    b = boardgen.Board("slab", nx, ny, nz, 0.5e-3, 0.5e-3, 0.1e-3, eps, mask, npml=(p,) * 6,
                       steps=steps, pml_eps_rw=eps_rw, sheet_R=0.02 if lossy else 0.0)
    if lossy:
        sig = np.zeros(eps.shape, np.float32)
        sig[k0:k0 + 6, p:ny - p, p:nx - p] = 0.05
        b.sigma_cell = sig
    b.sources = [boardgen.Source(nx // 3, ny // 2, k0 + 2, boardgen.GAUSS, 2.0, 4e-12, 1.2e-12, R=20.0),
                 boardgen.Source(2 * nx // 3, ny // 3, k0 + 4, boardgen.DGAUSS, 1e6, 5e-12, 1.5e-12)]
    b.probes = [(nx // 3 + 4, ny // 2, k0 + 3), (2 * nx // 3 - 5, ny // 3 + 3, k0 + 1),
                (nx // 3, ny // 2 + 6, k0 + 9)]
    b.plane_dft = (k0 + 1, np.array([3e9, 20e9]))
    return b


@pytest.mark.parametrize("lossy,eps_rw,shape,split", [(True, True, (70, 40, 44), 2),
                                                      (False, True, (512, 132, 30), 1),
                                                      (True, False, (70, 40, 44), 0),
                                                      (True, True, (512, 132, 30), 1)])
def test_slab_board_plain_and_material_pieces(F, oracle_mod, lossy, eps_rw, shape, split):
    """The split of a material board's tile planes between the plain kernel, its
    material variant (per plane on the small lossy eps_rw board, per tile on the
    wide ones) and the variant's conduction-only flavour (the lossy boards but
    the small eps_rw one; on the wide lossy one beside the material variant's
    pieces in the same pair): from an arbitrary state, 5 steps (two pairs and an
    odd one) give the node passes' bits and match the oracle; from zero, odd
    call splits, timed launches, the node passes alone and a checkpoint give the
    same bits, probes and the plane DFT against the oracle."""
    nx, ny, nz = shape
    b = slab_board(5, lossy, nx, ny, nz, eps_rw)
    st = random_state(oracle_mod, b, seed=31)
    if lossy:
        for n, bit in (("ex", 1), ("ey", 2)):        # the sheets' edges are state too
            on = (b.pec_edge_mask & bit) != 0
            st[n][on] = np.random.default_rng(bit).standard_normal(int(on.sum()))
    init = {n: st[n].copy() for n in FIELDS}
    announce(f"slab board lossy={lossy} {shape}: random state")
    ref = oracle_mod.run(b, state=st, threads=16)
    fields = two_step_equals_node_passes(F, b, init)
    info = two_step_equals_node_passes.info
    assert info.material_split == split, info.material_split
    if eps_rw:
        assert 0 < info.material_permille < 1000, info.material_permille
    else:
        assert info.material_permille == 0, info.material_permille
    assert (info.conduct_permille > 0) == (lossy and split != 2), info.conduct_permille
    compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)

    b = slab_board(71, lossy, nx, ny, nz, eps_rw)
    announce(f"slab board lossy={lossy} {shape}: from zero")
    ref = oracle_mod.run(b, threads=16)
    out = run(F, b)
    assert out[0].material_two_step == 1 and out[0].material_split == split
    for other in (run(F, b, chunks=[7, 1, 33, 30]), run(F, b, timing=True), run(F, b, tile=NODE_ONLY)):
        assert np.array_equal(other[1], out[1]) and np.array_equal(other[2], out[2])
        for n in FIELDS:
            assert np.array_equal(other[3][n], out[3][n]), n
    reach = max(np.abs(x).max() for x in ref.probes)
    for p in range(len(b.probes)):
        if np.abs(ref.probes[p]).max() > 1e-3 * reach:      # probes the pulse has reached
            assert rel_l2(out[1][p], ref.probes[p]) <= 1e-4, p
    for f in range(2):
        assert rel_l2(out[2][f], ref.plane_dft[f]) <= 1e-4, f
    # from zero after 71 steps: the stated 1e-4, with denominators at least 1e-2
    # of the whole E field's norm (in each array's units).  Between the nearly
    # perfect sheets the field is TM-like and has no Hz or Bz of its own: they
    # are residuals about 1e-3 of the other components (lossy board: Hz norm
    # 0.028 against 39 A/m for Hx and Hy in the oracle, and 6e-5 against 15 in
    # the slab's middle plane), so their own norms are no scale for FP32
    # round-off (8e-7 A/m there, 5e-8 of the H field).  The floor binds only for
    # such arrays.
    rep = compare_fields(ref.state, out[3], b, 1e-4, floor_rel=1e-2)
    for n, (whole, elem, reg, where) in rep.items():
        print(f"{n}: whole {whole:.2e} element {elem:.2e} worst region {reg:.2e} ({where})")
    g, _ = F.grid_from_board(b, max_steps=b.steps)
    g2, _ = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, 37)
        F.fdtd_load_state(g2, F.fdtd_save_state(g))
        F.fdtd_step_n(g2, 34)
        F.fdtd_synchronize(g2)
        fields = gpu_fields(F, g2, b)
        for n in FIELDS:
            assert np.array_equal(fields[n], out[3][n]), n
    finally:
        F.fdtd_destroy_grid(g)
        F.fdtd_destroy_grid(g2)
