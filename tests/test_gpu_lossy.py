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
