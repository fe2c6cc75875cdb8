"""Eq. 2's eps_rw on the HIP path: boards whose dielectric reaches into a PML slab
step in the node passes' arithmetic (pairs of steps on the material two-step
kernel, an odd step on the node passes; or, with a one-step shape set, every
step on the node passes), against the FP64 oracle.

Tolerances as for the fused kernels: all 12 arrays within a relative L2 of 2e-5
after a few steps from arbitrary states, probes and the plane DFT within 1e-4;
the two-step kernel and the node passes give the same bits, and so do call
splits, graphs, checkpoints and the batched call; with the PML in air the flag
changes nothing and the fused kernels run.
"""
import dataclasses

import numpy as np
import pytest

import boardgen
from _util import rel_l2
from test_gpu_parity import FIELDS, announce, compare_fields, gpu_fields, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1008_2602_amd import fdtd
    return fdtd


def eps_board(seed, steps, nx=30, ny=21, nz=14):
    """random_tiny with random eps_r in every cell (PML included), eps_rw on, a
    resistive source inside and the plane DFT on the PEC sheet's Ez row."""
    b = boardgen.random_tiny(seed, nx=nx, ny=ny, nz=nz, npml=3, steps=steps)
    rng = np.random.default_rng(seed + 5)
    b.eps_r_cell[:] = rng.choice([1.0, 2.2, 4.4], size=b.eps_r_cell.shape).astype(np.float32)
    b.pml_eps_rw = True
    p = b.npml
    i, j, k = (p[0] + nx - p[1]) // 2, (p[2] + ny - p[3]) // 2, (p[4] + nz - p[5]) // 2
    while b.pec_edge_mask[k, j, i] & 4 or any((s.i, s.j, s.k) == (i, j, k) for s in b.sources):
        i += 1
    b.sources.append(boardgen.Source(i, j, k, boardgen.DGAUSS, 2.0, 10e-12, 3e-12, R=25.0))
    kp = int(np.nonzero((b.pec_edge_mask & 3).any(axis=(1, 2)))[0][0])
    b.plane_dft = (kp, np.array([2e9, 11e9]))
    return b


NODE_ONLY = (64, 8, 1)   # a one-step shape: every step of a material board on the node passes


def step_from_state(F, b, init, tile=None):
    """All 12 arrays set from `init`, b.steps steps: (info, fields)."""
    g, _ = F.grid_from_board(b, max_steps=b.steps, tile=tile)
    try:
        for c, n in enumerate(FIELDS):
            F.fdtd_set_field(g, c, init[n].astype(np.float32))
        F.fdtd_step_n(g, b.steps)
        F.fdtd_synchronize(g)
        return F.fdtd_get_info(g), gpu_fields(F, g, b)
    finally:
        F.fdtd_destroy_grid(g)


def two_step_equals_node_passes(F, b, init):
    """The default (material two-step kernel, the odd step on the node passes)
    and the node passes alone from the same state: the same bits.  Returns the
    fields."""
    info, fields = step_from_state(F, b, init)
    info1, fields1 = step_from_state(F, b, init, tile=NODE_ONLY)
    assert info.node_passes == 1 and info1.node_passes == 1
    assert info.material_two_step == 1 and info1.material_two_step == 0
    assert (info.tile_x, info.tile_steps) == (64, 2)
    for n in FIELDS:
        assert np.array_equal(fields[n], fields1[n]), n
    two_step_equals_node_passes.info = info
    return fields


def run(F, b, chunks=None, timing=False, tile=None):
    g, ids = F.grid_from_board(b, max_steps=b.steps, tile=tile)
    try:
        if timing:
            F.fdtd_set_timing(g, True)
        for n in (chunks or [b.steps]):
            F.fdtd_step_n(g, n)
        F.fdtd_synchronize(g)
        info = F.fdtd_get_info(g)
        probes = np.stack([F.fdtd_get_probe(g, p, b.steps) for p in ids]) if ids else None
        plane = F.fdtd_get_plane_dft(g, b.ny, b.nx) if b.plane_dft is not None else None
        fields = gpu_fields(F, g, b)
    finally:
        F.fdtd_destroy_grid(g)
    return info, probes, plane, fields


@pytest.mark.parametrize("seed", [0, 1])
def test_eps_rw_from_zero_against_oracle(F, oracle_mod, seed):
    b = eps_board(seed, steps=67)
    announce(f"eps_rw board seed={seed} {b.nx}x{b.ny}x{b.nz}")
    ref = oracle_mod.run(b)
    info, probes, plane, fields = run(F, b)
    assert info.node_passes == 1
    for p in range(len(b.probes)):
        if np.abs(ref.probes[p]).max() > 0:
            assert rel_l2(probes[p], ref.probes[p]) <= 1e-4, p
    compare_fields(ref.state, fields, b, 2e-5)
    for f in range(2):
        assert rel_l2(plane[f], ref.plane_dft[f]) <= 1e-4, f
    # eps_rw matters on this board: the oracle without it differs
    ref0 = oracle_mod.run(dataclasses.replace(b, pml_eps_rw=False))
    assert rel_l2(ref0.state["ddx"], ref.state["ddx"]) > 1e-3


@pytest.mark.parametrize("shape,npml", [((30, 21, 14), (3, 3, 3, 3, 3, 3)),
                                        ((70, 13, 9), (4, 0, 2, 2, 3, 3)),
                                        ((9, 11, 7), (3, 2, 1, 3, 2, 2))])
def test_eps_rw_random_state_few_steps(F, oracle_mod, shape, npml):
    nx, ny, nz = shape
    eps, mask = boardgen.air(nx, ny, nz)
    rng = np.random.default_rng(nx * 7 + ny)
    eps[:] = rng.choice([1.0, 2.2, 4.4], size=eps.shape).astype(np.float32)
    if nz >= 4:
        boardgen.pec_sheet(mask, nz // 2, 0, nx // 2, 1, ny - 1)
    b = boardgen.Board(f"epsrand{nx}", nx, ny, nz, 0.7e-3, 0.9e-3, 0.4e-3, eps, mask,
                       npml=npml, steps=4, pml_eps_rw=True)
    st = random_state(oracle_mod, b, seed=nx + ny)
    init = {n: st[n].copy() for n in FIELDS}
    announce(f"eps_rw random state {shape} npml={npml}")
    ref = oracle_mod.run(b, state=st)
    fields = two_step_equals_node_passes(F, b, init)
    compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)


@pytest.mark.parametrize("shape,lossy", [((256, 128, 48), True), ((512, 256, 48), False)])
def test_node_pass_z_chunks_random_state(F, oracle_mod, shape, lossy):
    """Boards with enough columns that the node passes cut z into chunks that
    carry the previous plane in registers: 3 planes per chunk on the first board
    (4 x 32 column blocks), 12 on the second (8 x 64), as on the large benchmark
    board; the chunk seams (k0 > 0) lie at every third or twelfth plane.  Random
    eps_r in blocks everywhere (PML included), a PEC sheet, eps_rw on (and on the
    first board a lossy interior, in other blocks): three steps from an arbitrary
    state against the oracle, every array, element and region (each plane on
    its own)."""
    nx, ny, nz = shape
    eps, mask = boardgen.air(nx, ny, nz)
    rng = np.random.default_rng(nx + nz)
    # random eps_r in blocks of 32 x 16 x 4 cells (random per cell would exceed
    # the 65535 material classes on boards this size once the loss varies too)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    blocks = rng.choice([1.0, 2.2, 4.4], size=(nz // 4 + 1, ny // 16 + 1, nx // 32 + 1))
    eps[:] = blocks[kk // 4, jj // 16, ii // 32].astype(np.float32)
    boardgen.pec_sheet(mask, nz // 2, 0, nx // 2, 1, ny - 1)
    npml = (5, 4, 6, 3, 4, 5)
    b = boardgen.Board(f"epschunk{nx}", nx, ny, nz, 0.5e-3, 0.6e-3, 0.2e-3, eps, mask,
                       npml=npml, steps=3, pml_eps_rw=True)
    if lossy:
        sblocks = rng.choice([0.0, 0.4, 2.0], size=(nz // 4 + 1, ny // 16 + 1, nx // 32 + 1))
        sig = sblocks[(kk + 2) // 4, (jj + 8) // 16, (ii + 16) // 32].astype(np.float32)
        sig[:npml[4]] = 0.0
        sig[nz - npml[5]:] = 0.0
        sig[:, :npml[2]] = 0.0
        sig[:, ny - npml[3]:] = 0.0
        sig[:, :, :npml[0]] = 0.0
        sig[:, :, nx - npml[1]:] = 0.0
        b.sigma_cell = sig
    st = random_state(oracle_mod, b, seed=nx + ny)
    init = {n: st[n].copy() for n in FIELDS}
    announce(f"node-pass z chunks {shape} lossy={lossy}")
    ref = oracle_mod.run(b, state=st, threads=16)
    # every step on the node passes (their z chunks), then the default (one pair
    # on the two-step kernel, the last step on the node passes): the same bits
    fields = two_step_equals_node_passes(F, b, init)
    rep = compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)
    for n, (whole, elem, reg, where) in rep.items():
        print(f"{n}: whole {whole:.2e} element {elem:.2e} worst region {reg:.2e} ({where})")


def test_eps_rw_bitwise_across_calls_graphs_checkpoints_and_batches(F):
    """75 steps (two 32-step graph chunks and a tail with an odd step) against
    odd call splits (each odd count ends on the node passes), timed launches,
    the node passes alone, a checkpoint at step 40 and a batched call."""
    b = eps_board(3, steps=75)
    ref = run(F, b)
    assert ref[0].material_two_step == 1
    for out in (run(F, b, chunks=[7, 1, 33, 34]), run(F, b, timing=True), run(F, b, tile=NODE_ONLY)):
        assert np.array_equal(out[1], ref[1]) and np.array_equal(out[2], ref[2])
        for n in FIELDS:
            assert np.array_equal(out[3][n], ref[3][n]), n
    g, _ = F.grid_from_board(b, max_steps=b.steps)
    g2, _ = F.grid_from_board(b, max_steps=b.steps)
    try:
        F.fdtd_step_n(g, 40)
        F.fdtd_load_state(g2, F.fdtd_save_state(g))
        F.fdtd_step_n(g2, 35)
        F.fdtd_synchronize(g2)
        assert np.array_equal(F.fdtd_get_plane_dft(g2, b.ny, b.nx), ref[2])
        fields = gpu_fields(F, g2, b)
        for n in FIELDS:
            assert np.array_equal(fields[n], ref[3][n]), n
    finally:
        F.fdtd_destroy_grid(g)
        F.fdtd_destroy_grid(g2)
    # batched beside a board on the fused kernels
    other = boardgen.random_tiny(4, nx=40, ny=20, nz=10, npml=2, steps=50)
    alone = run(F, other)
    hs = [F.grid_from_board(x, max_steps=x.steps) for x in (other, b)]
    try:
        F.fdtd_step_many([h for h, _ in hs], [other.steps, b.steps])
        for (h, _), x, r in zip(hs, (other, b), (alone, ref)):
            F.fdtd_synchronize(h)
            fields = gpu_fields(F, h, x)
            for n in FIELDS:
                assert np.array_equal(fields[n], r[3][n]), n
    finally:
        for h, _ in hs:
            F.fdtd_destroy_grid(h)


def test_eps_rw_with_the_pml_in_air_is_the_fused_path(F):
    b = boardgen.small_board(steps=60)
    on = run(F, dataclasses.replace(b, pml_eps_rw=True))
    off = run(F, b)
    assert on[0].node_passes == 0
    assert np.array_equal(on[1], off[1])
    for n in FIELDS:
        assert np.array_equal(on[3][n], off[3][n]), n


def test_fig3_board_into_upml_against_oracle(F, oracle_mod):
    """The paper's Fig. 3 case (100 x 60 x 0.8 mm board running into the UPML,
    eps_rw on, dt = 1 ps, 1000 steps): the ground-row probes against the oracle and
    the decay the paper describes (below 5 % of the peak after 600 ps)."""
    b = boardgen.fig3_board(steps=1000)
    announce("fig3 board: oracle")
    ref = oracle_mod.run(b, threads=16)
    announce("fig3 board: gpu")
    info, probes, _, _ = run(F, b)
    assert info.node_passes == 1
    t = (np.arange(b.steps) + 1) * 1e-12
    for p in range(len(b.probes)):
        assert rel_l2(probes[p], ref.probes[p]) <= 1e-4, p
        assert np.abs(probes[p][t > 600e-12]).max() < 0.05 * np.abs(probes[p]).max(), p
