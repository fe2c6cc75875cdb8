"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances: probe series relative L2 <= 1e-4 per probe and identical FFT peak
bins (within one bin) for full runs; the DFT within 1e-4 per probe; for short
runs from arbitrary states (FP32 arithmetic over a few steps) every array
within a relative L2 of 2e-5, every element within 1e-5 of the array's largest
value and every region (PML faces, edges and corners, each node plane, row and
column, the PEC sheet rims) within 4e-5 (tests/_compare.py); runs from zero over
tens to hundreds of steps hold every element within the whole-array tolerance
of the largest value; batched, resumed and re-tiled runs are bitwise equal to
the plain run.
"""
import os
import sys

import numpy as np
import pytest

import boardgen
from _compare import FIELDS, aux_masks, compare_fields  # noqa: F401  (re-exported to the other GPU tests)
from _util import live_masks, rel_l2

pytestmark = pytest.mark.gpu

TWO_STEP = (64, 10, 2)   # a two-steps-per-pass shape other than the default 64x14x2


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


@pytest.fixture(scope="module")
def orc(oracle_mod):
    return oracle_mod


def gpu_fields(F, g, board):
    shp = (board.nz + 1, board.ny + 1, board.nx + 1)
    return {n: F.fdtd_get_field(g, c, shp).astype(np.float64) for c, n in enumerate(FIELDS)}


def gpu_run(F, board, steps=None, tile=None, init=None, chunks=None):
    steps = board.steps if steps is None else steps
    g, ids = F.grid_from_board(board, max_steps=max(steps, 1), tile=tile)
    try:
        if init is not None:
            for c, n in enumerate(FIELDS):
                F.fdtd_set_field(g, c, init[n].astype(np.float32))
        for n in (chunks or [steps]):
            F.fdtd_step_n(g, n)
        F.fdtd_synchronize(g)
        probes = np.stack([F.fdtd_get_probe(g, p, steps) for p in ids]) if ids else None
        fields = gpu_fields(F, g, board)
        dft = (np.stack([F.fdtd_get_dft(g, p) for p in ids])
               if board.dft_freqs is not None and ids else None)
        info = F.fdtd_get_info(g)
    finally:
        F.fdtd_destroy_grid(g)
    return probes, fields, dft, info


def random_state(orc, board, seed, scale_h=376.73):
    rng = np.random.default_rng(seed)
    st = orc.new_state(board)
    m = live_masks(board)
    am = aux_masks(board)
    axis = {"ddx": "x", "ddy": "y", "ddz": "z", "bbx": "x", "bby": "y", "bbz": "z"}
    eps0 = 8.854187817620389e-12
    mu0 = 4e-7 * np.pi
    for n in FIELDS:
        mask = m[n] & am[axis[n]] if n in axis else m[n]
        v = rng.standard_normal(st[n].shape, dtype=np.float32)
        v *= mask
        scale = {"h": 1.0 / scale_h, "d": eps0, "b": mu0 / scale_h}.get(n[0], 1.0)
        if n.startswith("e"):
            st[n][...] = v
        else:                                                   # both sides see FP32 inputs
            st[n][...] = (v.astype(np.float64) * scale).astype(np.float32)
    return st


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tiny_boards_from_zero(F, orc, seed):
    b = boardgen.random_tiny(seed, steps=60)
    dt = orc.time_step(b)
    for s in b.sources:
        s.t0, s.sigma = 20 * dt, 5 * dt
    announce(f"tiny board seed={seed} {b.nx}x{b.ny}x{b.nz} steps={b.steps}")
    ref = orc.run(b)
    probes, fields, dft, _ = gpu_run(F, b)
    for p in range(len(b.probes)):
        if np.abs(ref.probes[p]).max() > 0:
            assert rel_l2(probes[p], ref.probes[p]) <= 1e-4, p
    compare_fields(ref.state, fields, b, 2e-5)
    assert rel_l2(dft, ref.dft) <= 1e-4


@pytest.mark.parametrize("shape,npml", [((9, 11, 7), (3, 2, 1, 3, 2, 2)),
                                        ((70, 13, 9), (4, 4, 2, 2, 3, 3)),
                                        ((13, 17, 30), (0, 3, 2, 0, 5, 4)),
                                        ((2, 2, 2), (0, 0, 0, 0, 0, 0)),
                                        ((131, 9, 4), (1, 1, 1, 1, 1, 1))])
@pytest.mark.parametrize("tile", [None, TWO_STEP])
def test_random_state_few_steps(F, orc, shape, npml, tile):
    nx, ny, nz = shape
    eps, mask = boardgen.air(nx, ny, nz)
    rng = np.random.default_rng(nx * 1000 + ny)
    eps[:] = rng.choice([1.0, 2.2, 4.4], size=eps.shape).astype(np.float32)
    if nz >= 4:
        boardgen.pec_sheet(mask, nz // 2, 0, nx // 2, 1, ny - 1)
    b = boardgen.Board(f"rand{nx}x{ny}x{nz}", nx, ny, nz, 0.7e-3, 0.9e-3, 0.4e-3, eps, mask,
                       npml=npml, steps=4 if tile is None else 5)
    st = random_state(orc, b, seed=nx + ny + nz)
    init = {n: st[n].copy() for n in FIELDS}
    announce(f"random state {shape} npml={npml} tile={tile}")
    ref = orc.run(b, state=st)
    _, fields, _, _ = gpu_run(F, b, init=init, tile=tile)
    compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)


@pytest.mark.parametrize("shape,npml", [((64, 22, 5), (2, 2, 2, 2, 1, 1)),
                                        ((128, 14, 4), (1, 1, 1, 1, 1, 1)),
                                        ((2, 2, 2), (0, 0, 0, 0, 0, 0)),
                                        ((2, 9, 3), (0, 0, 1, 1, 0, 0)),
                                        ((65, 2, 2), (1, 1, 0, 0, 0, 0))])
@pytest.mark.parametrize("tile", [None, TWO_STEP, (64, 15, 1)])
def test_exact_tile_multiples_and_degenerate_shapes(F, orc, shape, npml, tile):
    """Grids whose cells fill the tiles exactly (nx a multiple of 64, ny of the
    owned rows: 11 for 64x14x2, 7 for 64x10x2, 14 for 64x15x1), so that the far
    wall's nodes fall outside every tile, and grids of the smallest size the
    library takes (two cells) in a direction.
    Three or four steps from an arbitrary state with sources, against the oracle."""
    nx, ny, nz = shape
    eps, mask = boardgen.air(nx, ny, nz)
    rng = np.random.default_rng(nx * 7 + ny * 3 + nz)
    eps[:] = rng.choice([1.0, 3.3], size=eps.shape).astype(np.float32)
    b = boardgen.Board(f"edge{nx}x{ny}x{nz}", nx, ny, nz, 0.5e-3, 0.6e-3, 0.3e-3, eps, mask,
                       npml=npml, steps=3 if tile == (64, 15, 1) else 4)
    b.sources = [boardgen.Source(nx // 2, ny // 2, nz // 2, boardgen.GAUSS, 1e6, 0.0, 1e-12)]
    b.probes = [(nx // 2, ny // 2, nz // 2), (nx - 1, ny - 1, nz - 1)]
    st = random_state(orc, b, seed=nx + 2 * ny + 5 * nz)
    init = {n: st[n].copy() for n in FIELDS}
    announce(f"exact multiples / degenerate {shape} npml={npml} tile={tile}")
    ref = orc.run(b, state=st)
    probes, fields, _, _ = gpu_run(F, b, init=init, tile=tile)
    compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)
    assert rel_l2(probes, ref.probes) <= 2e-5


def test_set_field_keeps_only_state_entries(F):
    """Entries outside the state (components that do not exist at a node, E
    tangential to the outer wall, H normal to the wall on it) are stored as zero,
    and a step leaves them zero."""
    b = boardgen.random_tiny(3, nx=70, ny=12, nz=6, npml=1, steps=2)
    shp = (b.nz + 1, b.ny + 1, b.nx + 1)
    m = live_masks(b)
    am = aux_masks(b)
    axis = {"ddx": "x", "ddy": "y", "ddz": "z", "bbx": "x", "bby": "y", "bbz": "z"}
    announce("set_field outside the state")
    g, _ = F.grid_from_board(b, max_steps=4)
    try:
        rng = np.random.default_rng(5)
        for c, n in enumerate(FIELDS):
            F.fdtd_set_field(g, c, rng.standard_normal(shp).astype(np.float32))
        for step in range(2):
            for c, n in enumerate(FIELDS):
                got = F.fdtd_get_field(g, c, shp)
                keep = m[n] & am[axis[n]] if n in axis else m[n].copy()
                if n in ("ex", "ey", "ez", "ddx", "ddy", "ddz"):
                    keep |= (b.pec_edge_mask & {"x": 1, "y": 2, "z": 4}[n[-1]]) != 0   # PEC edges: caller's business
                assert not got[~keep].any(), (step, n)
                if step == 0:
                    assert got[keep & m[n]].any(), n
            F.fdtd_step_n(g, 1)
    finally:
        F.fdtd_destroy_grid(g)


def test_small_board_full_run_parity(F, orc):
    b = boardgen.small_board()
    announce(f"small board full {b.nx}x{b.ny}x{b.nz} steps={b.steps}")
    ref = orc.run(b, threads=16)
    probes, _, _, _ = gpu_run(F, b)
    n_fft = orc.default_nfft(b.steps)
    f = orc.bin_freqs(n_fft, ref.dt)
    for p in range(len(b.probes)):
        e = rel_l2(probes[p], ref.probes[p])
        assert e <= 1e-4, (p, e)
        Xr = np.abs(orc.probe_fft(ref.probes[p], n_fft))
        Xg = np.abs(orc.probe_fft(probes[p].astype(np.float64), n_fft))
        pr = orc.find_peaks(Xr, f, f_min=0.5e9)
        pg = orc.find_peaks(Xg, f, f_min=0.5e9)
        assert len(pr) == len(pg)
        assert np.all(np.abs(pr - pg) <= 1.0 / (b.steps * ref.dt))


GOLDEN_REALISTIC = os.path.join(os.path.dirname(__file__), "golden", "realistic_board_probes.npz")


def test_realistic_board_full_run(F, orc):
    """The realistic board (444x364x60 cells, 16 probes) over its full 20000
    steps against the FP64 oracle's run stored by
    tests/golden/make_realistic_probes.py: per probe relative L2 <= 1e-4 on
    every 4th sample, and the spectral peaks of the full-resolution series
    within one bin of the oracle's."""
    d = np.load(GOLDEN_REALISTIC)
    b = boardgen.realistic_board()
    assert int(d["steps"]) == b.steps
    announce(f"realistic board full run {b.nx}x{b.ny}x{b.nz} steps={b.steps}")
    probes, _, _, info = gpu_run(F, b)
    assert abs(info.dt - float(d["dt"])) <= 1e-12 * float(d["dt"])
    dec = int(d["decimate"])
    n_fft = int(d["n_fft"])
    f = orc.bin_freqs(n_fft, float(d["dt"]))
    bin_hz = 1.0 / (b.steps * float(d["dt"]))
    for p in range(len(b.probes)):
        e = rel_l2(probes[p][::dec], d["series"][p])
        assert e <= 1e-4, (p, e)
        ref = d["peaks_hz"][p]
        ref = ref[~np.isnan(ref)]
        got = orc.find_peaks(np.abs(orc.probe_fft(probes[p].astype(np.float64), n_fft)), f, f_min=0.5e9)
        assert len(got) == len(ref), (p, got, ref)
        assert np.all(np.abs(got - ref) <= bin_hz), (p, got, ref)


def _bench_tile(board):
    """The tile the benchmark runs this board with (the tuner's cached choice)."""
    from paper_1008_2602_amd import tune
    return tune.tune_board(board)


def test_large_board_full_size_from_zero(F, orc):
    """The large-board workload at its full size (1048x792x88 cells, both PEC
    islands, 8 sources, 64 probes, 256 DFT frequencies) in the benchmark's tile:
    every field array, every probe series and the DFT against the oracle.  The
    sources fire inside the 200-step window (t0 = (24 + 4s) dt, sigma = 6 dt)."""
    b = boardgen.large_board(steps=200)
    dt = orc.time_step(b)
    for s_idx, s in enumerate(b.sources):
        s.t0, s.sigma = (24 + 4 * s_idx) * dt, 6 * dt
    tile = _bench_tile(b)
    announce(f"large board full size {b.nx}x{b.ny}x{b.nz} steps={b.steps} tile={tile}: oracle")
    ref = orc.run(b, threads=16)
    announce("large board full size: gpu")
    probes, fields, dft, _ = gpu_run(F, b, tile=tile)
    announce("large board full size: compare")
    peak = np.abs(ref.probes).max()
    assert peak > 0
    checked = 0
    for p in range(len(b.probes)):
        r = ref.probes[p]
        if np.abs(r).max() > 1e-6 * peak:      # probes the pulse has reached
            e = rel_l2(probes[p], r)
            assert e <= 1e-4, (p, e)
            checked += 1
        else:                                   # ahead of the front: tiny on both sides
            assert np.abs(probes[p] - r).max() <= 1e-4 * peak, p
    assert checked >= 4
    rep = compare_fields(ref.state, fields, b, 1e-4, floor_rel=1e-6)
    for n, (whole, elem, reg, where) in rep.items():
        print(f"{n}: whole {whole:.2e} element {elem:.2e} worst region {reg:.2e} ({where})")
    # the DFT per probe (256 frequencies each): within 1e-4 where the pulse arrived
    dmax = np.abs(ref.dft).max()
    for p in range(len(b.probes)):
        if np.abs(ref.probes[p]).max() > 1e-6 * peak:
            e = rel_l2(dft[p], ref.dft[p])
            assert e <= 1e-4, (p, e)
        else:
            assert np.abs(dft[p] - ref.dft[p]).max() <= 1e-4 * dmax, p


def test_large_board_full_size_random_state(F, orc):
    """Full-size large board from an arbitrary state (every live node and every
    kept D/B nonzero, so all PML slabs, edges, corners, island rims and tile
    seams are exercised), three steps in the benchmark's tile."""
    b = boardgen.large_board(steps=3)
    b.sources, b.probes, b.dft_freqs = [], [], None
    tile = _bench_tile(b)
    announce(f"large board full size random state tile={tile}: setup")
    st = random_state(orc, b, seed=3)
    init = {n: st[n].copy() for n in FIELDS}
    announce("large board full size random state: oracle")
    ref = orc.run(b, state=st, threads=16)
    announce("large board full size random state: gpu")
    _, fields, _, _ = gpu_run(F, b, init=init, tile=tile)
    del init
    announce("large board full size random state: compare")
    rep = compare_fields(ref.state, fields, b, 2e-5, elem_tol=1e-5)
    for n, (whole, elem, reg, where) in rep.items():
        print(f"{n}: whole {whole:.2e} element {elem:.2e} worst region {reg:.2e} ({where})")


def test_large_board_full_length_is_stable(F):
    """The large-board workload over its whole 10000 steps (2.7 ns) in the
    benchmark's tile: the watchdog stays quiet, every probe series and DFT value is
    finite, the probes see the pulses, and nothing grows: the swing of every
    probe over the last quarter of the run stays below the largest swing of the
    first half, which holds the pulses (the plane pair rings for a long time and
    keeps the static field the Gaussian sources leave, so the field need not decay
    monotonically)."""
    b = boardgen.large_board()
    tile = _bench_tile(b)
    announce(f"large board full length {b.steps} steps tile={tile}")
    probes, _, dft, info = gpu_run(F, b, tile=tile)
    assert info.step == b.steps
    assert np.all(np.isfinite(probes)) and np.all(np.isfinite(dft))
    peak = np.abs(probes).max()
    assert peak > 0
    n = b.steps
    late = np.ptp(probes[:, 3 * n // 4:], axis=1).max()
    early = np.ptp(probes[:, :n // 2], axis=1).max()
    assert late < early, (late, early)


def test_tile_shapes_bitwise(F):
    """Every shape, one- and two-step (an odd count ends on one single step),
    gives the same bits as the first."""
    b = boardgen.random_tiny(7, nx=150, ny=37, nz=12, npml=3, steps=31)
    for s in b.sources:
        s.t0, s.sigma = 5e-12, 2e-12
    outs = []
    for tile in F.fdtd_tile_shapes():
        announce(f"tile {tile}")
        probes, fields, _, _ = gpu_run(F, b, tile=tile)
        outs.append((probes, fields))
    for probes, fields in outs[1:]:
        assert np.array_equal(probes, outs[0][0])
        for n in FIELDS:
            assert np.array_equal(fields[n], outs[0][1][n]), n


def test_chunked_equals_single_call(F):
    b = boardgen.small_board(steps=240)
    announce("chunked vs single")
    p1, f1, _, _ = gpu_run(F, b)
    p2, f2, _, _ = gpu_run(F, b, chunks=[1, 7, 100, 0, 132])
    assert np.array_equal(p1, p2)
    for n in FIELDS:
        assert np.array_equal(f1[n], f2[n]), n


@pytest.mark.parametrize("tile", [None, TWO_STEP])
def test_checkpoint_resume_bitwise(F, tile):
    b = boardgen.small_board(steps=300)
    b.dft_freqs = np.linspace(1e9, 8e9, 16)
    announce(f"checkpoint/resume tile={tile}")
    g, ids = F.grid_from_board(b, tile=tile)
    F.fdtd_step_n(g, 121)
    image = F.fdtd_save_state(g)
    F.fdtd_step_n(g, 179)
    a_probe = F.fdtd_get_probe(g, ids[0], 300)
    a_dft = F.fdtd_get_dft(g, ids[0])
    a_ez = F.fdtd_get_field(g, F.FDTD_EZ, (b.nz + 1, b.ny + 1, b.nx + 1))
    F.fdtd_destroy_grid(g)
    g2, ids2 = F.grid_from_board(b, tile=tile)
    F.fdtd_load_state(g2, image)
    assert F.fdtd_get_info(g2).step == 121
    F.fdtd_step_n(g2, 179)
    assert np.array_equal(F.fdtd_get_probe(g2, ids2[0], 300), a_probe)
    assert np.array_equal(F.fdtd_get_dft(g2, ids2[0]), a_dft)
    assert np.array_equal(F.fdtd_get_field(g2, F.FDTD_EZ, a_ez.shape), a_ez)
    F.fdtd_destroy_grid(g2)


def test_dft_and_probe_fft(F, orc):
    b = boardgen.small_board(steps=1500)
    b.dft_freqs = np.linspace(0.5e9, 12e9, 64)
    announce("dft + probe fft")
    ref = orc.run(b, threads=16)
    g, ids = F.grid_from_board(b)
    F.fdtd_step_n(g, 700)
    F.fdtd_step_n(g, 800)
    dft = np.stack([F.fdtd_get_dft(g, p) for p in ids])
    series = np.stack([F.fdtd_get_probe(g, p, b.steps) for p in ids]).astype(np.float64)
    n_fft = 2048
    X = np.stack([F.fdtd_probe_fft(g, p, n_fft) for p in ids])
    with pytest.raises(F.FdtdError):
        F.fdtd_probe_fft(g, 0, 1024)      # shorter than the run
    F.fdtd_destroy_grid(g)
    for p in range(len(ids)):
        assert rel_l2(dft[p], ref.dft[p]) <= 1e-4
        # the device FFT of the device series equals numpy's FFT of the same samples
        np.testing.assert_allclose(X[p], np.fft.rfft(series[p], n_fft),
                                   rtol=0, atol=1e-9 * np.abs(X[p]).max())
        # and the oracle's spectrum of its own series
        assert rel_l2(X[p], orc.probe_fft(ref.probes[p], n_fft)) <= 1e-4
        # the running DFT equals the direct sum over the stored samples
        t = (np.arange(b.steps) + 1) * ref.dt
        direct = (series[p][None, :] * np.exp(-2j * np.pi * np.outer(b.dft_freqs, t))).sum(1) * ref.dt
        assert rel_l2(dft[p], direct) <= 1e-12


def test_info_and_state_errors(F):
    b = boardgen.small_board(steps=10)
    g, ids = F.grid_from_board(b)
    info = F.fdtd_get_info(g)
    assert info.cells == b.nx * b.ny * b.nz and info.n_probes == 4 and info.n_sources == 1
    F.fdtd_step_n(g, 10)
    with pytest.raises(F.FdtdError) as ei:
        F.fdtd_step_n(g, 1)               # beyond max_steps
    assert ei.value.code == F.FDTD_ESTATE
    with pytest.raises(F.FdtdError) as ei:
        F.fdtd_add_probe(g, 5, 5, 5)      # after the first step
    assert ei.value.code == F.FDTD_ESTATE
    info = F.fdtd_get_info(g)
    assert info.step == 10 and info.step_bytes >= 49 * info.cells
    F.fdtd_destroy_grid(g)


def test_unstable_run_is_reported(F):
    """A source whose time integral exceeds the FP32 range drives Ez at the source
    edge to inf; the watchdog reports it at the next synchronising call."""
    b = boardgen.small_board(steps=300)
    b.sources[0].J0 = 3e38
    g, ids = F.grid_from_board(b)
    F.fdtd_step_n(g, 300)
    with pytest.raises(F.FdtdError) as ei:
        F.fdtd_synchronize(g)
    assert ei.value.code == F.FDTD_EUNSTABLE
    F.fdtd_destroy_grid(g)


def _small_variants(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        b = boardgen.variant_board(rng, i, steps=int(rng.integers(40, 160)),
                                   n_xy=(int(rng.integers(40, 130)), int(rng.integers(40, 130))),
                                   nz=int(rng.integers(24, 40)))
        for s in b.sources:
            s.t0, s.sigma = 30e-12, 8e-12
        b.dft_freqs = np.linspace(1e9, 20e9, 8)
        out.append(b)
    return out


@pytest.mark.parametrize("tile", [None, TWO_STEP])
def test_step_many_bitwise_equals_alone(F, tile):
    boards = _small_variants(11, 6)
    # one board with a wide (uint16) class map: many distinct permittivities
    rng = np.random.default_rng(3)
    boards[2].eps_r_cell[:] = rng.choice([1.0, 2.5, 4.4],
                                         size=boards[2].eps_r_cell.shape).astype(np.float32)
    announce(f"step_many over {len(boards)} boards, steps {[b.steps for b in boards]}")
    alone = []
    for b in boards:
        p, f, d, info = gpu_run(F, b)
        alone.append((p, f, d))
        if b is boards[2]:
            assert info.n_classes > 256
    handles = [F.grid_from_board(b, tile=tile) for b in boards]
    gs = [h for h, _ in handles]
    # two batched calls with uneven counts, then the remainders (the lead handle's
    # shape runs the batch)
    first = [b.steps // 3 for b in boards]
    F.fdtd_step_many(gs, first)
    F.fdtd_step_many(gs[::-1], [b.steps - f for b, f in zip(boards, first)][::-1])
    for (g, ids), b, (p, f, d) in zip(handles, boards, alone):
        pb = np.stack([F.fdtd_get_probe(g, q, b.steps) for q in ids])
        assert np.array_equal(pb, p)
        fb = gpu_fields(F, g, b)
        for n in FIELDS:
            assert np.array_equal(fb[n], f[n]), (b.name, n)
        db = np.stack([F.fdtd_get_dft(g, q) for q in ids])
        assert np.allclose(db, d, rtol=1e-12, atol=0)
        F.fdtd_destroy_grid(g)


@pytest.mark.parametrize("tile", [None, TWO_STEP])
def test_graph_replays_match_eager(F, tile):
    """Graph-replayed chunks (timing off) against eager launches (timing on), with
    synchronisation and host reads between every replay."""
    b = boardgen.small_board(steps=32 * 6)
    ga, ida = F.grid_from_board(b, tile=tile)
    gb, idb = F.grid_from_board(b, tile=tile)
    F.fdtd_set_timing(gb, True)            # forces plain launches
    shp = (b.nz + 1, b.ny + 1, b.nx + 1)
    for c in range(6):
        announce(f"graph chunk {c}")
        F.fdtd_step_n(ga, 32)
        F.fdtd_step_n(gb, 32)
        F.fdtd_synchronize(ga)
        F.fdtd_synchronize(gb)
        for comp in (F.FDTD_EX, F.FDTD_EZ, F.FDTD_HY, F.FDTD_BZ):
            assert np.array_equal(F.fdtd_get_field(ga, comp, shp), F.fdtd_get_field(gb, comp, shp))
    assert np.array_equal(F.fdtd_get_probe(ga, ida[0], b.steps), F.fdtd_get_probe(gb, idb[0], b.steps))
    F.fdtd_destroy_grid(ga)
    F.fdtd_destroy_grid(gb)


def test_estimate_bytes_bounds_allocation(F):
    for b in _small_variants(5, 3) + [boardgen.small_board()]:
        est = F.board_bytes(b)
        g, _ = F.grid_from_board(b)
        F.fdtd_step_n(g, 1)
        used = F.fdtd_get_info(g).device_bytes
        F.fdtd_destroy_grid(g)
        assert used <= est < 1.3 * used + (2 << 20), (b.name, used, est)


def test_step_many_plans_replay_one_graph(F):
    """Repeated batched calls with the same handles and step counts replay one
    captured graph (one plan, captured); the results, read back between the
    calls, stay bitwise those of each board stepped alone.  Changing the set of
    handles makes a new plan; the lead keeps at most four, and evicted plans
    leave later calls correct."""
    boards = _small_variants(23, 5)
    for b in boards:
        b.steps = 32 * 12
    alone = []
    for b in boards:
        p, f, _, _ = gpu_run(F, b)
        alone.append((p, f))
    hs = [F.grid_from_board(b) for b in boards]
    gs = [g for g, _ in hs]
    shp = [(b.nz + 1, b.ny + 1, b.nx + 1) for b in boards]
    try:
        for c in range(4):
            announce(f"step_many plan replay {c}")
            F.fdtd_step_many(gs, [32] * len(gs))
            info = F.fdtd_get_info(gs[0])
            assert info.batch_plans == 1 and info.batch_graphs == 1, (info.batch_plans, info.batch_graphs)
            for g, s in zip(gs, shp):           # host reads between replays
                F.fdtd_get_field(g, F.FDTD_EZ, s)
        # six other sets led by the same handle: new plans, at most four kept
        done = [128] * len(gs)
        for sub in ([0, 1], [0, 2], [0, 3], [0, 4], [0, 1, 2], [0, 3, 4]):
            F.fdtd_step_many([gs[q] for q in sub], [8] * len(sub))
            for q in sub:
                done[q] += 8
            assert F.fdtd_get_info(gs[0]).batch_plans <= 4
        rest = [b.steps - d for b, d in zip(boards, done)]
        F.fdtd_step_many(gs, rest)
        for (g, ids), b, (p, f) in zip(hs, boards, alone):
            assert F.fdtd_get_info(g).step == b.steps
            pb = np.stack([F.fdtd_get_probe(g, q, b.steps) for q in ids])
            assert np.array_equal(pb, p), b.name
            fb = gpu_fields(F, g, b)
            for n in FIELDS:
                assert np.array_equal(fb[n], f[n]), (b.name, n)
    finally:
        for g in gs:
            F.fdtd_destroy_grid(g)
