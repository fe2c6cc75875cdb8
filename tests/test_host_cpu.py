"""The library's host-side planning against independent expectations, without a GPU.

`tests/host/host_logic.cpp` compiles the library's host source into a small
program that prints what the library would hand to the device (it launches no
kernel): the work list of a field launch and the FP32 coefficient tables.

* Work lists (the tiled launches of every field step, the batched ones
  included): every plane of every tile of the board is stepped by exactly one
  entry; each XCD's run is a contiguous stretch of the row-major tiles, padded
  with idle entries at its end only; runs carry about equal plane counts; z pieces
  keep at least two planes.
* Coefficient tables (set-up, the Eq. 5 grading rounded once to FP32): every
  entry of every axis equals the value built in FP64 from the oracle's own
  (sigma, kappa) at that node or half node, rounded once.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import boardgen

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def host_logic(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("host") / "host_logic")
    subprocess.check_call([hipcc, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1008_2602_amd", "csrc"),
                           os.path.join(HERE, "host", "host_logic.cpp"), "-o", exe,
                           "-Wl,--unresolved-symbols=ignore-all"],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)

    def run(*args):
        out = subprocess.run([exe, *map(str, args)], check=True, capture_output=True, text=True).stdout
        return [line.split() for line in out.splitlines()]
    return run


WORK_CASES = [
    # nx, ny, nz, tile columns, owned rows, concurrent blocks per XCD
    (1048, 792, 88, 64, 11, 32),   # the large board, 64x14x2
    (444, 364, 60, 64, 11, 32),    # the realistic board
    (800, 800, 64, 64, 11, 32),    # the served large boards
    (1048, 99, 88, 64, 11, 32),    # one y-slab of the large board
    (80, 72, 37, 64, 5, 32),       # the small board, 64x8x2
    (48, 43, 30, 64, 3, 64),       # the Table 1 board, 64x6x2 (two blocks per compute unit)
    (48, 43, 30, 64, 14, 32),      # the same in a one-step 64x15 shape
    (300, 200, 40, 128, 6, 7),     # a 128-wide one-step shape, an odd slot count
    (130, 130, 40, 64, 11, 1),     # one block per XCD
]


@pytest.mark.parametrize("case", WORK_CASES, ids=lambda c: "x".join(map(str, c)))
def test_work_list_steps_every_tile_plane_once(host_logic, case):
    nx, ny, nz, tx, rows, slots = case
    ent = np.array(host_logic("worklist", *case), dtype=np.int64)
    assert ent.ndim == 2 and ent.shape[1] == 5 and len(ent) % 8 == 0
    cx, cy = -(-nx // tx), -(-ny // rows)
    L = len(ent) // 8
    seen = {}
    run_planes = []
    prev_last = -1
    for x in range(8):
        run = ent[x * L:(x + 1) * L]
        real = run[:, 0] >= 0
        n_real = int(real.sum())
        assert real[:n_real].all() and not real[n_real:].any(), "idle entries only at a run's end"
        run = run[:n_real]
        assert (run[:, 0] == 0).all()
        # the run's tiles, a contiguous stretch of the row-major order, after the previous run's
        idx = sorted(set((run[:, 2] * cx + run[:, 1]).tolist()))
        if idx:
            assert idx == list(range(idx[0], idx[-1] + 1))
            assert idx[0] == prev_last + 1
            prev_last = idx[-1]
        run_planes.append(int((run[:, 4] - run[:, 3]).sum()))
        for b, ix, iy, kb, ke in run.tolist():
            assert 0 <= ix < cx and 0 <= iy < cy and 0 <= kb < ke <= nz
            seen.setdefault((ix, iy), []).append((kb, ke))
    assert prev_last == cx * cy - 1
    assert set(seen) == {(ix, iy) for ix in range(cx) for iy in range(cy)}
    for spans in seen.values():
        spans.sort()
        assert spans[0][0] == 0 and spans[-1][1] == nz
        assert all(a[1] == b[0] for a, b in zip(spans, spans[1:])), spans
        if len(spans) > 1:
            assert all(ke - kb >= 2 for kb, ke in spans), spans
    # about equal work per XCD: within one tile's planes (plus the pieces' extra planes)
    W = cx * cy * nz
    assert max(abs(p - W / 8) for p in run_planes) <= nz + 16


def _table(host_logic, b, axis, dt):
    n = (b.nx, b.ny, b.nz)[axis]
    rows = host_logic("coefs", b.nx, b.ny, b.nz, repr(b.dx), repr(b.dy), repr(b.dz), *b.npml,
                      repr(b.pml_m), repr(b.pml_R), repr(b.pml_kappa_max), repr(dt), axis)
    t = np.array(rows, dtype=np.float64).astype(np.float32)
    assert t.shape == (12, n + 1)
    return t.reshape(6, 2, n + 1)


def _boards():
    t1 = boardgen.table1_board(steps=10)
    odd = boardgen.table1_board(steps=10)
    odd.npml = (6, 9, 0, 7, 8, 5)      # uneven depths, one bare wall
    odd.pml_m, odd.pml_R, odd.pml_kappa_max = 4.0, 1e-8, 5.0
    odd.dx, odd.dy, odd.dz = 1.5e-3, 0.8e-3, 0.25e-3
    return [t1, odd]


@pytest.mark.parametrize("bi", [0, 1], ids=["table1", "graded_kappa"])
def test_coefficient_tables_match_the_oracle_profiles(host_logic, oracle_mod, bi):
    b = _boards()[bi]
    eps0 = oracle_mod.constants()["eps0"]
    dt = oracle_mod.time_step(b)
    for axis in range(3):
        n = (b.nx, b.ny, b.nz)[axis]
        got = _table(host_logic, b, axis, dt)
        want = np.zeros_like(got)
        for half in (0, 1):
            for i in range(n + 1):
                s, k = oracle_mod.sigma_kappa(b, axis, i + 0.5 * half)
                q = s * dt / eps0
                ph = k + 0.5 * q
                want[:, half, i] = np.array([-q / ph, (k - 0.5 * q) / ph, 1.0 / ph, ph, q, k])
        # the half node past the far wall (i = n) feeds only components held at zero
        # there; the library clamps its depth to the slab, so it is left out
        got[:, 1, n] = want[:, 1, n]
        np.testing.assert_array_equal(got, want)
        if any(b.npml[2 * axis:2 * axis + 2]):
            assert (got[4] > 0).any()                 # the grading is there
