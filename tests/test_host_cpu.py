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
* Material boards' split between the plain two-step kernel and its material
  variants: from a map of the nodes that need the rebuilt coefficients or
  conduct, every tile plane runs exactly once, on the kind of kernel that a brute
  force over its footprint (columns i0-2 .. i0+65, rows j0-2 .. j0+13, planes
  k-2 .. k+1) asks for; planes moved to the per-plane variant are covered by its
  64x10 tiles over the whole board; a tile's pieces are maximal runs of one kind.
* One round of a batched call (`fdtd_step_many`): boards go in launch order by
  group (class width, material or not) and falling step count; every board runs
  exactly its steps (passes of the shape, then one single step or, for a
  material board, a node-pass step when the count is odd); every pass of a span
  steps every plane of every tile (or piece) of exactly the boards still running,
  and no other.
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


HY, HROWS = 14, 11      # the hybrid grid: 64 x 14 x 2 tiles own 11 rows
MROWS = 7               # the per-plane material variant: 64 x 10 x 2 tiles own 7 rows


def _need_maps():
    """(name, nx, ny, nz, need[k, j, i]) with bit 1: rebuilt PML coefficients,
    bit 2: a conducting edge."""
    out = []
    nx, ny, nz = 200, 120, 24
    n = np.zeros((nz + 1, ny + 1, nx + 1), np.uint8)
    out.append(("none", nx, ny, nz, n.copy()))
    # a dielectric slab running into an 8-cell x/y PML (eps_rw): rebuilt nodes in
    # the PML columns and rows of planes 9 .. 12, on a board wide enough that few
    # tiles hold them (the per-tile split)
    ex, ey = 640, 330
    e = np.zeros((nz + 1, ey + 1, ex + 1), np.uint8)
    pml = np.zeros((ey + 1, ex + 1), bool)
    pml[:, :8] = pml[:, -8:] = True
    pml[:8, :] = pml[-8:, :] = True
    e[9:13][:, pml] = 1
    out.append(("eps_rw_slab", ex, ey, nz, e))
    # a lossy layer filling planes 6 .. 9 and a resistive sheet on plane 15
    c = n.copy()
    c[6:10] = 2
    c[15, 20:100, 30:170] = 2
    out.append(("lossy_layer", nx, ny, nz, c))
    # rebuilt nodes filling planes 3 .. 4 (the per-plane split) and a few conducting edges
    f = n.copy()
    f[3:5] = 1
    f[18, 50, 60] = 2
    out.append(("filled_planes", nx, ny, nz, f))
    # scattered nodes of both kinds on a board with ragged tiles
    rng = np.random.default_rng(5)
    nx, ny, nz = 170, 93, 17
    r = np.zeros((nz + 1, ny + 1, nx + 1), np.uint8)
    for bit, count in ((1, 6), (2, 9)):
        for _ in range(count):
            r[rng.integers(0, nz + 1), rng.integers(0, ny + 1), rng.integers(0, nx + 1)] |= bit
    out.append(("scattered", nx, ny, nz, r))
    return out


def _expected_kinds(need, nx, ny, nz):
    """kind[ty, tx, k] of the hybrid grid by brute force: 1 if the footprint on
    planes k-2 .. k+1 holds a rebuilt node, else 2 if it holds a conducting edge,
    else 0."""
    cx, cy = -(-nx // 64), -(-ny // HROWS)
    kind = np.zeros((cy, cx, nz), np.int64)
    for ty in range(cy):
        for tx in range(cx):
            j0, i0 = ty * HROWS, tx * 64
            fp = need[:, max(0, j0 - 2):min(ny, j0 + HY - 1) + 1, max(0, i0 - 2):min(nx, i0 + 65) + 1]
            per_plane = np.bitwise_or.reduce(fp.reshape(nz + 1, -1), axis=1)
            for k in range(nz):
                m = np.bitwise_or.reduce(per_plane[max(0, k - 2):min(nz, k + 1) + 1])
                kind[ty, tx, k] = 1 if m & 1 else (2 if m & 2 else 0)
    return kind


@pytest.mark.parametrize("case", _need_maps(), ids=lambda c: c[0])
def test_material_split_runs_every_tile_plane_on_the_kind_its_footprint_needs(host_logic, tmp_path, case):
    name, nx, ny, nz, need = case
    path = tmp_path / "need.bin"
    need.tofile(path)
    lines = host_logic("matsplit", nx, ny, nz, path)
    assert lines[0][0] == "split"
    split, mat_ty = int(lines[0][1]), int(lines[0][3])
    pieces = [(l[0], *map(int, l[1:])) for l in lines[1:]]
    want = _expected_kinds(need, nx, ny, nz)
    cy, cx = want.shape[:2]
    any_r = (want == 1).any(axis=(0, 1))
    # the documented choice between the two ways of splitting rebuilt planes
    f_tile, f_plane = (want == 1).mean(), any_r.mean()
    per_plane = any_r.any() and (1 - f_plane) * 0.615 + f_plane * 0.82 < (1 - f_tile) * 0.615 + f_tile * 1.00
    assert split == (0 if not any_r.any() else 2 if per_plane else 1)
    assert mat_ty == (10 if split == 2 else 14)
    if name == "none":
        assert split == 0 and all(p[0] == "plain" for p in pieces)
    if name == "filled_planes":
        assert split == 2
    if name == "eps_rw_slab":
        assert split == 1
    got = np.full((cy, cx, nz), -1, np.int64)
    mt_cx, mt_cy = -(-nx // 64), -(-ny // MROWS)
    mt_seen = np.zeros((mt_cy, mt_cx, nz), np.int64)
    code = {"plain": 0, "rb": 1, "cd": 2}
    per_tile = {}
    for kind, tx, ty, kb, ke in pieces:
        assert 0 <= kb < ke <= nz
        if kind == "rb" and split == 2:
            assert 0 <= tx < mt_cx and 0 <= ty < mt_cy
            mt_seen[ty, tx, kb:ke] += 1
            continue
        assert 0 <= tx < cx and 0 <= ty < cy
        assert (got[ty, tx, kb:ke] == -1).all(), "a tile plane in two pieces"
        got[ty, tx, kb:ke] = code[kind]
        per_tile.setdefault((tx, ty), []).append((kb, ke, kind))
    if split == 2:
        # the rebuilt planes: every 64x10 tile once, and no hybrid piece there
        assert (mt_seen[:, :, any_r] == 1).all() and (mt_seen[:, :, ~any_r] == 0).all()
        assert (got[:, :, any_r] == -1).all()
        assert (got[:, :, ~any_r] == want[:, :, ~any_r]).all()
    else:
        assert (got == want).all()
    for spans in per_tile.values():
        spans.sort()
        assert all(a[2] != b[2] or a[1] != b[0] for a, b in zip(spans, spans[1:])), "runs not merged"


def _parse_plan(lines):
    order, spans, node_tails, adv = None, [], [], {}
    for l in lines:
        if l[0] == "order":
            order = [int(v) for v in l[1:]]
        elif l[0] == "span":
            spans.append(dict(w=int(l[1]), steps=int(l[2]), s0=int(l[3]), s1=int(l[4]), tail=l[5] == "1",
                              lists=[]))
        elif l[0] == "list":
            spans[-1]["lists"].append((int(l[1]), []))
        elif l[0] == "e":
            spans[-1]["lists"][-1][1].append(tuple(int(v) for v in l[1:]))
        elif l[0] == "node_tail":
            node_tails.append(tuple(int(v) for v in l[1:]))
        elif l[0] == "adv":
            adv[int(l[1])] = (int(l[2]), int(l[3]))
    return order, spans, node_tails, adv


def _tiles(nx, ny, nz, tx, rows):
    return {(ix, iy) for ix in range(-(-nx // tx)) for iy in range(-(-ny // rows))}


def _check_cover(entries, tiles, nz, what):
    seen = {}
    for ix, iy, kb, ke in entries:
        assert (ix, iy) in tiles, what
        seen.setdefault((ix, iy), []).append((kb, ke))
    assert set(seen) == tiles, what
    for spans in seen.values():
        spans.sort()
        assert spans[0][0] == 0 and spans[-1][1] == nz and all(a[1] == b[0] for a, b in zip(spans, spans[1:])), what


PLAN_CASES = [
    # lead shape (tx, ty, steps per pass); boards (nx, ny, nz, steps, material need map or None, wide)
    ("plain_mixed", (64, 14, 2), [(100, 80, 20, 7, None, 0), (150, 90, 30, 4, None, 0), (90, 70, 20, 5, None, 1)]),
    ("plain_many", (64, 8, 2), [(130, 120, 25, n, None, 0) for n in (6, 6, 3, 1, 0, 9)]),
    ("one_step", (64, 15, 1), [(200, 90, 22, 5, None, 0), (70, 60, 18, 2, None, 0)]),
    ("material", (64, 14, 2), [(200, 120, 24, 7, "lossy_layer", 0), (640, 330, 24, 6, "eps_rw_slab", 0),
                               (200, 120, 24, 3, "filled_planes", 1), (300, 100, 24, 5, None, 0),
                               (120, 100, 24, 4, None, 0)]),
]


@pytest.mark.parametrize("case", PLAN_CASES, ids=lambda c: c[0])
def test_batched_round_runs_every_board_its_steps_on_every_tile(host_logic, tmp_path, case):
    name, (tx, ty, per), boards = case
    maps = {m[0]: m for m in _need_maps()}
    spec, split = [], {}
    for h, (nx, ny, nz, n, need, wide) in enumerate(boards):
        path = "-"
        if need is not None:
            mname, mx, my, mz, arr = maps[need]
            assert (mx, my, mz) == (nx, ny, nz)
            path = str(tmp_path / f"need{h}.bin")
            arr.tofile(path)
            lines = host_logic("matsplit", nx, ny, nz, path)
            mat_ty = int(lines[0][3])
            split[h] = {k: {(int(l[1]), int(l[2]), int(l[3]), int(l[4])) for l in lines[1:] if l[0] == k}
                        for k in ("plain", "cd", "rb")}
            split[h]["mat_ty"] = mat_ty
        spec.append(f"{nx} {ny} {nz} {n} {1 if need else 0} {wide} {path}")
    (tmp_path / "spec.txt").write_text("\n".join(spec) + "\n")
    order, spans, node_tails, adv = _parse_plan(host_logic("plan", tx, ty, per, 256, tmp_path / "spec.txt"))
    ng = len(boards)
    assert sorted(order) == list(range(ng))
    group = [2 * (boards[h][4] is not None) + boards[h][5] for h in range(ng)]
    keys = [(group[h], -boards[h][3]) for h in order]
    assert keys == sorted(keys), "launch order: by group, then falling step count"
    done = [0] * ng
    per_of = [2 if boards[h][4] is not None else per for h in range(ng)]
    npass = [boards[h][3] // per_of[h] for h in range(ng)]
    for sp in spans:
        in_span = {}
        for kind, ents in sp["lists"]:
            for b, ix, iy, kb, ke in ents:
                if b < 0:
                    continue
                in_span.setdefault(order[b], {}).setdefault(kind, []).append((ix, iy, kb, ke))
        for h, by_kind in in_span.items():
            nx, ny, nz, n, need, wide = boards[h]
            assert sp["w"] == wide
            if sp["tail"]:
                assert need is None and per == 2 and n % 2 == 1
                _check_cover(by_kind[0], _tiles(nx, ny, nz, 64, 14), nz, (name, h, "tail"))
                done[h] += 1
                continue
            assert sp["steps"] == per_of[h]
            if need is None:
                assert set(by_kind) == {0}
                _check_cover(by_kind[0], _tiles(nx, ny, nz, tx, ty - 3 if per == 2 else ty - 1), nz, (name, h))
            else:
                # each kind's list steps the planes of the board's pieces of that
                # kind once (the work list may cut a piece into shorter ones)
                sh = split[h]

                def planes(pcs):
                    out = [(ix, iy, k) for ix, iy, kb, ke in pcs for k in range(kb, ke)]
                    assert len(out) == len(set(out)), (name, h, "a plane twice")
                    return set(out)
                rb_kind = 3 if sh["mat_ty"] == 14 else 4
                for kind, key in ((1, "plain"), (2, "cd"), (rb_kind, "rb")):
                    assert planes(by_kind.get(kind, [])) == planes(sh[key]), (name, h, key)
                assert not by_kind.get(7 - rb_kind)
            done[h] += (sp["s1"] - sp["s0"]) * sp["steps"]
        # the boards of a span are exactly those of its group still running through it
        if not sp["tail"]:
            want = {h for h in range(ng) if group[h] == group[next(iter(in_span))] and npass[h] >= sp["s1"]}
            assert set(in_span) == want, (name, sp["s0"], sp["s1"])
    for h, rel, flip in node_tails:
        assert boards[h][4] is not None and boards[h][3] % 2 == 1
        assert rel == npass[h] * 2 and flip == npass[h] % 2
        done[h] += 1
    assert done == [b[3] for b in boards]
    for b, h in enumerate(order):
        n = boards[h][3]
        assert adv[b] == (n, npass[h] + n % per_of[h])
