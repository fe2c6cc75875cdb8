"""Seeded synthetic power/ground-plane boards (inputs only).

This module produces the *inputs* of a solve and nothing else: grid sizes, cell
spacings, a per-cell relative permittivity map, a per-node PEC edge mask, the
positions and pulse parameters of current sources, probe positions, step counts
and DFT frequencies.  It holds none of the time-stepping arithmetic: no time step,
no PML profile, no update coefficient, no edge-permittivity average and no pulse
sample is computed here.  Both the FP64 oracle and the HIP library consume these
inputs and each derives everything else on its own.

Geometry follows the paper's model (Model section, Fig. 1): a PEC ground plane and
a PEC power plane with a dielectric slab between them, an air layer around the
board, and a uniaxial PML wrapping the domain whose outer wall is PEC.

Conventions shared by every consumer (they are data layout, not arithmetic):

* ``nx, ny, nz`` count cells including air and PML; nodes run ``0..n``.
* ``eps_r_cell`` has shape ``(nz, ny, nx)`` (x fastest), dtype float32; cell
  ``(i, j, k)`` spans ``[i, i+1] x [j, j+1] x [k, k+1]`` in cell units.
* ``pec_edge_mask`` has shape ``(nz+1, ny+1, nx+1)``, dtype uint8; at node
  ``(i, j, k)`` bit 0 marks the edge Ex(i+1/2, j, k), bit 1 Ey(i, j+1/2, k) and
  bit 2 Ez(i, j, k+1/2) as perfect electric conductor.
* A current source or probe at ``(i, j, k)`` sits on the Ez edge (i, j, k+1/2).
* PEC sheets have zero thickness and lie on a z node plane (the paper models the
  planes as PEC by zeroing the tangential Ex and Ey there).  Every Ex/Ey edge on
  the plane whose span lies inside the sheet's footprint, perimeter included,
  is marked.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

GAUSS = 0   # J0 * exp(-(t - t0)^2 / (2 sigma^2))
DGAUSS = 1  # J0 * ((t - t0) / tau) * exp(-((t - t0) / tau)^2)   (Eq. 8, read as a pulse)

PEC_EX = 1
PEC_EY = 2
PEC_EZ = 4


@dataclass
class Source:
    i: int
    j: int
    k: int
    waveform: int = GAUSS
    J0: float = 1.0e6          # A/m^2 (1 A/mm^2, Results section)
    t0: float = 120e-12        # s
    sigma: float = 30e-12      # s (standard deviation for GAUSS, tau for DGAUSS)
    R: float = 0.0             # > 0: resistive voltage source, J0 is then V0 in volts
                               # (an EMF raising node k+1 over node k, in series with R)


@dataclass
class Board:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    eps_r_cell: np.ndarray
    pec_edge_mask: np.ndarray
    npml: Tuple[int, int, int, int, int, int] = (8, 8, 8, 8, 8, 8)
    courant: float = 0.99
    dt: float = 0.0                  # 0 => courant x CFL limit
    pml_m: float = 3.0
    pml_R: float = 1e-6
    pml_kappa_max: float = 1.0
    # Eq. 2's eps_rw: True divides each PML sigma by the relative permittivity at
    # the field location; False takes eps_rw = 1 (the same wherever the PML is air)
    pml_eps_rw: bool = False
    # conductivity per cell in S/m (lossy dielectric), None = lossless; zero in PML slabs
    sigma_cell: Optional[np.ndarray] = None
    # surface resistance (ohm per square) of the PEC-marked Ex/Ey edges, which then
    # are resistive sheets instead of perfect conductors; 0 = perfect conductors
    sheet_R: float = 0.0
    sources: List[Source] = field(default_factory=list)
    probes: List[Tuple[int, int, int]] = field(default_factory=list)
    steps: int = 1000
    dft_freqs: Optional[np.ndarray] = None
    # (k, frequencies in Hz): running DFT of Ez(i, j, k+1/2) over the whole plane k
    plane_dft: Optional[Tuple[int, np.ndarray]] = None
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def with_steps(self, steps: int) -> "Board":
        return dataclasses.replace(self, steps=int(steps))

    def check(self) -> None:
        """Shape and range checks of the inputs (no physics)."""
        assert self.eps_r_cell.shape == (self.nz, self.ny, self.nx)
        assert self.eps_r_cell.dtype == np.float32
        assert self.pec_edge_mask.shape == (self.nz + 1, self.ny + 1, self.nx + 1)
        assert self.pec_edge_mask.dtype == np.uint8
        for s in self.sources:
            assert 0 <= s.i <= self.nx and 0 <= s.j <= self.ny and 0 <= s.k < self.nz
        for (i, j, k) in self.probes:
            assert 0 <= i <= self.nx and 0 <= j <= self.ny and 0 <= k < self.nz


# ----------------------------------------------------------------------------
# rasterising helpers
# ----------------------------------------------------------------------------

def air(nx: int, ny: int, nz: int) -> Tuple[np.ndarray, np.ndarray]:
    return (np.ones((nz, ny, nx), np.float32),
            np.zeros((nz + 1, ny + 1, nx + 1), np.uint8))


def fill_box(eps: np.ndarray, i0: int, i1: int, j0: int, j1: int, k0: int, k1: int,
             eps_r: float) -> None:
    """Set cells [i0,i1) x [j0,j1) x [k0,k1) to eps_r."""
    eps[k0:k1, j0:j1, i0:i1] = np.float32(eps_r)


def pec_sheet(mask: np.ndarray, k: int, i0: int, i1: int, j0: int, j1: int) -> None:
    """Zero-thickness PEC rectangle on node plane k covering [i0,i1] x [j0,j1].

    Ex(i+1/2, j, k) is inside when i0 <= i < i1 and j0 <= j <= j1; Ey(i, j+1/2, k)
    when i0 <= i <= i1 and j0 <= j < j1 (perimeter edges included)."""
    mask[k, j0:j1 + 1, i0:i1] |= PEC_EX
    mask[k, j0:j1, i0:i1 + 1] |= PEC_EY


def cavity_box(nx: int, ny: int, nz: int, dx: float, dy: float, dz: float,
               eps_r: float, steps: int, name: str = "pec-cavity") -> Board:
    """Homogeneous box closed by the outer PEC wall on all six faces; no PML."""
    eps, mask = air(nx, ny, nz)
    eps[:] = np.float32(eps_r)
    return Board(name=name, nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz,
                 eps_r_cell=eps, pec_edge_mask=mask, npml=(0, 0, 0, 0, 0, 0),
                 steps=steps)


def plane_stack(name: str, board_cells: Tuple[int, int], diel_cells: int,
                air_xy: int, pml_xy: int, air_z_lo: int, air_z_hi: int, pml_z: int,
                dx: float, dy: float, dz: float, eps_r: float
                ) -> Tuple[Board, dict]:
    """Two full PEC planes with a dielectric slab between, air around, PML outside.

    Returns the board (no sources/probes yet) and a layout dict with the board
    footprint ``(bi0, bi1, bj0, bj1)`` in cells and the plane node indices."""
    bx, by = board_cells
    nx = bx + 2 * (air_xy + pml_xy)
    ny = by + 2 * (air_xy + pml_xy)
    nz = diel_cells + air_z_lo + air_z_hi + 2 * pml_z
    eps, mask = air(nx, ny, nz)
    bi0 = pml_xy + air_xy
    bj0 = pml_xy + air_xy
    bi1, bj1 = bi0 + bx, bj0 + by
    kg = pml_z + air_z_lo
    kt = kg + diel_cells
    fill_box(eps, bi0, bi1, bj0, bj1, kg, kt, eps_r)
    pec_sheet(mask, kg, bi0, bi1, bj0, bj1)
    pec_sheet(mask, kt, bi0, bi1, bj0, bj1)
    b = Board(name=name, nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz,
              eps_r_cell=eps, pec_edge_mask=mask,
              npml=(pml_xy, pml_xy, pml_xy, pml_xy, pml_z, pml_z))
    lay = dict(bi0=bi0, bi1=bi1, bj0=bj0, bj1=bj1, kg=kg, kt=kt)
    return b, lay


def _interior_xy(rng: np.random.Generator, lay: dict, n: int, margin: int = 1
                 ) -> List[Tuple[int, int]]:
    """n distinct (i, j) nodes strictly inside the board footprint."""
    out: List[Tuple[int, int]] = []
    seen = set()
    while len(out) < n:
        i = int(rng.integers(lay["bi0"] + margin, lay["bi1"] - margin + 1))
        j = int(rng.integers(lay["bj0"] + margin, lay["bj1"] - margin + 1))
        if (i, j) not in seen:
            seen.add((i, j))
            out.append((i, j))
    return out


# ----------------------------------------------------------------------------
# the five workload configurations
# ----------------------------------------------------------------------------

def small_board(seed: int = 1001, steps: int = 3000) -> Board:
    """48 x 40 mm board, 1 mm in-plane cells, 0.2 mm dz, 1.0 mm FR4 (eps_r 4.4)
    between two PEC sheets; 8 air + 8 PML cells on every side; grid 80 x 72 x 37;
    Gaussian Jz (t0 = 120 ps, sigma = 30 ps) at a seeded dielectric edge; four Ez
    probes on the first Ez row above the ground sheet; 3000 steps at 0.99 Courant."""
    rng = np.random.default_rng(seed)
    b, lay = plane_stack("small-48x40mm", (48, 40), 5, 8, 8, 8, 8, 8,
                         1e-3, 1e-3, 0.2e-3, 4.4)
    (si, sj), *pr = _interior_xy(rng, lay, 5)
    sk = int(rng.integers(lay["kg"], lay["kt"]))
    b.sources = [Source(si, sj, sk, GAUSS, 1.0e6, 120e-12, 30e-12)]
    b.probes = [(i, j, lay["kg"]) for (i, j) in pr]
    b.steps = steps
    b.meta = dict(layout=lay, seed=seed)
    b.check()
    return b


def realistic_board(seed: int = 1002, steps: int = 20000) -> Board:
    """200 x 160 mm board, 0.5 mm in-plane cells, 0.1 mm dz, 1.6 mm FR4 (eps_r 4.4);
    12-cell air gap, 10-cell PML; grid 444 x 364 x 60; Gaussian Jz with
    sigma = 20 ps (t0 = 4 sigma); 16 probes; 20000 steps."""
    rng = np.random.default_rng(seed)
    b, lay = plane_stack("realistic-200x160mm", (400, 320), 16, 12, 10, 12, 12, 10,
                         0.5e-3, 0.5e-3, 0.1e-3, 4.4)
    (si, sj), *pr = _interior_xy(rng, lay, 17)
    sk = int(rng.integers(lay["kg"], lay["kt"]))
    b.sources = [Source(si, sj, sk, GAUSS, 1.0e6, 80e-12, 20e-12)]
    b.probes = [(i, j, lay["kg"]) for (i, j) in pr]
    b.steps = steps
    b.meta = dict(layout=lay, seed=seed)
    b.check()
    return b


def _disjoint_islands(rng: np.random.Generator, bx: int, by: int
                      ) -> List[Tuple[int, int, int, int]]:
    """Two disjoint rectangles (in board cells), each spanning U(0.3, 0.6) of the
    board per axis, separated by at least 2 cells."""
    for _ in range(10000):
        rects = []
        for _r in range(2):
            w = int(round(rng.uniform(0.3, 0.6) * bx))
            h = int(round(rng.uniform(0.3, 0.6) * by))
            x0 = int(rng.integers(0, bx - w + 1))
            y0 = int(rng.integers(0, by - h + 1))
            rects.append((x0, x0 + w, y0, y0 + h))
        (a0, a1, b0, b1), (c0, c1, d0, d1) = rects
        if a1 + 2 <= c0 or c1 + 2 <= a0 or b1 + 2 <= d0 or d1 + 2 <= b0:
            return rects
    raise RuntimeError("could not place two disjoint islands")


def large_board(seed: int = 1003, steps: int = 10000) -> Board:
    """Large-board HBM stress case: 1024 x 768 x 64 interior cells plus a 12-cell
    PML on every face (grid 1048 x 792 x 88), dx = dy = 0.2 mm, dz = 0.1 mm,
    eps_r 4.2 slab of 16 cells centred in z (24 air cells above and below), a
    12-cell in-plane air gap (board 1000 x 744 cells), a full ground sheet and a
    power layer made of two seeded disjoint PEC islands; eight seeded Gaussian Jz
    sources under the islands (sigma = 20 ps, t0 = 4 sigma + U[0, 400) ps); 64
    probes; 10000 steps; DFT at (q+1) * 10 GHz / 256, q = 0..255."""
    rng = np.random.default_rng(seed)
    bx, by = 1000, 744
    nx, ny, nz = 1048, 792, 88
    eps, mask = air(nx, ny, nz)
    bi0 = bj0 = 24
    kg, kt = 36, 52
    fill_box(eps, bi0, bi0 + bx, bj0, bj0 + by, kg, kt, 4.2)
    pec_sheet(mask, kg, bi0, bi0 + bx, bj0, bj0 + by)
    islands = _disjoint_islands(rng, bx, by)
    for (x0, x1, y0, y1) in islands:
        pec_sheet(mask, kt, bi0 + x0, bi0 + x1, bj0 + y0, bj0 + y1)
    sources = []
    for (x0, x1, y0, y1) in islands:
        for _ in range(4):
            i = int(rng.integers(bi0 + x0 + 1, bi0 + x1))
            j = int(rng.integers(bj0 + y0 + 1, bj0 + y1))
            k = int(rng.integers(kg, kt))
            delay = float(rng.uniform(0.0, 400e-12))
            sources.append(Source(i, j, k, GAUSS, 1.0e6, 80e-12 + delay, 20e-12))
    lay = dict(bi0=bi0, bi1=bi0 + bx, bj0=bj0, bj1=bj0 + by, kg=kg, kt=kt,
               islands=islands)
    probes = [(i, j, kg) for (i, j) in _interior_xy(rng, lay, 64)]
    b = Board(name="large-1048x792x88", nx=nx, ny=ny, nz=nz,
              dx=0.2e-3, dy=0.2e-3, dz=0.1e-3, eps_r_cell=eps, pec_edge_mask=mask,
              npml=(12, 12, 12, 12, 12, 12), sources=sources, probes=probes,
              steps=steps,
              dft_freqs=np.array([(q + 1) * 10e9 / 256 for q in range(256)]),
              meta=dict(layout=lay, seed=seed))
    b.check()
    return b


def y_slab(board: Board, j0: int, j1: int) -> Board:
    """Cells j0 <= j < j1 of ``board`` as a board of its own: the y-slab that one
    rank of a slab decomposition along y would own.  A cut face (j0 > 0 or
    j1 < ny) gets no PML; with no halo exchanged it is an outer PEC wall, so
    the slab is the rank's share with its halo stubbed to zero.  Sources and
    probes strictly between the cut faces are kept (on a face an Ez edge is
    tangential and stays zero)."""
    assert 0 <= j0 < j1 <= board.ny
    npml = list(board.npml)
    if j0 > 0:
        npml[2] = 0
    if j1 < board.ny:
        npml[3] = 0
    assert npml[2] + npml[3] < j1 - j0
    def keep(j):
        return (j > j0 or j0 == 0) and (j < j1 or j1 == board.ny)

    b = dataclasses.replace(
        board, name=f"{board.name}-y{j0}-{j1}", ny=j1 - j0,
        eps_r_cell=np.ascontiguousarray(board.eps_r_cell[:, j0:j1, :]),
        pec_edge_mask=np.ascontiguousarray(board.pec_edge_mask[:, j0:j1 + 1, :]),
        sigma_cell=(None if board.sigma_cell is None
                    else np.ascontiguousarray(board.sigma_cell[:, j0:j1, :])),
        npml=tuple(npml),
        sources=[dataclasses.replace(s, j=s.j - j0) for s in board.sources if keep(s.j)],
        probes=[(i, j - j0, k) for (i, j, k) in board.probes if keep(j)],
        plane_dft=board.plane_dft,
        meta=dict(board.meta, slab=(j0, j1)))
    b.check()
    return b


def large_board_shard(rank: int, nranks: int = 8, seed: int = 1003, steps: int = 10000) -> Board:
    """Rank ``rank``'s share of the large board split into ``nranks`` equal y-slabs
    (792 / 8 = 99 cells each: grid 1048 x 99 x 88), halo stubbed (see y_slab).
    Only the first and last slab keep a y-PML face."""
    full = large_board(seed, steps)
    assert full.ny % nranks == 0 and 0 <= rank < nranks
    h = full.ny // nranks
    return y_slab(full, rank * h, (rank + 1) * h)


def variant_board(rng: np.random.Generator, idx: int, steps: int = 8000,
                  n_xy: Optional[Tuple[int, int]] = None,
                  nz: Optional[int] = None) -> Board:
    """One board of the batched-variant distribution: totals Nx, Ny ~ U{100..600}
    and Nz ~ U{24..64} including PML; dx = dy = 0.5 mm; 8-cell PML and 8-cell air
    gap in-plane; dielectric thickness U(0.2, 1.6) mm always 4 cells thick (so
    dz = thickness / 4); eps_r ~ U(3.5, 4.8); the rest of z is air split evenly
    around the slab; 8-cell PML in z; seeded source and four probes; sigma = 20 ps,
    t0 = 80 ps."""
    NX = int(rng.integers(100, 601)) if n_xy is None else n_xy[0]
    NY = int(rng.integers(100, 601)) if n_xy is None else n_xy[1]
    NZ = int(rng.integers(24, 65)) if nz is None else nz
    thick = float(rng.uniform(0.2e-3, 1.6e-3))
    eps_r = float(rng.uniform(3.5, 4.8))
    air_z = NZ - 4 - 16
    air_lo = air_z // 2
    air_hi = air_z - air_lo
    b, lay = plane_stack(f"variant{idx}-{NX}x{NY}x{NZ}", (NX - 32, NY - 32), 4,
                         8, 8, air_lo, air_hi, 8, 0.5e-3, 0.5e-3, thick / 4, eps_r)
    assert (b.nx, b.ny, b.nz) == (NX, NY, NZ)
    (si, sj), *pr = _interior_xy(rng, lay, 5)
    sk = int(rng.integers(lay["kg"], lay["kt"]))
    b.sources = [Source(si, sj, sk, GAUSS, 1.0e6, 80e-12, 20e-12)]
    b.probes = [(i, j, lay["kg"]) for (i, j) in pr]
    b.steps = steps
    b.meta = dict(layout=lay, thickness=thick, eps_r=eps_r)
    b.check()
    return b


def variant_batch(seed: int = 1004, n_boards: int = 64, steps: int = 8000) -> List[Board]:
    """64 uneven board variants for one batched launch (see variant_board)."""
    rng = np.random.default_rng(seed)
    return [variant_board(rng, i, steps) for i in range(n_boards)]


@dataclass
class Request:
    rid: int
    arrival_s: float
    board: Board


def served_requests(rate_per_s: float, seed: int = 1005, n_requests: int = 512,
                    steps: int = 8000, large_frac: float = 0.05,
                    large_xyz: Tuple[int, int, int] = (800, 800, 64)) -> List[Request]:
    """Served solves: Poisson arrivals at ``rate_per_s`` of boards drawn from the
    batched-variant distribution plus ``large_frac`` large boards."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        if rng.uniform() < large_frac:
            b = variant_board(rng, r, steps, n_xy=large_xyz[:2], nz=large_xyz[2])
        else:
            b = variant_board(rng, r, steps)
        out.append(Request(r, t, b))
    return out


# ----------------------------------------------------------------------------
# small boards used by tests
# ----------------------------------------------------------------------------

def table1_board(steps: int = 30000, air_cells: int = 6, pml_cells: int = 8,
                 source: str = "current") -> Board:
    """The geometry of the paper's Table 1 run: a 40 x 30 x 0.8 mm board with
    2 / 2 / 0.4 mm cells (20 x 15 x 2 board cells), dt = 1 ps, a source at one
    board corner and an Ez probe at the opposite corner, both on the first Ez row
    above the ground plane.  The paper does not state eps_r, the air gap or the
    PML depth; eps_r = 4.0 reproduces its predicted column.

    source "current": a DGAUSS current density of 1 A/mm^2 on the corner edge.
    source "resistive": the paper's resistive voltage source, V0 = 5 V and
    R = 10 ohm with the same DGAUSS shape, as a lumped element on that one edge
    (the other Ez edge of the two-cell gap stays dielectric, so the element sees
    the board through that edge's capacitance)."""
    b, lay = plane_stack("table1-40x30mm", (20, 15), 2, air_cells, pml_cells,
                         air_cells, air_cells, pml_cells, 2e-3, 2e-3, 0.4e-3, 4.0)
    b.dt = 1e-12
    si, sj, kg = lay["bi0"] + 1, lay["bj0"] + 1, lay["kg"]
    if source == "current":
        b.sources = [Source(si, sj, kg, DGAUSS, 1.0e6, 100e-12, 50e-12)]
    elif source == "resistive":
        b.sources = [Source(si, sj, kg, DGAUSS, 5.0, 100e-12, 50e-12, R=10.0)]
    else:
        raise ValueError(source)
    b.probes = [(lay["bi1"] - 1, lay["bj1"] - 1, kg)]
    b.steps = steps
    b.meta = dict(layout=lay, source=source)
    b.check()
    return b


def fig3_board(steps: int = 1000, pml_xy: int = 8, air_z: int = 6, pml_z: int = 8,
               eps_rw: bool = True) -> Board:
    """The paper's Fig. 3 case: the 100 x 60 x 0.8 mm board (2 / 2 / 0.4 mm cells,
    eps_r 4.0 as in Table 1) whose edges run into the UPML: the dielectric and both
    PEC planes continue through the x/y PML slabs to the outer wall, with air and
    PML above and below.  dt = 1 ps; the DGAUSS current source (1 A/mm^2, t0 =
    100 ps, tau = 50 ps) sits at the board centre on the first Ez row above the
    ground plane, with ground-row Ez probes at the centre offset by one cell, at
    10 mm and 20 mm along x, and one cell before the x PML.  eps_rw selects
    Eq. 2's sigma / eps_rw in the PML (the dielectric reaches it here)."""
    bx, by, nd = 50, 30, 2
    nx, ny = bx + 2 * pml_xy, by + 2 * pml_xy
    nz = nd + 2 * air_z + 2 * pml_z
    eps, mask = air(nx, ny, nz)
    kg = pml_z + air_z
    kt = kg + nd
    fill_box(eps, 0, nx, 0, ny, kg, kt, 4.0)
    pec_sheet(mask, kg, 0, nx, 0, ny)
    pec_sheet(mask, kt, 0, nx, 0, ny)
    b = Board(name="fig3-100x60mm", nx=nx, ny=ny, nz=nz, dx=2e-3, dy=2e-3, dz=0.4e-3,
              eps_r_cell=eps, pec_edge_mask=mask,
              npml=(pml_xy, pml_xy, pml_xy, pml_xy, pml_z, pml_z), pml_eps_rw=eps_rw)
    b.dt = 1e-12
    ci, cj = nx // 2, ny // 2
    b.sources = [Source(ci, cj, kg, DGAUSS, 1.0e6, 100e-12, 50e-12)]
    b.probes = [(ci + 1, cj, kg), (ci + 5, cj, kg), (ci + 10, cj, kg), (nx - pml_xy - 1, cj, kg)]
    b.steps = steps
    b.meta = dict(layout=dict(kg=kg, kt=kt, ci=ci, cj=cj))
    b.check()
    return b


def zconv_board(n_diel: int, steps: int = 4000, n_diel_max: int = 15, air_xy: int = 6,
                pml: int = 8) -> Board:
    """The z-convergence study of the Results section: the Table 1 board
    (40 x 30 mm, 2 mm in-plane cells, eps_r 4.0) with its 0.8 mm dielectric cut
    into n_diel z cells (dz = 0.8 mm / n_diel) and 1.6 mm of air above and below
    (2 n_diel cells), 8 PML cells.  The DGAUSS current filament (1 A/mm^2,
    t0 = 100 ps, tau = 50 ps) spans the whole gap at the board centre, so the
    injected current does not depend on dz; Ez is probed on the ground-plane row
    (the first Ez edge above the ground sheet) at the centre, off-centre and near
    a corner.  Every member of the family uses the time step of the finest grid
    (n_diel_max cells, 0.99 x Eq. 7), so their sample times coincide."""
    assert 1 <= n_diel <= n_diel_max
    dz = 0.8e-3 / n_diel
    b, lay = plane_stack(f"zconv-{n_diel}", (20, 15), n_diel, air_xy, pml,
                         2 * n_diel, 2 * n_diel, pml, 2e-3, 2e-3, dz, 4.0)
    c0 = 299792458.0
    dzf = 0.8e-3 / n_diel_max
    b.dt = 0.99 / (c0 * np.sqrt(2.0 / (2e-3) ** 2 + 1.0 / dzf ** 2))
    ci, cj = (lay["bi0"] + lay["bi1"]) // 2, (lay["bj0"] + lay["bj1"]) // 2
    b.sources = [Source(ci, cj, k, DGAUSS, 1.0e6, 100e-12, 50e-12)
                 for k in range(lay["kg"], lay["kt"])]
    kg = lay["kg"]
    b.probes = [(ci, cj, kg), (ci + 5, cj + 3, kg), (lay["bi1"] - 1, lay["bj1"] - 1, kg)]
    b.steps = steps
    b.meta = dict(layout=lay, n_diel=n_diel)
    b.check()
    return b


def lossy_dielectric(board: Board, tan_delta: float, f_ref: float = 5e9) -> Board:
    """Give the board's dielectric (cells with eps_r > 1) a loss tangent tan_delta
    at f_ref: conductivity sigma = 2 pi f_ref eps0 eps_r tan_delta per cell, cells
    in the PML slabs left lossless."""
    eps0 = 8.854187817620389e-12
    sig = np.where(board.eps_r_cell > 1.0,
                   2 * np.pi * f_ref * eps0 * board.eps_r_cell * tan_delta, 0.0).astype(np.float32)
    p = board.npml
    inner = np.zeros(sig.shape, bool)
    inner[p[4]:board.nz - p[5], p[2]:board.ny - p[3], p[0]:board.nx - p[1]] = True
    sig[~inner] = 0.0
    board.sigma_cell = sig
    return board


def conductor_loss(board: Board, sigma_metal: float = 5.8e7, f_ref: float = 5e9) -> Board:
    """Give the board's PEC sheets (the power and ground planes) the surface
    resistance of a good conductor of conductivity sigma_metal at f_ref,
    sqrt(pi f_ref mu0 / sigma_metal) ohms per square (copper at 5 GHz: 18.4
    milliohms per square), as one frequency-independent sheet resistance."""
    mu0 = 4e-7 * np.pi
    board.sheet_R = float(np.sqrt(np.pi * f_ref * mu0 / sigma_metal))
    return board


def random_tiny(seed: int, nx: int = 10, ny: int = 9, nz: int = 8, npml: int = 2,
                steps: int = 40) -> Board:
    """A tiny board with every feature: PML on all faces (may differ per face),
    a random eps_r block, a PEC sheet, two sources and three probes."""
    rng = np.random.default_rng(seed)
    eps, mask = air(nx, ny, nz)
    i0 = int(rng.integers(1, nx // 2)); i1 = int(rng.integers(nx // 2 + 1, nx))
    j0 = int(rng.integers(1, ny // 2)); j1 = int(rng.integers(ny // 2 + 1, ny))
    k0 = int(rng.integers(1, nz // 2)); k1 = int(rng.integers(nz // 2 + 1, nz))
    fill_box(eps, i0, i1, j0, j1, k0, k1, float(rng.uniform(2.0, 6.0)))
    pec_sheet(mask, k0, i0, i1, j0, j1)
    pml = tuple(int(x) for x in rng.integers(max(npml - 1, 0), npml + 2, size=6))
    srcs = [Source(int(rng.integers(i0 + 1, i1)), int(rng.integers(j0 + 1, j1)),
                   int(rng.integers(k0, k1)), w, 1.0e6, float(rng.uniform(5e-12, 20e-12)),
                   float(rng.uniform(2e-12, 5e-12))) for w in (GAUSS, DGAUSS)]
    probes = [(int(rng.integers(1, nx)), int(rng.integers(1, ny)), int(rng.integers(0, nz)))
              for _ in range(3)]
    b = Board(name=f"tiny{seed}", nx=nx, ny=ny, nz=nz, dx=1e-3, dy=1.2e-3, dz=0.5e-3,
              eps_r_cell=eps, pec_edge_mask=mask, npml=pml, sources=srcs,
              probes=probes, steps=steps,
              dft_freqs=np.array([1e9, 5e9, 20e9, 40e9]))
    b.check()
    return b


def random_fields(shape_nodes: Tuple[int, int, int], seed: int, count: int = 12,
                  scale: float = 1.0) -> List[np.ndarray]:
    """``count`` seeded standard-normal arrays of the padded node shape
    ``(nz+1, ny+1, nx+1)``; used as arbitrary initial states."""
    rng = np.random.default_rng(seed)
    return [(scale * rng.standard_normal(shape_nodes)).astype(np.float64)
            for _ in range(count)]
