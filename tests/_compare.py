"""Field comparison of the HIP path's state with the oracle's (no method
arithmetic): whole-array, element-wise and per-region bounds.

Regions checked for every array:
  * the 27 PML classes of a node (below, inside or above the PML slab on each
    axis): the interior, the 6 face slabs, the 12 edges and the 8 corners;
  * every node plane k, row j and column i on its own (tile seams in x and y,
    z-piece seams, the far-wall and low-wall layers);
  * the rims of the PEC sheets: nodes within two cells (in-plane) of a sheet's
    outline, on the sheet plane and the planes next to it.
A region's error is its relative L2.  Its denominator is at least
``region_floor`` times the region's share of the whole array's norm (the whole
norm times the square root of the region's fraction of the nodes), so a region
whose field is far below the array's typical level (one the wave has barely
reached, or that FP32 rounding near much stronger neighbours dominates) is held
to an absolute bound at that level instead of a relative one.
"""
import numpy as np

FIELDS = ("ex", "ey", "ez", "hx", "hy", "hz", "ddx", "ddy", "ddz", "bbx", "bby", "bbz")
_AXIS = {"ddx": "x", "ddy": "y", "ddz": "z", "bbx": "x", "bby": "y", "bbz": "z"}

# SI value -> E-like units (V/m): H by eta0, D by 1/eps0, B by c0
_EPS0 = 8.854187817620389e-12
_MU0 = 4e-7 * np.pi
TO_E_UNITS = {"e": 1.0, "h": np.sqrt(_MU0 / _EPS0), "d": 1.0 / _EPS0, "b": 1.0 / np.sqrt(_MU0 * _EPS0)}


def _pml_flags(n, lo, hi):
    return np.array([(i < lo) or (hi > 0 and i >= n - hi) for i in range(n + 1)])


def aux_masks(board):
    """Where the library keeps D/B: the component's own or cyclic-next axis is in
    a PML slab (elsewhere those auxiliaries never influence E or H)."""
    nx, ny, nz = board.nx, board.ny, board.nz
    p = board.npml
    X = _pml_flags(nx, p[0], p[1])[None, None, :]
    Y = _pml_flags(ny, p[2], p[3])[None, :, None]
    Z = _pml_flags(nz, p[4], p[5])[:, None, None]
    shp = (nz + 1, ny + 1, nx + 1)
    return {"x": np.broadcast_to(X | Y, shp), "y": np.broadcast_to(Y | Z, shp),
            "z": np.broadcast_to(Z | X, shp)}


def _axis_segments(n, lo, hi):
    """(name, slice) of the non-empty PML classes of the nodes 0..n on one axis."""
    segs = []
    a, b = lo, max(lo, n - hi if hi > 0 else n + 1)
    for name, s in (("lo", slice(0, a)), ("mid", slice(a, b)), ("hi", slice(b, n + 1))):
        if s.stop > s.start:
            segs.append((name, s))
    return segs


def rim_mask(board, width=2):
    """Boolean (nz+1, ny+1, nx+1) mask of the nodes within ``width`` cells
    in-plane of the outline of a PEC sheet, on the sheet's plane and the planes
    above and below it."""
    pec = board.pec_edge_mask
    out = np.zeros(pec.shape, bool)
    sheet_planes = np.nonzero((pec & 3).any(axis=(1, 2)))[0]
    for k in sheet_planes:
        m = (pec[k] & 3) != 0
        edge = np.zeros_like(m)
        edge[:, 1:] |= m[:, 1:] != m[:, :-1]
        edge[:, :-1] |= m[:, 1:] != m[:, :-1]
        edge[1:, :] |= m[1:, :] != m[:-1, :]
        edge[:-1, :] |= m[1:, :] != m[:-1, :]
        for _ in range(width):
            grown = edge.copy()
            grown[:, 1:] |= edge[:, :-1]
            grown[:, :-1] |= edge[:, 1:]
            grown[1:, :] |= edge[:-1, :]
            grown[:-1, :] |= edge[1:, :]
            edge = grown
        for kk in range(max(0, k - 1), min(pec.shape[0], k + 2)):
            out[kk] |= edge
    return out


def field_errors(r, g, board, floor=0.0, floor_max=0.0, region_floor=0.5, rim=None):
    """Errors of one array: (whole relative L2, element-wise max error over the
    largest reference value, worst region as (relative L2, region name)).
    ``floor`` and ``floor_max`` bound the whole-array norm and the largest
    reference value from below (absolute units of the array)."""
    d = g - r
    den = max(float(np.linalg.norm(r)), floor)
    whole = float(np.linalg.norm(d)) / den
    amax = max(float(np.abs(r).max()), floor_max)
    elem = float(np.abs(d).max()) / amax
    d2 = d * d
    r2 = r * r
    per_node = region_floor * den / np.sqrt(r.size)    # floor of a region of one node
    worst = (0.0, "")

    def upd(num2, den2, name, count):
        nonlocal worst
        e = float(np.sqrt(num2)) / max(float(np.sqrt(den2)), per_node * np.sqrt(count))
        if e > worst[0]:
            worst = (e, name)

    p = board.npml
    zs = _axis_segments(board.nz, p[4], p[5])
    ys = _axis_segments(board.ny, p[2], p[3])
    xs = _axis_segments(board.nx, p[0], p[1])
    for zn, zsl in zs:
        for yn, ysl in ys:
            for xn, xsl in xs:
                blk = d2[zsl, ysl, xsl]
                upd(blk.sum(), r2[zsl, ysl, xsl].sum(), f"pml z{zn} y{yn} x{xn}", blk.size)
    for ax, label in ((0, "plane k"), (1, "row j"), (2, "column i")):
        other = tuple(a for a in range(3) if a != ax)
        nums = d2.sum(axis=other)
        dens = r2.sum(axis=other)
        count = r.size // r.shape[ax]
        e = np.sqrt(nums) / np.maximum(np.sqrt(dens), per_node * np.sqrt(count))
        q = int(np.argmax(e))
        if e[q] > worst[0]:
            worst = (float(e[q]), f"{label}={q}")
    if rim is not None and rim.any():
        upd(d2[rim].sum(), r2[rim].sum(), "PEC sheet rims", int(rim.sum()))
    return whole, elem, worst


def compare_fields(ref, got, board, tol, floor_rel=None, elem_tol=None, region_tol=None,
                   region_floor=0.5):
    """Every array against the oracle: whole-array relative L2 <= tol, element-wise
    max|got - ref| <= elem_tol * max|ref| (default tol), and every region's
    relative L2 <= region_tol (default 2 tol).  With ``floor_rel`` the
    denominators are at least floor_rel times the norm (or, element-wise, the
    largest value) of the whole E field in each array's own units: an array
    that the pulse has only reached through the stencil's far tail (values many
    decades below the field, flushed or lost in FP32) is then held to an
    absolute bound instead."""
    elem_tol = tol if elem_tol is None else elem_tol
    region_tol = 2 * tol if region_tol is None else region_tol
    am = aux_masks(board)
    rim = rim_mask(board)
    e_norm = float(np.sqrt(sum(np.linalg.norm(ref[n]) ** 2 for n in ("ex", "ey", "ez"))))
    e_max = max(float(np.abs(ref[n]).max()) for n in ("ex", "ey", "ez"))
    report = {}
    for n in FIELDS:
        r = ref[n]
        if n in _AXIS:
            r = np.where(am[_AXIS[n]], r, 0.0)
        if np.abs(r).max() == 0:
            assert np.abs(got[n]).max() == 0, n
            continue
        u = TO_E_UNITS[n[0]]
        floor = floor_rel * e_norm / u if floor_rel is not None else 0.0
        floor_max = floor_rel * e_max / u if floor_rel is not None else 0.0
        whole, elem, (reg, where) = field_errors(r, got[n], board, floor, floor_max, region_floor, rim)
        report[n] = (whole, elem, reg, where)
    bad = [n for n, (w, e, g, _) in report.items() if w > tol or e > elem_tol or g > region_tol]
    for n in bad:
        w, e, g, where = report[n]
        print(f"compare_fields {n}: whole {w:.3e} (<= {tol:.1e}), element {e:.3e} "
              f"(<= {elem_tol:.1e}), region {g:.3e} (<= {region_tol:.1e}) at {where}", flush=True)
    for n in bad:
        whole, elem, reg, where = report[n]
        assert whole <= tol, (n, "whole", whole)
        assert elem <= elem_tol, (n, "element-wise", elem)
        assert reg <= region_tol, (n, "region", where, reg)
    return report
