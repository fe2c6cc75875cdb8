"""Small helpers shared by the tests (no method arithmetic)."""
import numpy as np


def live_masks(board):
    """Boolean masks of the entries each oracle array actually carries: E edges
    that are updated (not on the outer wall, not PEC) and H faces that exist and
    do not lie on the outer wall normal to themselves."""
    nx, ny, nz = board.nx, board.ny, board.nz
    kk = np.arange(nz + 1)[:, None, None]
    jj = np.arange(ny + 1)[None, :, None]
    ii = np.arange(nx + 1)[None, None, :]
    shp = (nz + 1, ny + 1, nx + 1)
    pec = board.pec_edge_mask
    m = {}
    m["ex"] = (ii < nx) & (jj >= 1) & (jj < ny) & (kk >= 1) & (kk < nz) & ((pec & 1) == 0)
    m["ey"] = (ii >= 1) & (ii < nx) & (jj < ny) & (kk >= 1) & (kk < nz) & ((pec & 2) == 0)
    m["ez"] = (ii >= 1) & (ii < nx) & (jj >= 1) & (jj < ny) & (kk < nz) & ((pec & 4) == 0)
    # an H face on the outer wall normal to it (Hx at i = 0 or nx, ...) touches only
    # E edges tangential to that wall, which stay zero: it carries nothing
    m["hx"] = (ii >= 1) & (ii < nx) & (jj < ny) & (kk < nz)
    m["hy"] = (jj >= 1) & (jj < ny) & (ii < nx) & (kk < nz)
    m["hz"] = (kk >= 1) & (kk < nz) & (ii < nx) & (jj < ny)
    for a, f in (("ddx", "ex"), ("ddy", "ey"), ("ddz", "ez"),
                 ("bbx", "hx"), ("bby", "hy"), ("bbz", "hz")):
        m[a] = m[f]
    return m


def rel_l2(a, b):
    """||a - b|| / ||b|| (real or complex)."""
    a = np.asarray(a)
    b = np.asarray(b)
    a = a.astype(np.complex128) if np.iscomplexobj(a) or np.iscomplexobj(b) else a.astype(np.float64)
    b = b.astype(a.dtype)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def rel_max(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))
