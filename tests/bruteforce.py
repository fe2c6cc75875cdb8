"""Brute-force sparse-matrix form of the Yee/UPML leapfrog (pins the oracle).

A different code path from the oracle's loops: the discrete curls are assembled
as Kronecker products of 1-D difference matrices, the stretched-coordinate loss
coefficients are diagonal matrices built from each component's coordinates, and
one step is a handful of sparse mat-vecs.  The equations are the paper's Eq. 4
(D from curl H, then E from D; B then H alike, with the same s as Eq. 1 gives
for mu), the Eq. 5 grading and the PEC planes of the Model section.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

C0 = 299792458.0
MU0 = 4e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 ** 2)
ETA0 = MU0 * C0

COMPS = ("ex", "ey", "ez", "hx", "hy", "hz")
AXES = "xyz"


def _fwd(n: int) -> sp.csr_matrix:
    """(F v)[i] = v[i+1] - v[i] on n+1 points (v[n+1] taken as 0)."""
    return sp.diags([-np.ones(n + 1), np.ones(n)], [0, 1], shape=(n + 1, n + 1), format="csr")


def _bwd(n: int) -> sp.csr_matrix:
    """(G v)[i] = v[i] - v[i-1] on n+1 points (v[-1] taken as 0)."""
    return sp.diags([np.ones(n + 1), -np.ones(n)], [0, -1], shape=(n + 1, n + 1), format="csr")


def _along(axis: str, m: sp.csr_matrix, nx: int, ny: int, nz: int) -> sp.csr_matrix:
    Ix, Iy, Iz = sp.identity(nx + 1), sp.identity(ny + 1), sp.identity(nz + 1)
    if axis == "x":
        return sp.kron(Iz, sp.kron(Iy, m)).tocsr()
    if axis == "y":
        return sp.kron(Iz, sp.kron(m, Ix)).tocsr()
    return sp.kron(m, sp.kron(Iy, Ix)).tocsr()


def _half(comp: str, axis: str) -> bool:
    """Does component ``comp`` sit at a half-integer coordinate along ``axis``?"""
    kind, c = comp[0], comp[1]
    return (c == axis) if kind == "e" else (c != axis)


def stretch(board, axis: str, pos: np.ndarray, dt: float):
    """sigma, kappa at coordinates ``pos`` (cell units) along ``axis``."""
    n = {"x": board.nx, "y": board.ny, "z": board.nz}[axis]
    lo = board.npml[2 * AXES.index(axis)]
    hi = board.npml[2 * AXES.index(axis) + 1]
    d = {"x": board.dx, "y": board.dy, "z": board.dz}[axis]
    sig = np.zeros_like(pos, dtype=float)
    kap = np.ones_like(pos, dtype=float)
    for npml, depth in ((lo, lo - pos), (hi, pos - (n - hi))):
        if npml <= 0:
            continue
        inside = depth > 0
        frac = np.where(inside, np.clip(depth, 0, None) / npml, 0.0) ** board.pml_m
        smax = -(board.pml_m + 1) * np.log(board.pml_R) / (2 * ETA0 * npml * d)
        sig = np.where(inside, frac * smax, sig)
        kap = np.where(inside, 1 + (board.pml_kappa_max - 1) * frac, kap)
    return sig, kap


class Stepper:
    def __init__(self, board, dt: float):
        b = board
        self.b, self.dt = b, dt
        nx, ny, nz = b.nx, b.ny, b.nz
        self.shape = (nz + 1, ny + 1, nx + 1)
        kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                                 indexing="ij")
        idx = {"x": ii, "y": jj, "z": kk}
        d = {"x": b.dx, "y": b.dy, "z": b.dz}
        F = {a: _along(a, _fwd(n), nx, ny, nz) / d[a] for a, n in zip(AXES, (nx, ny, nz))}
        G = {a: _along(a, _bwd(n), nx, ny, nz) / d[a] for a, n in zip(AXES, (nx, ny, nz))}
        # curl E at H positions, curl H at E positions
        self.curlE = {"hx": ("ez", F["y"], "ey", F["z"]),
                      "hy": ("ex", F["z"], "ez", F["x"]),
                      "hz": ("ey", F["x"], "ex", F["y"])}
        self.curlH = {"ex": ("hz", G["y"], "hy", G["z"]),
                      "ey": ("hx", G["z"], "hz", G["x"]),
                      "ez": ("hy", G["x"], "hx", G["y"])}
        # update masks (components that exist / are updated)
        pec = b.pec_edge_mask
        m = {}
        m["hx"] = (jj < ny) & (kk < nz)
        m["hy"] = (ii < nx) & (kk < nz)
        m["hz"] = (ii < nx) & (jj < ny)
        m["ex"] = (ii < nx) & (jj >= 1) & (jj < ny) & (kk >= 1) & (kk < nz) & ((pec & 1) == 0)
        m["ey"] = (ii >= 1) & (ii < nx) & (jj < ny) & (kk >= 1) & (kk < nz) & ((pec & 2) == 0)
        m["ez"] = (ii >= 1) & (ii < nx) & (jj >= 1) & (jj < ny) & (kk < nz) & ((pec & 4) == 0)
        self.mask = m
        self.pec0 = {"ex": (pec & 1) != 0, "ey": (pec & 2) != 0, "ez": (pec & 4) != 0}
        # coefficient arrays per component: cyclic (u, v, w) with u the component axis
        self.coef = {}
        for comp in COMPS:
            u = comp[1]
            v = AXES[(AXES.index(u) + 1) % 3]
            w = AXES[(AXES.index(u) + 2) % 3]
            sk = {}
            for a in (u, v, w):
                pos = idx[a] + (0.5 if _half(comp, a) else 0.0)
                sk[a] = stretch(b, a, pos.astype(float), dt)
            sv, kv = sk[v]
            sw, kw = sk[w]
            su, ku = sk[u]
            aux_a = (2 * EPS0 * kv - sv * dt) / (2 * EPS0 * kv + sv * dt)
            aux_b = 2 * EPS0 * dt / (2 * EPS0 * kv + sv * dt)
            fld_a = (2 * EPS0 * kw - sw * dt) / (2 * EPS0 * kw + sw * dt)
            pp_u = 2 * EPS0 * ku + su * dt
            pm_u = 2 * EPS0 * ku - su * dt
            pp_w = 2 * EPS0 * kw + sw * dt
            self.coef[comp] = (aux_a, aux_b, fld_a, pp_u, pm_u, pp_w)
        # edge permittivity: mean of the (up to) four cells touching the edge
        er = b.eps_r_cell.astype(np.float64)
        pad = np.zeros((nz + 2, ny + 2, nx + 2))
        pad[1:-1, 1:-1, 1:-1] = er  # cell (i,j,k) at pad[k+1, j+1, i+1]

        def cellavg(di, dj, dk):
            # average of cells (i - di_s, j - dj_s, k - dk_s) over the axes flagged 1
            acc = np.zeros(self.shape)
            cnt = 0
            for oi in ((0, 1) if di else (1,)):
                for oj in ((0, 1) if dj else (1,)):
                    for ok in ((0, 1) if dk else (1,)):
                        acc += pad[ok:ok + nz + 1, oj:oj + ny + 1, oi:oi + nx + 1]
                        cnt += 1
            acc = acc / cnt
            return np.where(acc == 0.0, 1.0, acc)  # only at never-updated wall edges

        self.eps = {"ex": EPS0 * cellavg(0, 1, 1), "ey": EPS0 * cellavg(1, 0, 1),
                    "ez": EPS0 * cellavg(1, 1, 0)}
        # sources as (flat index of Ez, waveform params)
        self.src = [(np.ravel_multi_index((s.k, s.j, s.i), self.shape), s) for s in b.sources]

    @staticmethod
    def wave(s, t):
        u = (t - s.t0) / s.sigma
        return s.J0 * (u * np.exp(-u * u) if s.waveform == 1 else np.exp(-0.5 * u * u))

    def step(self, st: dict, n: int) -> None:
        """One leapfrog step from E^n, H^{n-1/2} (state dict of flat arrays)."""
        dt = self.dt
        for h in ("hx", "hy", "hz"):
            e1, D1, e2, D2 = self.curlE[h]
            curl = D1 @ st[e1] - D2 @ st[e2]
            aa, bb, fa, ppu, pmu, ppw = (c.ravel() for c in self.coef[h])
            msk = self.mask[h].ravel()
            bo = st["b" + h[1]]
            bn = aa * bo - bb * curl
            hn = fa * st[h] + (ppu * bn - pmu * bo) / (MU0 * ppw)
            st["b" + h[1]] = np.where(msk, bn, bo)
            st[h] = np.where(msk, hn, st[h])
        tJ = (n + 0.5) * dt
        for e in ("ex", "ey", "ez"):
            h1, D1, h2, D2 = self.curlH[e]
            curl = D1 @ st[h1] - D2 @ st[h2]
            if e == "ez":
                J = np.zeros_like(curl)
                for fi, s in self.src:
                    J[fi] += self.wave(s, tJ)
                curl = curl - J
            aa, bb, fa, ppu, pmu, ppw = (c.ravel() for c in self.coef[e])
            msk = self.mask[e].ravel()
            do = st["d" + e[1]]
            dn = aa * do + bb * curl
            en = fa * st[e] + (ppu * dn - pmu * do) / (self.eps[e].ravel() * ppw)
            st["d" + e[1]] = np.where(msk, dn, do)
            en = np.where(msk, en, st[e])
            st[e] = np.where(self.pec0[e].ravel(), 0.0, en)


def run(board, dt: float, nsteps: int, init: dict | None = None):
    s = Stepper(board, dt)
    size = int(np.prod(s.shape))
    st = {k: np.zeros(size) for k in ("ex", "ey", "ez", "hx", "hy", "hz",
                                      "dx", "dy", "dz", "bx", "by", "bz")}
    if init:
        for k, v in init.items():
            st[k] = np.array(v, dtype=float).ravel().copy()
    probes = []
    for n in range(nsteps):
        s.step(st, n)
        probes.append([st["ez"][np.ravel_multi_index((k, j, i), s.shape)]
                       for (i, j, k) in board.probes])
    return {k: v.reshape(s.shape) for k, v in st.items()}, np.array(probes).T
