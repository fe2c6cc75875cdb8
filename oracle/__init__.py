"""FP64 CPU oracle for the Yee/UPML leapfrog and its probe spectrum.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product path
(``paper_1008_2602_amd``) never does and shares no code with it.

* ``fdtd_oracle.c`` is the stepper (plain triple loops, FP64, unified D/B
  storage), following the paper's Model section: Eqs. 1-2 (UPML medium and
  stretch factors), Eq. 4 (D from curl H, then E from D; B then H alike), Eq. 5
  (polynomial grading), Eq. 7 (time step) and the PEC planes.
* ``probe_fft`` is the post-run spectrum of a probe series (Results section, the
  FFT of the ground-plane Ez): rectangular window, zero padding to ``n_fft``,
  sample s taken at time (s+1) dt; numpy's FFT is the library primitive.

Parity pins live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdtd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FIELD_NAMES = ("ex", "ey", "ez", "hx", "hy", "hz", "ddx", "ddy", "ddz", "bbx", "bby", "bbz")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE arithmetic)."""
    stale = (not os.path.exists(_LIB)
             or os.path.getmtime(_LIB) < os.path.getmtime(_SRC))
    if force or stale:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("dt", C.c_double), ("courant", C.c_double),
                ("npml", C.c_int32 * 6),
                ("pml_m", C.c_double), ("pml_R", C.c_double), ("pml_kappa_max", C.c_double),
                ("eps_r_cell", C.c_void_p), ("sigma_cell", C.c_void_p), ("pec_mask", C.c_void_p),
                ("nsrc", C.c_int32), ("src_ijk", C.c_void_p), ("src_wave", C.c_void_p),
                ("src_J0", C.c_void_p), ("src_t0", C.c_void_p), ("src_sigma", C.c_void_p),
                ("src_R", C.c_void_p),
                ("nprobe", C.c_int32), ("probe_ijk", C.c_void_p),
                ("nfreq", C.c_int32), ("freqs", C.c_void_p),
                ("pml_eps_rw", C.c_int32),
                ("plane_k", C.c_int32), ("nplane_freq", C.c_int32), ("plane_freqs", C.c_void_p),
                ("sheet_R", C.c_double)]


class _State(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in FIELD_NAMES] + [("step", C.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = C.CDLL(_LIB)
        lib.or_run.argtypes = [C.POINTER(_Problem), C.POINTER(_State), C.c_int64,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.or_run.restype = C.c_int
        lib.or_time_step.argtypes = [C.POINTER(_Problem)]
        lib.or_time_step.restype = C.c_double
        lib.or_cfl_dt.argtypes = [C.c_double] * 3
        lib.or_cfl_dt.restype = C.c_double
        lib.or_waveform.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
        lib.or_waveform.restype = C.c_double
        lib.or_num_threads.restype = C.c_int
        lib.or_set_num_threads.argtypes = [C.c_int]
        lib.or_constants.argtypes = [C.POINTER(C.c_double)] * 4
        lib.or_sigma_kappa.argtypes = [C.POINTER(_Problem), C.c_int, C.c_double,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib = lib
    return _lib


def constants() -> Dict[str, float]:
    v = [C.c_double() for _ in range(4)]
    _load().or_constants(*[C.byref(x) for x in v])
    return dict(c0=v[0].value, mu0=v[1].value, eps0=v[2].value, eta0=v[3].value)


def set_threads(n: int) -> None:
    _load().or_set_num_threads(int(n))


def num_threads() -> int:
    return int(_load().or_num_threads())


class Problem:
    """Marshals a ``boardgen.Board`` into the oracle's C struct (keeps arrays alive)."""

    def __init__(self, board):
        b = board
        self.board = b
        self.eps = np.ascontiguousarray(b.eps_r_cell, dtype=np.float32)
        sig = getattr(b, "sigma_cell", None)
        self.sigma = None if sig is None else np.ascontiguousarray(sig, dtype=np.float32)
        if self.sigma is not None:
            assert self.sigma.shape == self.eps.shape and np.all(self.sigma >= 0)
            p_ = b.npml
            inner = np.zeros_like(self.sigma, dtype=bool)
            inner[p_[4]:b.nz - p_[5], p_[2]:b.ny - p_[3], p_[0]:b.nx - p_[1]] = True
            assert not np.any(self.sigma[~inner]), "conductivity only outside the PML slabs"
        self.pec = np.ascontiguousarray(b.pec_edge_mask, dtype=np.uint8)
        self.sheet_R = float(getattr(b, "sheet_R", 0.0) or 0.0)
        assert self.sheet_R >= 0.0 and np.isfinite(self.sheet_R)
        if self.sheet_R > 0.0:
            # sheet edges conduct like a lossy dielectric: only where every cell
            # touching them lies outside the PML slabs (edges on the outer wall are
            # never stepped and do not count)
            p_ = b.npml
            for bit, lo_i, lo_j in ((1, p_[0], p_[2] + 1), (2, p_[0] + 1, p_[2])):
                kk, jj, ii = np.nonzero(self.pec & bit)
                wall = ((kk == 0) | (kk == b.nz) | (ii == b.nx) | (jj == b.ny) |
                        ((jj == 0) if bit == 1 else (ii == 0)))
                ok = ((ii >= lo_i) & (ii < b.nx - p_[1]) & (jj >= lo_j) & (jj < b.ny - p_[3]) &
                      (kk > p_[4]) & (kk < b.nz - p_[5]))
                assert np.all(ok | wall), "resistive sheets only outside the PML slabs"
        ns = len(b.sources)
        self.src_ijk = np.array([[s.i, s.j, s.k] for s in b.sources], np.int32).reshape(ns, 3)
        self.src_wave = np.array([s.waveform for s in b.sources], np.int32)
        self.src_J0 = np.array([s.J0 for s in b.sources], np.float64)
        self.src_t0 = np.array([s.t0 for s in b.sources], np.float64)
        self.src_sigma = np.array([s.sigma for s in b.sources], np.float64)
        self.src_R = np.array([getattr(s, "R", 0.0) for s in b.sources], np.float64)
        for s in b.sources:
            if getattr(s, "R", 0.0) > 0.0:
                in_pml = ((s.i < b.npml[0] or s.i >= b.nx - b.npml[1]) or
                          (s.j < b.npml[2] or s.j >= b.ny - b.npml[3]) or
                          (s.k < b.npml[4] or s.k >= b.nz - b.npml[5]))
                assert not in_pml, "a resistive source must sit outside every PML slab"
        self.probe_ijk = np.array(b.probes, np.int32).reshape(len(b.probes), 3)
        self.freqs = (np.zeros(0) if b.dft_freqs is None
                      else np.ascontiguousarray(b.dft_freqs, dtype=np.float64))
        pd = getattr(b, "plane_dft", None)
        self.plane_k = -1 if pd is None else int(pd[0])
        self.plane_freqs = (np.zeros(0) if pd is None
                            else np.ascontiguousarray(pd[1], dtype=np.float64))
        assert self.plane_k < b.nz
        p = _Problem()
        p.nx, p.ny, p.nz = b.nx, b.ny, b.nz
        p.dx, p.dy, p.dz = b.dx, b.dy, b.dz
        p.dt, p.courant = b.dt, b.courant
        p.npml = (C.c_int32 * 6)(*b.npml)
        p.pml_m, p.pml_R, p.pml_kappa_max = b.pml_m, b.pml_R, b.pml_kappa_max
        p.eps_r_cell = self.eps.ctypes.data
        p.sigma_cell = None if self.sigma is None else self.sigma.ctypes.data
        p.pec_mask = self.pec.ctypes.data
        p.nsrc = ns
        p.src_ijk = self.src_ijk.ctypes.data
        p.src_wave = self.src_wave.ctypes.data
        p.src_J0 = self.src_J0.ctypes.data
        p.src_t0 = self.src_t0.ctypes.data
        p.src_sigma = self.src_sigma.ctypes.data
        p.src_R = self.src_R.ctypes.data
        p.nprobe = len(b.probes)
        p.probe_ijk = self.probe_ijk.ctypes.data
        p.nfreq = len(self.freqs)
        p.freqs = self.freqs.ctypes.data
        p.pml_eps_rw = 1 if getattr(b, "pml_eps_rw", False) else 0
        p.plane_k = self.plane_k
        p.nplane_freq = len(self.plane_freqs)
        p.plane_freqs = self.plane_freqs.ctypes.data
        p.sheet_R = self.sheet_R
        self.c = p

    @property
    def dt(self) -> float:
        return float(_load().or_time_step(C.byref(self.c)))


def new_state(board) -> Dict[str, np.ndarray]:
    shp = (board.nz + 1, board.ny + 1, board.nx + 1)
    st = {n: np.zeros(shp, np.float64) for n in FIELD_NAMES}
    st["step"] = 0
    return st


@dataclass
class Result:
    dt: float
    probes: np.ndarray           # (nprobe, nsteps) float64
    dft: Optional[np.ndarray]    # (nprobe, nfreq) complex128, accumulated over the run
    state: Dict[str, np.ndarray]
    plane_dft: Optional[np.ndarray] = None   # (nfreq, ny+1, nx+1) complex128, accumulated


def run(board, nsteps: Optional[int] = None, state: Optional[Dict[str, np.ndarray]] = None,
        threads: Optional[int] = None, dft: Optional[np.ndarray] = None,
        plane_dft: Optional[np.ndarray] = None) -> Result:
    """Advance ``state`` (zero fields if None) by ``nsteps`` (default board.steps).
    ``dft`` and ``plane_dft`` carry accumulators over from an earlier call."""
    lib = _load()
    if threads is not None:
        lib.or_set_num_threads(int(threads))
    prob = Problem(board)
    st = new_state(board) if state is None else state
    for n in FIELD_NAMES:
        a = st[n]
        assert a.dtype == np.float64 and a.flags.c_contiguous
        assert a.shape == (board.nz + 1, board.ny + 1, board.nx + 1)
    cs = _State(*[st[n].ctypes.data for n in FIELD_NAMES], int(st["step"]))
    n = board.steps if nsteps is None else int(nsteps)
    P = len(board.probes)
    series = np.zeros((P, max(n, 1)), np.float64)
    F = len(prob.freqs)
    if dft is None:
        dft = np.zeros((P, F), np.complex128)
    re = np.ascontiguousarray(dft.real.copy())
    im = np.ascontiguousarray(dft.imag.copy())
    FP = len(prob.plane_freqs) if prob.plane_k >= 0 else 0
    if plane_dft is None:
        plane_dft = np.zeros((FP, board.ny + 1, board.nx + 1), np.complex128)
    assert plane_dft.shape == (FP, board.ny + 1, board.nx + 1)
    pre = np.ascontiguousarray(plane_dft.real.copy())
    pim = np.ascontiguousarray(plane_dft.imag.copy())
    if n > 0:
        lib.or_run(C.byref(prob.c), C.byref(cs), n, series.ctypes.data,
                   re.ctypes.data if F else None, im.ctypes.data if F else None,
                   pre.ctypes.data if FP else None, pim.ctypes.data if FP else None)
    st["step"] = int(cs.step)
    return Result(dt=prob.dt, probes=series[:, :n], dft=(re + 1j * im) if F else None,
                  state=st, plane_dft=(pre + 1j * pim) if FP else None)


def sigma_kappa(board, axis: int, pos: float):
    """(sigma, kappa) of the Eq. 5 grading at coordinate ``pos`` along ``axis``."""
    prob = Problem(board)
    s, k = C.c_double(), C.c_double()
    _load().or_sigma_kappa(C.byref(prob.c), int(axis), float(pos), C.byref(s), C.byref(k))
    return s.value, k.value


def time_step(board) -> float:
    return Problem(board).dt


def waveform(wave: int, J0: float, t0: float, sigma: float, t: float) -> float:
    return float(_load().or_waveform(int(wave), J0, t0, sigma, t))


# ---------------------------------------------------------------------------
# post-run probe spectrum (Results section: FFT of the ground-plane Ez)
# ---------------------------------------------------------------------------

def probe_fft(series: np.ndarray, n_fft: int) -> np.ndarray:
    """Bins k = 0..n_fft/2 of X[k] = sum_{s<N} e[s] exp(-2 pi i k s / n_fft):
    rectangular window, no mean removal, zero padding to ``n_fft`` (>= N)."""
    e = np.asarray(series, np.float64)
    assert n_fft >= e.shape[-1]
    return np.fft.rfft(e, n=n_fft)


def default_nfft(nsteps: int) -> int:
    n = 1
    while n < nsteps:
        n *= 2
    return n


def bin_freqs(n_fft: int, dt: float) -> np.ndarray:
    return np.arange(n_fft // 2 + 1) / (n_fft * dt)


def find_peaks(mag: np.ndarray, freqs: np.ndarray, f_min: float, rel: float = 0.01
               ) -> np.ndarray:
    """Frequencies of local maxima of ``mag`` above ``rel`` * max (over f >= f_min)."""
    sel = freqs >= f_min
    m = np.where(sel, mag, 0.0)
    top = m.max()
    idx = [k for k in range(1, len(m) - 1)
           if sel[k] and m[k] >= m[k - 1] and m[k] > m[k + 1] and m[k] >= rel * top]
    return freqs[np.array(idx, dtype=int)] if idx else np.zeros(0)
