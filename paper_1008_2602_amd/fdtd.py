"""Thin ctypes binding of libfdtd (include/fdtd.h); same names as the C calls.

Argument marshalling only: every step of the solve runs in libfdtd's HIP
kernels.  PyTorch is used for plumbing alone: the caller's current HIP stream and,
optionally, device memory from its caching allocator.  Importing this module
fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

# PyTorch's ROCm build ships its own HIP runtime (SONAME libamdhip64.so.7).  Load
# it first so that libfdtd binds to that same runtime instead of a second copy:
# streams and device pointers then mean the same thing on both sides.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# FDTD_LIBRARY may point at another build of the same library (same ABI)
LIB_PATH = os.environ.get("FDTD_LIBRARY") or os.path.join(_HERE, "libfdtd.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fdtd.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libfdtd.so is not built ({LIB_PATH}); run __graft_entry__.build()")

_lib = C.CDLL(LIB_PATH)

FDTD_OK = 0
FDTD_EINVAL = -1
FDTD_ESTATE = -2
FDTD_ENOMEM = -3
FDTD_EDEVICE = -4
FDTD_EUNSTABLE = -5
FDTD_WAVE_GAUSS = 0
FDTD_WAVE_DGAUSS = 1
FDTD_EX, FDTD_EY, FDTD_EZ, FDTD_HX, FDTD_HY, FDTD_HZ = range(6)
FDTD_DX, FDTD_DY, FDTD_DZ, FDTD_BX, FDTD_BY, FDTD_BZ = range(6, 12)
COMPONENTS = ("ex", "ey", "ez", "hx", "hy", "hz", "dx", "dy", "dz", "bx", "by", "bz")

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class fdtd_grid_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("dt", C.c_double), ("courant", C.c_double),
                ("npml", C.c_int32 * 6),
                ("pml_m", C.c_double), ("pml_R", C.c_double), ("pml_kappa_max", C.c_double),
                ("max_steps", C.c_int64),
                ("hip_stream", C.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class fdtd_info(C.Structure):
    _fields_ = [("dt", C.c_double), ("step", C.c_int64), ("max_steps", C.c_int64),
                ("cells", C.c_int64), ("nodes", C.c_int64), ("step_bytes", C.c_int64),
                ("device_bytes", C.c_int64),
                ("n_sources", C.c_int32), ("n_probes", C.c_int32), ("n_freqs", C.c_int32),
                ("n_classes", C.c_int32), ("tile_x", C.c_int32), ("tile_y", C.c_int32),
                ("tile_steps", C.c_int32), ("plane_k", C.c_int32), ("plane_nf", C.c_int32),
                ("node_passes", C.c_int32), ("material_two_step", C.c_int32),
                ("material_permille", C.c_int32),
                ("material_split", C.c_int32),
                ("conduct_permille", C.c_int32),
                ("batch_plans", C.c_int32), ("batch_graphs", C.c_int32)]


class FdtdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfdtd error {code}: {msg}")
        self.code = code


_P = C.c_void_p
_sigs = {
    "fdtd_create_grid": ([C.POINTER(fdtd_grid_desc), C.POINTER(C.c_void_p)], C.c_int),
    "fdtd_set_materials": ([_P, _P, _P], C.c_int),
    "fdtd_add_source": ([_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                         C.c_double, C.POINTER(C.c_int)], C.c_int),
    "fdtd_add_voltage_source": ([_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int)],
                                C.c_int),
    "fdtd_add_probe": ([_P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)], C.c_int),
    "fdtd_add_voltage_probe": ([_P, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)],
                               C.c_int),
    "fdtd_get_voltage": ([_P, C.c_int, _P, C.c_int64], C.c_int),
    "fdtd_set_dft_freqs": ([_P, _P, C.c_int], C.c_int),
    "fdtd_set_plane_dft": ([_P, C.c_int, _P, C.c_int], C.c_int),
    "fdtd_set_pml_eps_rw": ([_P, C.c_int], C.c_int),
    "fdtd_set_conductivity": ([_P, _P], C.c_int),
    "fdtd_set_sheet_resistance": ([_P, C.c_double], C.c_int),
    "fdtd_get_plane_dft": ([_P, _P, _P], C.c_int),
    "fdtd_get_plane": ([_P, C.c_int, C.c_int, _P], C.c_int),
    "fdtd_step_n": ([_P, C.c_int64], C.c_int),
    "fdtd_step_many": ([_P, C.c_int, _P], C.c_int),
    "fdtd_probe_fft": ([_P, C.c_int, C.c_int, _P, _P], C.c_int),
    "fdtd_probe_fft_noalloc": ([_P, C.c_int, C.c_int, _P, _P], C.c_int),
    "fdtd_get_probe": ([_P, C.c_int, _P, C.c_int64], C.c_int),
    "fdtd_get_dft": ([_P, C.c_int, _P, _P], C.c_int),
    "fdtd_get_field": ([_P, C.c_int, _P], C.c_int),
    "fdtd_set_field": ([_P, C.c_int, _P], C.c_int),
    "fdtd_state_bytes": ([_P], C.c_int64),
    "fdtd_estimate_bytes": ([C.POINTER(fdtd_grid_desc), C.c_int, C.c_int, C.c_int], C.c_int64),
    "fdtd_save_state": ([_P, _P, C.c_int64], C.c_int),
    "fdtd_load_state": ([_P, _P, C.c_int64], C.c_int),
    "fdtd_get_info": ([_P, C.POINTER(fdtd_info)], C.c_int),
    "fdtd_set_tile": ([_P, C.c_int, C.c_int, C.c_int], C.c_int),
    "fdtd_tile_shapes": ([_P, C.c_int], C.c_int),
    "fdtd_set_timing": ([_P, C.c_int], C.c_int),
    "fdtd_get_timing": ([_P, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    "fdtd_synchronize": ([_P], C.c_int),
    "fdtd_get_stream": ([_P, C.POINTER(C.c_void_p)], C.c_int),
    "fdtd_destroy_grid": ([_P], C.c_int),
    "fdtd_last_error": ([], C.c_char_p),
}
for _name, (_args, _res) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def header_symbols() -> List[str]:
    """Function names declared in include/fdtd.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(fdtd_\w+)\s*\(", text, re.M)))


def library():
    return _lib


def fdtd_last_error() -> str:
    return _lib.fdtd_last_error().decode()


def _check(rc: int) -> int:
    if rc != FDTD_OK:
        raise FdtdError(rc, fdtd_last_error())
    return rc


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# --------------------------------------------------------------------------
# optional device memory from PyTorch's caching allocator

class TorchAllocator:
    """Hands libfdtd device memory owned by torch tensors on the current device."""

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self._live: Dict[int, object] = {}
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, _ctx):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self._live[p] = t
        return p

    def _free(self, ptr, _ctx):
        self._live.pop(int(ptr) if ptr else 0, None)

    @property
    def live_bytes(self) -> int:
        return sum(t.numel() for t in self._live.values())


# --------------------------------------------------------------------------
# the C calls

def _desc(nx, ny, nz, dx, dy, dz, dt, courant, npml, pml_m, pml_R, pml_kappa_max, max_steps,
          hip_stream, allocator):
    d = fdtd_grid_desc()
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.dx, d.dy, d.dz = float(dx), float(dy), float(dz)
    d.dt, d.courant = float(dt), float(courant)
    d.npml = (C.c_int32 * 6)(*[int(v) for v in npml])
    d.pml_m, d.pml_R, d.pml_kappa_max = float(pml_m), float(pml_R), float(pml_kappa_max)
    d.max_steps = int(max_steps)
    d.hip_stream = hip_stream
    if allocator is not None:
        d.dev_alloc, d.dev_free = allocator.alloc, allocator.free
    return d


def fdtd_create_grid(nx, ny, nz, dx, dy, dz, *, dt=0.0, courant=0.99, npml=(8,) * 6,
                     pml_m=3.0, pml_R=1e-6, pml_kappa_max=1.0, max_steps=1,
                     hip_stream=None, allocator: Optional[TorchAllocator] = None):
    d = _desc(nx, ny, nz, dx, dy, dz, dt, courant, npml, pml_m, pml_R, pml_kappa_max,
              max_steps, hip_stream, allocator)
    h = C.c_void_p()
    _check(_lib.fdtd_create_grid(C.byref(d), C.byref(h)))
    return h


def fdtd_set_materials(g, eps_r_cell: np.ndarray, pec_edge_mask: Optional[np.ndarray] = None):
    eps = np.ascontiguousarray(eps_r_cell, dtype=np.float32)
    pec = None if pec_edge_mask is None else np.ascontiguousarray(pec_edge_mask, dtype=np.uint8)
    _check(_lib.fdtd_set_materials(g, _ptr(eps), _ptr(pec)))


def fdtd_add_source(g, i, j, k, waveform, J0, t0, sigma) -> int:
    out = C.c_int()
    _check(_lib.fdtd_add_source(g, int(i), int(j), int(k), int(waveform), float(J0),
                                float(t0), float(sigma), C.byref(out)))
    return out.value


def fdtd_add_voltage_source(g, i, j, k, waveform, V0, t0, sigma, R) -> int:
    out = C.c_int()
    _check(_lib.fdtd_add_voltage_source(g, int(i), int(j), int(k), int(waveform), float(V0),
                                        float(t0), float(sigma), float(R), C.byref(out)))
    return out.value


def fdtd_add_probe(g, i, j, k) -> int:
    out = C.c_int()
    _check(_lib.fdtd_add_probe(g, int(i), int(j), int(k), C.byref(out)))
    return out.value


def fdtd_add_voltage_probe(g, i, j, k0, k1) -> int:
    out = C.c_int()
    _check(_lib.fdtd_add_voltage_probe(g, int(i), int(j), int(k0), int(k1), C.byref(out)))
    return out.value


def fdtd_set_dft_freqs(g, f_hz: Sequence[float]):
    f = np.ascontiguousarray(f_hz, dtype=np.float64)
    _check(_lib.fdtd_set_dft_freqs(g, _ptr(f), len(f)))


def fdtd_set_conductivity(g, sigma_cell: Optional[np.ndarray]):
    sig = None if sigma_cell is None else np.ascontiguousarray(sigma_cell, dtype=np.float32)
    _check(_lib.fdtd_set_conductivity(g, _ptr(sig)))


def fdtd_set_sheet_resistance(g, ohms_per_square: float):
    _check(_lib.fdtd_set_sheet_resistance(g, float(ohms_per_square)))


def fdtd_set_pml_eps_rw(g, on: bool):
    _check(_lib.fdtd_set_pml_eps_rw(g, 1 if on else 0))


def fdtd_set_plane_dft(g, k: int, f_hz: Sequence[float]):
    f = np.ascontiguousarray(f_hz, dtype=np.float64)
    _check(_lib.fdtd_set_plane_dft(g, int(k), _ptr(f), len(f)))


def fdtd_get_plane_dft(g, ny: int, nx: int) -> np.ndarray:
    """(nf, ny+1, nx+1) complex128."""
    nf = fdtd_get_info(g).plane_nf
    re = np.zeros((nf, ny + 1, nx + 1))
    im = np.zeros((nf, ny + 1, nx + 1))
    _check(_lib.fdtd_get_plane_dft(g, _ptr(re), _ptr(im)))
    return re + 1j * im


def fdtd_get_plane(g, comp: int, k: int, ny: int, nx: int) -> np.ndarray:
    out = np.zeros((ny + 1, nx + 1), np.float32)
    _check(_lib.fdtd_get_plane(g, int(comp), int(k), _ptr(out)))
    return out


def fdtd_step_n(g, n: int):
    _check(_lib.fdtd_step_n(g, int(n)))


def fdtd_step_many(grids: Sequence, n: Sequence[int]):
    arr = (C.c_void_p * len(grids))(*[h.value if isinstance(h, C.c_void_p) else h for h in grids])
    ns = np.ascontiguousarray(n, dtype=np.int64)
    _check(_lib.fdtd_step_many(arr, len(grids), _ptr(ns)))


def fdtd_probe_fft(g, pid: int, n_fft: int) -> np.ndarray:
    re = np.zeros(n_fft // 2 + 1)
    im = np.zeros(n_fft // 2 + 1)
    _check(_lib.fdtd_probe_fft(g, int(pid), int(n_fft), _ptr(re), _ptr(im)))
    return re + 1j * im


def fdtd_probe_fft_noalloc(g, pid: int, n_fft: int) -> np.ndarray:
    re = np.zeros(n_fft // 2 + 1)
    im = np.zeros(n_fft // 2 + 1)
    _check(_lib.fdtd_probe_fft_noalloc(g, int(pid), int(n_fft), _ptr(re), _ptr(im)))
    return re + 1j * im


def fdtd_get_probe(g, pid: int, n: int) -> np.ndarray:
    out = np.zeros(int(n), np.float32)
    _check(_lib.fdtd_get_probe(g, int(pid), _ptr(out) if n else None, int(n)))
    return out


def fdtd_get_voltage(g, vid: int, n: int) -> np.ndarray:
    out = np.zeros(int(n), np.float64)
    _check(_lib.fdtd_get_voltage(g, int(vid), _ptr(out) if n else None, int(n)))
    return out


def fdtd_get_dft(g, pid: int) -> np.ndarray:
    nf = fdtd_get_info(g).n_freqs
    re = np.zeros(nf)
    im = np.zeros(nf)
    _check(_lib.fdtd_get_dft(g, int(pid), _ptr(re), _ptr(im)))
    return re + 1j * im


def fdtd_get_field(g, comp: int, shape) -> np.ndarray:
    out = np.zeros(shape, np.float32)
    _check(_lib.fdtd_get_field(g, int(comp), _ptr(out)))
    return out


def fdtd_set_field(g, comp: int, values: np.ndarray):
    v = np.ascontiguousarray(values, dtype=np.float32)
    _check(_lib.fdtd_set_field(g, int(comp), _ptr(v)))


def fdtd_state_bytes(g) -> int:
    n = _lib.fdtd_state_bytes(g)
    if n < 0:
        raise FdtdError(int(n), fdtd_last_error())
    return int(n)


def fdtd_save_state(g) -> bytes:
    n = fdtd_state_bytes(g)
    buf = (C.c_char * n)()
    _check(_lib.fdtd_save_state(g, buf, n))
    return bytes(buf)


def fdtd_load_state(g, image: bytes):
    buf = C.create_string_buffer(image, len(image))
    _check(_lib.fdtd_load_state(g, buf, len(image)))


def fdtd_estimate_bytes(nx, ny, nz, dx, dy, dz, *, n_sources=0, n_probes=0, n_freqs=0,
                        dt=0.0, courant=0.99, npml=(8,) * 6, pml_m=3.0, pml_R=1e-6,
                        pml_kappa_max=1.0, max_steps=1) -> int:
    d = _desc(nx, ny, nz, dx, dy, dz, dt, courant, npml, pml_m, pml_R, pml_kappa_max,
              max_steps, None, None)
    v = _lib.fdtd_estimate_bytes(C.byref(d), int(n_sources), int(n_probes), int(n_freqs))
    if v < 0:
        raise FdtdError(int(v), fdtd_last_error())
    return int(v)


def board_bytes(board, max_steps: Optional[int] = None) -> int:
    """Upper bound of the device bytes a handle for ``board`` holds."""
    b = board
    return fdtd_estimate_bytes(b.nx, b.ny, b.nz, b.dx, b.dy, b.dz, n_sources=len(b.sources),
                               n_probes=len(b.probes),
                               n_freqs=0 if b.dft_freqs is None else len(b.dft_freqs),
                               dt=b.dt, courant=b.courant, npml=b.npml, pml_m=b.pml_m,
                               pml_R=b.pml_R, pml_kappa_max=b.pml_kappa_max,
                               max_steps=int(max_steps if max_steps is not None else b.steps))


def fdtd_get_info(g) -> fdtd_info:
    out = fdtd_info()
    _check(_lib.fdtd_get_info(g, C.byref(out)))
    return out


def fdtd_set_tile(g, tile_x: int, tile_y: int, steps: int = 1):
    _check(_lib.fdtd_set_tile(g, int(tile_x), int(tile_y), int(steps)))


def fdtd_tile_shapes() -> List[tuple]:
    """(tile_x, tile_y, steps per pass) of every supported field-kernel shape."""
    buf = (C.c_int * 96)()
    n = _lib.fdtd_tile_shapes(buf, 32)
    return [(buf[3 * s], buf[3 * s + 1], buf[3 * s + 2]) for s in range(min(n, 32))]


def fdtd_set_timing(g, on: bool):
    _check(_lib.fdtd_set_timing(g, 1 if on else 0))


def fdtd_get_timing(g):
    ms = C.c_double()
    n = C.c_int64()
    _check(_lib.fdtd_get_timing(g, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def fdtd_get_stream(g) -> int:
    """The handle's hipStream_t as an integer (e.g. for torch.cuda.ExternalStream)."""
    p = C.c_void_p()
    _check(_lib.fdtd_get_stream(g, C.byref(p)))
    return int(p.value or 0)


def fdtd_synchronize(g):
    _check(_lib.fdtd_synchronize(g))


def fdtd_destroy_grid(g):
    _check(_lib.fdtd_destroy_grid(g))


# --------------------------------------------------------------------------
# marshalling a board description (any object with the boardgen.Board fields)

def grid_from_board(board, max_steps: Optional[int] = None, hip_stream=None,
                    allocator: Optional[TorchAllocator] = None, tile=None):
    """Create a handle and pass the board's materials, sources, probes and DFT
    frequencies to it.  Returns (handle, probe ids)."""
    b = board
    g = fdtd_create_grid(b.nx, b.ny, b.nz, b.dx, b.dy, b.dz, dt=b.dt, courant=b.courant,
                         npml=b.npml, pml_m=b.pml_m, pml_R=b.pml_R,
                         pml_kappa_max=b.pml_kappa_max,
                         max_steps=int(max_steps if max_steps is not None else b.steps),
                         hip_stream=hip_stream, allocator=allocator)
    try:
        fdtd_set_materials(g, b.eps_r_cell, b.pec_edge_mask)
        if getattr(b, "pml_eps_rw", False):
            fdtd_set_pml_eps_rw(g, True)
        if getattr(b, "sigma_cell", None) is not None:
            fdtd_set_conductivity(g, b.sigma_cell)
        if getattr(b, "sheet_R", 0.0):
            fdtd_set_sheet_resistance(g, b.sheet_R)
        for s in b.sources:
            if getattr(s, "R", 0.0) > 0.0:
                fdtd_add_voltage_source(g, s.i, s.j, s.k, s.waveform, s.J0, s.t0, s.sigma, s.R)
            else:
                fdtd_add_source(g, s.i, s.j, s.k, s.waveform, s.J0, s.t0, s.sigma)
        ids = [fdtd_add_probe(g, i, j, k) for (i, j, k) in b.probes]
        if b.dft_freqs is not None and len(b.dft_freqs):
            fdtd_set_dft_freqs(g, b.dft_freqs)
        if getattr(b, "plane_dft", None) is not None:
            fdtd_set_plane_dft(g, b.plane_dft[0], b.plane_dft[1])
        if tile is not None:
            fdtd_set_tile(g, *tile)
    except Exception:
        fdtd_destroy_grid(g)
        raise
    return g, ids


def node_shape(board) -> tuple:
    return (board.nz + 1, board.ny + 1, board.nx + 1)
