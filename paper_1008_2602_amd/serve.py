"""Continuous-batching solve server over libfdtd.

Board-solve requests arrive over time.  At every chunk boundary the server
  1. admits waiting requests, oldest first, while their device footprint fits in
     the budget (a younger request may pass an older one that does not fit, until
     the older one has waited ``max_bypass_s``; after that nothing passes it);
  2. advances every resident board by up to ``chunk`` steps in shared launches
     (``fdtd_step_many``), so requests that arrived while others were running
     join them on the device;
  3. finishes the boards that reached their step count (probe series and DFT
     read back, handle destroyed, footprint released).
Fields stay resident on the device between chunks.  Latency is completion time
minus arrival time.  The executor is pluggable: ``GpuExecutor`` drives the
library, tests drive the same scheduler with a modelled executor on the CPU.

With an executor that can enqueue a chunk without waiting for it
(``step_async``) and ``workers`` > 0, the loop is pipelined: admitted requests
are set up (device buffers, material classes, tables) on worker threads while
the device runs the current chunks, and finished boards are read back and
released on workers too; up to ``depth`` chunks are in flight, the next one
enqueued before the previous one ends, so the device does not idle at chunk
boundaries.  A prepared board joins the first chunk enqueued after its set-up
is done; the budget counts a board from admission until it is released.
"""
from __future__ import annotations

import heapq
import threading
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor
from concurrent.futures import wait as wait_futures
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class SolveRequest:
    rid: int
    arrival_s: float
    board: Any                      # boardgen.Board-like (geometry, sources, probes, steps)
    steps: Optional[int] = None     # default board.steps

    @property
    def n_steps(self) -> int:
        return int(self.steps if self.steps is not None else self.board.steps)


@dataclass
class SolveResult:
    rid: int
    arrival_s: float
    admit_s: float
    finish_s: float
    steps: int
    cells: int
    probes: Optional[np.ndarray] = None
    dft: Optional[np.ndarray] = None

    @property
    def latency_s(self) -> float:
        return self.finish_s - self.arrival_s

    @property
    def wait_s(self) -> float:
        return self.admit_s - self.arrival_s


@dataclass
class _Resident:
    req: SolveRequest
    handle: Any
    probe_ids: List[int]
    done: int
    bytes: int
    admit_s: float


class _StreamPool:
    """HIP streams (non-blocking, default priority) owned by the executor for its
    whole life: each resident board has one to itself, and a finished board's
    stream goes back to the pool.  Streams outlive every event recorded on them,
    and no two live boards share one (a batched call captures its launches on
    its first board's stream, which no other thread may touch meanwhile)."""

    def __init__(self):
        import ctypes
        # the HIP runtime the library and PyTorch already use
        self._hip = ctypes.CDLL("libamdhip64.so.7")
        self._c = ctypes
        self._free: List[int] = []
        self._all: List[int] = []
        self._lock = threading.Lock()

    def get(self) -> int:
        with self._lock:
            if self._free:
                return self._free.pop()
        s = self._c.c_void_p()
        rc = self._hip.hipStreamCreateWithFlags(self._c.byref(s), 1)   # hipStreamNonBlocking
        if rc != 0 or not s.value:
            raise RuntimeError(f"hipStreamCreateWithFlags failed ({rc})")
        with self._lock:
            self._all.append(int(s.value))
        return int(s.value)

    def put(self, stream: int) -> None:
        with self._lock:
            self._free.append(stream)

    def close(self) -> None:
        with self._lock:
            for st in self._all:
                self._hip.hipStreamSynchronize(self._c.c_void_p(st))
                self._hip.hipStreamDestroy(self._c.c_void_p(st))
            self._all, self._free = [], []


class GpuExecutor:
    """Runs boards through libfdtd on the current device.  Every resident board
    runs on a stream of its own from the executor's pool; a chunk runs on its
    first board's stream, bracketed by events for the device-busy figure."""

    def __init__(self, allocator=None, tile=None, collect=True):
        import torch
        from . import fdtd as F
        self.F = F
        self.torch = torch
        self.allocator = allocator
        self.tile = tile
        self.collect = collect
        self.pool = _StreamPool()
        self.streams = {}               # id(handle) -> (raw stream, torch view of it)
        self._lock = threading.Lock()
        self.chunk_events = []          # (start, end) events of every chunk

    def footprint(self, req: SolveRequest) -> int:
        return self.F.board_bytes(req.board, max_steps=req.n_steps)

    def create(self, req: SolveRequest):
        """Set up a board (device buffers, classes, tables, work lists) on its own
        stream; returns when the board is ready to step."""
        raw = self.pool.get()
        try:
            g, ids = self.F.grid_from_board(req.board, max_steps=req.n_steps,
                                            allocator=self.allocator, tile=self.tile,
                                            hip_stream=raw)
        except Exception:
            self.pool.put(raw)
            raise
        self.F.fdtd_step_n(g, 0)               # finalise now, not inside a chunk
        self.F.fdtd_synchronize(g)
        with self._lock:
            self.streams[id(g)] = (raw, self.torch.cuda.ExternalStream(raw))
        return g, ids

    def step_async(self, handles: Sequence, ns: Sequence[int]):
        """Enqueue one chunk (no wait); returns its completion token."""
        st = self.streams[id(handles[0])][1]
        start = self.torch.cuda.Event(enable_timing=True)
        end = self.torch.cuda.Event(enable_timing=True)
        start.record(st)
        self.F.fdtd_step_many(list(handles), list(ns))
        end.record(st)
        self.chunk_events.append((start, end))
        return end

    def wait(self, token) -> None:
        token.synchronize()

    def step(self, handles: Sequence, ns: Sequence[int]) -> None:
        self.wait(self.step_async(handles, ns))

    def busy_fraction(self) -> Optional[float]:
        """Share of the time from the first chunk's start to the last chunk's end
        that some chunk ran on the device."""
        if not self.chunk_events:
            return None
        self.chunk_events[-1][1].synchronize()     # chunks run in order
        first = self.chunk_events[0][0]
        busy = 0.0
        last_end = 0.0
        for s, e in self.chunk_events:
            t0 = max(first.elapsed_time(s), last_end)
            t1 = first.elapsed_time(e)
            busy += max(0.0, t1 - t0)
            last_end = max(last_end, t1)
        return busy / last_end if last_end > 0 else None

    def finish(self, handle, probe_ids, req: SolveRequest):
        F = self.F
        probes = dft = None
        if self.collect:
            probes = np.stack([F.fdtd_get_probe(handle, p, req.n_steps) for p in probe_ids]) \
                if probe_ids else np.zeros((0, req.n_steps), np.float32)
            if req.board.dft_freqs is not None and probe_ids:
                dft = np.stack([F.fdtd_get_dft(handle, p) for p in probe_ids])
        F.fdtd_destroy_grid(handle)             # waits for the handle's stream
        with self._lock:
            raw, _ = self.streams.pop(id(handle), (None, None))
        if raw is not None:
            self.pool.put(raw)
        return probes, dft

    def close(self) -> None:
        """Release the stream pool (after every board is finished)."""
        self.pool.close()

    def now(self) -> float:
        return time.perf_counter()

    def wait_until(self, t: float) -> None:
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)


def _cells(req: SolveRequest) -> int:
    b = req.board
    return b.nx * b.ny * b.nz


class Server:
    def __init__(self, executor, budget_bytes: int, chunk: int = 500,
                 max_resident: Optional[int] = None, max_bypass_s: float = 5.0,
                 log: Optional[Callable[[dict], None]] = None, workers: int = 0,
                 depth: int = 2, solo_cells: Optional[int] = None):
        if budget_bytes <= 0 or chunk <= 0:
            raise ValueError("budget and chunk must be positive")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.max_resident = max_resident
        self.max_bypass_s = float(max_bypass_s)
        self.log = log
        self.workers = int(workers)
        self.depth = max(1, int(depth))
        # boards of at least solo_cells cells run their chunks without the
        # smaller resident boards (which wait, resident, until none is left):
        # a large solve then runs at about its own rate instead of pacing, and
        # being paced by, every chunk it shares; None: every chunk holds every
        # resident board
        self.solo_cells = solo_cells
        self.chunks = 0
        self.peak_bytes = 0
        self.peak_resident = 0
        self.rejected: List[int] = []

    def _chunk_boards(self, resident: List["_Resident"]) -> List["_Resident"]:
        """The resident boards the next chunk advances."""
        if self.solo_cells is None:
            return resident
        solo = [e for e in resident if _cells(e.req) >= self.solo_cells]
        return solo or resident

    def run(self, requests: Sequence[SolveRequest]) -> List[SolveResult]:
        if self.workers > 0 and hasattr(self.ex, "step_async"):
            return self._run_pipelined(requests)
        ex = self.ex
        pending = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        foot = {}
        for r in pending:
            foot[r.rid] = ex.footprint(r)
            if foot[r.rid] > self.budget:
                self.rejected.append(r.rid)
        pending = [r for r in pending if r.rid not in set(self.rejected)]
        t0 = ex.now()
        waiting: List[SolveRequest] = []
        resident: List[_Resident] = []
        used = 0
        results: List[SolveResult] = []
        nxt = 0
        while nxt < len(pending) or waiting or resident:
            now = ex.now() - t0
            while nxt < len(pending) and pending[nxt].arrival_s <= now:
                waiting.append(pending[nxt])
                nxt += 1
            # admission: oldest first; younger requests may pass a blocked one until
            # it has waited max_bypass_s
            admitted = []
            blocked_since = None
            for r in list(waiting):
                if self.max_resident is not None and len(resident) >= self.max_resident:
                    break
                fits = used + foot[r.rid] <= self.budget
                if not fits:
                    if blocked_since is None:
                        blocked_since = r.arrival_s
                    if now - blocked_since >= self.max_bypass_s:
                        break
                    continue
                h, ids = ex.create(r)
                used += foot[r.rid]
                resident.append(_Resident(r, h, ids, 0, foot[r.rid], ex.now() - t0))
                waiting.remove(r)
                admitted.append(r.rid)
            self.peak_bytes = max(self.peak_bytes, used)
            self.peak_resident = max(self.peak_resident, len(resident))
            if not resident:
                if nxt < len(pending):
                    ex.wait_until(t0 + pending[nxt].arrival_s)
                    continue
                if waiting:
                    raise RuntimeError("a waiting request can never be admitted")
                break
            batch = self._chunk_boards(resident)
            ns = [min(self.chunk, e.req.n_steps - e.done) for e in batch]
            ex.step([e.handle for e in batch], ns)
            self.chunks += 1
            for e, n in zip(batch, ns):
                e.done += n
            fin_t = ex.now() - t0
            still = []
            for e in resident:
                if e.done >= e.req.n_steps:
                    probes, dft = ex.finish(e.handle, e.probe_ids, e.req)
                    used -= e.bytes
                    b = e.req.board
                    results.append(SolveResult(e.req.rid, e.req.arrival_s, e.admit_s, fin_t,
                                               e.req.n_steps, b.nx * b.ny * b.nz, probes, dft))
                else:
                    still.append(e)
            resident = still
            if self.log:
                self.log(dict(t=fin_t, chunk=self.chunks, resident=len(resident),
                              waiting=len(waiting), used=used, admitted=admitted))
        return sorted(results, key=lambda r: r.rid)


    # ------------------------------------------------------------------ pipelined
    def _admit(self, waiting, foot, used, n_live, now):
        """Requests to admit now, oldest first, within the budget (younger ones may
        pass a blocked one until it has waited max_bypass_s)."""
        out = []
        blocked_since = None
        for r in waiting:
            if self.max_resident is not None and n_live + len(out) >= self.max_resident:
                break
            if used + foot[r.rid] > self.budget:
                if blocked_since is None:
                    blocked_since = r.arrival_s
                if now - blocked_since >= self.max_bypass_s:
                    break
                continue
            out.append(r)
            used += foot[r.rid]
        return out

    def _run_pipelined(self, requests: Sequence[SolveRequest]) -> List[SolveResult]:
        ex = self.ex
        pending = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        foot = {r.rid: ex.footprint(r) for r in pending}
        self.rejected = [r.rid for r in pending if foot[r.rid] > self.budget]
        rejected = set(self.rejected)
        pending = [r for r in pending if r.rid not in rejected]
        t0 = ex.now()
        waiting: List[SolveRequest] = []
        preparing = {}                 # future -> (request, admit time)
        resident: List[_Resident] = []
        inflight = []                  # (token, [boards that complete in that chunk])
        finishing = {}                 # future -> _Resident
        results: List[SolveResult] = []
        used = 0
        nxt = 0
        pool = ThreadPoolExecutor(max_workers=self.workers)

        def finish_job(e: _Resident):
            # the board's reads wait on its own stream, which the batched call
            # orders after the chunk the board completed in; only the main
            # thread waits on chunk tokens
            probes, dft = ex.finish(e.handle, e.probe_ids, e.req)
            b = e.req.board
            return SolveResult(e.req.rid, e.req.arrival_s, e.admit_s, ex.now() - t0,
                               e.req.n_steps, b.nx * b.ny * b.nz, probes, dft)

        try:
            while nxt < len(pending) or waiting or preparing or resident or inflight or finishing:
                now = ex.now() - t0
                while nxt < len(pending) and pending[nxt].arrival_s <= now:
                    waiting.append(pending[nxt])
                    nxt += 1
                # boards whose set-up is done join the next chunk
                for f in [f for f in preparing if f.done()]:
                    r, adm = preparing.pop(f)
                    h, ids = f.result()
                    resident.append(_Resident(r, h, ids, 0, foot[r.rid], adm))
                # released boards give their budget back
                for f in [f for f in finishing if f.done()]:
                    e = finishing.pop(f)
                    results.append(f.result())
                    used -= e.bytes
                admitted = self._admit(waiting, foot, used,
                                       len(resident) + len(preparing), now)
                for r in admitted:
                    waiting.remove(r)
                    used += foot[r.rid]
                    preparing[pool.submit(ex.create, r)] = (r, now)
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_resident = max(self.peak_resident, len(resident))
                if resident and len(inflight) < self.depth:
                    batch = self._chunk_boards(resident)
                    ns = [min(self.chunk, e.req.n_steps - e.done) for e in batch]
                    token = ex.step_async([e.handle for e in batch], ns)
                    self.chunks += 1
                    for e, n in zip(batch, ns):
                        e.done += n
                    done = [e for e in batch if e.done >= e.req.n_steps]
                    resident = [e for e in resident if e.done < e.req.n_steps]
                    inflight.append((token, done))
                    for e in done:
                        finishing[pool.submit(finish_job, e)] = e
                    if self.log:
                        self.log(dict(t=ex.now() - t0, chunk=self.chunks, resident=len(resident),
                                      waiting=len(waiting), used=used,
                                      admitted=[r.rid for r in admitted]))
                    continue
                if inflight:
                    # the oldest chunk in flight ends before the next is enqueued
                    token, _ = inflight.pop(0)
                    ex.wait(token)
                    continue
                if preparing or finishing:
                    wait_futures(list(preparing) + list(finishing), return_when=FIRST_COMPLETED,
                                 timeout=(None if nxt >= len(pending) else
                                          max(0.0, pending[nxt].arrival_s - (ex.now() - t0))))
                    continue
                if nxt < len(pending):
                    ex.wait_until(t0 + pending[nxt].arrival_s)
                    continue
                if waiting:
                    raise RuntimeError("a waiting request can never be admitted")
        finally:
            pool.shutdown(wait=True)
        return sorted(results, key=lambda r: r.rid)


def summarize(results: Sequence[SolveResult], wall_s: Optional[float] = None) -> Dict[str, float]:
    if not results:
        return {"completed": 0}
    lat = np.array([r.latency_s for r in results])
    wait = np.array([r.wait_s for r in results])
    span = wall_s if wall_s is not None else max(r.finish_s for r in results) - min(
        r.arrival_s for r in results)
    cell_updates = float(sum(r.cells * r.steps for r in results))
    return {
        "completed": len(results),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_wait_s": float(wait.mean()),
        "solves_per_s": len(results) / span if span > 0 else float("inf"),
        "gcell_updates_per_s": cell_updates / span / 1e9 if span > 0 else float("inf"),
        "span_s": span,
    }
