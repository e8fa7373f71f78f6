"""Serving loop: continuous batching of energy + gradient requests.

Requests (an instance: qubit count, reference, ansatz strings, grouped
Hamiltonian, angles) arrive over time.  The server keeps one device arena
allocated for its lifetime and never allocates or frees device memory while
serving (hipFree would synchronize the device).  Scheduling:

* admission: requests wait FIFO; the head of the queue is admitted when its
  device footprint (tables + two states, exact size from
  qf_batch_create_arena's size query) fits a free range of the arena;
* continuous batching: whenever one of `slots` launch slots (one HIP stream
  each) is idle, everything admissible in the queue (up to `max_wave`
  requests) becomes one wave, a persistent batched launch on that slot's
  stream.  Waves on different slots overlap on the device: a new wave's
  workgroups start on compute units as soon as they are free;
* completion per request: each slot owns a mailbox (coherent pinned host
  memory); the kernel publishes an instance's energy and gradient there and
  then raises its flag as soon as that instance's team is done, so a short
  request in a wave completes without waiting for the wave's long ones.  A
  wave's arena range and slot are released when the whole launch finishes;
* solo lane (solo_qubits): a request of at least that many qubits fills the
  device by itself, and the single-instance kernels (a plan: blocked apply,
  sigma, blocked adjoint, each a full-grid launch) run it faster than a team
  of the persistent kernel, which has to meet at a barrier after every pass.
  Such requests queue FIFO for one solo lane: a host thread that runs the
  plan path on its own stream while the batched waves of the smaller
  requests go on beside it.  The plan's tables and the request's two states
  share one arena range (qf_plan_create_arena), released when the request
  finishes, so the lane never allocates or frees device memory and its
  footprint is bounded by one request;
* co-residency: up to `slots` persistent launches overlap, so every team is
  capped at (resident grid) / slots workgroups (the library enforces it and
  the server checks it): overlapping waves can always gather their teams;
* failures: a request whose team barrier times out (its wave's mailbox flag
  reads 2) or whose solo-lane call raises is marked failed with its error;
  the other requests of the wave and of the trace complete normally.

Latency is measured from a request's arrival to its completion (mailbox
flag or solo-lane return).  The plain path (`serve_plain`) runs the same
trace one request at a time with the single-instance kernels.
"""
from __future__ import annotations

import ctypes
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import api
from ._lib import QF_OK, QFError, check, lib, ptr, stream_handle

ALIGN = 256
QF_E_HIP = -4
# Requests of at least this many qubits take the solo lane (on MI355X a
# 24-qubit request takes 235 ms on the plan kernels and 292 ms as a team of
# the persistent kernel; below 20 qubits the batched waves win).
SOLO_QUBITS = 20


@dataclass
class Request:
    rid: int
    arrival: float
    n: int
    occ: int
    A: np.ndarray
    H: np.ndarray
    off: np.ndarray
    theta: np.ndarray
    E: float | None = None
    grad: np.ndarray | None = None
    t_admit: float | None = None
    t_done: float | None = None
    footprint: int = 0
    team: int = 0  # workgroups the request's instance ran with (0: solo lane)
    solo: bool = False  # ran on the solo lane (plan kernels)
    plan_bytes: int = 0  # solo lane: arena bytes of the plan's tables
    error: str | None = None  # set when the request failed (t_done is then its failure time)


class RangeAllocator:
    """First-fit allocator of 256-byte aligned ranges in [0, nbytes)."""

    def __init__(self, nbytes: int):
        self.nbytes = (int(nbytes) // ALIGN) * ALIGN
        self.free = [(0, self.nbytes)]  # sorted, coalesced (offset, size)

    def alloc(self, size: int):
        size = (int(size) + ALIGN - 1) // ALIGN * ALIGN
        for i, (o, s) in enumerate(self.free):
            if s >= size:
                if s == size:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + size, s - size)
                return o, size
        return None

    def release(self, off: int, size: int):
        self.free.append((off, size))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def largest(self) -> int:
        return max((s for _, s in self.free), default=0)


class Arena(RangeAllocator):
    """A RangeAllocator over one device buffer held for the server's lifetime."""

    def __init__(self, nbytes: int):
        import torch
        super().__init__(nbytes)
        self.buf = torch.empty(self.nbytes + ALIGN, dtype=torch.uint8, device="cuda")
        self.base = (self.buf.data_ptr() + ALIGN - 1) // ALIGN * ALIGN


def _arrays(reqs, team_table, share: bool = False, concurrent: int = 1):
    """C arrays of a wave.  share: ask the library to split the resident grid
    by work (team < 0), with the table's team size as each floor;
    concurrent: persistent launches that may overlap (caps the teams)."""
    c = len(reqs)
    keep = [np.ascontiguousarray(r.off, dtype=np.int64) for r in reqs]
    n = (ctypes.c_int * c)(*[r.n for r in reqs])
    occ = (ctypes.c_uint64 * c)(*[r.occ for r in reqs])
    K = (ctypes.c_int64 * c)(*[len(r.A) for r in reqs])
    A = (ctypes.c_void_p * c)(*[ptr(r.A) for r in reqs])
    H = (ctypes.c_void_p * c)(*[ptr(r.H) for r in reqs])
    O = (ctypes.c_void_p * c)(*[ptr(o) for o in keep])
    G = (ctypes.c_int64 * c)(*[len(o) - 1 for o in keep])
    base = [int(team_table.get(r.n, 0)) if team_table else 0 for r in reqs]
    T = (ctypes.c_int * c)(*[-max(1, w) if share else w for w in base])
    return (c, n, occ, A, K, H, O, G, T, int(concurrent)), keep


def default_team_table() -> dict:
    """The tuned team sizes for this device ({} if none match it)."""
    from .autotune import device_arch, load_table
    return load_table(device_arch()) or {}


def footprint(reqs, team_table=None, share: bool = False, concurrent: int = 1) -> int:
    """Exact arena bytes a wave of these requests needs (with the same team
    policy as the launch).  With share, a request's team in a wave is never
    larger than alone, so footprint([r], ..., share=True) bounds its part."""
    args, keep = _arrays(reqs, team_table, share, concurrent)
    need = ctypes.c_int64()
    check(lib.qf_batch_create_arena(*args, None, 0, ctypes.byref(need), None, None), "qf_batch_create_arena(size)")
    return need.value


@dataclass
class Wave:
    reqs: list
    handle: ctypes.c_void_p
    slot: int
    arena_range: tuple
    t_launch: float
    keep: list = field(default_factory=list)
    E: np.ndarray | None = None      # mailbox views
    grad: np.ndarray | None = None
    flag: np.ndarray | None = None
    koff: list = field(default_factory=list)
    open: int = 0                    # requests not yet published


class _Addr:
    """A device address in the arena, passed where the API takes a buffer."""

    def __init__(self, addr: int):
        self.addr = addr

    def data_ptr(self) -> int:
        return self.addr


def _align(v: int) -> int:
    return (int(v) + ALIGN - 1) // ALIGN * ALIGN


def solo_footprint(r) -> int:
    """Arena bytes of a solo-lane request: its plan's tables, then its two
    states (phi, lambda)."""
    if not r.plan_bytes:
        r.plan_bytes = _align(api.Plan.arena_bytes(r.n, r.A, r.H, r.off))
    return r.plan_bytes + 2 * (1 << r.n) * 16


def _view(addr: int, ctype, count: int) -> np.ndarray:
    return np.ctypeslib.as_array(ctypes.cast(ctypes.c_void_p(addr), ctypes.POINTER(ctype)), shape=(count,))


class Server:
    def __init__(self, arena_bytes: int, slots: int = 2, max_wave: int = 64, team_table=None,
                 mailbox_bytes: int = 32 << 20, share: bool = True, solo_qubits: int | None = SOLO_QUBITS,
                 spin_limit: int | None = None):
        """spin_limit: polls before a wave's team barrier gives up (None: the
        library default); a tiny value forces barrier timeouts from the host."""
        import torch
        if team_table is None:
            team_table = default_team_table()
        self.team = team_table
        self.share = share  # split the grid among a wave's requests by work
        self.solo_qubits = solo_qubits  # None: every request goes through batched waves
        self.spin_limit = spin_limit
        self.arena = Arena(arena_bytes)
        self.solo_stream = torch.cuda.Stream()
        self.solo_job = None      # (thread, request, arena range)
        self.solo_runs = 0
        self.solo_live = 0        # solo-lane plans alive now / at most (one request at a time)
        self.solo_live_max = 0
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.busy = [None] * slots
        self.max_wave = max_wave
        self.mb_bytes = int(mailbox_bytes)
        self.mailbox = []
        for _ in range(slots):
            m = ctypes.c_void_p()
            check(lib.qf_mailbox_alloc(self.mb_bytes, ctypes.byref(m)), "qf_mailbox_alloc")
            self.mailbox.append(m)
        self.waves = 0
        self.wave_sizes = []
        self.max_busy = 0  # most waves in flight at once (overlap on the device)

    def close(self):
        for m in self.mailbox:
            lib.qf_mailbox_free(m)
        self.mailbox = []

    def __del__(self):
        if getattr(self, "mailbox", None):
            self.close()

    def _launch(self, reqs, slot, now):
        args, keep = _arrays(reqs, self.team, self.share, len(self.streams))
        need = ctypes.c_int64()
        check(lib.qf_batch_create_arena(*args, None, 0, ctypes.byref(need), None, None), "arena size")
        rng = self.arena.alloc(need.value)
        if rng is None:
            return None
        h = ctypes.c_void_p()
        st = stream_handle(self.streams[slot])
        check(lib.qf_batch_create_arena(*args, ctypes.c_void_p(self.arena.base + rng[0]), rng[1],
                                        ctypes.byref(need), st, ctypes.byref(h)), "qf_batch_create_arena")
        teams = (ctypes.c_int * len(reqs))()
        grid = ctypes.c_int()
        check(lib.qf_batch_info(h, teams, None, ctypes.byref(grid)), "qf_batch_info")
        # co-residency of overlapping waves: no team above the grid's share
        # (the grid is already trimmed to the wave's tickets, so compare with
        # what the library used: resident grid / slots >= any team it made)
        cap = max(1, self.resident_grid // len(self.streams))
        if max(teams) > cap:
            raise RuntimeError(f"team of {max(teams)} workgroups above the co-residency cap {cap}")
        for r, w in zip(reqs, teams):
            r.team = int(w)
        if self.spin_limit is not None:
            check(lib.qf_batch_set_spin_limit(h, int(self.spin_limit)), "qf_batch_set_spin_limit")
        theta = np.ascontiguousarray(np.concatenate([r.theta for r in reqs]), dtype=np.float64)
        keep.append(theta)
        mb = self.mailbox[slot].value
        check(lib.qf_batch_launch_mailbox(h, ptr(theta), ctypes.c_void_p(mb), self.mb_bytes, st),
              "qf_batch_launch_mailbox")
        for r in reqs:
            r.t_admit = now
        self.waves += 1
        self.wave_sizes.append(len(reqs))
        c, kt = len(reqs), sum(len(r.A) for r in reqs)
        koff = np.concatenate([[0], np.cumsum([len(r.A) for r in reqs])]).tolist()
        return Wave(reqs, h, slot, rng, now, keep, E=_view(mb, ctypes.c_double, c),
                    grad=_view(mb + 8 * c, ctypes.c_double, max(kt, 1)),
                    flag=_view(mb + 8 * c + 8 * kt, ctypes.c_uint32, c), koff=koff, open=c)

    def _publish(self, w: Wave, now):
        """Complete every request of w whose mailbox flag is up (1: result,
        2: its team barrier timed out)."""
        for i, r in enumerate(w.reqs):
            if r.t_done is None and w.flag[i] in (1, 2):
                if w.flag[i] == 1:
                    r.E = float(w.E[i])
                    r.grad = w.grad[w.koff[i]:w.koff[i + 1]].copy()
                else:
                    r.error = "team barrier timed out"
                r.t_done = now
                w.open -= 1

    def _solo_run(self, r, addr: int, t0: float):
        """Solo lane body (host thread): arena plan, energy + gradient.  A
        failure marks this request only."""
        try:
            plan = api.Plan(r.n, r.A, r.H, r.off, arena=(addr, r.plan_bytes), stream=self.solo_stream)
            self.solo_live += 1
            self.solo_live_max = max(self.solo_live_max, self.solo_live)
            try:
                r.E, r.grad = plan.energy_grad(r.occ, r.theta, _Addr(addr + r.plan_bytes), self.solo_stream)
            finally:
                plan.close()
                self.solo_live -= 1
        except Exception as e:  # recorded on the request; the loop goes on
            r.error = f"{type(e).__name__}: {e}"
        r.t_done = time.perf_counter() - t0

    def _solo_poll(self, pending_solo, t0) -> int:
        """Retire a finished solo request, start the next if it fits.
        Returns the number of requests completed (or failed)."""
        done = 0
        if self.solo_job is not None and not self.solo_job[0].is_alive():
            th, r, rng = self.solo_job
            th.join()
            self.solo_job = None
            self.arena.release(*rng)
            done += 1
        if self.solo_job is None and pending_solo:
            r = pending_solo[0]
            rng = self.arena.alloc(r.footprint)
            if rng is not None:
                pending_solo.pop(0)
                r.t_admit = time.perf_counter() - t0
                r.solo, r.team = True, 0
                th = threading.Thread(target=self._solo_run, args=(r, self.arena.base + rng[0], t0), daemon=True)
                self.solo_job = (th, r, rng)
                self.solo_runs += 1
                th.start()
        return done

    def _finish(self, w: Wave, now):
        E = np.zeros(len(w.reqs))
        g = np.zeros(max(1, sum(len(r.A) for r in w.reqs)))
        st = lib.qf_batch_collect(w.handle, ptr(E), ptr(g))
        status = (ctypes.c_int * len(w.reqs))()
        check(lib.qf_batch_status(w.handle, status), "qf_batch_status")
        if st != QF_OK and not (st == QF_E_HIP and any(v != QF_OK for v in status)):
            raise QFError(st, "qf_batch_collect", lib.qf_last_error().decode())
        lib.qf_batch_destroy(w.handle)
        self._publish(w, now)
        for i, r in enumerate(w.reqs):  # requests whose flag the host had not seen
            if r.t_done is None:
                if status[i] == QF_OK:
                    r.E = float(E[i])
                    r.grad = g[w.koff[i]:w.koff[i + 1]].copy()
                else:
                    r.error = "team barrier timed out"
                r.t_done = now
                w.open -= 1
        self.arena.release(*w.arena_range)

    def serve(self, requests, poll_s: float = 50e-6):
        """Replay `requests` (sorted by arrival, seconds from start).  Returns stats."""
        def is_solo(r):
            return self.solo_qubits is not None and r.n >= self.solo_qubits

        self.resident_grid = resident_grid()

        def size(r):
            if not r.footprint and r.error is None:
                try:
                    r.footprint = (solo_footprint(r) if is_solo(r)
                                   else footprint([r], self.team, self.share, len(self.streams)))
                except QFError as e:  # an invalid request is rejected at its arrival
                    r.error = f"rejected: {e}"

        # the size queries are host work of the library (they release the
        # interpreter lock): taken before the replay, 16 at a time
        with ThreadPoolExecutor(max_workers=16) as ex:
            list(ex.map(size, requests))
        for r in requests:
            if r.footprint > self.arena.nbytes:
                raise ValueError(f"request {r.rid} needs {r.footprint} bytes, arena has {self.arena.nbytes}")
        pending, pending_solo = [], []
        t0 = time.perf_counter()
        try:
            self._replay(requests, is_solo, pending, pending_solo, t0, poll_s)
        finally:
            if self.solo_job is not None:
                self.solo_job[0].join()
                self.arena.release(*self.solo_job[2])
                self.solo_job = None
            import torch
            torch.cuda.synchronize()
        out = stats(requests, self.waves, self.wave_sizes)
        out["max_waves_in_flight"] = self.max_busy
        out["solo_requests"] = self.solo_runs
        return out

    def _replay(self, requests, is_solo, pending, pending_solo, t0, poll_s):
        nxt = 0
        done = 0
        while done < len(requests):
            now = time.perf_counter() - t0
            while nxt < len(requests) and requests[nxt].arrival <= now:
                r = requests[nxt]
                nxt += 1
                if r.error is not None:  # rejected at admission
                    r.t_done = now
                    done += 1
                    continue
                (pending_solo if is_solo(r) else pending).append(r)
            done += self._solo_poll(pending_solo, t0)
            for s, w in enumerate(self.busy):
                if w is None:
                    continue
                before = w.open
                self._publish(w, time.perf_counter() - t0)
                done += before - w.open
                if lib.qf_batch_poll(w.handle) == 0:
                    before = w.open
                    self._finish(w, time.perf_counter() - t0)
                    done += before
                    self.busy[s] = None
            for s in range(len(self.busy)):
                if self.busy[s] is not None or not pending:
                    continue
                # FIFO admission by footprint: the head must fit before anything behind it
                wave, budget, mb = [], self.arena.largest(), 0
                for r in pending[:self.max_wave]:
                    mb_r = 12 + 8 * len(r.A)
                    if r.footprint > budget or mb + mb_r > self.mb_bytes:
                        break
                    wave.append(r)
                    budget -= r.footprint
                    mb += mb_r
                if not wave:
                    break
                w = self._launch(wave, s, time.perf_counter() - t0)
                if w is None:
                    break
                self.busy[s] = w
                pending = pending[len(wave):]
                self.max_busy = max(self.max_busy, sum(b is not None for b in self.busy))
            idle = not pending and not pending_solo and self.solo_job is None and all(b is None for b in self.busy)
            if nxt < len(requests) and idle:
                time.sleep(max(0.0, min(requests[nxt].arrival - (time.perf_counter() - t0), 1e-3)))
            else:
                time.sleep(poll_s)


def resident_grid() -> int:
    """Workgroups of the persistent batched kernel resident on this device."""
    g = ctypes.c_int()
    check(lib.qf_batch_resident_grid(ctypes.byref(g)), "qf_batch_resident_grid")
    return g.value


def serve_plain(requests, max_qubits: int, arena_bytes: int | None = None):
    """One request at a time, FIFO, single-instance kernels (qf_plan_*), each
    request's plan tables and states in one preallocated arena (no device
    allocation per request)."""
    import torch
    # plan sizes are taken before the replay, as the server takes footprints
    with ThreadPoolExecutor(max_workers=16) as ex:
        sizes = list(ex.map(lambda r: _align(api.Plan.arena_bytes(r.n, r.A, r.H, r.off)), requests))
    need = max(pb + 2 * (1 << r.n) * 16 for pb, r in zip(sizes, requests)) if arena_bytes is None \
        else int(arena_bytes)
    arena = Arena(need)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    for r, pb in zip(requests, sizes):
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.t_admit = time.perf_counter() - t0
        try:
            plan = api.Plan(r.n, r.A, r.H, r.off, arena=(arena.base, pb), stream=stream)
            try:
                r.E, r.grad = plan.energy_grad(r.occ, r.theta, _Addr(arena.base + pb), stream)
            finally:
                plan.close()
        except Exception as e:
            r.error = f"{type(e).__name__}: {e}"
        r.t_done = time.perf_counter() - t0
    return stats(requests, len(requests), [1] * len(requests))


def stats(requests, waves, wave_sizes):
    ok = [r for r in requests if r.error is None]
    lat = np.array([r.t_done - r.arrival for r in ok]) if ok else np.zeros(1)
    span = max(r.t_done for r in requests) - min(r.arrival for r in requests)
    return {"requests": len(requests), "completed": len(ok), "failed": len(requests) - len(ok),
            "throughput_req_per_s": len(ok) / span,
            "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
            "latency_ms_max": float(lat.max() * 1e3), "makespan_s": span, "waves": waves,
            "mean_wave_size": float(np.mean(wave_sizes)) if wave_sizes else 0.0}


def make_requests(qf, qi, trace, workers: int = 16):
    """Requests for (arrival, recipe) pairs; tables are built on the host
    before the replay (a request carries its tables), `workers` at a time
    (the builder calls release the interpreter lock)."""
    def one(item):
        j, (t, rcp) = item
        h, g = qi.integrals(rcp["n_orb"], rcp["n_elec"], rcp["seed"])
        H, off, _ = qf.build_paulis("hamiltonian", rcp["n_orb"], rcp["n_elec"], h, g)
        A, aoff, _ = qf.build_paulis("uccsd", rcp["n_orb"], rcp["n_elec"])
        theta = qf.ansatz_angles(A, aoff, qi.amplitudes(len(aoff) - 1, rcp["seed"], rcp["t_scale"]))
        return Request(j, float(t), 2 * rcp["n_orb"], (1 << rcp["n_elec"]) - 1, A, H, off, theta)
    with ThreadPoolExecutor(max_workers=max(1, int(workers))) as ex:
        return list(ex.map(one, enumerate(trace)))
