"""Continuous-batching server for two-star simulation requests.

Requests (N elements, mass ratio q, seed, step count) arrive over time. The server keeps every
admitted system's state on the GPU and advances all of them together: each round replays one
captured HIP graph that holds K leap-frog steps of every active system (one launch per kernel per
step over the whole segment table). Between rounds it retires finished systems, admits waiting
requests first-come first-served while their device footprint fits the memory budget, and builds
newly admitted systems on a second stream in a worker thread, so admission overlaps the running
rounds. A request whose footprint exceeds the whole budget is rejected. The budget bounds the
summed footprint of admitted systems; the server also records PyTorch's peak allocation over the
run, which the footprints bound (up to the allocator's rounding), and its peak cache, which may
exceed them when freed blocks of retired systems cannot be reused as they are.

Rounds are queued ``depth`` (default 2) ahead on the compute stream: while one round runs, the
host picks the next round's systems, builds its graph if needed and queues it, and only then waits
for the older round to retire the systems it finished (their final state is copied on a separate
stream after that round's event), so the GPU does not idle during the host's bookkeeping.

Which admitted systems take part in a round is a policy choice. ``"all"`` steps every resident
system each round (processor sharing: all requests finish together). ``"srpt"`` (default) orders
the resident systems by remaining work (steps left times N^2) and takes the shortest ones until
the round's per-step work reaches ``fill`` pair interactions, enough to keep the GPU busy, so short
requests finish first while large ones still fill the machine.

The one-at-a-time baseline runs the same trace through the single-system path (nb_step with one
system, same precision mode): each request, in arrival order, is created and stepped alone to
completion before the next one starts.

Each system's kernels, work split and reduction orders depend on its own size only, so its result
is bitwise the same alone and in any mix; both runs record a digest of every final state.

After every round the server reads each of the round's systems' non-finite counts (positions or
velocities that are NaN or infinite after the round's last step). A system that has one is
evicted at once with status ``"failed"``: queued rounds are drained first (they may still hold
it), then its graphs and device memory are released. Other systems are unaffected, since no
kernel reads another system's state.
"""

from __future__ import annotations

import collections
import dataclasses
import hashlib
import queue
import threading
import time

import numpy as np

from . import (
    MODES,
    NB_FP64,
    NbParams,
    nb_graph_create,
    nb_graph_destroy,
    nb_graph_launch,
    nb_nonfinite_async,
    nb_scratch_bytes,
)
from .system import System


@dataclasses.dataclass
class Record:
    rid: int
    n: int
    q: float
    steps: int
    t_arrive: float
    t_admit: float = float("nan")
    t_done: float = float("nan")
    bytes: int = 0
    status: str = "pending"
    digest: str = ""
    state: tuple = ()  # (positions, velocities) of the final state, with keep_states


def footprint_bytes(n: int, q: float, mode: str = "kahan") -> int:
    """Device bytes one system holds: nine state arrays, the side flags and the workspace."""
    import synth

    n1, _ = synth.particle_counts(n, q)
    m = MODES[mode]
    p = NbParams(n=n, n1=n1, G=1.0, m=1.0, dt=1e-4, D1=1.0, D2=1.0, q=q, a=1.0, R2_0=1.0,
                 growth_rate=1e-4, growth_on=1, mode=m)
    elem = 8 if m == NB_FP64 else 4
    return 9 * max(n, 1) * elem + max(n, 1) + nb_scratch_bytes(p) + 256


def state_digest(system: System, stream=None, after=None) -> str:
    """Hash of the final positions and velocities. With ``stream`` the copies run there, after
    ``after`` (an event) when given, and only that stream is waited for."""
    import torch

    h = hashlib.sha256()
    if stream is None:
        system.synchronize()
        for t in (system.x, system.y, system.z, system.vx, system.vy, system.vz):
            h.update(t[: system.n].cpu().numpy().tobytes())
        return h.hexdigest()[:32]
    with torch.cuda.stream(stream):
        if after is not None:
            stream.wait_event(after)
        host = [t[: system.n].to("cpu", non_blocking=True) for t in
                (system.x, system.y, system.z, system.vx, system.vy, system.vz)]
        stream.synchronize()
    for t in host:
        h.update(t.numpy().tobytes())
    return h.hexdigest()[:32]


def _build(req, mode: str, dt: float, stream) -> System:
    import synth

    ic = synth.make_binary(req.n, req.q, seed=req.seed)
    return System.from_ic(ic, mode=mode, dt=dt, stream=stream)


def _final_state(system: System) -> tuple:
    system.synchronize()
    return system.positions(), system.velocities()


def summarize(records, t0: float = 0.0) -> dict:
    done = [r for r in records if r.status == "done"]
    if not done:
        return {"completed": 0}
    lat = np.array([r.t_done - r.t_arrive for r in done])
    span = max(r.t_done for r in done) - min(r.t_arrive for r in records)
    inter = float(sum(float(r.n) ** 2 * r.steps for r in done))
    return {
        "completed": len(done),
        "rejected": sum(r.status == "rejected" for r in records),
        "failed": sum(r.status == "failed" for r in records),
        "span_s": span,
        "sims_per_s": len(done) / span if span > 0 else float("nan"),
        "interactions_per_s": inter / span if span > 0 else float("nan"),
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "latency_max_s": float(lat.max()),
    }


class BatchServer:
    def __init__(self, budget_bytes: int, round_steps: int = 10, max_active: int = 512,
                 mode: str = "kahan", dt: float = 1e-4, use_graphs: bool = True,
                 keep_digests: bool = True, policy: str = "srpt", fill: float = 1.2e10,
                 workers: int = 2, depth: int = 2, keep_states: bool = False):
        if policy not in ("srpt", "all"):
            raise ValueError("policy must be 'srpt' or 'all'")
        import torch

        self.torch = torch
        self.budget = int(budget_bytes)
        self.round_steps = int(round_steps)
        self.max_active = int(max_active)
        self.mode = mode
        self.dt = dt
        self.use_graphs = use_graphs
        self.keep_digests = keep_digests
        self.policy = policy
        self.fill = float(fill)
        self.workers = max(1, int(workers))
        self.depth = max(1, int(depth))
        self.compute = torch.cuda.Stream()
        self.copy_stream = torch.cuda.Stream()
        self.admit_stream = torch.cuda.Stream()
        self.keep_states = keep_states
        self.rounds = 0
        self.graphs_built = 0
        self.evicted = 0
        # memory of the last run: the largest summed footprint admitted at once, and PyTorch's
        # peak device allocation (live tensors) and peak cache (held blocks) during it, over the
        # allocation already live when the run started
        self.peak_footprint_bytes = 0
        self.peak_allocated_bytes = 0
        self.peak_cached_bytes = 0
        # pinned host slots for the per-round non-finite counts
        self._flags = torch.zeros(self.max_active, dtype=torch.int32, pin_memory=True)

    # -------------------------------------------------------------- hooks

    def build_system(self, req) -> System:
        """Creates the system of a request on the admission stream (runs in a worker thread)."""
        return _build(req, self.mode, self.dt, self.admit_stream)

    def on_round_queued(self, systems) -> None:
        """Called after each round is queued on the compute stream, with the round's systems
        (a subclass may queue its own work there)."""

    def _nonfinite(self, entries, ev) -> list:
        """Entries of a completed round whose system holds a non-finite element."""
        if not entries:
            return []
        if len(entries) > self._flags.numel():
            self._flags = self.torch.zeros(len(entries), dtype=self.torch.int32, pin_memory=True)
        self.copy_stream.wait_event(ev)
        nb_nonfinite_async([a[0].handle for a in entries], self._flags, self.copy_stream)
        self.copy_stream.synchronize()
        flags = self._flags[: len(entries)].tolist()
        return [a for a, f in zip(entries, flags) if f != 0]

    # -------------------------------------------------------------- admission worker

    def _worker(self, todo: "queue.Queue", ready: "queue.Queue"):
        while True:
            item = todo.get()
            if item is None:
                return
            req, rec = item
            try:
                sysm = self.build_system(req)
                sysm.use_on(self.compute)
                ready.put((req, rec, sysm, None))
                del sysm  # the main loop owns it now
            except Exception as e:  # reported by the main loop
                ready.put((req, rec, None, e))

    # -------------------------------------------------------------- main loop

    def run(self, trace, log=None) -> list:
        recs = {r.rid: Record(r.rid, r.n, r.q, r.steps, r.t_arrive) for r in trace}
        pending = collections.deque(sorted(trace, key=lambda r: (r.t_arrive, r.rid)))
        waiting = collections.deque()
        todo, ready = queue.Queue(), queue.Queue()
        workers = [threading.Thread(target=self._worker, args=(todo, ready), daemon=True)
                   for _ in range(self.workers)]
        for w in workers:
            w.start()
        active = []  # [System, Record, steps not yet queued]
        inflight = collections.deque()  # queued rounds: (event, systems it finishes, graph key)
        reserved = 0
        in_flight = 0
        graphs = {}  # (request ids of the round's systems, k) -> graph
        cuda = self.torch.cuda
        base_alloc, base_cache = cuda.memory_allocated(), cuda.memory_reserved()
        cuda.reset_peak_memory_stats()
        self.peak_footprint_bytes = 0
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        try:
            while pending or waiting or active or in_flight or inflight:
                t = now()
                while pending and pending[0].t_arrive <= t:
                    req = pending.popleft()
                    rec = recs[req.rid]
                    rec.bytes = footprint_bytes(req.n, req.q, self.mode)
                    if rec.bytes > self.budget:
                        rec.status = "rejected"
                        continue
                    waiting.append(req)
                while (waiting and reserved + recs[waiting[0].rid].bytes <= self.budget
                       and len(active) + in_flight < self.max_active):
                    req = waiting.popleft()
                    rec = recs[req.rid]
                    reserved += rec.bytes
                    self.peak_footprint_bytes = max(self.peak_footprint_bytes, reserved)
                    rec.t_admit = now()
                    rec.status = "admitted"
                    in_flight += 1
                    todo.put((req, rec))
                while True:
                    try:
                        req, rec, sysm, err = ready.get_nowait()
                    except queue.Empty:
                        break
                    in_flight -= 1
                    if err is not None:
                        raise err
                    active.append([sysm, rec, req.steps])
                    sysm = None
                if not active and not inflight:
                    # idle: wait for an arrival or a system under construction
                    nxt = pending[0].t_arrive - now() if pending else 0.002
                    if in_flight:
                        try:
                            item = ready.get(timeout=max(1e-4, min(nxt, 0.05)))
                            ready.put(item)
                        except queue.Empty:
                            pass
                    elif nxt > 0:
                        time.sleep(min(nxt, 0.05))
                    continue
                # systems with steps left that no queued round will finish
                open_ = [a for a in active if a[2] > 0]
                if open_ and len(inflight) < self.depth:
                    if self.policy == "srpt":
                        order = sorted(open_, key=lambda a: (a[2] * float(a[1].n) ** 2,
                                                             a[1].t_arrive, a[1].rid))
                        chosen, work = [], 0.0
                        for a in order:
                            chosen.append(a)
                            work += float(a[1].n) ** 2
                            if work >= self.fill:
                                break
                    else:
                        chosen = open_
                    k = min(self.round_steps, min(a[2] for a in chosen))
                    key = (tuple(a[1].rid for a in chosen), k)
                    if self.use_graphs:
                        graph = graphs.get(key)
                        if graph is None:
                            graph = nb_graph_create([a[0].handle for a in chosen], k,
                                                    self.compute)
                            graphs[key] = graph
                            self.graphs_built += 1
                        nb_graph_launch(graph, self.compute)
                    else:
                        from . import nb_step

                        nb_step([a[0].handle for a in chosen], k, self.compute)
                    self.on_round_queued([a[0] for a in chosen])
                    ev = self.torch.cuda.Event()
                    ev.record(self.compute)
                    self.rounds += 1
                    finishing = []
                    for a in chosen:
                        a[2] -= k
                        if a[2] <= 0:
                            finishing.append(a)
                    inflight.append((ev, finishing, key, chosen))
                    continue
                if not inflight:
                    continue
                # the oldest queued round: wait for it, check its systems, then retire the ones
                # it finished
                ev, finishing, _, chosen = inflight.popleft()
                ev.synchronize()
                t = now()
                failed = self._nonfinite([a for a in chosen if a[1].status != "failed"], ev)
                if failed:
                    # rounds queued after this one may still step them: drain the queue first
                    self.compute.synchronize()
                    for a in failed:
                        a[1].status = "failed"
                        a[1].t_done = t
                        a[2] = 0
                    self.evicted += len(failed)
                finishing = [a for a in finishing if a[1].status != "failed"]
                if finishing or failed:
                    for a in finishing:
                        sysm, rec = a[0], a[1]
                        rec.t_done = t
                        rec.status = "done"
                        if self.keep_digests:
                            rec.digest = state_digest(sysm, self.copy_stream, ev)
                        if self.keep_states:
                            self.copy_stream.wait_event(ev)
                            self.copy_stream.synchronize()
                            rec.state = _final_state(sysm)
                    gone = {a[1].rid for a in finishing + failed}
                    for gk in [gk for gk in graphs if gone.intersection(gk[0])]:
                        nb_graph_destroy(graphs.pop(gk))
                    for a in finishing + failed:
                        reserved -= a[1].bytes
                        a[0].close()
                    active = [a for a in active if a[1].rid not in gone]
                    if log:
                        log("t=%.2fs active=%d waiting=%d done=%d" % (
                            t, len(active), len(waiting),
                            sum(r.status == "done" for r in recs.values())))
                if len(graphs) > 64:  # bound the cache: drop graphs no queued round uses
                    busy = {q[2] for q in inflight}
                    for gk in list(graphs)[:-16]:
                        if gk not in busy:
                            nb_graph_destroy(graphs.pop(gk))
        finally:
            for _ in workers:
                todo.put(None)
            for w in workers:
                w.join(timeout=60)
            self.compute.synchronize()
            for g in graphs.values():
                nb_graph_destroy(g)
            for a in active:
                a[0].close()
            self.peak_allocated_bytes = cuda.max_memory_allocated() - base_alloc
            self.peak_cached_bytes = cuda.max_memory_reserved() - base_cache
        return [recs[r.rid] for r in trace]


def run_sequential(trace, mode: str = "kahan", dt: float = 1e-4, chunk: int = 100,
                   keep_digests: bool = True, log=None, keep_states: bool = False) -> list:
    """One system at a time, in arrival order, each stepped alone to completion. A system whose
    final state holds a non-finite element is reported ``"failed"``."""
    import torch

    stream = torch.cuda.Stream()
    recs = [Record(r.rid, r.n, r.q, r.steps, r.t_arrive) for r in trace]
    order = sorted(range(len(trace)), key=lambda i: (trace[i].t_arrive, trace[i].rid))
    t0 = time.perf_counter()
    for i in order:
        req, rec = trace[i], recs[i]
        wait = req.t_arrive - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        rec.t_admit = time.perf_counter() - t0
        sysm = _build(req, mode, dt, stream)
        left = req.steps
        while left > 0:
            k = min(chunk, left)
            sysm.step(k)
            left -= k
        sysm.synchronize()
        rec.t_done = time.perf_counter() - t0
        rec.status = "failed" if sysm.diagnostics()["nonfinite"] else "done"
        if keep_digests:
            rec.digest = state_digest(sysm)
        if keep_states:
            rec.state = _final_state(sysm)
        sysm.close()
        if log:
            log("seq t=%.2fs done rid=%d n=%d" % (rec.t_done, rec.rid, rec.n))
    return recs
