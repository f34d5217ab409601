"""Continuous-batching layout server over one tfdp_batch.

Requests arrive over time (a trace of synthgraphs.Request objects); the
loop admits them while batch slots and the HBM budget allow, steps every
active graph together in chunks of at most `chunk` iterations (fewer when the
members' iterations are long, so that a chunk takes about CHUNK_SECONDS),
and retires a
graph as soon as its iterations are done, so requests that arrive while
others are on the device join the running batch at the next chunk.

* layout request: the graph's CSR and initial positions are uploaded and a
  layout handle is created with the autotuner's start choice (exact method
  for small graphs, else the size-rule grid; workspace sized for the largest
  final grid the tuner may choose); `iters` iterations of the k schedule
  over T = iters.
* re-tune request (Sec. 5, global refinement): a finished graph stays
  resident; the request sets alpha, beta, gamma and the repulsion weight,
  restarts the counter with T = iters and a unit step cap, and runs again
  from the current positions (start grid again). A re-tune waits for its
  graph to be idle. A graph evicted to make room (least recently used idle
  graph first) keeps its positions on the host and is uploaded again when a
  re-tune needs it.
* final stage at the requested force accuracy (Sec. 3.4, "Choices of k"):
  for every request on a grid, the box of its positions BOX_LEAD iterations
  before its first k = 3 iteration fixes the last stage's method
  (autotune.final_choice: the grid whose k = 3 repulsion is within `tol` of
  the exact sums, or the exact method where that is cheaper), applied at the
  switch. The rule depends only on the request's own positions and counter,
  so a request gets the same choice and the same result alone (run_alone)
  and in the mix.
* admission by HBM footprint: CSR + positions + workspace bytes
  (tfdp_workspace_size) must fit the budget left by the resident graphs.

Admission work (uploads, handle creation) runs on BUILD_WORKERS worker
threads and a stream of its own, so that it waits neither for the chunk on
the device nor holds up the stepping loop, and a large graph's handle
(tens of milliseconds of host work) does not hold up the smaller ones behind
it; the stepping stream waits for it before the new member's first chunk.
Members are stepped in three cost classes, each a batch on a stream of its
own with chunks of its own length: light members
(iterations below LIGHT_ITERATION: grids of graphs up to about 1e5 nodes,
exact stages up to about 1.4e4), the rest, and members whose iterations are
long (an exact stage of a large graph, EXPENSIVE_ITERATION). The
compute-bound exact passes then run beside the latency-bound grid passes,
and a small request advances at the pace of the light class instead of that
of every graph on the device. Each class keeps at most two chunks in flight;
a graph that changes class, or is re-tuned, evicted or copied after a chunk
on another stream, is ordered after that chunk by its event. Kernels are
launched directly (no stream
capture) in both legs, since the worker thread's GPU work runs concurrently
with the stepping thread. Latency of a request = completion - arrival, completion
being the device time of the event recorded after the chunk (or, plain, the
call) that finished it, measured from an event recorded at the start of the
run on the idle stream.

plain=True serves the same trace one request at a time with
tfdp_layout_step on the same stream (the sequential baseline), with the
same final-stage rule.
"""
from __future__ import annotations

import time
from collections import OrderedDict, deque
from dataclasses import dataclass

import numpy as np

from . import autotune
from . import tfdp as T

BOX_LEAD = 10  # iterations between reading the box and the switch to k = 3
CHUNK_SECONDS = 2e-3  # target device time of one chunk (admission points this far apart)
EXPENSIVE_ITERATION = 2.5e-4  # members with longer iterations are stepped as a batch of their own
LIGHT_ITERATION = 4.0e-5  # members with shorter ones form a class of their own (None: two classes)
BUILD_WORKERS = 4  # worker threads creating handles (uploads, CSR check, edge schedule)


def iteration_seconds(n: int, nnz: int, exact: bool) -> float:
    """Rough device time of one iteration of a graph on MI355X (for chunk
    sizing only): the exact method at about 5e12 pair terms per second,
    else a launch floor plus the per-node and per-entry passes."""
    if exact:
        return n * n / 5.0e12
    return 25e-6 + 6e-11 * n + 7e-12 * nnz


@dataclass
class _Graph:
    key: int              # rid of the layout request that brought the graph
    graph: object         # synthgraphs.Graph (host CSR)
    lay: object = None    # Layout while resident
    host_pos: np.ndarray | None = None  # positions while evicted
    bytes: int = 0
    busy: bool = False
    ws_n_int: int = 0     # largest grid the workspace holds
    last_ev: object = None      # event after the graph's latest chunk
    last_stream: object = None  # the stream it was recorded on


@dataclass
class Record:
    rid: int
    kind: str
    n: int
    iters: int
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    start_pos: object = None   # positions at admission (kept when record_inputs)
    params: object = None      # TfdpParams at admission
    final: tuple | None = None  # (k_mode, n_int) of the last stage
    ws_n_int: int = 0          # largest grid of the graph's workspace (cap of the last stage's grid)
    final_pos: object = None   # positions at completion (kept when record_outputs)

    @property
    def latency(self):
        return self.done - self.arrival


def footprint(n: int, nnz: int, ws_params) -> int:
    return 8 * n + 4 * (n + 1) + 4 * nnz + T.tfdp_workspace_size(n, nnz, ws_params) + 256


def final_stage_points(iters: int):
    """(t_read, t_switch): the counter at which the box is read and the first
    k = 3 iteration of a schedule over T = iters."""
    t_switch = (19 * iters) // 20
    return max(0, t_switch - BOX_LEAD), t_switch


def box_extremes(pos):
    """(min x, min y, max x, max y) of the positions, on the current stream."""
    import torch
    return torch.cat([pos.amin(0), pos.amax(0)])


def final_params(lay, ext, tol: float, cap: int):
    """Parameters of the last stage from the box extremes `ext` (host)."""
    e = np.asarray(ext, dtype=np.float64)
    w = float(max(e[2] - e[0], e[3] - e[1]))
    if not np.isfinite(w) or w <= 0:
        w = 1.0
    cur = lay.params
    k_mode, ni = autotune.final_choice(lay.n, w, tol, gamma=cur.gamma, tau=cur.tau, cap=cap)
    if k_mode == 0:
        return T.TfdpParams(**{**cur.as_dict(), "k_mode": 0})
    return T.TfdpParams(**{**cur.as_dict(), "n_int": max(cur.n_int, ni)})


def run_alone(lay, iters: int, tol: float, cap: int):
    """One request on its own handle with tfdp_layout_step, with the same
    final-stage rule as the server. Returns the last stage's (k_mode, n_int)."""
    if lay.params.k_mode != -1:
        lay.step(iters)
        return (lay.params.k_mode, lay.params.n_int)
    t_read, t_switch = final_stage_points(iters)
    lay.step(t_read)
    ext = box_extremes(lay.pos).cpu().numpy()
    lay.step(t_switch - t_read)
    lay.set_params(final_params(lay, ext, tol, cap))
    lay.step(iters - t_switch)
    return (lay.params.k_mode, lay.params.n_int)


def request_params(n: int, iters: int, extra: dict | None = None, t0: float = 0.0):
    k_mode, n_int = autotune.start_params(n)
    return T.tfdp_params_default(n_int=n_int, total_iters=iters, k_mode=k_mode, t0=t0, **(extra or {}))


class _Run:
    """A request on the device: its graph, record and counter-driven events."""

    def __init__(self, g, rec, iters):
        self.g = g
        self.rec = rec
        self.iters = iters
        self.done = 0
        self.t_read, self.t_switch = final_stage_points(iters)
        self.tuned = g.lay.params.k_mode != -1  # exact from the start: no final choice
        self.ext = None      # pinned host extremes
        self.ext_ev = None   # event after their copy

    def next_stop(self):
        """Iterations to the next counter at which the server must act."""
        stops = [self.iters]
        if not self.tuned:
            stops += [t for t in (self.t_read, self.t_switch) if t > self.done]
        return min(stops) - self.done


class Server:
    def __init__(self, pool, budget_bytes: int, slots: int = 256, chunk: int = 10, tol: float = 1e-3,
                 stream=None, record_inputs: bool = False, record_outputs: bool = False, plain: bool = False,
                 workers: int = BUILD_WORKERS, light_iteration: float | None = LIGHT_ITERATION):
        import torch
        from concurrent.futures import ThreadPoolExecutor
        self.torch = torch
        self.pool = pool                    # index -> (Graph, pos0)
        self.budget = int(budget_bytes)
        self.slots = slots
        self.chunk = chunk
        self.tol = tol
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.admit_stream = torch.cuda.Stream(device=self.stream.device)
        # one stream per cost class (default priority), so that the long
        # chunks of one class run beside the short ones of another. Classes:
        # light members (short iterations; None: no such
        # class), the rest, and members whose iterations are long. Five runs
        # of each load, median p50 / p99 (ms) with and without the light
        # class: 0.8x 36 / 218 against 55 / 263, 1.2x 67 / 253 against
        # 80 / 294 (a threshold of 3e-5 s, which moves graphs of 4e4 - 1e5
        # nodes out of the light class, measured worse than two classes)
        self.light_iteration = light_iteration
        ncls = 1 if plain else (3 if light_iteration is not None else 2)
        self.streams = [self.stream] + [torch.cuda.Stream(device=self.stream.device) for _ in range(ncls - 1)]
        # chunks in flight per class (one for the expensive class: p99 at
        # 0.8x load within run-to-run spread, at 1.2x load 595 ms against
        # 285 ms with two)
        self.max_inflight = [2] * ncls
        # handles are created on worker threads (uploads, the CSR check and
        # the host-side edge schedule of tfdp_layout_init take up to about
        # 100 ms for the largest graphs; the stepping loop keeps the GPU busy
        # meanwhile). With one worker, admissions under load queued behind
        # those builds (p50 / p99 at 0.8x load 38-56 / 229-353 ms against
        # 27-34 / 221-229 ms with four)
        self.worker = ThreadPoolExecutor(max_workers=1 if plain else workers)
        self.graphs = OrderedDict()         # key -> _Graph (LRU order of idle use)
        self.used = 0
        self.record_inputs = record_inputs
        self.record_outputs = record_outputs
        # plain: one request at a time, stepped by tfdp_layout_step alone
        # (the sequential baseline)
        self.plain = plain
        if plain:
            self.slots = 1
        # the cost classes are stepped as separate batches, so that members
        # with long iterations (an exact stage of a large graph) do not hold
        # the others to their chunk length
        self.batches = [] if plain else [T.Batch(slots, map_entries=1 << 22) for _ in range(ncls)]
        # no stream capture in the server (batches and served handles launch
        # directly, in both legs): the worker thread's uploads and handle
        # set-up run concurrently with the stepping thread, and a capture in
        # progress on the stepping stream must not meet them (a chunk event
        # was once recorded inside a capture that way)
        for b in self.batches:
            b.set_graphs(False)

    # ---------------------------------------------------------------- memory
    def _evict_for(self, need: int) -> bool:
        while self.used + need > self.budget:
            victim = next((g for g in self.graphs.values() if g.lay is not None and not g.busy), None)
            if victim is None:
                return False
            with self.torch.cuda.stream(self.stream):
                if victim.last_ev is not None and victim.last_stream is not self.stream:
                    self.stream.wait_event(victim.last_ev)
                victim.host_pos = victim.lay.pos.cpu().numpy()
            victim.lay.close()
            victim.lay = None
            self.used -= victim.bytes
        return True

    def _build(self, g: _Graph, pos_host, params, ws):
        """Worker thread: upload and create the graph's handle."""
        torch = self.torch
        with torch.cuda.stream(self.admit_stream):
            pos = torch.as_tensor(pos_host).to(self.stream.device)
            lay = T.Layout(g.graph.row_ptr, g.graph.col_idx, pos, params, workspace_params=ws)
            T.tfdp_layout_set_graphs(lay.handle, 0)
            # the tensors are used on the stepping streams from now on
            for t in (lay.row_ptr, lay.col_idx, lay.pos, lay.workspace):
                for st in self.streams:
                    t.record_stream(st)
        return lay

    def _reserve(self, g: _Graph, params):
        """Reserve the HBM footprint of the graph's handle (evicting idle
        graphs if needed); returns the workspace parameters or None."""
        n, nnz = g.graph.n, g.graph.nnz
        ws = params if params.k_mode == 0 else T.TfdpParams(
            **{**params.as_dict(), "n_int": max(params.n_int, autotune.workspace_grid(n)), "k_mode": -1})
        need = footprint(n, nnz, ws)
        if not self._evict_for(need):
            return None
        g.bytes = need
        g.ws_n_int = ws.n_int
        self.used += need
        return ws

    # ---------------------------------------------------------------- admission
    def _admit(self, req, active: dict, preparing: dict) -> bool:
        if len(active) + len(preparing) >= self.slots:
            return False
        if req.kind == "layout":
            graph, pos0 = self.pool[req.graph]
            g = _Graph(req.rid, graph)
            p = request_params(graph.n, req.iters)
            ws = self._reserve(g, p)
            if ws is None:
                return False
            self.graphs[req.rid] = g
            g.busy = True
            preparing[req.rid] = (req, g, self.worker.submit(self._build, g, pos0, p, ws))
            return True
        g = self.graphs.get(req.target)
        if g is None or g.busy:
            return False  # target not laid out yet, or still running
        p = request_params(g.graph.n, req.iters, req.params, t0=1.0)
        self.graphs.move_to_end(req.target)
        if g.lay is None:
            ws = self._reserve(g, p)
            if ws is None:
                return False
            g.busy = True
            preparing[req.rid] = (req, g, self.worker.submit(self._build, g, g.host_pos, p, ws))
            g.host_pos = None
            return True
        g.lay.set_params(p)
        g.lay.iteration = 0
        g.busy = True
        preparing[req.rid] = (req, g, None)
        return True

    def _activate(self, req, g: _Graph, rec: Record, active: dict):
        torch = self.torch
        rec.n = g.graph.n
        rec.params = g.lay.params
        rec.ws_n_int = g.ws_n_int
        for st in self.streams:
            st.wait_stream(self.admit_stream)
            if g.last_ev is not None and g.last_stream is not st:
                st.wait_event(g.last_ev)  # a re-tune after a chunk on another stream
        if self.record_inputs:
            rec.start_pos = g.lay.pos.clone()  # on self.stream
            copied = torch.cuda.Event()
            copied.record(self.stream)
            g.last_ev, g.last_stream = copied, self.stream  # the first chunk waits for the copy
        run = _Run(g, rec, req.iters)
        run.group = -1
        active[req.rid] = run

    def _retire(self, run: _Run, event, stream):
        rec = run.rec
        rec.done_event = event
        rec.final = (run.g.lay.params.k_mode, run.g.lay.params.n_int)
        if self.record_outputs:
            with self.torch.cuda.stream(stream):
                rec.final_pos = run.g.lay.pos.clone()
                # the graph's next run (a re-tune, possibly on another
                # stream) waits for this copy, not only for the chunk
                # before it: otherwise its first chunk could move the
                # positions while they are being copied
                copied = self.torch.cuda.Event()
                copied.record(stream)
            run.g.last_ev, run.g.last_stream = copied, stream
        if not self.plain and run.group >= 0:
            self.batches[run.group].remove(run.g.lay)
        run.g.busy = False
        self.graphs.move_to_end(run.g.key)

    # ---------------------------------------------------------------- loop
    def _final_stage_events(self, active):
        """Box read at t_read (device reduction, copy to pinned memory) and the
        last stage's parameters at t_switch, for runs that reached them."""
        torch = self.torch
        for run in active.values():
            if run.tuned:
                continue
            if run.done == run.t_read and run.ext is None:
                st = run.g.last_stream if run.g.last_stream is not None else self.stream
                with torch.cuda.stream(st):
                    ext = box_extremes(run.g.lay.pos)
                    run.ext = torch.empty(4, dtype=ext.dtype, pin_memory=True)
                    run.ext.copy_(ext, non_blocking=True)
                    run.ext_ev = torch.cuda.Event()
                    run.ext_ev.record(st)
            if run.done == run.t_switch:
                run.ext_ev.synchronize()
                run.g.lay.set_params(final_params(run.g.lay, run.ext.numpy(), self.tol, run.g.ws_n_int))
                run.tuned = True

    def _cost_class(self, cost: float) -> int:
        if cost > EXPENSIVE_ITERATION:
            return len(self.streams) - 1
        if self.light_iteration is not None and cost > self.light_iteration:
            return 1
        return 0

    def _issue(self, active, inflight):
        """A chunk of the active runs of every cost class whose stream has
        fewer than two chunks in flight; returns the finished runs (with the
        event and stream of their last chunk) and whether anything was
        issued."""
        torch = self.torch
        for q in inflight:
            while q and q[0].query():
                q.popleft()
        self._final_stage_events(active)
        groups = tuple([] for _ in self.streams)
        for run in active.values():
            cost = iteration_seconds(run.g.graph.n, run.g.graph.nnz, run.g.lay.params.k_mode == 0)
            groups[self._cost_class(cost)].append((run, cost))
        # every member into the batch of its class first: a batch steps all
        # its slots, so a graph whose class changed (its last stage chosen)
        # must have left its old batch before that batch steps again, or it
        # would be stepped twice in one pass of the loop
        for grp, members in enumerate(groups):
            for run, _ in members:
                if run.group != grp:
                    if run.group >= 0:
                        self.batches[run.group].remove(run.g.lay)
                    self.batches[grp].add(run.g.lay)
                    run.group = grp
        finished, issued = [], False
        for grp, members in enumerate(groups):
            if not members or len(inflight[grp]) >= self.max_inflight[grp]:
                continue
            stream = self.streams[grp]
            for run, _ in members:
                g = run.g
                # a graph last stepped on the other stream (class change,
                # or a re-tune after a request of the other class)
                if g.last_ev is not None and g.last_stream is not stream:
                    stream.wait_event(g.last_ev)
            # at most `chunk` iterations, fewer when the members' iterations
            # are long, so that a chunk takes about CHUNK_SECONDS
            per_iter = sum(c for _, c in members)
            cap_iters = max(1, min(self.chunk, int(CHUNK_SECONDS / max(per_iter, 1e-9))))
            step = min(cap_iters, min(r.next_stop() for r, _ in members))
            self.batches[grp].step(step, stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            inflight[grp].append(ev)
            issued = True
            for r, _ in members:
                r.done += step
                r.g.last_ev, r.g.last_stream = ev, stream
                if r.done == r.iters:
                    finished.append((r, ev, stream))
        return finished, issued

    def run(self, trace):
        """Serve the trace; returns the list of Records in request order."""
        torch = self.torch
        recs = {r.rid: Record(r.rid, r.kind, 0, r.iters, r.arrival) for r in trace}
        pending = sorted(trace, key=lambda r: r.arrival)
        waiting = []
        active = {}      # rid -> _Run
        preparing = {}   # rid -> (request, graph, future or None)
        inflight = [deque() for _ in self.streams]
        i = 0
        with torch.cuda.stream(self.stream):
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev0.record(self.stream)
            t_start = time.perf_counter()
            while i < len(pending) or waiting or active or preparing:
                now = time.perf_counter() - t_start
                while i < len(pending) and pending[i].arrival <= now:
                    waiting.append(pending[i])
                    i += 1
                still = []
                for req in waiting:
                    if self._admit(req, active, preparing):
                        recs[req.rid].admitted = time.perf_counter() - t_start
                    else:
                        still.append(req)
                waiting = still
                for rid in [r for r, (_, _, f) in preparing.items() if f is None or f.done()]:
                    req, g, fut = preparing.pop(rid)
                    if fut is not None:
                        g.lay = fut.result()
                    self._activate(req, g, recs[rid], active)
                if not active:
                    if preparing:
                        time.sleep(2e-4)
                    elif i < len(pending):
                        time.sleep(max(0.0, min(pending[i].arrival - (time.perf_counter() - t_start), 0.002)))
                    elif waiting:
                        raise RuntimeError("requests cannot be admitted: budget or slots too small")
                    continue
                if self.plain:
                    rid = next(iter(active))
                    run = active.pop(rid)
                    run_alone(run.g.lay, run.iters, self.tol, run.g.ws_n_int)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(self.stream)
                    run.done = run.iters
                    run.g.last_ev, run.g.last_stream = ev, self.stream
                    self._retire(run, ev, self.stream)
                    inflight[0].append(ev)
                    while len(inflight[0]) > 2:
                        inflight[0].popleft().synchronize()
                    continue
                finished, issued = self._issue(active, inflight)
                for run, ev, st in finished:
                    self._retire(active.pop(run.rec.rid), ev, st)
                for q in inflight:
                    while q and q[0].query():
                        q.popleft()
                if not issued:
                    # the classes with members had two chunks in flight: wait
                    # until one of those still in flight ends (none left, if
                    # they all ended since the check)
                    blocked = [q for g, q in enumerate(inflight) if q and len(q) >= self.max_inflight[g]]
                    while blocked and not any(q[0].query() for q in blocked):
                        time.sleep(5e-5)
            torch.cuda.synchronize()
            for r in recs.values():
                r.done = ev0.elapsed_time(r.done_event) * 1e-3
                del r.done_event
            for g in self.graphs.values():
                if g.lay is not None and g.lay.sync_status() != 0:
                    raise RuntimeError(f"graph of request {g.key}: non-finite positions")
        return [recs[r.rid] for r in trace]

    def close(self):
        self.worker.shutdown(wait=True)
        for b in self.batches:
            b.close()
        for g in self.graphs.values():
            if g.lay is not None:
                g.lay.close()
                g.lay = None
        self.graphs.clear()


def summarize(records, wall_s: float | None = None):
    lat = np.array([r.latency for r in records])
    node_its = float(sum(r.n * r.iters for r in records))
    span = wall_s if wall_s is not None else max(r.done for r in records) - min(r.arrival for r in records)
    return {
        "requests": len(records),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "node_iterations_per_s": node_its / span,
        "span_s": span,
    }
