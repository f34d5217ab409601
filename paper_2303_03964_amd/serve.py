"""Continuous-batching layout server over one tfdp_batch.

Requests arrive over time (a trace of synthgraphs.Request objects); the
loop admits them while batch slots and the HBM budget allow, steps every
active graph together in chunks of `chunk` iterations, and retires a graph
as soon as its iterations are done, so requests that arrive while others are
on the device join the running batch at the next chunk.

* layout request: the graph's CSR and initial positions are uploaded, a
  layout handle is created with the autotuner's start choice (exact method
  for small graphs, else its grid; workspace sized for the largest final
  grid the tuner may choose) and added to the batch for `iters` iterations
  (k schedule over T = iters).
* re-tune request (Sec. 5, global refinement): a finished graph stays
  resident; the request changes alpha, beta, gamma and the repulsion weight,
  restarts the counter with T = iters and a unit step cap, and runs again
  from the current positions. A re-tune waits for its graph to be idle. A
  graph evicted to make room (least recently used idle graph first) keeps
  its positions on the host and is uploaded again when a re-tune needs it.
* admission by HBM footprint: CSR + positions + workspace bytes
  (tfdp_workspace_size) must fit the budget left by the resident graphs.

Latency of a request = completion (positions final on the device, observed
after a stream synchronisation at the end of the chunk that finished it)
minus arrival. The loop runs in wall-clock time against the trace's arrival
times; all device work is enqueued on one stream.
"""
from __future__ import annotations

import time
from collections import OrderedDict
from dataclasses import dataclass, field

import numpy as np

from . import autotune
from . import tfdp as T


@dataclass
class _Graph:
    key: int              # rid of the layout request that brought the graph
    graph: object         # synthgraphs.Graph (host CSR)
    lay: object = None    # Layout while resident
    host_pos: np.ndarray | None = None  # positions while evicted
    bytes: int = 0
    busy: bool = False


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
    params: object = None      # TfdpParams used
    final_pos: object = None   # positions at completion (kept when record_outputs)

    @property
    def latency(self):
        return self.done - self.arrival


def footprint(n: int, nnz: int, ws_params) -> int:
    return 8 * n + 4 * (n + 1) + 4 * nnz + T.tfdp_workspace_size(n, nnz, ws_params) + 256


class Server:
    def __init__(self, pool, budget_bytes: int, slots: int = 256, chunk: int = 10, tol: float = 1e-3,
                 stream=None, record_inputs: bool = False, record_outputs: bool = False, plain: bool = False):
        import torch
        self.torch = torch
        self.pool = pool                    # index -> (Graph, pos0)
        self.budget = int(budget_bytes)
        self.slots = slots
        self.chunk = chunk
        self.tol = tol
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.batch = T.Batch(slots)
        self.graphs = OrderedDict()         # key -> _Graph (LRU order of idle use)
        self.used = 0
        self.record_inputs = record_inputs
        self.record_outputs = record_outputs
        # plain: one request at a time, stepped by tfdp_layout_step alone
        # (the sequential baseline)
        self.plain = plain
        if plain:
            self.slots = 1

    # ---------------------------------------------------------------- memory
    def _evict_for(self, need: int) -> bool:
        while self.used + need > self.budget:
            victim = next((g for g in self.graphs.values() if g.lay is not None and not g.busy), None)
            if victim is None:
                return False
            victim.host_pos = victim.lay.pos.cpu().numpy()
            victim.lay.close()
            victim.lay = None
            self.used -= victim.bytes
        return True

    def _make_layout(self, g: _Graph, pos, params):
        n, nnz = g.graph.n, g.graph.nnz
        ws = params if params.k_mode == 0 else T.TfdpParams(
            **{**params.as_dict(), "n_int": max(params.n_int, autotune.workspace_grid(n)), "k_mode": -1})
        need = footprint(n, nnz, ws)
        if not self._evict_for(need):
            return False
        g.lay = T.Layout(g.graph.row_ptr, g.graph.col_idx, pos, params, workspace_params=ws)
        g.bytes = need
        self.used += need
        return True

    # ---------------------------------------------------------------- admission
    def _admit(self, req, rec: Record, active: dict) -> bool:
        torch = self.torch
        if len(active) >= self.slots:
            return False
        if req.kind == "layout":
            graph, pos0 = self.pool[req.graph]
            g = _Graph(req.rid, graph)
            k_mode, n_int = autotune.start_params(graph.n)
            p = T.tfdp_params_default(n_int=n_int, total_iters=req.iters, k_mode=k_mode)
            if not self._make_layout(g, torch.as_tensor(pos0).cuda(), p):
                return False
            self.graphs[req.rid] = g
        else:
            g = self.graphs.get(req.target)
            if g is None or g.busy:
                return False  # target not laid out yet, or still running
            base = g.lay.params if g.lay is not None else self._last_params[req.target]
            p = T.TfdpParams(**{**base.as_dict(), **req.params, "total_iters": req.iters, "t0": 1.0})
            if g.lay is None:
                if not self._make_layout(g, torch.as_tensor(g.host_pos).cuda(), p):
                    return False
                g.host_pos = None
            else:
                g.lay.set_params(p)
            g.lay.iteration = 0
            self.graphs.move_to_end(req.target)
        g.busy = True
        rec.n = g.graph.n
        rec.params = g.lay.params
        if self.record_inputs:
            rec.start_pos = g.lay.pos.clone()
        if not self.plain:
            self.batch.add(g.lay)
        active[req.rid] = (g, req.iters, rec)
        return True

    # ---------------------------------------------------------------- loop
    def run(self, trace):
        """Serve the trace; returns the list of Records in request order."""
        torch = self.torch
        self._last_params = {}
        recs = {r.rid: Record(r.rid, r.kind, 0, r.iters, r.arrival) for r in trace}
        pending = sorted(trace, key=lambda r: r.arrival)
        waiting = []
        active = {}   # rid -> (graph, remaining, record)
        i = 0
        t_start = time.perf_counter()
        with torch.cuda.stream(self.stream):
            while i < len(pending) or waiting or active:
                now = time.perf_counter() - t_start
                while i < len(pending) and pending[i].arrival <= now:
                    waiting.append(pending[i])
                    i += 1
                still = []
                for req in waiting:
                    if self._admit(req, recs[req.rid], active):
                        recs[req.rid].admitted = time.perf_counter() - t_start
                    else:
                        still.append(req)
                waiting = still
                if not active:
                    if i < len(pending):
                        time.sleep(max(0.0, min(pending[i].arrival - (time.perf_counter() - t_start), 0.01)))
                    elif waiting:
                        raise RuntimeError("requests cannot be admitted: budget or slots too small")
                    continue
                if self.plain:
                    step = min(rem for _, rem, _ in active.values())
                    for g, _, _ in active.values():
                        g.lay.step(step)
                else:
                    step = min(self.chunk, min(rem for _, rem, _ in active.values()))
                    self.batch.step(step)
                finished = []
                for rid in list(active):
                    g, rem, rec = active[rid]
                    rem -= step
                    active[rid] = (g, rem, rec)
                    if rem == 0:
                        finished.append(rid)
                if finished:
                    torch.cuda.synchronize()
                    t_done = time.perf_counter() - t_start
                    for rid in finished:
                        g, _, rec = active.pop(rid)
                        rec.done = t_done
                        if self.record_outputs:
                            rec.final_pos = g.lay.pos.clone()
                        if g.lay.sync_status() != 0:
                            raise RuntimeError(f"request {rid}: non-finite positions")
                        if not self.plain:
                            self.batch.remove(g.lay)
                        self._last_params[g.key] = g.lay.params
                        g.busy = False
                        self.graphs.move_to_end(g.key)
        return [recs[r.rid] for r in trace]

    def close(self):
        self.batch.close()
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
