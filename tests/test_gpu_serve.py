"""Continuous-batching server: every request's result is the same alone and
in the mix.

A short Poisson trace of layout and re-tune requests over small Chung-Lu
graphs is served with a tight HBM budget (so that requests queue, graphs are
evicted and re-uploaded) and chunked batched steps (so that requests join
and leave a running batch). Each request is then replayed alone: a fresh
layout handle with the request's parameters and starting positions, stepped
by tfdp_layout_step for the request's iterations. Tolerance: bit-identical
positions (the batch runs the plain kernels' code per graph).
"""
import sys

import numpy as np
import pytest

import synthgraphs as sg
from tests._lib import ensure_built

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()
    import paper_2303_03964_amd as lib
    lib.load_library()
    return lib


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_pool(count):
    out = []
    for i in range(count):
        rng = np.random.default_rng([99, i])
        n = int(rng.integers(800, 6000))
        g = sg.chung_lu(n, float(rng.uniform(2.0, 3.0)), 10.0, 1000 + i)
        out.append((g, sg.uniform_positions(g.n, 2000 + i)))
    return out


def test_results_same_alone_and_in_the_mix(T):
    import torch
    from paper_2303_03964_amd import autotune, serve
    pool = small_pool(6)
    trace = sg.serving_trace(14, rate=400.0, pool=len(pool), seed=7, layout_iters=40, retune_iters=20)
    kinds = [r.kind for r in trace]
    say(f"trace: {kinds}")
    assert "retune" in kinds
    stream = torch.cuda.Stream()
    # budget: room for about three graphs at a time
    ws = [serve.footprint(g.n, g.nnz, T.tfdp_params_default(n_int=autotune.workspace_grid(g.n)))
          for g, _ in pool]
    budget = 3 * max(ws)
    srv = serve.Server(pool, budget, slots=4, chunk=7, stream=stream, record_inputs=True, record_outputs=True)
    recs = srv.run(trace)
    srv.close()
    s = serve.summarize(recs)
    say(f"served: {s}")
    assert all(r.done > 0 for r in recs)
    with torch.cuda.stream(stream):
        for r, req in zip(recs, trace):
            g = pool[req.graph][0] if req.kind == "layout" else pool[trace[req.target].graph][0]
            lay = T.Layout(g.row_ptr, g.col_idx, r.start_pos.clone(), r.params)
            lay.step(r.iters)
            torch.cuda.synchronize()
            same = torch.equal(lay.pos, r.final_pos)
            say(f"request {r.rid} {r.kind} n={r.n} latency {r.latency * 1e3:.1f} ms same={same}")
            assert same
            lay.close()


def test_sequential_baseline_serves_everything(T):
    import torch
    from paper_2303_03964_amd import serve
    pool = small_pool(4)
    trace = sg.serving_trace(8, rate=1000.0, pool=len(pool), seed=8, layout_iters=20, retune_iters=10)
    stream = torch.cuda.Stream()
    srv = serve.Server(pool, 1 << 34, stream=stream, plain=True)
    recs = srv.run(trace)
    srv.close()
    assert all(r.done >= r.arrival for r in recs)
    s = serve.summarize(recs)
    assert s["p99_ms"] >= s["p50_ms"] > 0
