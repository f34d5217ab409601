#!/usr/bin/env python3
"""Benchmark of the t-FDP layout iteration on one MI355X.

One step = one iteration of the whole hot path over the graph: box, interval
binning, spreading, FFT convolution, gather, CSR attraction and the move.
Default workload: Chung-Lu power-law graph, 1,000,000 nodes, exponent 2.5,
mean degree 10, int32 CSR, FP32 positions uniform in [-1, 1]^2, N_int = 256,
T = 500 iterations of the k schedule (k = 1/2/3 for 450/25/25 iterations).
With --steps >= T (default 500) the timed region is the whole layout. With
fewer steps K it is a schedule-weighted sample of it: K - 2m iterations at
k = 1 from the start and m = round(K/20) at k = 2 and at k = 3, started from
the positions and counters saved at the two switches by an untimed pass over
the whole schedule (which also gives the quality of the final layout).

Prints one JSON line. ``value`` = n * steps / seconds (node-iterations/s)
with the inputs resident in HBM. ``roofline`` prices the dominant kernel
(the attraction pass, which runs beside the grid passes on a second stream
at this size; the fused gather + attraction + update pass otherwise) by its
algorithmic bytes per launch over its average launch time, measured with HIP
events on the stream it is launched on in a second pass over the same
iterations. ``cpu_baseline`` times the FP64 CPU
oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="chung_lu_1m", choices=["chung_lu_1m", "mesh_100k", "sbm_1k"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=0, help="oracle iterations (0: about 15 s of work)")
    ap.add_argument("--repeats", type=int, default=5, help="timed repeats of the K steps; value is the median")
    ap.add_argument("--no-graphs", action="store_true", help="launch every kernel directly")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-workload section")
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--batch-iters", type=int, default=300)
    ap.add_argument("--no-batch-sequential", action="store_true",
                    help="skip the sequential comparison of the batched section (short profiles)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="copy this many MiB device-to-device once before the run (a plain copy kernel "
                         "of known size for scaling hardware byte counters)")
    return ap.parse_args()


def workload(name):
    import synthgraphs as sg
    if name == "chung_lu_1m":
        return sg.chung_lu_1m()
    if name == "mesh_100k":
        return sg.mesh_100k()
    return sg.sbm_1k()


def gather_bytes(n, nnz, m):
    """Algorithmic HBM bytes of one gather + attraction + update launch:
    read own position (8 B), write new position (8 B), row_ptr (4 B) per
    node; column index (4 B) and neighbour position (8 B) per CSR entry; the
    M x M grid of potentials (16 B per grid node) once."""
    return 20.0 * n + 12.0 * nnz + 16.0 * m * m


def attract_bytes(n, nnz):
    """Algorithmic HBM bytes of one overlapped attraction launch: read own
    position (8 B) and row_ptr (4 B), write the row's attraction sum (8 B)
    per node; column index (4 B) and neighbour position (8 B) per CSR entry."""
    return 20.0 * n + 12.0 * nnz


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_file, summary):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    profiles/<summary>, if it was taken on the current kernel source; else
    None."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256_16") != source_digest([kernel_file, "paper_2303_03964_amd/csrc/tfdp_internal.h"]):
        return None
    return rec.get("hbm_bytes_per_launch")


def gather_reference(torch, lay, stream, reps=20):
    """Time of a plain gather of every CSR entry's neighbour position
    (torch.index_select with the int32 column indices, 8-byte rows) on the
    same graph and stream: a reference for the random-gather part of the
    edge pass, which reads the same neighbours (and writes no copy)."""
    pos = lay.pos.view(-1, 2)
    col = lay.col_idx
    with torch.cuda.stream(stream):
        out = torch.empty((col.numel(), 2), dtype=pos.dtype, device=pos.device)
        for _ in range(3):
            torch.index_select(pos, 0, col, out=out)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            torch.index_select(pos, 0, col, out=out)
        e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del out
    return {"op": "torch.index_select of the nnz neighbour positions (int32 indices, 8-byte rows)",
            "avg_ms": ms, "gathers": int(col.numel()), "gathers_per_s": col.numel() / (ms * 1e-3)}


def cpu_baseline(w, iters, budget=15.0):
    """The FP64 oracle (as it stands) on the same graph: `iters` iterations of
    forces + move at k = 1 from the initial positions (iters = 0: as many as
    fit in `budget` seconds)."""
    from oracle import tfdp as ot
    p = ot.Params(n_int=w.n_int, total_iters=w.iters, k_mode=-1)
    x = w.pos0.astype(np.float64)
    g = w.graph
    t0 = ot.default_t0(g.n)
    c0 = time.process_time()
    s0 = time.perf_counter()
    done = 0
    target = iters if iters > 0 else 10 ** 9
    while done < target:
        k = ot.k_for_iteration(done, w.iters)
        _, _, d = ot.forces(x, g.row_ptr, g.col_idx, p, k)
        x = ot.capped_move(x, d, ot.step_cap(done, w.iters, t0))
        done += 1
        if iters <= 0 and time.perf_counter() - s0 > budget:
            break
    wall = time.perf_counter() - s0
    cpu = time.process_time() - c0
    return {
        "value": g.n * done / wall,
        "unit": "node-iterations/s",
        "cores": max(1, int(round(cpu / wall))),
        "kind": "oracle",
        "sample": f"{done} iterations (k=1) of the FP64 NumPy oracle on the same {g.n}-node graph; "
                  f"{wall:.1f} s wall, {cpu:.1f} s CPU; host os.cpu_count()={os.cpu_count()}",
    }


def batched_section(T, torch, stream, graphs, iters, accuracy=True, sequential=True):
    """Batched workload: `graphs` SBMs with n log-uniform in [200, 20000]
    (2..20 blocks, mean degree 8), T = iters, grids from the autotuner: the
    size rule for the k = 1 and k = 2 stages and, with `accuracy`, at the
    switch to k = 3 the final grid from each layout's box for a k = 3
    repulsion error of 1e-3 (workspaces sized for the cap at creation).
    Times the whole schedule stepped by one tfdp_batch against the same
    graphs stepped one after another with tfdp_layout_step on the same
    stream, from the same positions, with the same re-tune in between."""
    import synthgraphs as sg
    from paper_2303_03964_amd import autotune
    t_gen = time.perf_counter()
    members = [sg.sbm_batch_member(i) for i in range(graphs)]
    gen_s = time.perf_counter() - t_gen
    lays, pos0, p1 = [], [], []
    for g, pos in members:
        k_mode, n_int = autotune.start_params(g.n)
        p = T.tfdp_params_default(n_int=n_int, total_iters=iters, k_mode=k_mode)
        ws = (T.tfdp_params_default(n_int=max(n_int, autotune.workspace_grid(g.n)), total_iters=iters)
              if accuracy and k_mode != 0 else p)
        pt = torch.as_tensor(pos).cuda()
        pos0.append(pt.clone())
        p1.append(p)
        lays.append(T.Layout(g.row_ptr, g.col_idx, pt, p, workspace_params=ws))
    n_tot = sum(l.n for l in lays)
    nnz_tot = sum(l.nnz for l in lays)
    stage1 = (19 * iters) // 20 if accuracy else iters  # first k = 3 iteration
    B = T.Batch(len(lays))
    for lay in lays:
        B.add(lay)
    # tile schedule of the batched grid passes, chosen by the autotuner for
    # the FFT lengths of each stage (k = 1 at t = 0, then the k = 2 and k = 3
    # grids at their switches)
    t_tune = time.perf_counter()
    tiles, done = {}, set()
    for t_at in (0, (9 * iters) // 10, (19 * iters) // 20):
        want = autotune.batch_lengths(lays, t_at) - done
        if want:
            tiles.update(autotune.tune_batch_tiles(B, lays, lengths=want, at_iteration=t_at))
            done |= want
    tune_s = time.perf_counter() - t_tune

    def reset():
        for lay, p0, p in zip(lays, pos0, p1):
            lay.set_params(p)
            lay.pos.copy_(p0)
            lay.iteration = 0
        torch.cuda.synchronize()

    def run(batched):
        reset()
        t0 = time.perf_counter()
        if batched:
            B.step(stage1)
        else:
            for lay in lays:
                lay.step(stage1)
        torch.cuda.synchronize()
        if stage1 < iters:
            grids = autotune.retune_many(lays)
            if batched:
                B.step(iters - stage1)
            else:
                for lay in lays:
                    lay.step(iters - stage1)
            torch.cuda.synchronize()
        else:
            grids = [lay.params.n_int for lay in lays]
        return time.perf_counter() - t0, grids

    run(True)   # warm-up: device tables, captured graphs of both stages
    if sequential:
        run(False)
    t_batch, grids = run(True)
    final_batch = [lay.pos.clone() for lay in lays]
    if sequential:
        t_seq, grids_seq = run(False)
        same = all(torch.equal(a, lay.pos) for a, lay in zip(final_batch, lays)) and grids == grids_seq
    else:
        t_seq, same = float("nan"), None
    bad = [lay.sync_status() for lay in lays]
    # repulsion error of the last stage's method at the final positions
    # (k = 3 grid against the exact sums; 0 for the exact method), on every
    # 16th graph
    errs = []
    for lay in lays[::16]:
        if lay.params.k_mode == 0:
            errs.append(0.0)
            continue
        ex, _, _ = lay.forces(k=0)
        fr, _, _ = lay.forces(k=3)
        torch.cuda.synchronize()
        errs.append(float(torch.linalg.norm((fr - ex).double()) / torch.linalg.norm(ex.double())))
    B.close()
    for lay in lays:
        lay.close()
    return {
        "workload": f"sbm_batch_{graphs}: SBMs, n log-uniform [200, 20000], 2..20 blocks, mean degree 8",
        "graphs": graphs,
        "nodes": n_tot,
        "nnz": nnz_tot,
        "iters": iters,
        "grid_rule": ("n <= 1024: exact method; else k=1,2: N_int = 64 (n/1000)^(1/5) rounded down to a "
                      "power of two when within 25%; k=3 stage: N_int = ceil(1.4 W / h3(1e-3)) from the box at "
                      "the switch, or the exact method where it costs less"
                      if accuracy else "n <= 1024: exact method; else the k=1,2 grid for the whole schedule"),
        "exact_method_graphs": sum(1 for q in p1 if q.k_mode == 0),
        "final_stage_exact_graphs": sum(1 for v in grids if v == 0),
        "final_n_int": ({"min": min(v for v in grids if v), "median": int(np.median([v for v in grids if v])),
                         "max": max(grids)} if any(grids) else None),
        "final_stage_rel_err_vs_exact": {"graphs": len(errs), "median": float(np.median(errs)), "max": max(errs)},
        "value": n_tot * iters / t_batch,
        "unit": "node-iterations/s",
        "ms": t_batch * 1e3,
        "sequential_value": n_tot * iters / t_seq,
        "sequential_ms": t_seq * 1e3,
        "speedup_vs_sequential": t_seq / t_batch,
        "bitwise_equal_to_sequential": same if same is None else bool(same),
        "tiles": {str(L): {"rows_per_block": r, "column_groups": g, "trial_ms": round(ms, 3)}
                  for L, (r, g, ms) in sorted(tiles.items())},
        "tile_tuning_s": tune_s,
        "nonfinite_members": int(sum(1 for v in bad if v != 0)),
        "generation_s": gen_s,
    }


def final_stage_accuracy(T, torch, pool, trace, recs, stream, every=8):
    """Repulsion error of the last stage's method against the exact sums at
    the final positions of every `every`-th served request (0 for requests
    whose last stage is the exact method), and the mix of last stages."""
    errs, grid_errs = [], []
    with torch.cuda.stream(stream):
        for r, req in list(zip(recs, trace))[::every]:
            k_mode, n_int = r.final
            if k_mode == 0:
                errs.append(0.0)
                continue
            g = pool[req.graph][0] if req.kind == "layout" else pool[trace[req.target].graph][0]
            p = T.TfdpParams(**{**r.params.as_dict(), "n_int": n_int, "k_mode": -1})
            ws = T.TfdpParams(**{**p.as_dict(), "n_int": max(n_int, r.ws_n_int)})
            lay = T.Layout(g.row_ptr, g.col_idx, r.final_pos.clone(), p, workspace_params=ws)
            ex, _, _ = lay.forces(k=0)
            fr, _, _ = lay.forces(k=3)
            torch.cuda.synchronize()
            e = float(torch.linalg.norm((fr - ex).double()) / torch.linalg.norm(ex.double()))
            errs.append(e)
            grid_errs.append(e)
            lay.close()
    last = [r.final for r in recs]
    return {
        "tol": 1e-3,
        "sampled_requests": len(errs),
        "rel_err_vs_exact": {"median": float(np.median(errs)), "max": float(max(errs)),
                             "grid_requests": len(grid_errs),
                             "grid_max": float(max(grid_errs)) if grid_errs else None},
        "last_stage_exact_requests": sum(1 for f in last if f[0] == 0),
        "last_stage_grid_requests": sum(1 for f in last if f[0] != 0),
        "rule": "box read 10 iterations before the first k = 3 iteration; N_int = ceil(1.4 W / h3(1e-3)) "
                "(capped by the workspace), or the exact method where it costs less",
    }


def serving_section(T, torch, stream, requests):
    """Serving workload: Poisson arrivals of layout requests (Chung-Lu, n
    log-uniform in [1000, 200000], exponent in [2, 3], 200 iterations) and
    re-tune requests (30%: new alpha, beta, gamma, repulsion weight on a
    resident graph, 50 iterations). The sequential capacity is measured
    first (every request arriving at once, served one by one with
    tfdp_layout_step); the continuous-batching server then runs at offered
    loads of 0.5, 0.8 and 1.2 times that capacity."""
    import synthgraphs as sg
    from paper_2303_03964_amd import serve
    pool_n = 48
    t_gen = time.perf_counter()
    pool = [sg.serving_graph(i) for i in range(pool_n)]
    gen_s = time.perf_counter() - t_gen
    free, total = torch.cuda.mem_get_info()
    budget = int(0.5 * free)
    out = {"workload": "serving: Chung-Lu n log-uniform [1e3, 2e5], exponent [2, 3], mean degree 10; "
                       "30% re-tunes (alpha, beta, gamma, w_r) of resident graphs",
           "pool_graphs": pool_n, "requests": requests, "layout_iters": 200, "retune_iters": 50,
           "hbm_budget_bytes": budget, "chunk": 10, "generation_s": gen_s,
           "final_stage_tol": 1e-3}
    # warm-up: kernels, allocator
    warm = sg.serving_trace(6, 1e6, pool_n, seed=1)
    for plain in (True, False):
        srv = serve.Server(pool, budget, stream=stream, plain=plain)
        srv.run(warm)
        srv.close()
    burst = sg.serving_trace(requests, 1e9, pool_n, seed=sg.SEED_BASE + 7)
    srv = serve.Server(pool, budget, stream=stream, plain=True, record_outputs=True)
    t0 = time.perf_counter()
    recs_seq = srv.run(burst)
    seq_s = time.perf_counter() - t0
    srv.close()
    cap = requests / seq_s
    seq = serve.summarize(recs_seq, seq_s)
    out["sequential"] = {"capacity_req_per_s": cap, **seq}
    srv = serve.Server(pool, budget, stream=stream, record_outputs=True)
    t0 = time.perf_counter()
    recs = srv.run(burst)
    bat_s = time.perf_counter() - t0
    srv.close()
    same = all(torch.equal(a.final_pos, b.final_pos) and a.final == b.final for a, b in zip(recs, recs_seq))
    out["batched_burst"] = {"req_per_s": requests / bat_s, **serve.summarize(recs, bat_s),
                            "bitwise_equal_to_sequential": bool(same)}
    out["final_stage"] = final_stage_accuracy(T, torch, pool, burst, recs, stream)
    print(f"# serving final stage: {json.dumps(out['final_stage'])}", file=sys.stderr, flush=True)
    del recs, recs_seq
    loads = {}
    for f in (0.5, 0.8, 1.2):
        trace = sg.serving_trace(requests, f * cap, pool_n, seed=sg.SEED_BASE + 7)
        srv = serve.Server(pool, budget, stream=stream)
        t0 = time.perf_counter()
        recs = srv.run(trace)
        wall = time.perf_counter() - t0
        srv.close()
        seq_trace = serve.Server(pool, budget, stream=stream, plain=True)
        t1 = time.perf_counter()
        recs_seq = seq_trace.run(trace)
        wall_seq = time.perf_counter() - t1
        seq_trace.close()
        loads[f"{f}x"] = {"offered_req_per_s": f * cap, "batched": serve.summarize(recs, wall),
                          "sequential": serve.summarize(recs_seq, wall_seq)}
        print(f"# serving load {f}x: {json.dumps(loads[f'{f}x'])}", file=sys.stderr, flush=True)
    out["loads"] = loads
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2303_03964_amd as T

    t_gen = time.perf_counter()
    w = workload(args.workload)
    g = w.graph
    print(f"# workload {w.name}: n={g.n} nnz={g.nnz} n_int={w.n_int} T={w.iters} "
          f"(generated in {time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    # a side stream (default priority): iteration pairs are captured as HIP
    # graphs, which the legacy default stream does not allow
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    pos0 = torch.as_tensor(w.pos0).to(dev)
    params = T.tfdp_params_default(n_int=w.n_int, total_iters=w.iters, k_mode=-1)
    lay = T.Layout(g.row_ptr, g.col_idx, pos0.clone(), params, device=dev)
    if args.no_graphs:
        T.tfdp_layout_set_graphs(lay.handle, 0)
    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def reset(pos=pos0, t=0):
        lay.pos.copy_(pos)
        lay.iteration = t
        torch.cuda.synchronize()

    # untimed pass over the whole schedule (T iterations from the start): the
    # quality of the final layout, and the states at the k = 2 and k = 3
    # switches from which a timed region shorter than T starts its k = 2 and
    # k = 3 iterations
    T_all = w.iters
    t_k2, t_k3 = (9 * T_all) // 10, (19 * T_all) // 20
    reset()
    lay.step(t_k2)
    pos_k2 = lay.pos.clone()
    lay.step(t_k3 - t_k2)
    pos_k3 = lay.pos.clone()
    lay.step(T_all - t_k3)
    torch.cuda.synchronize()
    if lay.sync_status() != 0:
        raise RuntimeError("non-finite positions in the schedule pass")
    # quality of the final layout: stress error and neighbourhood preservation
    # over 64 seeded sources (BFS, sums and the radix select on the device)
    t_q = time.perf_counter()
    src = torch.as_tensor(np.random.default_rng(20230307).choice(g.n, 64, replace=False), dtype=torch.int32).to(dev)
    se, nps, levels = T.tfdp_quality_sampled(lay.row_ptr, lay.col_idx, lay.pos, src)
    quality = {"after_iters": T_all, "se_sampled": se, "np1_sampled": nps[0], "np2_sampled": nps[1],
               "sources": 64, "bfs_levels": levels, "seconds": round(time.perf_counter() - t_q, 4)}

    # timed region: K iterations. K >= T: the schedule from the start (its
    # first K iterations). K < T: a schedule-weighted sample, K - 2 m
    # iterations at k = 1 from the start and m = round(K / 20) (at least one
    # when K >= 3) at k = 2 and at k = 3, each from the state saved at its
    # switch: the 90/5/5 % mix of the whole layout
    if args.steps >= T_all or args.steps < 3:
        segments = [(pos0, 0, args.steps)]
    else:
        m = max(1, int(round(args.steps / 20)))
        segments = [(pos0, 0, args.steps - 2 * m), (pos_k2, t_k2, m), (pos_k3, t_k3, m)]
    k_mix = {}
    for p_, t_, c_ in segments:
        for it in range(t_, t_ + c_):
            kk = 1 if it < t_k2 else (2 if it < t_k3 else 3)
            k_mix[f"k{kk}"] = k_mix.get(f"k{kk}", 0) + 1

    if args.warmup > 0:
        reset()
        lay.step(args.warmup)
        torch.cuda.synchronize()
        if lay.sync_status() != 0:
            raise RuntimeError("non-finite positions during warm-up")
    times = []
    for _ in range(max(1, args.repeats)):
        total = 0.0
        for p_, t_, c_ in segments:
            reset(p_, t_)
            t0 = time.perf_counter()
            lay.step(c_)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
        times.append(total)
    st = lay.sync_status()
    if st != 0:
        raise RuntimeError(f"layout status {st}")
    secs = float(np.median(times))
    print(f"# timed {args.steps} iterations {k_mix}: {secs * 1e3:.2f} ms (runs: {[round(t * 1e3, 2) for t in times]})",
          file=sys.stderr, flush=True)

    # per-phase times with HIP events recorded by the library on the launch
    # stream: the k = 1 iterations of the timed region from the start, and a
    # few iterations from each switch
    reset()
    k1_iters = max(1, min(args.steps, t_k2))
    T.tfdp_layout_set_profiling(lay.handle, 1)
    lay.step(k1_iters)
    ph1 = T.tfdp_layout_phase_times(lay.handle)
    ph_k = {}
    for kk, (p_, t_) in ((2, (pos_k2, t_k2)), (3, (pos_k3, t_k3))):
        reset(p_, t_)
        lay.step(min(5, T_all - t_))
        ph_k[kk] = T.tfdp_layout_phase_times(lay.handle)
    T.tfdp_layout_set_profiling(lay.handle, 0)
    torch.cuda.synchronize()

    gather_ref = gather_reference(torch, lay, stream)
    # dominant kernel: the attraction pass when it runs beside the grid passes
    # (events on its own stream), else the fused edge pass
    overlapped = ph1.get("attract", (0.0, 0))[1] > 0
    if overlapped:
        gm_ms, gm_n = ph1["attract"]
        kernel = "k_attract (attraction sums of every row, on a second stream beside the grid passes; k=1)"
        bytes_launch = attract_bytes(g.n, g.nnz)
        summary = "attract_chung_lu_1m_traffic.json"
    else:
        gm_ms, gm_n = ph1["gather_update"]
        kernel = "k_edges<1,2> (edge pass + gather + update, k=1)"
        bytes_launch = gather_bytes(g.n, g.nnz, w.n_int)
        summary = "gather_update_chung_lu_1m_traffic.json"
    avg_ms = gm_ms / max(gm_n, 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic("paper_2303_03964_amd/csrc/node_forces.hip", summary)
    phases = {name: round(ms / cnt, 4) for name, (ms, cnt) in ph1.items() if cnt}
    phases_k23 = {f"k{kk}": {name: round(ms / cnt, 4) for name, (ms, cnt) in ph.items() if cnt}
                  for kk, ph in ph_k.items()}
    # summed kernel time per k = 1 iteration (phases that run concurrently on
    # the two streams are counted separately)
    kernel_ms_k1 = sum(ms for ms, _ in ph1.values()) / max(k1_iters, 1)
    dbar = g.nnz / g.n
    # bytes per node-iteration: algorithmic (positions read by the spreading
    # and by the edge pass, written once, row_ptr, column index and neighbour
    # position per CSR entry) and compulsory (neighbour positions served from
    # the on-chip caches)
    alg_node_it = 28.0 + 12.0 * dbar
    comp_node_it = 28.0 + 4.0 * dbar
    step_s = secs / args.steps

    rec = {
        "metric": "t-FDP node-iterations/s at 1M nodes" if w.name == "chung_lu_1m"
        else f"t-FDP node-iterations/s ({w.name})",
        "value": g.n * args.steps / secs,
        "unit": "node-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "n": g.n,
            "nnz": g.nnz,
            "n_int": w.n_int,
            "total_iters": w.iters,
            "k_schedule": "1/2/3 over 90/5/5%",
            "timed_k_mix": k_mix,
            "timed_segments_start_iter": [t_ for _, t_, _ in segments],
            "params": {"alpha": 0.1, "beta": 8.0, "gamma": 2.0},
            "positions": "uniform [-1,1]^2 float32, seeded",
        },
        "roofline": {
            "kernel": kernel,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_launch,
            "avg_launch_ms": avg_ms,
            "launches": gm_n,
            "gather_reference": gather_ref,
        },
        "step_bytes": {
            "algorithmic_per_node_iter": alg_node_it,
            "compulsory_per_node_iter": comp_node_it,
            "algorithmic_GBps": alg_node_it * g.n / step_s / 1e9,
            "algorithmic_frac": alg_node_it * g.n / step_s / 1e9 / HBM_PEAK_GBS,
            "compulsory_GBps": comp_node_it * g.n / step_s / 1e9,
            "compulsory_frac": comp_node_it * g.n / step_s / 1e9 / HBM_PEAK_GBS,
        },
        "phase_ms_k1": phases,
        "phase_ms_k23": phases_k23,
        "kernel_ms_sum_k1_events": kernel_ms_k1,
        "edge_pass_overlapped": overlapped,
        "final_layout_quality": quality,
        "hip_graphs": not args.no_graphs,
    }
    lay.close()
    if not args.no_batch:
        seq = not args.no_batch_sequential
        rec["batched"] = batched_section(T, torch, stream, args.batch_graphs, args.batch_iters, sequential=seq)
        print(f"# batched: {json.dumps(rec['batched'])}", file=sys.stderr, flush=True)
        rec["batched_size_rule_grids"] = batched_section(T, torch, stream, args.batch_graphs, args.batch_iters,
                                                         accuracy=False, sequential=seq)
        print(f"# batched (size-rule grids): {json.dumps(rec['batched_size_rule_grids'])}", file=sys.stderr,
              flush=True)
    if not args.no_serve:
        rec["serving"] = serving_section(T, torch, stream, args.serve_requests)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_iters)
        if w.name == "chung_lu_1m":
            # the oracle on the 100k-mesh workload as well (about 5 s)
            rec["cpu_baseline_mesh_100k"] = cpu_baseline(workload("mesh_100k"), 0, budget=5.0)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
