"""Batched stepping (tfdp_batch_*) against plain tfdp_layout_step.

A batch runs the plain kernels' code for every graph inside shared launches,
so each member's positions and counter after a batched call must equal,
bit for bit, those of the same handle stepped alone with the same calls.
The plain path itself is pinned to the FP64 oracle by test_gpu_parity.py.
Cases: graphs of uneven sizes and grids (several FFT-length classes in one
launch), k schedules crossing 1 -> 2 -> 3 inside a call, odd call lengths,
fixed-k and exact-method members, non-default parameters, members joining
with another counter, re-tuned parameters between calls, removal, and
captured graphs against direct launches.
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


@pytest.fixture(scope="module")
def stream():
    import torch
    s = torch.cuda.Stream()
    return s


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (batch member index, N_int, extra parameters)
MEMBERS = [
    (0, 32, {}),
    (1, 64, {}),
    (2, 16, {}),
    (3, 128, {}),
    (5, 48, {"k_mode": 2}),
    (6, 24, {"alpha": 0.05, "beta": 4.0, "gamma": 3.0, "rep_weight": 2.0}),
    (7, 40, {}),
    (9, 8, {"k_mode": 1}),
]


def graphs(indices):
    return [sg.sbm_batch_member(i) for i in indices]


def pair(T, g, pos, n_int, total, extra):
    import torch
    p = T.tfdp_params_default(n_int=n_int, total_iters=total, **extra)
    a = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), p)
    b = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), p)
    return a, b


def run_case(T, stream, calls, total=40, graphs_on=True, members=MEMBERS, exact_n=0):
    import torch
    with torch.cuda.stream(stream):
        gs = graphs([m[0] for m in members])
        batch_lays, plain_lays = [], []
        for (idx, n_int, extra), (g, pos) in zip(members, gs):
            a, b = pair(T, g, pos, n_int, total, extra)
            batch_lays.append(a)
            plain_lays.append(b)
        if exact_n:
            g = sg.sbm([exact_n // 2, exact_n - exact_n // 2], 0.1, 0.01, 17)
            pos = sg.uniform_positions(g.n, 18)
            a, b = pair(T, g, pos, 16, total, {"k_mode": 0})
            batch_lays.append(a)
            plain_lays.append(b)
        say(f"batch of {len(batch_lays)}: n = {[l.n for l in batch_lays]}")
        B = T.Batch(len(batch_lays) + 2)
        B.set_graphs(graphs_on)
        for lay in batch_lays:
            B.add(lay)
        for c in calls:
            B.step(c)
            for lay in plain_lays:
                lay.step(c)
        torch.cuda.synchronize()
        for a, b in zip(batch_lays, plain_lays):
            assert a.sync_status() == 0 and b.sync_status() == 0
            assert a.iteration == b.iteration == sum(calls)
            same = torch.equal(a.pos, b.pos)
            if not same:
                d = (a.pos - b.pos).abs().max().item()
                say(f"  n={a.n}: max |diff| = {d}")
            assert same
        B.close()
        return batch_lays, plain_lays


def test_batch_matches_plain_bitwise(T, stream):
    # 7 + 20 + 13 iterations with T = 40: k switches at t = 36 and 38
    run_case(T, stream, [7, 20, 13], exact_n=300)


def test_batch_direct_launches(T, stream):
    run_case(T, stream, [5, 6], graphs_on=False)


def test_batch_single_iterations_and_long_calls(T, stream):
    run_case(T, stream, [1, 1, 30, 1, 3], total=36, members=MEMBERS[:4])


def test_batch_membership_and_retune(T, stream):
    import torch
    with torch.cuda.stream(stream):
        gs = graphs([0, 2, 4])
        lays = [pair(T, g, pos, 32, 60, {}) for g, pos in gs]
        B = T.Batch(4)
        B.add(lays[0][0])
        B.add(lays[1][0])
        B.step(9)
        lays[0][1].step(9)
        lays[1][1].step(9)
        # a member joins with counter 0 while the others are at 9
        B.add(lays[2][0])
        # re-tune member 1 (Sec. 5 global refinement: weights changed)
        p = T.tfdp_params_default(n_int=32, total_iters=60, alpha=0.2, beta=2.0, rep_weight=3.0)
        lays[1][0].set_params(p)
        lays[1][1].set_params(p)
        B.step(12)
        for a, b in lays:
            b.step(12)
        # member 0 leaves; its counter moves through the plain API meanwhile
        B.remove(lays[0][0])
        lays[2][0].iteration = 40
        lays[2][1].iteration = 40
        B.step(11)
        for a, b in lays[1:]:
            b.step(11)
        torch.cuda.synchronize()
        for a, b in lays:
            assert a.iteration == b.iteration
            assert torch.equal(a.pos, b.pos)
        B.close()


def test_batch_many_uneven_graphs(T, stream):
    """48 graphs of the batched workload (n log-uniform 200..20000) with the
    size-driven grid choice; one call over the whole schedule."""
    import torch
    from paper_2303_03964_amd import autotune
    members = []
    for i in range(48):
        g, pos = sg.sbm_batch_member(i)
        members.append((i, autotune.n_int_for_size(g.n), {}))
    run_case(T, stream, [30], total=30, members=members)


def test_batch_with_tau_and_refinement_weights(T, stream):
    """Members with tau != 1 and local-refinement weights, bit-identical to
    their plain steps (weights and tau reach the batched kernels through the
    member descriptors)."""
    import torch
    with torch.cuda.stream(stream):
        gs = graphs([0, 1, 3])
        rng = np.random.default_rng(4)
        lays = []
        for q, (g, pos) in enumerate(gs):
            extra = {"tau": [0.5, 1.0, 2.0][q], "gamma": 2.3}
            a, b = pair(T, g, pos, 32, 40, extra)
            if q != 1:
                rw = torch.as_tensor(rng.uniform(0.5, 2.0, g.n).astype(np.float32))
                aw = torch.as_tensor(rng.uniform(0.5, 2.0, g.n).astype(np.float32))
                a.set_node_weights(rw, aw)
                b.set_node_weights(rw, aw)
            lays.append((a, b))
        B = T.Batch(4)
        for a, _ in lays:
            B.add(a)
        B.step(17)
        for _, b in lays:
            b.step(17)
        # weights changed between calls reach the batch
        w2 = torch.full((lays[1][0].n,), 1.7)
        lays[1][0].set_node_weights(None, w2)
        lays[1][1].set_node_weights(None, w2)
        B.step(23)
        for _, b in lays:
            b.step(23)
        torch.cuda.synchronize()
        for a, b in lays:
            assert a.iteration == b.iteration == 40
            assert torch.equal(a.pos, b.pos)
        B.close()
