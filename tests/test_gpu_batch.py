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


def test_batch_exact_symmetric_member_bitwise(T, stream):
    # an exact member of 5,000 nodes takes the pair-symmetric passes (tile
    # pairs and node pass in the batched launches), beside a small exact one
    run_case(T, stream, [3, 4], members=MEMBERS[:2], exact_n=5000)
    run_case(T, stream, [2, 5], members=MEMBERS[:1], exact_n=300)


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


def test_batch_members_match_oracle_one_step(T, stream):
    """One batched iteration of members of every class against the FP64
    oracle's forces and capped move (Sec. 3.3 Eq.5-7 and Sec. 3.4 applied to
    each member): the exact method, fixed k = 2, the k schedule at t = 0
    (k = 1), t = 275 (k = 2) and t = 290 (k = 3) of T = 300, and a member
    with tau and local-refinement weights. Positions are spread to about a
    laid-out extent (side ~ sqrt(n)), so that the grids are coarse and the
    update caps some moves. Bound: relative L2 of the move <= 1e-5 and the
    per-node bound of the plain parity tests."""
    import torch
    from oracle import tfdp as ot
    from tests.test_gpu_parity import NODE_TOL
    # (label, batch member index, parameters, counter, weights)
    cases = [
        ("exact", 1, dict(k_mode=0, n_int=16), 0, False),
        ("fixed k=2", 2, dict(k_mode=2, n_int=48), 0, False),
        ("schedule t=0", 0, dict(k_mode=-1, n_int=64), 0, False),
        ("schedule t=275", 3, dict(k_mode=-1, n_int=32), 275, False),
        ("schedule t=290", 19, dict(k_mode=-1, n_int=40), 290, False),
        ("tau + weights", 18, dict(k_mode=1, n_int=24, tau=0.6, alpha=0.05, beta=6.0, rep_weight=1.5), 0, True),
    ]
    rng = np.random.default_rng(8)
    with torch.cuda.stream(stream):
        B = T.Batch(len(cases))
        items = []
        for label, idx, extra, t, weighted in cases:
            g, pos = sg.sbm_batch_member(idx)
            pos = (pos * (0.5 * np.sqrt(g.n))).astype(np.float32)
            p = T.tfdp_params_default(total_iters=300, **extra)
            lay = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), p)
            lay.iteration = t
            rw = aw = None
            if weighted:
                rw = rng.uniform(0.5, 3.0, g.n).astype(np.float32)
                aw = rng.uniform(0.2, 4.0, g.n).astype(np.float32)
                lay.set_node_weights(torch.as_tensor(rw), torch.as_tensor(aw))
            B.add(lay)
            items.append((label, g, pos, extra, t, rw, aw, lay))
        B.step(1)
        torch.cuda.synchronize()
        for label, g, pos, extra, t, rw, aw, lay in items:
            assert lay.sync_status() == 0 and lay.iteration == t + 1
            got = lay.pos.cpu().numpy().astype(np.float64)
            op = ot.Params(total_iters=300, **extra)
            k = extra["k_mode"] if extra["k_mode"] >= 0 else ot.k_for_iteration(t, 300)
            x = pos.astype(np.float64)
            _, _, disp = ot.forces(x, g.row_ptr, g.col_idx, op, k,
                                   rep_w=None if rw is None else rw.astype(np.float64),
                                   att_w=None if aw is None else aw.astype(np.float64))
            want = ot.capped_move(x, disp, ot.step_cap(t, 300, ot.default_t0(g.n)))
            err = float(np.linalg.norm((got - x) - (want - x)) / np.linalg.norm(want - x))
            mv = np.linalg.norm(want - x, axis=1)
            node = float((np.linalg.norm(got - want, axis=1) / (mv + np.median(mv))).max())
            say(f"{label}: n={g.n} k={k} move rel L2 {err:.2e}, per node {node:.2e}")
            assert err <= 1e-5
            assert node <= NODE_TOL
        B.close()
        for it in items:
            it[-1].close()


def test_batch_churn_reuse_and_arena_resets(T, stream):
    """Members join, leave and re-join over many short calls (the serving
    pattern), with an arena of the minimum size, so that compositions are
    built, reused (captured on their second use) and dropped by arena resets;
    every member stays bit-identical to its plain twin."""
    import torch
    with torch.cuda.stream(stream):
        gs = graphs([0, 1, 2, 4, 7])
        lays = [pair(T, g, pos, [32, 48, 16, 24, 40][q], 80, {}) for q, (g, pos) in enumerate(gs)]
        B = T.Batch(3, map_entries=3000)  # room for a few compositions: resets
        plan = [  # (members in the batch during the call, iterations)
            ({0, 1}, 4), ({0, 1}, 4), ({0, 1, 2}, 3), ({1, 2}, 5), ({1, 2, 3}, 6), ({1, 2, 3}, 6),
            ({2, 3, 4}, 7), ({0, 3, 4}, 2), ({0, 3, 4}, 2), ({0, 1, 4}, 9), ({0, 1}, 4), ({0, 1}, 4),
        ]
        inside = set()
        for members, iters in plan:
            for q in sorted(inside - members):
                B.remove(lays[q][0])
            for q in sorted(members - inside):
                B.add(lays[q][0])
            inside = set(members)
            B.step(iters)
            for q in members:
                lays[q][1].step(iters)
        torch.cuda.synchronize()
        for q, (a, b) in enumerate(lays):
            assert a.sync_status() == 0
            assert a.iteration == b.iteration, q
            assert torch.equal(a.pos, b.pos), q
        B.close()


def test_batch_arena_too_small_is_reported(T, stream):
    """A composition larger than the whole arena is refused with
    TFDP_ERR_WORKSPACE (nothing stepped); a larger arena then runs it."""
    import torch
    with torch.cuda.stream(stream):
        lays = []
        for q, g in enumerate([sg.chung_lu(60_000, 2.5, 10.0, 5), sg.sbm([400, 300], 0.02, 0.002, 6)]):
            pos = sg.uniform_positions(g.n, 6 + q)
            lays.append(T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(),
                                 T.tfdp_params_default(n_int=[96, 32][q])))
        B = T.Batch(2, map_entries=0)  # the minimum arena (256 entries)
        for lay in lays:
            B.add(lay)
        with pytest.raises(T.TfdpError) as e:
            B.step(2)
        assert e.value.status == -2 and "map entries" in str(e.value)
        # the same members step in a batch whose arena holds their composition
        B.close()
        B2 = T.Batch(2, map_entries=1 << 16)
        for lay in lays:
            B2.add(lay)
        B2.step(2)
        torch.cuda.synchronize()
        for lay in lays:
            assert lay.sync_status() == 0 and lay.iteration == 2
        B2.close()
        for lay in lays:
            lay.close()


def test_single_member_batch_equals_plain(T, stream):
    """A batch of one steps its member by the plain call; joining and
    leaving members switch between that and the batched launches without
    changing any result."""
    import torch
    with torch.cuda.stream(stream):
        gs = graphs([3, 5])
        lays = [pair(T, g, pos, [48, 32][q], 50, {}) for q, (g, pos) in enumerate(gs)]
        B = T.Batch(2)
        B.add(lays[0][0])
        for calls, members in (((7, 5), (0,)), ((9,), (0, 1)), ((6, 3), (0,)), ((20,), (0, 1))):
            for q in (0, 1):
                inside = any(m is lays[q][0] for m in B.members)
                if q in members and not inside:
                    B.add(lays[q][0])
                elif q not in members and inside:
                    B.remove(lays[q][0])
            for c in calls:
                B.step(c)
                for q in members:
                    lays[q][1].step(c)
        torch.cuda.synchronize()
        for a, b in lays:
            assert a.iteration == b.iteration
            assert torch.equal(a.pos, b.pos)
        B.close()


@pytest.mark.parametrize("rows,groups", [(2, 1), (4, 2), (8, 1)])
def test_batch_tiles_bitwise(T, stream, rows, groups):
    """Every tile of the batched grid passes gives the plain results bit for
    bit (members at FFT lengths 128, 256, 384 and 512 across the k switches)."""
    import torch
    members = [(0, 32, {}), (1, 64, {}), (3, 96, {}), (7, 40, {}), (5, 48, {"k_mode": 2})]
    with torch.cuda.stream(stream):
        gs = graphs([m[0] for m in members])
        lays = [pair(T, g, pos, n_int, 40, extra) for (idx, n_int, extra), (g, pos) in zip(members, gs)]
        B = T.Batch(len(lays))
        for L in (64, 128, 256, 384, 512):
            B.set_tiles(L, rows, groups)
            assert B.tiles(L) == (rows, groups)
        for a, _ in lays:
            B.add(a)
        for c in (9, 20, 11):
            B.step(c)
            for _, b in lays:
                b.step(c)
        torch.cuda.synchronize()
        for a, b in lays:
            assert a.iteration == b.iteration == 40
            assert torch.equal(a.pos, b.pos)
        B.close()


def test_tile_autotuner_restores_state(T, stream):
    import torch
    from paper_2303_03964_amd import autotune
    with torch.cuda.stream(stream):
        gs = graphs([0, 1, 3, 4])
        lays = [pair(T, g, pos, autotune.n_int_for_size(g.n), 60, {})[0] for g, pos in gs]
        B = T.Batch(len(lays))
        for lay in lays:
            B.add(lay)
        B.step(3)
        torch.cuda.synchronize()
        before = [(lay.pos.clone(), lay.iteration) for lay in lays]
        chosen = autotune.tune_batch_tiles(B, lays, iters=2, repeats=1)
        say(f"tiles chosen: {chosen}")
        assert chosen and all(L in autotune.TUNABLE_LENGTHS for L in chosen)
        for L, (r, g, ms) in chosen.items():
            assert B.tiles(L) == (r, g) and ms > 0
        for lay, (p, t) in zip(lays, before):
            assert lay.iteration == t and torch.equal(lay.pos, p)
        B.close()
