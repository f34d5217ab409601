"""Sampled stress error on the device (Sec. 4, "Metrics") against the FP64
oracle's metric with the same sources: multi-source BFS hop distances and
the optimal-scale stress over (source, node) pairs."""
import sys

import numpy as np
import pytest

import synthgraphs as sg
from oracle import metrics as om
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


def gpu_se(T, g, pos, sources):
    import torch
    rp = torch.as_tensor(g.row_ptr, dtype=torch.int32).cuda()
    ci = torch.as_tensor(g.col_idx, dtype=torch.int32).cuda()
    p = torch.as_tensor(pos, dtype=torch.float32).cuda()
    src = torch.as_tensor(np.asarray(sources), dtype=torch.int32).cuda()
    return T.tfdp_stress_sampled(rp, ci, p, src)


@pytest.mark.parametrize("case", ["sbm_1k", "two_components", "mesh_100k"])
def test_sampled_stress_matches_oracle(T, case):
    rng = np.random.default_rng(3)
    if case == "sbm_1k":
        w = sg.sbm_1k()
        g, pos = w.graph, sg.uniform_positions(w.graph.n, 4, -20, 20)
        src = rng.choice(g.n, 64, replace=False)
    elif case == "two_components":
        a = sg.sbm([150, 150], 0.05, 0.01, 5)
        b = sg.sbm([100, 100], 0.05, 0.01, 6)
        e = np.concatenate([a.edges(), b.edges() + a.n])
        g = sg.csr_from_edges(a.n + b.n, e)
        pos = sg.uniform_positions(g.n, 7, -10, 10)
        src = rng.choice(g.n, 17, replace=False)
    else:
        w = sg.mesh_100k()
        g, pos = w.graph, sg.uniform_positions(w.graph.n, 8, -300, 300)
        src = rng.choice(g.n, 64, replace=False)
    se, levels = gpu_se(T, g, pos, src)
    want = om.stress_error(pos.astype(np.float64), g.row_ptr, g.col_idx, sources=src)
    d = om.graph_distances(g.n, g.row_ptr, g.col_idx, src)
    ecc = int(np.nanmax(np.where(np.isfinite(d), d, np.nan)))
    say(f"{case}: n={g.n} SE gpu {se:.12f} oracle {want:.12f} levels {levels} (max distance {ecc})")
    assert abs(se - want) <= 1e-9 * abs(want)
    assert levels == ecc + 1


def test_invalid_csr_is_rejected(T):
    import torch
    rp = torch.tensor([0, 1, 2], dtype=torch.int32).cuda()
    ci = torch.tensor([1, 5], dtype=torch.int32).cuda()  # column out of range
    p = torch.zeros((2, 2), dtype=torch.float32).cuda()
    src = torch.tensor([0], dtype=torch.int32).cuda()
    with pytest.raises(T.TfdpError):
        T.tfdp_stress_sampled(rp, ci, p, src)


def gpu_quality(T, g, pos, sources):
    import torch
    rp = torch.as_tensor(g.row_ptr, dtype=torch.int32).cuda()
    ci = torch.as_tensor(g.col_idx, dtype=torch.int32).cuda()
    p = torch.as_tensor(pos, dtype=torch.float32).cuda()
    src = torch.as_tensor(np.asarray(sources), dtype=torch.int32).cuda()
    return T.tfdp_quality_sampled(rp, ci, p, src)


def np_case(case):
    rng = np.random.default_rng(11)
    if case == "sbm_1k":
        w = sg.sbm_1k()
        g, pos = w.graph, sg.uniform_positions(w.graph.n, 4, -20, 20)
        src = rng.choice(g.n, 64, replace=False)
    elif case == "two_components_isolated":
        # two components plus isolated nodes (empty rings), some of them sources
        a = sg.sbm([150, 150], 0.05, 0.01, 5)
        b = sg.sbm([100, 100], 0.05, 0.01, 6)
        e = np.concatenate([a.edges(), b.edges() + a.n])
        g = sg.csr_from_edges(a.n + b.n + 5, e)
        pos = sg.uniform_positions(g.n, 7, -10, 10)
        src = np.concatenate([rng.choice(a.n + b.n, 20, replace=False), [g.n - 1, g.n - 3]])
    elif case == "grid_ties":
        # the lattice's own integer coordinates (node i at column i % 316,
        # row i // 316): rings are mostly preserved and many distances tie
        # exactly, so the k-th nearest is often decided by the node index
        w = sg.mesh_100k()
        g = w.graph
        idx = np.arange(g.n)
        pos = np.stack([idx % 316, idx // 316], axis=1).astype(np.float32)
        src = rng.choice(g.n, 64, replace=False)
    elif case == "coincident":
        # every node at one point: all distances tie
        w = sg.sbm_1k()
        g = w.graph
        pos = np.full((g.n, 2), 3.25, dtype=np.float32)
        src = rng.choice(g.n, 9, replace=False)
    else:
        # jittered lattice coordinates: high NP without ties
        w = sg.mesh_100k()
        g = w.graph
        idx = np.arange(g.n)
        pos = (np.stack([idx % 316, idx // 316], axis=1)
               + sg.uniform_positions(g.n, 8, -0.3, 0.3)).astype(np.float32)
        src = rng.choice(g.n, 33, replace=False)
    return g, pos, src


@pytest.mark.parametrize("case", ["sbm_1k", "two_components_isolated", "grid_ties", "coincident", "mesh_100k"])
def test_sampled_np_matches_oracle(T, case):
    g, pos, src = np_case(case)
    se, nps, levels = gpu_quality(T, g, pos, src)
    se_only, _ = gpu_se(T, g, pos, src)
    assert se == se_only or (np.isnan(se) and np.isnan(se_only))
    for r in (1, 2):
        want = om.neighborhood_preservation(pos, g.row_ptr, g.col_idx, r, nodes=[int(s) for s in src])
        say(f"{case}: n={g.n} NP_{r} gpu {nps[r - 1]:.15f} oracle {want:.15f}")
        # the same sets on both sides: equal up to the order of the mean
        assert abs(nps[r - 1] - want) <= 1e-12
        if case in ("grid_ties", "mesh_100k"):
            assert want > 0.3  # the case exercises large overlaps


def test_np_without_rings_is_nan(T):
    g = sg.csr_from_edges(6, np.array([[0, 1]]))
    pos = sg.uniform_positions(6, 2, 0, 1)
    se, nps, _ = gpu_quality(T, g, pos, [3, 4])
    assert np.isnan(nps[0]) and np.isnan(nps[1]) and np.isnan(se)


def test_source_out_of_range_is_rejected(T):
    g = sg.csr_from_edges(6, np.array([[0, 1], [1, 2]]))
    pos = sg.uniform_positions(6, 2, 0, 1)
    with pytest.raises(T.TfdpError, match="source"):
        gpu_quality(T, g, pos, [1, 6])
    with pytest.raises(T.TfdpError, match="source"):
        gpu_se(T, g, pos, [-1])


def test_quality_1m_bench_configuration(T):
    """SE, NP_1 and NP_2 on the 1M-node Chung-Lu graph after 40 layout
    iterations, from the first 16 of the 64 seeded sources bench.py uses
    (the oracle's distances and sorts over 1M nodes take seconds per
    source), against the oracle metrics over the same sources."""
    import torch
    w = sg.chung_lu_1m()
    g = w.graph
    p = T.tfdp_params_default(n_int=w.n_int, total_iters=w.iters)
    lay = T.Layout(g.row_ptr, g.col_idx, w.pos0, p)
    lay.step(40)
    torch.cuda.synchronize()
    pos = lay.pos.cpu().numpy()
    src = np.random.default_rng(20230307).choice(g.n, 64, replace=False)[:16]
    se, nps, levels = T.tfdp_quality_sampled(lay.row_ptr, lay.col_idx, lay.pos,
                                             torch.as_tensor(src, dtype=torch.int32).cuda())
    say(f"1M: device metrics done (SE {se:.6f}); oracle SE ...")
    want = om.stress_error(pos.astype(np.float64), g.row_ptr, g.col_idx, sources=src)
    say(f"1M: SE gpu {se:.12f} oracle {want:.12f}, BFS levels {levels}")
    assert abs(se - want) <= 1e-9 * abs(want)
    for r in (1, 2):
        want = om.neighborhood_preservation(pos, g.row_ptr, g.col_idx, r, nodes=[int(s) for s in src])
        say(f"1M: NP_{r} gpu {nps[r - 1]:.15f} oracle {want:.15f}")
        assert abs(nps[r - 1] - want) <= 1e-12
    lay.close()


@pytest.mark.parametrize("case", ["path_400", "lattice_200"])
def test_metrics_beyond_255_hops(T, case):
    """Graphs whose hop distances exceed 255 (a 400-node path; an unrewired
    200 x 200 lattice, diameter 398: the mesh family of Sec. 4): SE and NP
    over the same sources as the oracle metrics, every distance counted."""
    rng = np.random.default_rng(5)
    if case == "path_400":
        n = 400
        g = sg.csr_from_edges(n, np.stack([np.arange(n - 1), np.arange(1, n)], axis=1))
        pos = (np.stack([np.arange(n), np.zeros(n)], axis=1) + sg.uniform_positions(n, 3, -2, 2)).astype(np.float32)
        src = np.array([0, 7, 200, 399])
    else:
        g = sg.lattice_rewired(200, 0.0, 1)
        idx = np.arange(g.n)
        pos = (np.stack([idx % 200, idx // 200], axis=1) + sg.uniform_positions(g.n, 4, -0.4, 0.4)).astype(np.float32)
        src = np.concatenate([[0, g.n - 1], rng.choice(g.n, 10, replace=False)])
    se, nps, levels = gpu_quality(T, g, pos, src)
    d = om.graph_distances(g.n, g.row_ptr, g.col_idx, src)
    ecc = int(d[np.isfinite(d)].max())
    want = om.stress_error(pos.astype(np.float64), g.row_ptr, g.col_idx, sources=src)
    say(f"{case}: max hop distance {ecc}, BFS levels {levels}; SE gpu {se:.12f} oracle {want:.12f}")
    assert ecc > 255 and levels == ecc + 1
    assert abs(se - want) <= 1e-9 * abs(want)
    for r in (1, 2):
        w_np = om.neighborhood_preservation(pos, g.row_ptr, g.col_idx, r, nodes=[int(s) for s in src])
        say(f"  NP_{r} gpu {nps[r - 1]:.15f} oracle {w_np:.15f}")
        assert abs(nps[r - 1] - w_np) <= 1e-12


def test_bfs_beyond_16_bit_distances_is_refused(T):
    """A path of 66,000 nodes from one end: the BFS still finds nodes at hop
    distance 65534, the largest 16-bit distance, so the call is refused with
    TFDP_ERR_UNSUPPORTED rather than counting farther nodes as unreachable."""
    n = 66000
    g = sg.csr_from_edges(n, np.stack([np.arange(n - 1), np.arange(1, n)], axis=1))
    pos = sg.uniform_positions(n, 9, -5, 5)
    say("path of 66,000 nodes: one BFS level per launch up to level 65534")
    with pytest.raises(T.TfdpError) as e:
        gpu_se(T, g, pos, [0])
    assert e.value.status == -5
    # the same path from its middle node has eccentricity 33,000: measured
    se, levels = gpu_se(T, g, pos, [n // 2])
    assert levels == n // 2 + 1 and np.isfinite(se)
