"""The overlapped edge pass (attraction on a second stream beside the grid
passes, then a node pass) against the fused edge pass and the FP64 oracle.

Both schedules run the same arithmetic per node (the same segmented row sums,
repulsion gather and capped move), so positions and forces must be equal bit
for bit, across k switches, with captured graphs and with direct launches,
and with local-refinement weights; the overlapped forces are also held to the
oracle (relative L2 and the per-node bound of the parity tests)."""
import sys

import numpy as np
import pytest

import synthgraphs as sg
from oracle import tfdp as ot
from tests._lib import ensure_built, rel_l2

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


def hub_graph(n=20000, seed=4):
    """Random graph with two heavy rows (degree 1500 and 900: the edge pass's
    block-wide path) and a ragged tail of ordinary rows."""
    rng = np.random.default_rng(seed)
    e = [(0, j) for j in range(1, 1501)]
    e += [(1, j) for j in range(3000, 3900)]
    u = rng.integers(0, n, size=5 * n)
    v = rng.integers(0, n, size=5 * n)
    e += list(zip(u.tolist(), v.tolist()))
    return sg.csr_from_edges(n, np.array(e, dtype=np.int64))


def pair(T, g, pos, graphs=True, **kw):
    import torch
    p = T.tfdp_params_default(**kw)
    out = []
    for mode in (0, 1):
        lay = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), p)
        lay.set_overlap(mode)
        if not graphs:
            T.tfdp_layout_set_graphs(lay.handle, 0)
        out.append(lay)
    return out


@pytest.mark.parametrize("case", ["hub_20k", "mesh_100k"])
@pytest.mark.parametrize("graphs", [True, False])
def test_overlap_steps_bitwise_equal_fused(T, case, graphs):
    import torch
    if case == "hub_20k":
        g, n_int = hub_graph(), 64
        pos = sg.uniform_positions(g.n, 31, -1, 1)
    else:
        w = sg.mesh_100k()
        g, n_int, pos = w.graph, w.n_int, w.pos0
    iters = 40  # k = 1 for 36 iterations, k = 2 for 2, k = 3 for 2
    fused, over = pair(T, g, pos, graphs, n_int=n_int, total_iters=iters)
    for chunk in (13, 17, 10):  # calls that end inside and across the k switches
        for lay in (fused, over):
            lay.step(chunk)
        torch.cuda.synchronize()
        same = bool(torch.equal(fused.pos, over.pos))
        say(f"{case} graphs={graphs}: after t={fused.iteration}: bitwise equal {same}")
        assert same
    assert fused.sync_status() == 0 and over.sync_status() == 0
    for k in (1, 2, 3):
        a = fused.forces(k=k)
        b = over.forces(k=k)
        torch.cuda.synchronize()
        assert all(bool(torch.equal(x, y)) for x, y in zip(a, b)), k
    fused.close()
    over.close()


def test_overlap_with_node_weights_bitwise_equal_fused(T):
    import torch
    g = hub_graph(seed=5)
    pos = sg.uniform_positions(g.n, 32, -20, 20)
    rng = np.random.default_rng(33)
    rep_w = rng.uniform(0.5, 3.0, size=g.n).astype(np.float32)
    att_w = rng.uniform(0.2, 4.0, size=g.n).astype(np.float32)
    fused, over = pair(T, g, pos, n_int=48, total_iters=30, tau=0.6, rep_weight=1.3)
    for lay in (fused, over):
        lay.set_node_weights(rep_w, att_w)
        lay.step(30)
    torch.cuda.synchronize()
    assert bool(torch.equal(fused.pos, over.pos))
    fused.close()
    over.close()


@pytest.mark.parametrize("k", [1, 3])
def test_overlap_forces_match_oracle(T, k):
    import torch
    g = hub_graph(seed=6)
    pos = sg.uniform_positions(g.n, 34, -1, 1)
    n_int = 64
    lay = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), T.tfdp_params_default(n_int=n_int))
    lay.set_overlap(1)
    fr, fa, ft = (t.cpu().numpy().astype(np.float64) for t in lay.forces(k=k))
    x = pos.astype(np.float64)
    wr = ot.repulsion_ibfft_stable(x, 2.0, n_int, k)
    wa = ot.attraction(x, g.row_ptr, g.col_idx, 0.1, 8.0)
    errs = [rel_l2(fr, wr), rel_l2(fa, wa), rel_l2(ft, wr + wa)]
    # per-node bound as in the parity tests
    node = []
    for got, want, sc in ((fr, wr, np.linalg.norm(wr, axis=1)), (fa, wa, np.linalg.norm(wa, axis=1)),
                          (ft, wr + wa, np.linalg.norm(wr, axis=1) + np.linalg.norm(wa, axis=1))):
        den = sc + np.median(sc)
        node.append(float((np.linalg.norm(got - want, axis=1) / den).max()))
    say(f"overlapped k={k}: rel L2 rep/att/tot {errs}; per node {node}")
    assert max(errs) <= 1e-5
    assert max(node) <= 1e-4
    lay.close()


def test_set_overlap_arguments(T):
    import torch
    g = sg.sbm([300, 200], 0.05, 0.01, 7)
    lay = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(sg.uniform_positions(g.n, 35)).cuda(),
                   T.tfdp_params_default(n_int=32))
    for bad in (-2, 2):
        with pytest.raises(T.TfdpError):
            lay.set_overlap(bad)
    for mode in (-1, 0, 1, -1):
        lay.set_overlap(mode)
    lay.close()
