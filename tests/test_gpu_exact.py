"""The pair-symmetric exact method (each unordered pair once, the row and
the column sums in 64-bit fixed point) against the FP64 oracle's all-pairs
sums (Sec. 3.4, exact method; Eq.5, 11): relative L2 <= 1e-5 and the
per-node bound of the parity tests, at sizes with one to dozens of tiles and
ragged last tiles, for gamma = 2 (hardware reciprocal) and other gamma and
tau. Integer accumulation makes the result independent of the block order,
so repeated evaluations and repeated layouts are bit-identical; batched
exact members reproduce plain ones bit for bit."""
import sys

import numpy as np
import pytest

import synthgraphs as sg
from oracle import tfdp as ot
from tests._lib import ensure_built, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5
NODE_TOL = 1e-4


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


def forces(T, g, pos, **params):
    import torch
    lay = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), T.tfdp_params_default(n_int=16, **params))
    out = [t.cpu().numpy().astype(np.float64) for t in lay.forces(k=0)]
    again = [t.cpu().numpy().astype(np.float64) for t in lay.forces(k=0)]
    torch.cuda.synchronize()
    lay.close()
    # the accumulators are cleared by every evaluation: a second one is equal
    assert all(np.array_equal(a, b) for a, b in zip(out, again))
    return out


def node_error(got, want):
    s = np.linalg.norm(want, axis=1)
    den = s + np.median(s)
    dn = np.linalg.norm(got - want, axis=1)
    # a graph whose exact forces all vanish (one node) compares absolutely
    return float(np.where(den > 0, dn / np.where(den > 0, den, 1.0), dn).max())


def compare(T, g, pos, gamma=2.0, tau=1.0, alpha=0.1, beta=8.0):
    say(f"case n={g.n} gamma={gamma} tau={tau}")
    got = forces(T, g, pos, gamma=gamma, tau=tau, alpha=alpha, beta=beta)
    x = pos.astype(np.float64)
    wr = ot.repulsion_exact(x, gamma, tau=tau)
    wa = ot.attraction(x, g.row_ptr, g.col_idx, alpha, beta, tau=tau)
    err = [rel_l2(got[0], wr), rel_l2(got[1], wa), rel_l2(got[2], wr + wa)]
    node = node_error(got[0], wr)
    say(f"  rel L2 rep/att/tot {err}; per node (repulsion) {node}")
    assert max(err) <= TOL
    assert node <= NODE_TOL


@pytest.mark.parametrize("n", [4096, 5000, 9001])
def test_symmetric_exact_matches_oracle(T, n):
    # 16, 20 and 36 tiles of 256 nodes; the last two with ragged last tiles
    g = sg.chung_lu(n, 2.5, 8.0, 40 + n % 97)
    pos = sg.uniform_positions(n, 41, -30.0, 30.0)
    compare(T, g, pos)


@pytest.mark.parametrize("n", [20000, 70001])
def test_large_graphs_sampled_rows(T, n):
    # 3,160 and 37,401 tile pairs: every node's repulsion against the
    # one-launch kernel, and sampled rows (with the first and the last node)
    # against the FP64 oracle
    import torch
    g = sg.chung_lu(n, 2.5, 8.0, 53)
    pos = sg.uniform_positions(n, 54, -60.0, 60.0)
    got = forces(T, g, pos)
    rows = np.random.default_rng(55).choice(n, size=1500, replace=False)
    rows = np.sort(np.concatenate([rows, [0, n - 1]]))
    want = ot.repulsion_exact(pos.astype(np.float64), 2.0, rows=rows, block=256)
    err = rel_l2(got[0][rows], want)
    node = node_error(got[0][rows], want)
    say(f"n={n}: sampled rows rel L2 {err:.2e}, per node {node:.2e}")
    assert err <= TOL and node <= NODE_TOL
    import os
    old = os.environ.get("TFDP_SYM_MIN_NODES")
    os.environ["TFDP_SYM_MIN_NODES"] = "2000000000"
    try:
        one = forces(T, g, pos)
    finally:
        if old is None:
            del os.environ["TFDP_SYM_MIN_NODES"]
        else:
            os.environ["TFDP_SYM_MIN_NODES"] = old
    d = rel_l2(got[0], one[0])
    say(f"  against the one-launch kernel: rel L2 {d:.2e}")
    assert d <= TOL
    torch.cuda.synchronize()


@pytest.mark.parametrize("gamma,tau", [(1.5, 1.0), (3.0, 0.5), (2.0, 0.25)])
def test_symmetric_exact_other_gamma_tau(T, gamma, tau):
    g = sg.sbm([2500, 2300], 0.004, 0.0005, 43)
    pos = sg.uniform_positions(g.n, 44, -20.0, 20.0)
    compare(T, g, pos, gamma=gamma, tau=tau)


@pytest.mark.parametrize("n", [1, 2, 255, 257, 1000])
def test_symmetric_exact_small_graphs_forced(T, n, monkeypatch):
    # the pair-symmetric kernels on graphs below their default size: one
    # node, one pair, a single ragged tile, a tile and one node
    monkeypatch.setenv("TFDP_SYM_MIN_NODES", "1")
    if n >= 3:
        g = sg.sbm([n // 2, n - n // 2], 0.05, 0.01, 45)
    else:
        g = sg.csr_from_edges(n, np.array([[0, 1]] if n == 2 else [], dtype=np.int64).reshape(-1, 2))
    pos = sg.uniform_positions(n, 46, -5.0, 5.0)
    compare(T, g, pos)


def test_coincident_and_far_apart_nodes(T):
    # many nodes on a few points (zero terms within a point) and one node far
    # away (terms near the underflow of (1 + d^2)^-2 d)
    rng = np.random.default_rng(47)
    n = 4500
    pos = rng.integers(0, 4, size=(n, 2)).astype(np.float32)
    pos[-1] = (3.0e4, -2.0e4)
    g = sg.chung_lu(n, 2.5, 6.0, 48)
    compare(T, g, pos)


def test_symmetric_layout_is_deterministic_and_near_one_launch_kernel(T, monkeypatch):
    """Steps of the exact method: two runs of 20 iterations are bit-identical
    (integer sums); one step of the one-launch kernel (other summation
    order) is within float rounding of one symmetric step."""
    import torch
    g = sg.chung_lu(6000, 2.5, 8.0, 49)
    pos = sg.uniform_positions(g.n, 50, -20.0, 20.0)
    p = T.tfdp_params_default(n_int=16, k_mode=0, total_iters=20)
    runs = []
    for env, iters in (("", 20), ("", 20), ("", 1), ("1000000000", 1)):
        if env:
            monkeypatch.setenv("TFDP_SYM_MIN_NODES", env)
        lay = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), p)
        lay.step(iters)
        torch.cuda.synchronize()
        assert lay.sync_status() == 0
        runs.append(lay.pos.cpu().numpy().astype(np.float64))
        lay.close()
    assert np.array_equal(runs[0], runs[1])
    d = rel_l2(runs[2] - pos, runs[3] - pos)
    say(f"one step, symmetric vs one-launch kernel: relative difference of the moves {d:.2e}")
    assert d <= 1e-5


def test_symmetric_single_step_matches_oracle(T):
    import torch
    g = sg.chung_lu(5000, 2.5, 8.0, 51)
    pos = sg.uniform_positions(g.n, 52, -10.0, 10.0)
    t = 3
    p = T.tfdp_params_default(n_int=16, k_mode=0, total_iters=20)
    lay = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), p)
    lay.iteration = t
    lay.step(1)
    torch.cuda.synchronize()
    got = lay.pos.cpu().numpy().astype(np.float64)
    op = ot.Params(n_int=16, k_mode=0, total_iters=20)
    x = pos.astype(np.float64)
    _, _, disp = ot.forces(x, g.row_ptr, g.col_idx, op, 0)
    want = ot.capped_move(x, disp, ot.step_cap(t, 20, ot.default_t0(g.n)))
    err = rel_l2(got - x, want - x)
    say(f"one exact step at n={g.n}: relative error of the move {err:.2e}")
    assert err <= 1e-5
    lay.close()
