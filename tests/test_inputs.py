"""The seeded input generators: structure and statistics of the workloads."""
import numpy as np

import synthgraphs as sg


def check_csr(g):
    rp, ci = g.row_ptr, g.col_idx
    assert rp.dtype == np.int32 and ci.dtype == np.int32
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == ci.size
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(rows != ci)                                  # no self-loops
    key = rows.astype(np.int64) * g.n + ci
    assert np.unique(key).size == key.size                      # no duplicates
    rev = ci.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(key), np.sort(rev))           # symmetric


def test_csr_from_edges_hygiene():
    g = sg.csr_from_edges(4, np.array([[0, 1], [1, 0], [2, 2], [3, 1], [0, 1]]))
    check_csr(g)
    assert g.m == 2 and list(g.row_ptr) == [0, 1, 3, 3, 4]


def test_sbm_1k():
    w = sg.sbm_1k()
    check_csr(w.graph)
    assert w.graph.n == 1000 and w.n_int == 64 and w.iters == 300
    # expected m = 10 * C(100,2) * 0.08 + C(10,2) * 100^2 * 0.002 = 3960 + 900 = 4860
    assert abs(w.graph.m - 4860) < 4 * np.sqrt(4860)
    e = w.graph.edges()
    intra = (e[:, 0] // 100 == e[:, 1] // 100).mean()
    assert abs(intra - 3960 / 4860) < 0.03
    assert w.pos0.dtype == np.float32 and w.pos0.min() >= -1 and w.pos0.max() <= 1
    w2 = sg.sbm_1k()
    assert np.array_equal(w.graph.col_idx, w2.graph.col_idx) and np.array_equal(w.pos0, w2.pos0)


def test_lattice_small():
    g = sg.lattice_rewired(20, 0.0, 1)
    check_csr(g)
    assert g.m == 2 * 20 * 19
    g2 = sg.lattice_rewired(20, 0.1, 1)
    check_csr(g2)
    assert g2.m == g.m and not np.array_equal(g.col_idx, g2.col_idx)


def test_chung_lu_small():
    g = sg.chung_lu(20000, 2.5, 10.0, 3)
    check_csr(g)
    w = sg.chung_lu_weights(20000, 2.5, 10.0)
    assert abs(w.mean() - 10) < 1e-9 and w.max() <= np.sqrt(w.sum()) * (1 + 1e-6)
    assert 8.5 < g.nnz / g.n < 10.0
    assert g.degrees()[:10].mean() > 20 * g.degrees().mean()


def test_batch_member():
    g, pos = sg.sbm_batch_member(3)
    check_csr(g)
    assert 200 <= g.n <= 20000 and pos.shape == (g.n, 2)
    assert 5.0 < g.nnz / g.n < 11.0
