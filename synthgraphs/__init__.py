"""Seeded synthetic graphs and initial positions.

This module only produces inputs: undirected graphs stored as symmetric CSR
arrays and uniform random FP32 starting positions. It holds none of the layout
method's arithmetic, so the FP64 oracle and the GPU library can both be fed
from it without sharing any part of the computation.

The graph families stand in for the real-world graphs of the paper's
evaluation (Sec. 4, "Datasets"), which are not available here:

* stochastic block model  -> the clustered graphs (Sec. 4, synthetic graphs)
* rewired square lattice  -> mesh-like graphs
* Chung-Lu power law      -> large social networks (Sec. 4.2, runtime study)

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 20230307


@dataclass
class Graph:
    """Undirected simple graph as symmetric CSR (int32 indices)."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz], nnz = 2m, columns sorted within a row

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def edges(self) -> np.ndarray:
        """Undirected edge list (u < v), int64[m, 2]."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        cols = self.col_idx.astype(np.int64)
        keep = rows < cols
        return np.stack([rows[keep], cols[keep]], axis=1)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def csr_from_edges(n: int, edges: np.ndarray) -> Graph:
    """Symmetric CSR from an undirected edge list.

    Self-loops and duplicate edges (in either orientation) are dropped; each
    remaining edge {u, v} is stored as u->v and v->u. Columns are sorted
    within each row.
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("edge endpoint out of range")
    u = np.minimum(e[:, 0], e[:, 1])
    v = np.maximum(e[:, 0], e[:, 1])
    keep = u != v
    key = np.unique(u[keep] * n + v[keep])
    u = key // n
    v = key % n
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    order = np.argsort(rows * n + cols, kind="stable")
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32")
    return Graph(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=cols.astype(np.int32))


def uniform_positions(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """FP32 positions uniform in [lo, hi]^2, shape (n, 2), C-contiguous."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(lo, hi, size=(n, 2)).astype(np.float32))


def _sample_distinct_pairs(rng, count, n_a, n_b, same_block):
    """`count` distinct index pairs drawn uniformly from a block pair.

    For a diagonal block (same_block) the pairs are unordered (i < j) from
    n_a nodes; otherwise ordered (i in A, j in B).
    """
    if count == 0:
        return np.zeros((0, 2), dtype=np.int64)
    if same_block:
        total = n_a * (n_a - 1) // 2
        if count * 3 >= total:
            iu, ju = np.triu_indices(n_a, k=1)
            pick = rng.choice(total, size=count, replace=False)
            return np.stack([iu[pick], ju[pick]], axis=1).astype(np.int64)
        keys = np.zeros(0, dtype=np.int64)
        while keys.size < count:
            need = 2 * (count - keys.size) + 16
            i = rng.integers(0, n_a, size=need)
            j = rng.integers(0, n_a, size=need)
            ok = i < j
            keys = np.unique(np.concatenate([keys, i[ok] * n_a + j[ok]]))
        keys = rng.permutation(keys)[:count]
        return np.stack([keys // n_a, keys % n_a], axis=1)
    total = n_a * n_b
    if count * 3 >= total:
        flat = rng.choice(total, size=count, replace=False).astype(np.int64)
    else:
        flat = np.zeros(0, dtype=np.int64)
        while flat.size < count:
            draw = rng.integers(0, total, size=2 * (count - flat.size) + 16)
            flat = np.unique(np.concatenate([flat, draw]))
        flat = rng.permutation(flat)[:count]
    return np.stack([flat // n_b, flat % n_b], axis=1)


def sbm(block_sizes, p_in: float, p_out: float, seed: int) -> Graph:
    """Stochastic block model: every node pair is an edge independently with
    probability p_in (same block) or p_out (different blocks).

    Sampled per block pair as a binomial edge count followed by a uniform
    choice of that many distinct pairs, which has the same distribution as
    independent per-pair draws.
    """
    rng = np.random.default_rng(seed)
    sizes = [int(s) for s in block_sizes]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(offs[-1])
    parts = []
    for a in range(len(sizes)):
        for b in range(a, len(sizes)):
            same = a == b
            total = sizes[a] * (sizes[a] - 1) // 2 if same else sizes[a] * sizes[b]
            if total == 0:
                continue
            cnt = int(rng.binomial(total, p_in if same else p_out))
            pr = _sample_distinct_pairs(rng, cnt, sizes[a], sizes[b], same)
            pr[:, 0] += offs[a]
            pr[:, 1] += offs[b]
            parts.append(pr)
    edges = np.concatenate(parts) if parts else np.zeros((0, 2), dtype=np.int64)
    return csr_from_edges(n, edges)


def lattice_rewired(side: int, p_rewire: float, seed: int) -> Graph:
    """side x side 4-neighbour lattice; each edge (u, v) is, with probability
    p_rewire, replaced by (u, w) with w uniform, w != u and not already a
    neighbour of u (Watts-Strogatz style rewiring)."""
    rng = np.random.default_rng(seed)
    n = side * side
    idx = np.arange(n, dtype=np.int64).reshape(side, side)
    horiz = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1)
    vert = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], axis=1)
    edges = np.concatenate([horiz, vert])
    adj = [set() for _ in range(n)]
    for u, v in edges:
        adj[u].add(int(v))
        adj[v].add(int(u))
    flip = rng.random(edges.shape[0]) < p_rewire
    out = edges.copy()
    for e in np.nonzero(flip)[0]:
        u, v = int(edges[e, 0]), int(edges[e, 1])
        for _ in range(64):
            w = int(rng.integers(0, n))
            if w != u and w not in adj[u]:
                break
        else:
            continue
        adj[u].discard(v)
        adj[v].discard(u)
        adj[u].add(w)
        adj[w].add(u)
        out[e, 1] = w
    return csr_from_edges(n, out)


def chung_lu_weights(n: int, exponent: float, mean_degree: float) -> np.ndarray:
    """Expected degrees w_i = c (i + i0)^(-1/(exponent-1)), with c chosen so
    that mean(w) = mean_degree and i0 so that max(w) <= sqrt(sum(w))."""
    a = 1.0 / (exponent - 1.0)
    i = np.arange(n, dtype=np.float64)
    wmax_target = math.sqrt(mean_degree * n)

    def wmax(i0):
        base = (i + i0) ** (-a)
        c = mean_degree * n / base.sum()
        return c * i0 ** (-a)

    lo, hi = 1e-3, float(n)
    if wmax(lo) <= wmax_target:
        i0 = lo
    else:
        for _ in range(200):
            mid = math.sqrt(lo * hi)
            if wmax(mid) > wmax_target:
                lo = mid
            else:
                hi = mid
        i0 = hi
    base = (i + i0) ** (-a)
    return mean_degree * n / base.sum() * base


def chung_lu(n: int, exponent: float, mean_degree: float, seed: int) -> Graph:
    """Chung-Lu power-law graph: m = round(sum(w)/2) edges with both
    endpoints drawn i.i.d. proportional to w; self-loops and duplicates are
    dropped afterwards (so the realised mean degree is slightly below the
    target)."""
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, exponent, mean_degree)
    m = int(round(w.sum() / 2))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = np.searchsorted(cdf, rng.random(m), side="right")
    v = np.searchsorted(cdf, rng.random(m), side="right")
    u = np.minimum(u, n - 1)
    v = np.minimum(v, n - 1)
    return csr_from_edges(n, np.stack([u, v], axis=1))


# --------------------------------------------------------------------------
# Named workloads (sizes of the plain-layout study; seeds fixed)
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    graph: Graph
    pos0: np.ndarray  # float32[n, 2]
    n_int: int
    iters: int


def sbm_1k(seed: int = SEED_BASE + 1) -> Workload:
    """1,000-node SBM, 10 blocks of 100, p_in = 0.08, p_out = 0.002."""
    g = sbm([100] * 10, 0.08, 0.002, seed)
    return Workload("sbm_1k", g, uniform_positions(g.n, seed + 1000), 64, 300)


def mesh_100k(seed: int = SEED_BASE + 2) -> Workload:
    """316 x 316 lattice with 2% rewiring (99,856 nodes)."""
    g = lattice_rewired(316, 0.02, seed)
    return Workload("mesh_100k", g, uniform_positions(g.n, seed + 1000), 128, 500)


def chung_lu_1m(seed: int = SEED_BASE + 3, n: int = 1_000_000) -> Workload:
    """Chung-Lu, exponent 2.5, mean degree 10, one million nodes."""
    g = chung_lu(n, 2.5, 10.0, seed)
    return Workload("chung_lu_1m" if n == 1_000_000 else f"chung_lu_{n}", g,
                    uniform_positions(g.n, seed + 1000), 256, 500)


def sbm_batch_member(index: int, seed: int = SEED_BASE + 4):
    """One graph of the batched workload: n log-uniform in [200, 20000],
    B uniform in {2..20} equal blocks, mean degree 8 with 80% of the expected
    degree inside the block."""
    rng = np.random.default_rng([seed, index])
    n = int(round(math.exp(rng.uniform(math.log(200), math.log(20000)))))
    nb = int(rng.integers(2, 21))
    sizes = [n // nb + (1 if i < n % nb else 0) for i in range(nb)]
    bs = n / nb
    p_in = min(1.0, 0.8 * 8.0 / max(bs - 1.0, 1.0))
    p_out = min(1.0, 0.2 * 8.0 / max(n - bs, 1.0))
    g = sbm(sizes, p_in, p_out, int(rng.integers(0, 2**31 - 1)))
    return g, uniform_positions(g.n, int(rng.integers(0, 2**31 - 1)))


# --------------------------------------------------------------------------
# Request stream of the serving workload
# --------------------------------------------------------------------------

def serving_graph(index: int, seed: int = SEED_BASE + 5):
    """One graph of the serving workload: Chung-Lu with n log-uniform in
    [1000, 200000], exponent uniform in [2.0, 3.0], mean degree 10."""
    rng = np.random.default_rng([seed, index])
    n = int(round(math.exp(rng.uniform(math.log(1000), math.log(200000)))))
    expo = float(rng.uniform(2.0, 3.0))
    g = chung_lu(n, expo, 10.0, int(rng.integers(0, 2**31 - 1)))
    return g, uniform_positions(g.n, int(rng.integers(0, 2**31 - 1)))


@dataclass
class Request:
    """One request of a serving trace. kind "layout": lay out pool graph
    `graph` from its initial positions for `iters` iterations; kind
    "retune": `iters` more iterations of the graph of layout request
    `target` (resident, from its current positions) with the parameter
    values in `params`."""

    rid: int
    arrival: float  # seconds after the start of the trace
    kind: str
    graph: int = -1
    target: int = -1
    params: dict | None = None
    iters: int = 200


def serving_trace(count: int, rate: float, pool: int, seed: int = SEED_BASE + 6, retune_share: float = 0.3,
                  layout_iters: int = 200, retune_iters: int = 50):
    """Poisson arrivals at `rate` requests/s. A request is a re-tune with
    probability retune_share once a layout request exists; it targets a
    uniformly chosen earlier layout request and draws alpha in [0.01, 0.5],
    beta in [1, 50], gamma in [1.5, 8] and rep_weight in [0.5, 4] uniformly.
    Layout requests take pool graphs round robin from a random start."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    layouts = []
    g0 = int(rng.integers(0, pool))
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        if layouts and rng.random() < retune_share:
            params = {
                "alpha": float(rng.uniform(0.01, 0.5)),
                "beta": float(rng.uniform(1.0, 50.0)),
                "gamma": float(rng.uniform(1.5, 8.0)),
                "rep_weight": float(rng.uniform(0.5, 4.0)),
            }
            out.append(Request(rid, t, "retune", target=int(layouts[rng.integers(0, len(layouts))]),
                               params=params, iters=retune_iters))
        else:
            out.append(Request(rid, t, "layout", graph=(g0 + len(layouts)) % pool, iters=layout_iters))
            layouts.append(rid)
    return out
