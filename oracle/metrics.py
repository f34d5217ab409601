"""Layout quality metrics of Sec. 4 ("Metrics"), FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see oracle/tfdp.py): used to compare final layouts
of the GPU library with those of the oracle.

* Normalised stress error SE over node pairs with finite graph distance,
  with the optimal uniform scale s of the layout (closed form below).
* Neighbourhood preservation NP_r: mean Jaccard similarity between the
  r-ring graph neighbourhood of a node and its k_i nearest neighbours in the
  layout, k_i = |N_G(i, r)|.
* Relative metric error (M(X_s) - M(X_t)) / M(X_t).

Readings: SE is averaged over the pairs with finite distance (the paper's
2/(n(n-1)) prefactor counts all pairs, which differs only for disconnected
graphs). In NP the layout neighbours exclude the node itself, distance ties
are broken towards the lower node index, and nodes with an empty graph
neighbourhood are skipped.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path


def _adjacency(n, row_ptr, col_idx):
    data = np.ones(len(col_idx))
    return csr_matrix((data, np.asarray(col_idx), np.asarray(row_ptr)), shape=(n, n))


def graph_distances(n, row_ptr, col_idx, sources=None):
    """Hop distances (inf when unreachable) from ``sources`` (all nodes by
    default), rows indexed like ``sources``."""
    a = _adjacency(n, row_ptr, col_idx)
    return shortest_path(a, method="D", unweighted=True, directed=False, indices=sources)


def optimal_scale(lay_d, graph_d):
    """Minimiser of sum (s D - d)^2 / d^2 over s: s = sum(D/d) / sum(D^2/d^2)."""
    r = lay_d / graph_d
    return float(r.sum() / (r * r).sum())


def stress_pairs(pos, row_ptr, col_idx, sources=None):
    """Layout distances d and hop distances D of the pairs that the stress
    error counts (Sec. 4, "Metrics"): all unordered pairs {i, j}, i != j,
    with finite D; with ``sources`` every ordered pair (s, v), s taken from
    ``sources`` (row q of the distance matrix belongs to sources[q]),
    v != s, with finite D (a sampled estimate: over all nodes as sources each
    unordered pair appears twice, which changes neither the optimal scale
    nor the mean)."""
    x = np.asarray(pos, dtype=np.float64)
    n = x.shape[0]
    src = np.arange(n) if sources is None else np.asarray(sources)
    d = graph_distances(n, row_ptr, col_idx, src)
    lay = np.sqrt(((x[src, None, :] - x[None, :, :]) ** 2).sum(-1))
    mask = np.isfinite(d) & (d > 0)
    if sources is None:
        mask &= np.arange(n)[None, :] > np.arange(n)[:, None]
    return lay[mask], d[mask]


def stress_error(pos, row_ptr, col_idx, sources=None):
    """Normalised stress error with the optimal scale, the mean of
    ((s d - D) / D)^2 over the pairs of ``stress_pairs``."""
    ll, dd = stress_pairs(pos, row_ptr, col_idx, sources)
    s = optimal_scale(ll, dd)
    return float((((s * ll - dd) / dd) ** 2).mean())


def ring_neighbours(n, row_ptr, col_idx, r):
    """N_G(i, r): nodes at hop distance 1..r from i, as sets."""
    rp = np.asarray(row_ptr)
    ci = np.asarray(col_idx)
    out = []
    for i in range(n):
        seen = {i}
        frontier = [i]
        for _ in range(r):
            nxt = []
            for u in frontier:
                for v in ci[rp[u]:rp[u + 1]]:
                    v = int(v)
                    if v not in seen:
                        seen.add(v)
                        nxt.append(v)
            frontier = nxt
        seen.discard(i)
        out.append(seen)
    return out


def sampled_rings(n, row_ptr, col_idx, r, nodes):
    """N_G(i, r) for the listed nodes only, from their hop distances (the
    same sets as ring_neighbours, without a search from every node)."""
    d = graph_distances(n, row_ptr, col_idx, list(nodes))
    return {int(i): set(int(v) for v in np.nonzero((d[q] >= 1) & (d[q] <= r))[0]) for q, i in enumerate(nodes)}


def neighborhood_preservation(pos, row_ptr, col_idx, r, nodes=None):
    """NP_r (Sec. 4, Metrics). Brute-force layout distances per node; with
    ``nodes`` the mean over those nodes (sampled estimate)."""
    x = np.asarray(pos, dtype=np.float64)
    n = x.shape[0]
    if nodes is None:
        rings = ring_neighbours(n, row_ptr, col_idx, r)
        sel = range(n)
    else:
        sel = [int(i) for i in nodes]
        rings = sampled_rings(n, row_ptr, col_idx, r, sel)
    vals = []
    idx = np.arange(n)
    for i in sel:
        ng = rings[i]
        ki = len(ng)
        if ki == 0:
            continue
        d2 = ((x - x[i]) ** 2).sum(axis=1)
        d2[i] = np.inf
        order = np.lexsort((idx, d2))   # distance, then lower index
        nl = set(int(v) for v in order[:ki])
        vals.append(len(ng & nl) / len(ng | nl))
    return float(np.mean(vals)) if vals else float("nan")


def relative_error(source_value, target_value):
    """(M(X_s) - M(X_t)) / M(X_t) (Sec. 4, Metrics)."""
    return (source_value - target_value) / target_value
