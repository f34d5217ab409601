"""Grid choice for the interpolated repulsion (Sec. 3.4).

The cost of one iteration is a per-node part (spreading, gather, edges) and
a grid part that grows like (N_int k)^2 log(N_int k); the accuracy of the
interpolation is set by the interval width h = W / N_int (W = side of the
layout box) and by k.

``n_int_for_size`` is the starting grid of a graph of n nodes: it follows
the grids used for 10^3 (64), 10^5 (128) and 10^6 (256) nodes, i.e.
N_int = 64 (n / 1000)^(1/5), rounded up to a multiple of 8.
"""
from __future__ import annotations

import math


def n_int_for_size(n: int) -> int:
    v = 64.0 * (max(n, 1) / 1000.0) ** 0.2
    return int(min(1024, max(8, 8 * math.ceil(v / 8.0))))
