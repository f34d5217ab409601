"""Grid choice for the interpolated repulsion (Sec. 3.4).

The cost of one iteration has a per-node part (spreading, gather, edges) and
a grid part that grows like (N_int k)^2 log(N_int k); the accuracy of the
interpolation is set by the interval width h = W / N_int (W = side of the
layout box) and by k: the relative L2 error of the repulsion behaves like
C_k h^k (k-point Lagrange interpolation per interval).

The tuner works in two stages, matching the k schedule of Sec. 3.4
(graphs of at most EXACT_MAX_N nodes use the exact method instead):

* start (k = 1 and 2, the first 95% of the iterations): N_int from the
  graph size, ``n_int_for_size``: N_int = 64 (n / 1000)^(1/5), a multiple
  of 8, which passes through the grids of the 10^3-node (64) and
  10^6-node (256) workloads; ``start_params`` rounds it down to a power of
  two when it exceeds one by at most 25% (half the FFT length, a quarter of
  the grid work);
* final (k = 3, the last 5%): at the switch, the box side W of the current
  layout fixes N_int = ceil(margin W / h_k(tol)) with h_k(tol) =
  (tol / C_k)^(1/k) and margin 1.4 for the growth of the box over the last
  iterations, so that the repulsion of the last iterations is within ``tol``
  of the exact sums (k = 2 keeps the starting grid: 1e-3 at k = 2 would need
  h ~ 0.1); C_3 grows with the kernel's narrowing for other gamma and tau
  (``kernel_scale``). Where the exact method costs less than that grid, or
  the grid would exceed the largest one the workspace holds (a layout wider
  than about 87 / sqrt(kernel_scale) length units cannot meet 1e-3 on an
  FFT of at most 2048 points per side), the last stage switches to the exact
  method instead (``final_choice``). ``retune`` applies a grid with
  tfdp_layout_set_params (the workspace is sized for the cap at creation,
  ``workspace_grid``).

C_k comes from ``calibrate``: exact (k = 0) against interpolated forces of
the library on laid-out graphs at several N_int, fitted in log space.
``DEFAULT_C`` holds fits for gamma = 2 (calibrate() on MI355X agrees within
a factor of three; the GPU tests check that).
"""
from __future__ import annotations

import math

import numpy as np

# C_k of err ~ C_k h^k for gamma = 2 (relative L2 of the repulsion): fits to
# the errors of the interpolated against the exact sums on four SBM layouts
# of 357..2047 nodes after 300 iterations, N_int 8..128 (calibrate() measures
# the same on the device)
DEFAULT_C = {1: 2.0, 2: 0.095, 3: 0.022}
MAX_N_INT_K3 = 341  # N_int * 3 * 2 <= 2048 (largest FFT length)


def n_int_for_size(n: int) -> int:
    v = 64.0 * (max(n, 1) / 1000.0) ** 0.2
    return int(min(1024, max(8, 8 * math.ceil(v / 8.0))))


EXACT_MAX_N = 1024  # at most this many nodes: the exact O(n^2) method


def fft_rounded(n_int: int, slack: float = 1.25) -> int:
    """The FFT length per side is the smallest 2^a (or 3 * 2^a for 384, 768,
    1536) >= 2 N_int k: a grid just above a power of two takes a longer FFT
    in every pass. Round N_int down to that power of two when it exceeds it
    by at most `slack`."""
    p = 1 << max(0, (n_int - 1).bit_length() - 1)  # largest power of two < n_int
    return p if p >= 8 and n_int <= slack * p else n_int


def start_params(n: int):
    """(k_mode, N_int) for the start of a layout of n nodes: the exact method
    up to EXACT_MAX_N nodes (cheaper than a grid there, and exact), else the
    k schedule on the size-rule grid rounded down to an FFT-friendly size."""
    if n <= EXACT_MAX_N:
        return 0, 8
    return -1, fft_rounded(n_int_for_size(n))


def kernel_scale(gamma: float = 2.0, tau: float = 1.0, k: int = 3) -> float:
    """Factor of C_k for other t-force parameters: the kernel
    (1 + tau d^2)^-gamma narrows as gamma and tau grow, and the k = 3 error
    at a given h grows with it. Fit on FP64 oracle errors (a 475-node SBM
    layout, N_int 16..64): C_3 relative to gamma = 2 was 0.21, 9.1 and 31 at
    gamma = 1.5, 4 and 8; (gamma / 2)^3 bounds all three (0.42, 8, 64 --
    at gamma = 4 the margin of final_n_int covers the rest). tau rescales
    lengths by sqrt(tau): tau^(k/2)."""
    return (gamma / 2.0) ** k * tau ** (k / 2.0)


def interval_width(tol: float, k: int, consts=None, gamma: float = 2.0, tau: float = 1.0) -> float:
    c = (consts or DEFAULT_C)[k] * kernel_scale(gamma, tau, k)
    return (tol / c) ** (1.0 / k)


def final_n_int(width: float, tol: float = 1e-3, k: int = 3, consts=None, margin: float = 1.4,
                lo: int = 8, hi: int = MAX_N_INT_K3, gamma: float = 2.0, tau: float = 1.0) -> int:
    """Intervals per side for a box of side `width` so that k-point
    interpolation stays within `tol` (relative L2 of the repulsion), clamped
    to [lo, hi]."""
    v = math.ceil(margin * width / interval_width(tol, k, consts, gamma, tau))
    return int(min(hi, max(lo, v)))


def workspace_grid(n: int, cap: int = MAX_N_INT_K3) -> int:
    """Largest N_int a graph's workspace is sized for: the final grid of a
    box whose side is 3 sqrt(n) (final boxes of SBM layouts with the default
    parameters measured 0.8..1.6 sqrt(n)), capped."""
    return final_n_int(3.0 * math.sqrt(max(n, 1)), hi=cap, lo=n_int_for_size(n))


def box_side(pos) -> float:
    """Side of the square layout box (max of the x and y ranges) from the
    positions (torch tensor or array, [n, 2])."""
    p = pos.detach().float().cpu().numpy() if hasattr(pos, "detach") else np.asarray(pos, dtype=np.float32)
    p = p[np.all(np.isfinite(p), axis=1)]
    if p.size == 0:
        return 1.0
    ext = p.max(axis=0) - p.min(axis=0)
    return float(max(ext.max(), 1e-6))


def box_sides(positions) -> np.ndarray:
    """box_side of each of a list of [n_i, 2] float32 tensors (every n_i at
    least 1), reduced where the tensors live (one pass on the device, then a
    copy of two extremes per tensor): the same float32 extremes, so the same
    widths as box_side on each tensor."""
    import torch
    if not positions:
        return np.zeros(0)
    dev = positions[0].device
    counts = torch.tensor([int(p.shape[0]) for p in positions], device=dev)
    if int(counts.min()) < 1:
        raise ValueError("every layout needs at least one row")
    pos = torch.cat([p.float() for p in positions])
    seg = torch.repeat_interleave(torch.arange(len(positions), device=dev), counts)[:, None].expand(-1, 2)
    fin = torch.isfinite(pos).all(dim=1, keepdim=True)  # rows with a non-finite coordinate are left out
    inf = torch.tensor(float("inf"), device=dev)
    lo = torch.full((len(positions), 2), float("inf"), device=dev).scatter_reduce(
        0, seg, torch.where(fin, pos, inf), "amin")
    hi = torch.full((len(positions), 2), -float("inf"), device=dev).scatter_reduce(
        0, seg, torch.where(fin, pos, -inf), "amax")
    ext = (hi - lo).amax(dim=1).cpu().numpy().astype(np.float64)  # -inf: no finite row
    return np.where(np.isfinite(ext), np.maximum(ext, 1e-6), 1.0)


def retune(lay, tol: float = 1e-3, consts=None, k: int = 3, cap: int | None = None) -> int:
    """Set the final-stage grid of a Layout from its current box; returns
    the new N_int (never below the current one; at most `cap`)."""
    from . import tfdp as T
    cur = lay.params.n_int
    hi = cap if cap is not None else MAX_N_INT_K3
    new = max(cur, final_n_int(box_side(lay.pos), tol, k, consts, hi=hi, gamma=lay.params.gamma,
                               tau=lay.params.tau))
    if new != cur:
        p = T.TfdpParams(**{**lay.params.as_dict(), "n_int": new})
        lay.set_params(p)
    return new


# Exact against interpolated cost per iteration, measured on MI355X in
# batches: n^2 pair terms of the exact method cost about as much as 12^2 L^2
# grid points of the k = 3 passes (L = FFT length per side)
EXACT_PER_FFT_LENGTH = 12


def fft_length(n_int: int, k: int) -> int:
    """FFT length per side the library uses for N_int and k: the smallest
    power of two >= max(64, 2 N_int k), or three quarters of it when that is
    still >= 2 N_int k and one of the radix-3 lengths 384, 768, 1536."""
    m2 = 2 * n_int * k
    L = 64
    while L < m2:
        L *= 2
    l3 = 3 * L // 4
    return l3 if l3 >= m2 and l3 in (384, 768, 1536) else L


def final_choice(n: int, width: float, tol: float = 1e-3, consts=None, gamma: float = 2.0, tau: float = 1.0,
                 cap: int = MAX_N_INT_K3):
    """(k_mode, N_int) for the k = 3 stage: the grid that meets `tol`, or the
    exact method when that is cheaper than the grid or when the grid that
    meets `tol` is larger than `cap` (the largest grid of the workspace)."""
    ni = final_n_int(width, tol, 3, consts, hi=10 ** 9, gamma=gamma, tau=tau)
    if ni > cap:
        return 0, None
    if n <= EXACT_PER_FFT_LENGTH * fft_length(ni, 3):
        return 0, None
    return -1, ni


def retune_many(layouts, tol: float = 1e-3, consts=None, allow_exact: bool = True, caps=None):
    """The k = 3 stage choice for many Layouts (their boxes from one device
    reduction): the exact method where it is cheaper or where the grid
    that meets `tol` exceeds the layout's cap (caps[i], default
    MAX_N_INT_K3), else the grid from each box. Exact-method layouts keep
    their parameters. Returns the N_int of each layout (0 for the exact
    method)."""
    from . import tfdp as T
    # every box in one reduction on the device (a copy of all positions and
    # a loop of box_side over 512 layouts took 130-170 ms of host time inside
    # a timed batched run)
    widths = box_sides([lay.pos for lay in layouts])
    out = []
    for q, lay in enumerate(layouts):
        w = float(widths[q])
        cur = lay.params
        if cur.k_mode == 0:
            out.append(0)
            continue
        cap = caps[q] if caps is not None else MAX_N_INT_K3
        k_mode, ni = final_choice(lay.n, w, tol, consts, cur.gamma, cur.tau, cap)
        if k_mode == 0 and allow_exact:
            lay.set_params(T.TfdpParams(**{**cur.as_dict(), "k_mode": 0}))
            out.append(0)
            continue
        ni = max(cur.n_int, ni if ni is not None else final_n_int(w, tol, 3, consts, hi=cap, gamma=cur.gamma,
                                                                    tau=cur.tau))
        if ni != cur.n_int:
            lay.set_params(T.TfdpParams(**{**cur.as_dict(), "n_int": ni}))
        out.append(ni)
    return out


def calibrate(T, layouts, n_ints=(16, 24, 32, 48, 64, 96), ks=(1, 2, 3)):
    """Fit C_k from the library's own forces: for each Layout (positions of
    a laid-out graph; workspace large enough for max(n_ints)), the relative
    L2 error of the k-point repulsion against the exact sums at every N_int,
    then log err = log C_k + k log h by least squares on log C_k.
    Returns ({k: C_k}, samples). Restores each layout's parameters."""
    import torch
    samples = {k: [] for k in ks}
    for lay in layouts:
        keep = lay.params
        exact, _, _ = lay.forces(k=0)
        torch.cuda.synchronize()
        ex = exact.double()
        norm = torch.linalg.norm(ex).item()
        w = box_side(lay.pos)
        for ni in n_ints:
            for k in ks:
                if ni * k > 1024:
                    continue
                p = T.TfdpParams(**{**keep.as_dict(), "n_int": ni, "k_mode": k})
                lay.set_params(p)
                fr, _, _ = lay.forces(k=k)
                torch.cuda.synchronize()
                err = torch.linalg.norm(fr.double() - ex).item() / max(norm, 1e-300)
                samples[k].append((w / ni, err))
        lay.set_params(keep)
    consts = {}
    for k in ks:
        h = np.array([s[0] for s in samples[k]])
        e = np.array([s[1] for s in samples[k]])
        ok = (e > 0) & np.isfinite(e)
        consts[k] = float(np.exp(np.mean(np.log(e[ok]) - k * np.log(h[ok])))) if ok.any() else DEFAULT_C[k]
    return consts, samples


TILE_CANDIDATES = [(r, g) for r in (2, 4, 8) for g in (1, 2)]
TUNABLE_LENGTHS = (64, 128, 256, 384, 512, 768)


def k_of(params, t: int) -> int:
    """k of iteration t (the schedule of Sec. 3.4 for k_mode -1)."""
    if params.k_mode >= 0:
        return params.k_mode
    T = params.total_iters
    return 1 if t < (9 * T) // 10 else 2 if t < (19 * T) // 20 else 3


def batch_lengths(layouts, at_iteration=None):
    """Tunable FFT lengths the members use at their current counters (or at
    counter `at_iteration`)."""
    out = set()
    for lay in layouts:
        k = k_of(lay.params, lay.iteration if at_iteration is None else at_iteration)
        if k > 0 and fft_length(lay.params.n_int, k) in TUNABLE_LENGTHS:
            out.add(fft_length(lay.params.n_int, k))
    return out


def tune_batch_tiles(batch, layouts, iters: int = 4, repeats: int = 2, lengths=None, at_iteration=None,
                     stream=None):
    """Tile schedule of a batch's grid passes, chosen by measurement: for
    every tunable FFT length the members use (at their current counters, or
    with every counter set to `at_iteration` during the trials), time `iters`
    batched iterations with each candidate tile (rows per block of the row
    passes, column groups of the column pass; the best of `repeats` runs
    after a first one that builds the maps) and keep the fastest. Tiles do
    not change results, and every member's positions and counter are restored
    afterwards. Returns {length: (rows, groups, ms)}."""
    import time
    import torch
    if lengths is None:
        lengths = batch_lengths(layouts, at_iteration)
    saved = [(lay.pos.clone(), lay.iteration) for lay in layouts]

    def restore(trial=True):
        for lay, (p, t) in zip(layouts, saved):
            lay.pos.copy_(p)
            lay.iteration = at_iteration if (trial and at_iteration is not None) else t
        torch.cuda.synchronize()

    chosen = {}
    for L in sorted(lengths):
        best = None
        for rows, groups in TILE_CANDIDATES:
            batch.set_tiles(L, rows, groups, stream)
            times = []
            for rep in range(repeats + 1):
                restore()
                t0 = time.perf_counter()
                batch.step(iters, stream)
                torch.cuda.synchronize()
                if rep > 0:  # the first run builds the maps and launches directly
                    times.append(time.perf_counter() - t0)
            ms = 1e3 * min(times)
            if best is None or ms < best[2]:
                best = (rows, groups, ms)
        batch.set_tiles(L, best[0], best[1], stream)
        chosen[L] = best
    restore(trial=False)
    return chosen
