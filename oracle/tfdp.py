"""FP64 CPU oracle of the t-FDP force evaluation and layout step.

TEST INFRASTRUCTURE ONLY. This module is the slow, plain reference that the
GPU library is checked against. Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library never does. It
shares no code with the GPU path: the only common input is the seeded graph
and position generator module, which holds none of the arithmetic below.

Everything is float64 NumPy. Each function names the passage of the paper it
follows: "Force-directed graph layouts revisited: a new force based on the
t-Distribution" (Zhong et al., arXiv 2303.03964).

Readings of points the paper leaves open (each one is also listed in the
design notes of the repository):

* Sign convention. Eq.5-7 give the repulsive force with a minus sign and the
  attraction with a plus sign along x_i - x_j, i.e. the gradient of an
  energy; Eq.11 writes the repulsion with a plus sign. The displacement used
  here moves a node away from every other node and towards its neighbours:
      D_i = w_r * sum_j K_ij (x_i - x_j)
            - alpha * sum_{j in N(i)} (1 + beta / (1 + |x_i - x_j|^2)) (x_i - x_j)
  with K_ij = (1 + |x_i - x_j|^2)^(-gamma) (Eq.11-12). w_r (default 1) is
  the repulsion multiplier of global refinement (Sec. 5); with w_r = 1 this
  is exactly Eq.7 taken as a motion.
* Update rule. The paper only says that the resultant force moves the node
  until convergence (Sec. 3.1). Used here: a synchronous capped step with
  linear cooling, x_i <- x_i + D_i * min(1, T_t / |D_i|), T_t = T0 (1 - t/T),
  T0 = max(1, sqrt(n)/10) unless given.
* k schedule (Sec. 3.4, "Choices of k"): k = 1 for t < floor(0.9 T),
  k = 2 for t < floor(0.95 T), k = 3 afterwards.
* Box (Sec. 3.4, the garbled [x_min, x_max] x [x_min, x_max]): a square of
  side W = max(x range, y range) centred on the per-axis mid-range; W = 1 if
  all points coincide. Binning in float64 with this exact operation order:
  h = W / N_int, r = (x - lo) / h, c = min(max(floor(r), 0), N_int - 1),
  t = r - c.
* Interpolation nodes: k equispaced nodes per interval at (j + 1/2)/k of the
  interval (j = 0..k-1), so all intervals together form one uniform grid of
  M = N_int * k nodes per side with spacing s = h / k; grid node g sits at
  lo + (g + 1/2) s. Lagrange interpolation uses only the k nodes of the
  point's own interval, per axis, as a tensor product.
* Kernel in layout units at the grid spacing: K(a, b) = (1 + s^2 (a^2 + b^2))^-gamma
  for integer node offsets (a, b).
* Self term: the sums of Eq.11 run over all j including i; the self
  contribution is (x_i - x_i) K_ii = 0 in the exact sums and cancels in the
  interpolated ones, so it is not special-cased.
"""
from __future__ import annotations

import math

import numpy as np

# Defaults of Sec. 3.3 ("Parameter Analysis"): alpha = 0.1, beta = 8, gamma = 2.
DEFAULT_ALPHA = 0.1
DEFAULT_BETA = 8.0
DEFAULT_GAMMA = 2.0


# ---------------------------------------------------------------------------
# Pair forces (Sec. 3.2 and 3.3)
# ---------------------------------------------------------------------------

def t_force_general(d, tau, phi_t):
    """Generalised t-force, Eq.3: 2 tau phi d / (1 + tau d^2)^(phi + 1)."""
    d = np.asarray(d, dtype=np.float64)
    return 2.0 * tau * phi_t * d / (1.0 + tau * d * d) ** (phi_t + 1.0)


def t_force(d, phi):
    """t-force, Eq.4 (tau = 1): d / (1 + d^2)^phi."""
    d = np.asarray(d, dtype=np.float64)
    return d / (1.0 + d * d) ** phi


def repulsive_magnitude(d, gamma):
    """Magnitude of the pairwise repulsive t-force, Eq.5."""
    return t_force(d, gamma)


def attractive_magnitude(d, beta):
    """Magnitude of the pairwise attraction, Eq.6: a linear spring plus the
    attractive t-force with exponent 1 weighted by beta."""
    d = np.asarray(d, dtype=np.float64)
    return d + beta * t_force(d, 1.0)


def kernel(d2, gamma, tau=1.0):
    """The kernel of Eq.12 as a function of the squared distance; with tau
    the generalised t-force of Eq.3 (the paper's model has tau = 1):
    (1 + tau d^2)^-gamma."""
    return (1.0 + tau * np.asarray(d2, dtype=np.float64)) ** (-gamma)


# ---------------------------------------------------------------------------
# Exact sums
# ---------------------------------------------------------------------------

def repulsion_exact(pos, gamma, rows=None, block=2048, tau=1.0):
    """Exact all-pairs repulsion, Eq.11: F_i = sum_j K_ij (x_i - x_j).

    ``rows`` selects the nodes i to evaluate (all by default); every j is
    summed. O(n * len(rows)) work, processed in blocks of rows.
    """
    x = np.asarray(pos, dtype=np.float64)
    idx = np.arange(x.shape[0]) if rows is None else np.asarray(rows)
    out = np.zeros((idx.size, 2))
    for b0 in range(0, idx.size, block):
        sel = idx[b0:b0 + block]
        diff = x[sel, None, :] - x[None, :, :]
        d2 = diff[..., 0] ** 2 + diff[..., 1] ** 2
        k = kernel(d2, gamma, tau)
        out[b0:b0 + block, 0] = (k * diff[..., 0]).sum(axis=1)
        out[b0:b0 + block, 1] = (k * diff[..., 1]).sum(axis=1)
    return out


def attraction(pos, row_ptr, col_idx, alpha, beta, rows=None, tau=1.0, weights=None):
    """Attraction along edges (Eq.6, weighted by alpha as in Eq.7), as a
    motion towards the neighbours:
        F^a_i = -alpha * sum_{j in N(i)} (1 + beta / (1 + d_ij^2)) (x_i - x_j).
    (|Delta| + beta |Delta| / (1 + |Delta|^2)) * Delta / |Delta| simplifies to
    the factor above, so no square root is needed.) With tau the attractive
    t-force is the generalised one of Eq.3 (1 + tau d^2 in the denominator);
    with per-node ``weights`` a (local refinement, Sec. 5) the term of edge
    (i, j) is scaled by (a_i + a_j) / 2, the same for both ends.
    """
    x = np.asarray(pos, dtype=np.float64)
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    n = x.shape[0]
    idx = np.arange(n) if rows is None else np.asarray(rows)
    out = np.zeros((idx.size, 2))
    if rows is None:
        src = np.repeat(np.arange(n), np.diff(rp))
        diff = x[src] - x[ci]
        d2 = diff[:, 0] ** 2 + diff[:, 1] ** 2
        fac = 1.0 + beta / (1.0 + tau * d2)
        if weights is not None:
            a = np.asarray(weights, dtype=np.float64)
            fac = fac * 0.5 * (a[src] + a[ci])
        f = fac[:, None] * diff
        out[:, 0] = np.bincount(src, weights=f[:, 0], minlength=n)
        out[:, 1] = np.bincount(src, weights=f[:, 1], minlength=n)
    else:
        for o, i in enumerate(idx):
            nb = ci[rp[i]:rp[i + 1]]
            diff = x[i] - x[nb]
            d2 = diff[:, 0] ** 2 + diff[:, 1] ** 2
            fac = 1.0 + beta / (1.0 + tau * d2)
            if weights is not None:
                a = np.asarray(weights, dtype=np.float64)
                fac = fac * 0.5 * (a[i] + a[nb])
            out[o] = (fac[:, None] * diff).sum(axis=0)
    return -alpha * out


# ---------------------------------------------------------------------------
# Interpolation-based FFT (Sec. 3.4, Eq.11-15)
# ---------------------------------------------------------------------------

def square_box(pos):
    """Square box around the points: (lo_x, lo_y, W). See module notes."""
    x = np.asarray(pos, dtype=np.float64)
    xmin, ymin = x.min(axis=0)
    xmax, ymax = x.max(axis=0)
    w = max(xmax - xmin, ymax - ymin)
    if not w > 0.0:
        w = 1.0
    cx = (xmin + xmax) / 2.0
    cy = (ymin + ymax) / 2.0
    return (cx - w / 2.0, cy - w / 2.0, w)


def bin_points(pos, box, n_int):
    """Interval index c (int64[n, 2]) and in-interval coordinate t in [0, 1]
    (float64[n, 2]) of every point, per axis, for N_int intervals per side."""
    x = np.asarray(pos, dtype=np.float64)
    lo = np.array([box[0], box[1]], dtype=np.float64)
    h = box[2] / n_int
    r = (x - lo) / h
    c = np.minimum(np.maximum(np.floor(r), 0.0), n_int - 1.0)
    t = r - c
    return c.astype(np.int64), t, h


def node_offsets(k):
    """In-interval coordinates tau_j = (j + 1/2) / k of the k nodes."""
    return (np.arange(k, dtype=np.float64) + 0.5) / k


def lagrange_weights(t, k):
    """Lagrange basis L_j(t) = prod_{m != j} (t - tau_m) / (tau_j - tau_m)
    over the k nodes of one interval; t has any shape, result t.shape + (k,)."""
    t = np.asarray(t, dtype=np.float64)
    tau = node_offsets(k)
    out = np.ones(t.shape + (k,))
    for j in range(k):
        for m in range(k):
            if m != j:
                out[..., j] *= (t - tau[m]) / (tau[j] - tau[m])
    return out


class Interp:
    """Per-point interpolation data for one (box, N_int, k): interval index,
    per-axis Lagrange weights and per-axis offsets delta = x - y_g from each
    of the point's k grid nodes (Sec. 3.4, piecewise interpolation)."""

    def __init__(self, pos, n_int, k, box=None):
        self.pos = np.asarray(pos, dtype=np.float64)
        self.box = square_box(self.pos) if box is None else tuple(float(v) for v in box)
        self.n_int = int(n_int)
        self.k = int(k)
        self.m = self.n_int * self.k
        self.c, self.t, self.h = bin_points(self.pos, self.box, self.n_int)
        self.s = self.h / self.k
        self.w = lagrange_weights(self.t, self.k)            # [n, 2, k]
        tau = node_offsets(self.k)
        self.delta = (self.t[:, :, None] - tau[None, None, :]) * self.h  # [n, 2, k]
        self.g = self.c[:, :, None] * self.k + np.arange(self.k)[None, None, :]  # [n, 2, k]

    def taps(self):
        """Iterate over the k x k taps: (gx, gy, weight, dx, dy), each [n]."""
        for a in range(self.k):
            for b in range(self.k):
                yield (self.g[:, 0, a], self.g[:, 1, b],
                       self.w[:, 0, a] * self.w[:, 1, b],
                       self.delta[:, 0, a], self.delta[:, 1, b])

    def spread(self, values):
        """Projection onto the grid: q(g) = sum_i w_ig v_i (Sec. 3.4, first
        step). ``values`` is a list of per-point arrays, or callables
        f(dx, dy) -> per-point array evaluated per tap. Returns [len, M, M]
        indexed [channel, gy, gx]."""
        out = np.zeros((len(values), self.m, self.m))
        for gx, gy, w, dx, dy in self.taps():
            flat = gy * self.m + gx
            for ch, v in enumerate(values):
                vv = v(dx, dy) if callable(v) else v
                out[ch] += np.bincount(flat, weights=w * vv,
                                       minlength=self.m * self.m).reshape(self.m, self.m)
        return out

    def gather(self, grid, combine):
        """Back-projection (Sec. 3.4, third step): per point
        sum_g w_ig * combine(grid values at g, dx, dy)."""
        acc = None
        for gx, gy, w, dx, dy in self.taps():
            val = combine(grid[:, gy, gx], dx, dy)
            acc = w * val if acc is None else acc + w * val
        return acc


def kernel_tables(m, s, gamma, tau=1.0):
    """Kernel on the node offsets (a, b), a, b in (-M, M), as arrays indexed
    [b + M - 1, a + M - 1]: K = (1 + tau s^2 (a^2 + b^2))^-gamma, and the two
    tables of the displacement-weighted kernel H_x = K s a, H_y = K s b."""
    off = np.arange(-(m - 1), m, dtype=np.float64)
    a = off[None, :]
    b = off[:, None]
    k = kernel(s * s * (a * a + b * b), gamma, tau)
    return k, k * s * a, k * s * b


def fft_length(m):
    """FFT length per side: the smallest power of two >= 2M. Any length
    >= 2M - 1 gives the same linear convolution."""
    return 1 << int(math.ceil(math.log2(2 * m)))


def convolve_fft(grids, table, length=None):
    """Grid interaction by FFT (Sec. 3.4, second step):
    phi(g) = sum_g' T(g - g') q(g') for g, g' in [0, M)^2, computed by
    embedding the Toeplitz operator in a circulant of side L and multiplying
    spectra. ``grids`` is [C, M, M], ``table`` is [2M-1, 2M-1] indexed as in
    kernel_tables."""
    grids = np.asarray(grids, dtype=np.float64)
    m = grids.shape[-1]
    L = fft_length(m) if length is None else int(length)
    if L < 2 * m - 1:
        raise ValueError("FFT length too short for a linear convolution")
    emb = np.zeros((L, L))
    off = np.arange(-(m - 1), m)
    emb[np.ix_(off % L, off % L)] = table
    spec = np.fft.rfft2(emb)
    pad = np.zeros(grids.shape[:-2] + (L, L))
    pad[..., :m, :m] = grids
    out = np.fft.irfft2(np.fft.rfft2(pad) * spec, s=(L, L))
    return out[..., :m, :m]


def convolve_direct(grids, table):
    """The same grid interaction as an explicit double sum (small M only)."""
    grids = np.asarray(grids, dtype=np.float64)
    m = grids.shape[-1]
    ii = np.arange(m)
    dy = ii[:, None, None, None] - ii[None, None, :, None] + (m - 1)   # gy - gy'
    dx = ii[None, :, None, None] - ii[None, None, None, :] + (m - 1)   # gx - gx'
    op = table[dy, dx].reshape(m * m, m * m)
    flat = grids.reshape(grids.shape[:-2] + (m * m,))
    return (flat @ op.T).reshape(grids.shape)


def repulsion_ibfft_paper(pos, gamma, n_int, k, box=None, direct=False, tau=1.0):
    """Interpolated repulsion in the paper's form (Eq.13-15): three kernel
    sums psi_v with charges v in {1, x, y}, then
    F_x(i) = x_i psi_1(i) - psi_x(i), F_y(i) = y_i psi_1(i) - psi_y(i)."""
    it = Interp(pos, n_int, k, box)
    x = it.pos
    q = it.spread([np.ones(x.shape[0]), x[:, 0], x[:, 1]])
    kt, _, _ = kernel_tables(it.m, it.s, gamma, tau)
    phi = convolve_direct(q, kt) if direct else convolve_fft(q, kt)
    psi1 = it.gather(phi, lambda v, dx, dy: v[0])
    psix = it.gather(phi, lambda v, dx, dy: v[1])
    psiy = it.gather(phi, lambda v, dx, dy: v[2])
    return np.stack([x[:, 0] * psi1 - psix, x[:, 1] * psi1 - psiy], axis=1)


def repulsion_ibfft_stable(pos, gamma, n_int, k, box=None, direct=False, tau=1.0):
    """Interpolated repulsion in offset form: the same algebra as Eq.13-15
    with every position written relative to the grid node it is spread to or
    gathered from, x = y_g + delta. Charges {1, delta_x, delta_y};
    phi_1 = K * q_1, G_x = H_x * q_1 - K * q_dx, G_y = H_y * q_1 - K * q_dy
    (* = grid convolution), and F(i) = sum_g w_ig (delta_ig phi_1(g) + G(g)).
    Substituting x_i = y_g + delta_ig and x_j = y_g' + delta_jg' into
    x_i psi_1 - psi_x gives this identity exactly, so it equals the paper form
    up to rounding while avoiding the cancellation of two large terms."""
    it = Interp(pos, n_int, k, box)
    n = it.pos.shape[0]
    q = it.spread([np.ones(n), lambda dx, dy: dx, lambda dx, dy: dy])
    kt, hx, hy = kernel_tables(it.m, it.s, gamma, tau)
    conv = convolve_direct if direct else convolve_fft
    k_q = conv(q, kt)                  # [K*q1, K*qdx, K*qdy]
    hx_q1 = conv(q[0:1], hx)[0]
    hy_q1 = conv(q[0:1], hy)[0]
    phi1 = k_q[0]
    gx = hx_q1 - k_q[1]
    gy = hy_q1 - k_q[2]
    grid = np.stack([phi1, gx, gy])
    fx = it.gather(grid, lambda v, dx, dy: dx * v[0] + v[1])
    fy = it.gather(grid, lambda v, dx, dy: dy * v[0] + v[2])
    return np.stack([fx, fy], axis=1)


# ---------------------------------------------------------------------------
# Resultant force, k schedule, update, layout loop
# ---------------------------------------------------------------------------

class Params:
    """Model and schedule parameters (defaults of Sec. 3.3)."""

    def __init__(self, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA, gamma=DEFAULT_GAMMA,
                 rep_weight=1.0, n_int=64, k_mode=-1, total_iters=300, t0=0.0, tau=1.0):
        self.alpha = float(alpha)
        self.beta = float(beta)
        self.gamma = float(gamma)
        self.rep_weight = float(rep_weight)
        self.n_int = int(n_int)
        self.k_mode = int(k_mode)
        self.total_iters = int(total_iters)
        self.t0 = float(t0)
        self.tau = float(tau)


AUTO_GRID_MIN = 50
AUTO_GRID_CHUNK = 10


def auto_n_int(pos, cap):
    """Automatic grid: one interval per unit of layout length, at least 50,
    N_int = max(50, ceil(W)) for the side W of the square box (the rule of
    Linderman et al. that Sec. 3.4 cites for t-SNE), capped at `cap`; chosen
    every AUTO_GRID_CHUNK iterations (reading of this implementation)."""
    w = square_box(pos)[2]
    return int(min(cap, max(AUTO_GRID_MIN, math.ceil(w))))


def k_for_iteration(t, total):
    """Dynamic k of Sec. 3.4: 1 for the first 90% of the iterations, 2 for
    the next 5%, 3 for the rest (boundaries rounded down)."""
    if t < (9 * total) // 10:
        return 1
    if t < (19 * total) // 20:
        return 2
    return 3


def default_t0(n):
    """Initial step cap T0 = max(1, sqrt(n) / 10)."""
    return max(1.0, math.sqrt(n) / 10.0)


def step_cap(t, total, t0):
    """Linear cooling T_t = T0 (1 - t / T)."""
    return t0 * (1.0 - t / total)


def forces(pos, row_ptr, col_idx, params, k, rep_w=None, att_w=None):
    """Repulsion, attraction and displacement D = w_r F^r + F^a (Eq.7 as a
    motion). k = 0 evaluates the repulsion exactly, k >= 1 by the
    interpolation scheme (offset form). Local refinement (Sec. 5): per-node
    weights r (``rep_w``) scale each node's repulsion in D,
    D_i = w_r r_i F^r_i + F^a_i, and a (``att_w``) the attraction of its
    edges (see attraction); F^r is returned unweighted."""
    tau = getattr(params, "tau", 1.0)
    if k == 0:
        fr = repulsion_exact(pos, params.gamma, tau=tau)
    else:
        fr = repulsion_ibfft_stable(pos, params.gamma, params.n_int, k, tau=tau)
    fa = attraction(pos, row_ptr, col_idx, params.alpha, params.beta, tau=tau, weights=att_w)
    r = 1.0 if rep_w is None else np.asarray(rep_w, dtype=np.float64)[:, None]
    return fr, fa, params.rep_weight * r * fr + fa


def capped_move(pos, disp, cap):
    """x <- x + D min(1, cap / |D|); a node with D = 0 stays put."""
    x = np.asarray(pos, dtype=np.float64)
    d = np.asarray(disp, dtype=np.float64)
    norm = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    scale = np.ones_like(norm)
    big = norm > cap
    scale[big] = cap / norm[big]
    return x + d * scale[:, None]


def layout(pos0, row_ptr, col_idx, params, iters=None, t_start=0,
           round_fp32=False, callback=None, rep_w=None, att_w=None):
    """Run the iteration loop: at each t pick k (fixed or scheduled),
    evaluate the forces at the current positions, move every node
    synchronously. Returns the final positions (float64; rounded to float32
    after every step if ``round_fp32``)."""
    x = np.asarray(pos0, dtype=np.float64).copy()
    n = x.shape[0]
    total = params.total_iters
    t0 = params.t0 if params.t0 > 0 else default_t0(n)
    iters = total - t_start if iters is None else iters
    auto = params.n_int == 0
    if auto:
        params = Params(**{**params.__dict__})
        kmax = params.k_mode if params.k_mode in (1, 2) else 3
        params.n_int = auto_n_int(x, 1024 // kmax)
    for t in range(t_start, t_start + iters):
        if auto and t % AUTO_GRID_CHUNK == 0:
            params.n_int = auto_n_int(x, 1024 // kmax)
        k = params.k_mode if params.k_mode >= 0 else k_for_iteration(t, total)
        _, _, disp = forces(x, row_ptr, col_idx, params, k, rep_w, att_w)
        x = capped_move(x, disp, step_cap(t, total, t0))
        if round_fp32:
            x = x.astype(np.float32).astype(np.float64)
        if callback is not None:
            callback(t, x)
    return x
