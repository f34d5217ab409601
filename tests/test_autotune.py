"""Grid autotuner rules (host only) and its error model against the FP64
oracle: on laid-out graphs, the final-stage grid it picks keeps the k = 3
repulsion within the requested tolerance of the exact sums."""
import math

import numpy as np
import pytest

import synthgraphs as sg
from oracle import tfdp as ot
from paper_2303_03964_amd import autotune


def test_size_rule_passes_through_workload_grids():
    assert autotune.n_int_for_size(1000) == 64
    assert autotune.n_int_for_size(1_000_000) == 256
    vals = [autotune.n_int_for_size(n) for n in (200, 2000, 20000, 200000)]
    assert vals == sorted(vals) and all(v % 8 == 0 for v in vals)


def test_final_grid_meets_model_tolerance():
    for w in (5.0, 40.0, 120.0):
        for tol in (1e-2, 1e-3, 1e-4):
            m = 1.4
            ni = autotune.final_n_int(w, tol, margin=m, hi=10 ** 6)
            # the widened box meets the tolerance, one interval fewer would not
            assert autotune.DEFAULT_C[3] * (m * w / ni) ** 3 <= tol * (1 + 1e-9)
            assert ni == 8 or autotune.DEFAULT_C[3] * (m * w / (ni - 1)) ** 3 > tol * 0.999


def test_workspace_grid_caps():
    assert autotune.workspace_grid(20000) == autotune.MAX_N_INT_K3
    assert autotune.n_int_for_size(200) <= autotune.workspace_grid(200) <= autotune.MAX_N_INT_K3


def test_box_side():
    p = np.array([[0, 0], [3, 1], [1, -1], [np.nan, 5]], np.float32)
    assert autotune.box_side(p) == pytest.approx(3.0)


def test_box_sides_equal_box_side_per_layout():
    # the one-reduction widths of many layouts equal box_side of each: rows
    # with a non-finite coordinate left out, a layout without a finite row
    # 1.0, a single row (zero extent) 1e-6
    import torch
    rng = np.random.default_rng(3)
    parts = []
    for i in range(40):
        n = int(rng.integers(1, 60))
        p = (rng.standard_normal((n, 2)) * rng.uniform(0.01, 500)).astype(np.float32)
        if i % 7 == 3:
            p[rng.integers(0, n)] = (np.nan, 1.0)
        if i % 11 == 5:
            p[rng.integers(0, n), 1] = np.inf
        if i == 20:
            p[:] = np.nan
        parts.append(torch.from_numpy(p))
    parts.append(torch.zeros((1, 2)))
    got = autotune.box_sides(parts)
    want = [autotune.box_side(p) for p in parts]
    assert got.tolist() == want
    assert got[20] == 1.0 and got[-1] == 1e-6


@pytest.mark.parametrize("index,gamma", [(1, 2.0), (11, 2.0), (13, 2.0), (1, 4.0), (1, 1.5)])
def test_error_model_against_oracle(index, gamma):
    """Lay out a batch-workload graph with the oracle (gamma = 2), pick the
    final grid for tol = 1e-3 and the given gamma (a re-tune that changes
    gamma starts from such a layout) and check the oracle's k = 3
    interpolated repulsion against its exact sums."""
    g, pos0 = sg.sbm_batch_member(index)
    if g.n > 1500:
        pytest.skip("kept small for the CPU suite")
    p = ot.Params(n_int=autotune.n_int_for_size(g.n), total_iters=300, k_mode=1)
    x = ot.layout(pos0.astype(np.float64), g.row_ptr, g.col_idx, p, iters=270)
    tol = 1e-3
    ni = autotune.final_n_int(autotune.box_side(x), tol, gamma=gamma)
    assert ni < autotune.MAX_N_INT_K3  # the tested grids are within the cap
    ex = ot.repulsion_exact(x, gamma)
    fr = ot.repulsion_ibfft_stable(x, gamma, ni, 3)
    err = np.linalg.norm(fr - ex) / np.linalg.norm(ex)
    assert err <= tol, (g.n, ni, err)


def test_final_choice_prefers_exact_when_cheaper():
    # a few thousand nodes in a wide box: a 1e-3 grid is far costlier than n^2
    assert autotune.final_choice(5000, 60.0)[0] == 0
    # a million nodes in a box the largest grid resolves: the grid
    k_mode, ni = autotune.final_choice(1_000_000, 60.0)
    assert k_mode == -1 and ni == math.ceil(1.4 * 60.0 / autotune.interval_width(1e-3, 3))
    # a box too wide for 1e-3 on the largest grid (or on the workspace's
    # cap): the exact method, whatever it costs
    assert autotune.final_choice(1_000_000, 300.0) == (0, None)
    assert autotune.final_choice(1_000_000, 60.0, cap=200) == (0, None)
    # a narrower kernel (gamma 8) needs a finer grid at the same box
    assert autotune.final_choice(1_000_000, 30.0)[0] == -1
    assert autotune.final_choice(1_000_000, 30.0, gamma=8.0) == (0, None)
    assert autotune.kernel_scale(2.0, 1.0) == 1.0 and autotune.kernel_scale(4.0, 1.0) == 8.0
    assert autotune.kernel_scale(2.0, 4.0) == 8.0
    assert autotune.fft_length(64, 1) == 128 and autotune.fft_length(341, 3) == 2048
    # radix-3 lengths where 3 * 2^a >= 2M is shorter than the power of two
    assert [autotune.fft_length(n, 3) for n in (64, 128, 256, 300)] == [384, 768, 1536, 2048]
    assert autotune.fft_length(192, 1) == 384 and autotune.fft_length(200, 1) == 512
    lengths = {autotune.fft_length(n, k) for k in (1, 2, 3) for n in range(1, 342)}
    assert lengths == {64, 128, 256, 384, 512, 768, 1024, 1536, 2048}


def test_start_params():
    assert autotune.start_params(500) == (0, 8)
    k_mode, ni = autotune.start_params(2000)
    assert k_mode == -1 and ni == 64  # size rule 80 rounded to the FFT-friendly 64
    assert autotune.start_params(1_000_000) == (-1, 256)
    assert autotune.fft_rounded(72) == 64 and autotune.fft_rounded(88) == 88
