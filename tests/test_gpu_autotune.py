"""Grid autotuner on the device: the error constants measured from the
library's own forces agree with the defaults (fitted to the FP64 oracle), and
the final-stage grid it picks keeps the k = 3 repulsion within the requested
tolerance of the exact sums (the library's exact sums are pinned to the
oracle by test_gpu_parity.py)."""
import sys

import numpy as np
import pytest

import synthgraphs as sg
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


def laid_out(T, index, iters):
    import torch
    from paper_2303_03964_amd import autotune
    g, pos = sg.sbm_batch_member(index)
    p = T.tfdp_params_default(n_int=autotune.n_int_for_size(g.n), total_iters=300)
    ws = T.tfdp_params_default(n_int=autotune.workspace_grid(g.n), total_iters=300)
    lay = T.Layout(g.row_ptr, g.col_idx, torch.as_tensor(pos).cuda(), p, workspace_params=ws)
    lay.step(iters)
    torch.cuda.synchronize()
    return lay


def test_calibrated_constants_match_defaults(T):
    from paper_2303_03964_amd import autotune
    lays = [laid_out(T, i, 300) for i in (1, 3, 7)]
    consts, samples = autotune.calibrate(T, lays)
    say(f"calibrated C_k = {consts}, defaults {autotune.DEFAULT_C}")
    for k in (1, 2, 3):
        assert len(samples[k]) >= 6
        assert autotune.DEFAULT_C[k] / 3 <= consts[k] <= autotune.DEFAULT_C[k] * 3
    for lay in lays:
        lay.close()


@pytest.mark.parametrize("index", [0, 3, 9])
def test_retuned_grid_meets_tolerance(T, index):
    import torch
    from paper_2303_03964_amd import autotune
    lay = laid_out(T, index, 285)
    ni = autotune.retune(lay, tol=1e-3)  # at the switch to k = 3
    lay.step(15)
    ex, _, _ = lay.forces(k=0)
    fr, _, _ = lay.forces(k=3)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm((fr - ex).double()) / torch.linalg.norm(ex.double()))
    say(f"graph {index}: n={lay.n} final N_int={ni} k=3 error {err:.2e}")
    assert err <= 1e-3
    lay.close()
