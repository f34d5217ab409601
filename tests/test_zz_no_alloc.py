"""tfdp_quality_sampled_noalloc (the library's static scratch, no device
allocation) against tfdp_quality_sampled with a caller workspace: the same
kernels on the same inputs, so SE, NP_1, NP_2 and the BFS level count must
agree exactly. Two calls in a row, the second on a smaller graph with fewer
sources, so that the second call runs over the first one's leftovers."""
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


def device_case(g, pos, src):
    import torch
    return (torch.as_tensor(g.row_ptr, dtype=torch.int32).cuda(),
            torch.as_tensor(g.col_idx, dtype=torch.int32).cuda(),
            torch.as_tensor(pos, dtype=torch.float32).cuda(),
            torch.as_tensor(np.asarray(src), dtype=torch.int32).cuda())


def test_noalloc_matches_workspace_entry_point(T):
    rng = np.random.default_rng(11)
    big = sg.mesh_100k().graph
    small = sg.sbm([150, 120, 90], 0.06, 0.004, 9)
    cases = [
        ("mesh_100k, 64 sources", big, sg.uniform_positions(big.n, 21, -300, 300), rng.choice(big.n, 64, replace=False)),
        ("sbm 360, 9 sources", small, sg.uniform_positions(small.n, 22, -10, 10), rng.choice(small.n, 9, replace=False)),
    ]
    for name, g, pos, src in cases:
        rp, ci, p, s = device_case(g, pos, src)
        say(f"noalloc: {name}: n={g.n} nnz={int(ci.numel())} "
            f"scratch need {T.tfdp_stress_workspace_size(g.n, len(src))} bytes")
        se0, np0, lv0 = T.tfdp_quality_sampled(rp, ci, p, s)
        se1, np1, lv1 = T.tfdp_quality_sampled_noalloc(rp, ci, p, s)
        say(f"  workspace: SE {se0!r} NP {np0!r} levels {lv0}")
        say(f"  static:    SE {se1!r} NP {np1!r} levels {lv1}")
        assert lv1 == lv0
        assert se1 == se0
        assert np1 == np0


def test_noalloc_refuses_beyond_its_limit(T):
    import torch
    n, nsrc = 600_000, 64  # ~88 MB of metric scratch, above the 64 MiB array
    assert T.tfdp_stress_workspace_size(n, nsrc) > 64 << 20
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    s = torch.arange(nsrc, dtype=torch.int32, device="cuda")
    with pytest.raises(T.TfdpError) as e:
        T.tfdp_quality_sampled_noalloc(rp, ci, p, s)
    assert e.value.status == -5
    assert "static scratch" in str(e.value)
