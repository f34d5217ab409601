"""C ABI checks that need no GPU: the library loads, exports every function
of include/tfdp.h, and its host-side validation returns the documented
status codes without touching a device."""
import ctypes

import pytest

from tests._lib import ensure_built, header_functions

ensure_built()
import paper_2303_03964_amd as T  # noqa: E402
from paper_2303_03964_amd.tfdp import TfdpParams  # noqa: E402

OK, INVALID, WORKSPACE, HIPERR, NONFINITE, UNSUPPORTED = 0, -1, -2, -3, -4, -5


def test_exports_every_header_function():
    lib = ctypes.CDLL(T.library_path())
    names = header_functions()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name


def test_defaults_match_paper():
    p = T.tfdp_params_default()
    assert p.alpha == pytest.approx(0.1) and p.beta == 8.0 and p.gamma == 2.0
    assert p.rep_weight == 1.0 and p.k_mode == -1 and p.t0 == 0.0 and p.tau == 1.0


@pytest.mark.parametrize("field,value,code", [
    ("gamma", 1.0, INVALID), ("gamma", 0.5, INVALID), ("gamma", float("nan"), INVALID),
    ("alpha", -0.1, INVALID), ("alpha", float("inf"), INVALID), ("beta", -1.0, INVALID),
    ("rep_weight", -2.0, INVALID), ("n_int", -1, INVALID), ("n_int", 1025, INVALID),
    ("k_mode", 4, INVALID), ("k_mode", -2, INVALID), ("total_iters", 0, INVALID),
    ("t0", float("inf"), INVALID), ("n_int", 400, UNSUPPORTED),
    ("tau", 0.0, INVALID), ("tau", -1.0, INVALID), ("tau", float("nan"), INVALID),
])
def test_validate_rejects(field, value, code):
    p = T.tfdp_params_default(**{field: value})
    assert T.tfdp_params_validate(p, 100, 10) == code
    assert T.tfdp_last_error() != ""
    assert T.tfdp_workspace_size(100, 10, p) == 0


def test_validate_sizes_and_limits():
    p = T.tfdp_params_default()
    assert T.tfdp_params_validate(p, 0, 0) == INVALID
    assert T.tfdp_params_validate(p, 10, -1) == INVALID
    assert T.tfdp_params_validate(p, 10, 2 ** 31) == INVALID
    assert T.tfdp_params_validate(p, 1, 0) == OK
    # k_mode 1 allows a 1024-interval grid, the schedule does not
    assert T.tfdp_params_validate(T.tfdp_params_default(n_int=1024, k_mode=1), 10, 0) == OK
    assert T.tfdp_params_validate(T.tfdp_params_default(n_int=341), 10, 0) == OK
    assert T.tfdp_params_validate(T.tfdp_params_default(n_int=342), 10, 0) == UNSUPPORTED
    # automatic grid: valid, workspace sized for the largest grid of the k range
    auto = T.tfdp_params_default(n_int=0)
    assert T.tfdp_params_validate(auto, 10, 0) == OK
    assert T.tfdp_workspace_size(1000, 0, auto) == T.tfdp_workspace_size(1000, 0, T.tfdp_params_default(n_int=341))


def test_contact_condition_is_a_warning():
    p = T.tfdp_params_default(alpha=0.2, beta=8.0)
    assert T.tfdp_params_validate(p, 10, 0) == OK
    assert "Eq.9" in T.tfdp_last_error()
    assert T.tfdp_params_validate(T.tfdp_params_default(), 10, 0) == OK
    assert T.tfdp_last_error() == ""


def test_workspace_size_monotone():
    p = T.tfdp_params_default(n_int=256, total_iters=500)
    a = T.tfdp_workspace_size(1000, 0, p)
    b = T.tfdp_workspace_size(1_000_000, 10_000_000, p)
    assert 0 < a < b and a % 256 == 0
    # 1M nodes, 256 intervals, k up to 3: well under 1 GB
    assert b < 200 * 2 ** 20


def test_init_rejects_before_device_work():
    lib = T.load_library()
    p = T.tfdp_params_default()
    h = ctypes.c_void_p(1)
    fake = ctypes.c_void_p(0x100000)
    # NULL handle slot
    assert lib.tfdp_layout_init(None, 10, 0, fake, fake, fake, fake, 1 << 20, ctypes.byref(p), None) == INVALID
    # NULL device pointers
    assert lib.tfdp_layout_init(ctypes.byref(h), 10, 4, None, fake, fake, fake, 1 << 20, ctypes.byref(p), None) == INVALID
    assert h.value is None
    # invalid parameters
    bad = T.tfdp_params_default(gamma=0.9)
    assert lib.tfdp_layout_init(ctypes.byref(h), 10, 4, fake, fake, fake, fake, 1 << 20, ctypes.byref(bad), None) == INVALID
    # workspace missing, too small, misaligned
    need = T.tfdp_workspace_size(10, 4, p)
    assert lib.tfdp_layout_init(ctypes.byref(h), 10, 4, fake, fake, fake, None, need, ctypes.byref(p), None) == WORKSPACE
    assert lib.tfdp_layout_init(ctypes.byref(h), 10, 4, fake, fake, fake, fake, need - 1, ctypes.byref(p), None) == WORKSPACE
    odd = ctypes.c_void_p(0x100010)
    assert lib.tfdp_layout_init(ctypes.byref(h), 10, 4, fake, fake, fake, odd, need, ctypes.byref(p), None) == WORKSPACE
    assert "workspace" in T.tfdp_last_error()


def test_null_handle_calls():
    lib = T.load_library()
    assert lib.tfdp_layout_step(None, 1, None) == INVALID
    assert lib.tfdp_layout_forces(None, None, 1, None, None, None, None) == INVALID
    assert lib.tfdp_layout_set_params(None, None) == INVALID
    assert lib.tfdp_layout_get_iter(None, None) == INVALID
    assert lib.tfdp_layout_set_iter(None, 3) == INVALID
    assert lib.tfdp_layout_sync_status(None, None) == INVALID
    assert lib.tfdp_layout_set_profiling(None, 1) == INVALID
    assert lib.tfdp_layout_set_graphs(None, 1) == INVALID
    assert lib.tfdp_layout_set_overlap(None, 1) == INVALID
    assert lib.tfdp_layout_set_node_weights(None, None, None) == INVALID
    assert lib.tfdp_layout_get_params(None, None) == INVALID
    lib.tfdp_layout_destroy(None)


def test_phase_names():
    names = [T.tfdp_phase_name(i) for i in range(T.tfdp_phase_count())]
    assert "gather_update" in names and "spread" in names and "rowfft" in names and "colconv" in names
    assert "attract" in names and "node_update" in names
    assert T.tfdp_phase_name(-1) == "" and T.tfdp_phase_name(999) == ""


def test_params_struct_layout(tmp_path):
    """The ctypes mirror has the C struct's size and field offsets (compiled
    from include/tfdp.h with the host C compiler)."""
    import os
    import subprocess
    assert ctypes.sizeof(TfdpParams) == 36
    fields = [name for name, _ in TfdpParams._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"tfdp.h\"\nint main(void) {\n"
                   '  printf("%zu", sizeof(tfdp_params));\n'
                   + "".join(f'  printf(" %zu", offsetof(tfdp_params, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"),
                        "-I", "/opt/rocm/include", str(src), "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("no host C compiler for the HIP headers: " + r.stderr[-200:])
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(TfdpParams)
    assert vals[1:] == [getattr(TfdpParams, f).offset for f in fields]


def test_batch_host_bookkeeping():
    lib = T.load_library()
    out = ctypes.c_void_p()
    need = T.tfdp_batch_workspace_size(4, 0)
    assert need > 0 and T.tfdp_batch_workspace_size(0, 10) == 0 and T.tfdp_batch_workspace_size(4, -1) == 0
    assert T.tfdp_batch_workspace_size(4, 1 << 20) >= need + (1 << 20) * 8 - 8 * 256
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: no step runs with members
    assert lib.tfdp_batch_create(None, 4, fake, need) == INVALID
    assert lib.tfdp_batch_create(ctypes.byref(out), 0, fake, need) == INVALID
    assert lib.tfdp_batch_create(ctypes.byref(out), 4, None, need) == WORKSPACE
    assert lib.tfdp_batch_create(ctypes.byref(out), 4, fake, need - 1) == WORKSPACE
    assert lib.tfdp_batch_create(ctypes.byref(out), 4, ctypes.c_void_p(0x100040), need) == WORKSPACE
    assert lib.tfdp_batch_create(ctypes.byref(out), 4, fake, need) == OK and out.value
    b = out
    assert lib.tfdp_batch_count(b) == 0 and lib.tfdp_batch_count(None) == 0
    # NULL members and removal of a non-member are rejected without device work
    assert lib.tfdp_batch_add(b, None) == INVALID
    assert lib.tfdp_batch_add(None, ctypes.c_void_p(8)) == INVALID
    assert lib.tfdp_batch_remove(b, ctypes.c_void_p(8)) == INVALID
    assert "not a member" in T.tfdp_last_error()
    # an empty batch steps without touching a device; negative counts fail
    assert lib.tfdp_batch_step(b, 5, None) == OK
    assert lib.tfdp_batch_step(b, -1, None) == INVALID
    assert lib.tfdp_batch_step(None, 1, None) == INVALID
    assert lib.tfdp_batch_set_graphs(b, 0) == OK and lib.tfdp_batch_set_graphs(None, 1) == INVALID
    # tile schedule: defaults, validation (no device work when nothing changes)
    assert T.tfdp_batch_get_tiles(b, 256) == (8, 2) and T.tfdp_batch_get_tiles(b, 512) == (2, 1)
    assert T.tfdp_batch_get_tiles(b, 768) == (4, 1)
    assert lib.tfdp_batch_set_tiles(b, 256, 8, 2, None) == OK and lib.tfdp_batch_set_tiles(b, 256, 0, 0, None) == OK
    assert lib.tfdp_batch_set_tiles(None, 256, 8, 2, None) == INVALID
    assert lib.tfdp_batch_set_tiles(b, 300, 8, 2, None) == INVALID
    assert lib.tfdp_batch_set_tiles(b, 256, 3, 1, None) == UNSUPPORTED
    assert lib.tfdp_batch_set_tiles(b, 256, 4, 3, None) == UNSUPPORTED
    assert lib.tfdp_batch_set_tiles(b, 1024, 8, 1, None) == UNSUPPORTED
    lib.tfdp_batch_destroy(b)
    lib.tfdp_batch_destroy(None)


def test_stress_metric_host_checks():
    lib = T.load_library()
    assert T.tfdp_stress_workspace_size(0, 4) == 0
    assert T.tfdp_stress_workspace_size(10, 0) == 0 and T.tfdp_stress_workspace_size(10, 65) == 0
    assert T.tfdp_stress_workspace_size(1000, 64) > 64 * 1000
    se = ctypes.c_double()
    fake = ctypes.c_void_p(0x100000)
    assert lib.tfdp_stress_sampled(10, 4, fake, fake, fake, fake, 0, fake, 1 << 20, ctypes.byref(se), None,
                                   None) == INVALID
    assert lib.tfdp_stress_sampled(10, 4, None, fake, fake, fake, 4, fake, 1 << 20, ctypes.byref(se), None,
                                   None) == INVALID
    assert lib.tfdp_stress_sampled(10, 4, fake, fake, fake, fake, 4, None, 1 << 20, ctypes.byref(se), None,
                                   None) == WORKSPACE
    assert lib.tfdp_stress_sampled(10, 4, fake, fake, fake, fake, 4, fake, 16, ctypes.byref(se), None,
                                   None) == WORKSPACE


def test_quality_metric_host_checks():
    lib = T.load_library()
    se = ctypes.c_double()
    np2 = (ctypes.c_double * 2)()
    fake = ctypes.c_void_p(0x100000)
    # np output required; misaligned workspace rejected
    assert lib.tfdp_quality_sampled(10, 4, fake, fake, fake, fake, 4, fake, 1 << 20, ctypes.byref(se), None, None,
                                    None) == INVALID
    assert lib.tfdp_quality_sampled(10, 4, fake, fake, fake, fake, 4, ctypes.c_void_p(0x100040), 1 << 20,
                                    ctypes.byref(se), np2, None, None) == WORKSPACE
    assert lib.tfdp_quality_sampled(10, 4, fake, fake, fake, fake, 65, fake, 1 << 20, ctypes.byref(se), np2, None,
                                    None) == INVALID


def test_noalloc_metric_host_checks():
    """The allocation-free metric refuses bad arguments and sizes above its
    static scratch before any device work."""
    lib = T.load_library()
    se = ctypes.c_double()
    np2 = (ctypes.c_double * 2)()
    fake = ctypes.c_void_p(0x100000)
    assert lib.tfdp_quality_sampled_noalloc(10, 4, fake, fake, fake, fake, 4, ctypes.byref(se), None, None,
                                            None) == INVALID
    assert lib.tfdp_quality_sampled_noalloc(10, 4, fake, fake, fake, fake, 0, ctypes.byref(se), np2, None,
                                            None) == INVALID
    assert lib.tfdp_quality_sampled_noalloc(0, 4, fake, fake, fake, fake, 4, ctypes.byref(se), np2, None,
                                            None) == INVALID
    n = 600_000
    assert T.tfdp_stress_workspace_size(n, 64) > 64 << 20
    assert lib.tfdp_quality_sampled_noalloc(n, 4, fake, fake, fake, fake, 64, ctypes.byref(se), np2, None,
                                            None) == UNSUPPORTED
    assert "static scratch" in T.tfdp_last_error()
