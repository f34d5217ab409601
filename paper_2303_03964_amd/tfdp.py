"""ctypes binding of libtfdp.so (C ABI in include/tfdp.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the computation runs in the library's
kernels. torch is imported before the library is loaded so that both share
one HIP runtime.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libtfdp.so"

TFDP_OK = 0
STATUS_NAMES = {
    0: "TFDP_OK",
    -1: "TFDP_ERR_INVALID_ARG",
    -2: "TFDP_ERR_WORKSPACE",
    -3: "TFDP_ERR_HIP",
    -4: "TFDP_ERR_NONFINITE",
    -5: "TFDP_ERR_UNSUPPORTED",
}


class TfdpParams(ctypes.Structure):
    """Mirror of ``tfdp_params``."""

    _fields_ = [
        ("alpha", c_float),
        ("beta", c_float),
        ("gamma", c_float),
        ("rep_weight", c_float),
        ("n_int", c_int32),
        ("k_mode", c_int32),
        ("total_iters", c_int32),
        ("t0", c_float),
        ("tau", c_float),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TfdpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


# C signatures: name -> (restype, argtypes)
_SIGS = {
    "tfdp_params_default": (None, [POINTER(TfdpParams)]),
    "tfdp_params_validate": (c_int32, [POINTER(TfdpParams), c_int32, c_int64]),
    "tfdp_workspace_size": (c_size_t, [c_int32, c_int64, POINTER(TfdpParams)]),
    "tfdp_layout_init": (c_int32, [POINTER(c_void_p), c_int32, c_int64, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_size_t, POINTER(TfdpParams), c_void_p]),
    "tfdp_layout_step": (c_int32, [c_void_p, c_int32, c_void_p]),
    "tfdp_layout_forces": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "tfdp_layout_set_params": (c_int32, [c_void_p, POINTER(TfdpParams)]),
    "tfdp_layout_set_node_weights": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "tfdp_layout_get_params": (c_int32, [c_void_p, POINTER(TfdpParams)]),
    "tfdp_layout_get_iter": (c_int32, [c_void_p, POINTER(c_int32)]),
    "tfdp_layout_set_iter": (c_int32, [c_void_p, c_int32]),
    "tfdp_layout_sync_status": (c_int32, [c_void_p, c_void_p]),
    "tfdp_layout_destroy": (None, [c_void_p]),
    "tfdp_last_error": (c_char_p, []),
    "tfdp_layout_set_profiling": (c_int32, [c_void_p, c_int32]),
    "tfdp_layout_set_graphs": (c_int32, [c_void_p, c_int32]),
    "tfdp_layout_set_overlap": (c_int32, [c_void_p, c_int32]),
    "tfdp_phase_count": (c_int32, []),
    "tfdp_phase_name": (c_char_p, [c_int32]),
    "tfdp_layout_phase_times": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64), c_int32]),
    "tfdp_stress_workspace_size": (c_size_t, [c_int32, c_int32]),
    "tfdp_stress_sampled": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                      c_size_t, POINTER(c_double), POINTER(c_int32), c_void_p]),
    "tfdp_quality_sampled": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                       c_size_t, POINTER(c_double), POINTER(c_double), POINTER(c_int32),
                                       c_void_p]),
    "tfdp_quality_sampled_noalloc": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                               POINTER(c_double), POINTER(c_double), POINTER(c_int32), c_void_p]),
    "tfdp_batch_workspace_size": (c_size_t, [c_int32, c_int64]),
    "tfdp_batch_create": (c_int32, [POINTER(c_void_p), c_int32, c_void_p, c_size_t]),
    "tfdp_batch_add": (c_int32, [c_void_p, c_void_p]),
    "tfdp_batch_remove": (c_int32, [c_void_p, c_void_p]),
    "tfdp_batch_count": (c_int32, [c_void_p]),
    "tfdp_batch_step": (c_int32, [c_void_p, c_int32, c_void_p]),
    "tfdp_batch_set_graphs": (c_int32, [c_void_p, c_int32]),
    "tfdp_batch_set_tiles": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p]),
    "tfdp_batch_get_tiles": (c_int32, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "tfdp_batch_destroy": (None, [c_void_p]),
}

_lib = None


def library_path() -> str:
    return os.environ.get("TFDP_LIBRARY", os.path.join(_HERE, _LIB_NAME))


def load_library():
    """Load libtfdp.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} not found: build it first (python -m paper_2303_03964_amd.build)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status):
    if status != TFDP_OK:
        raise TfdpError(status, tfdp_last_error())
    return status


def _stream(stream):
    if stream is None:
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return c_void_p(stream.cuda_stream)
    return c_void_p(int(stream))


def _ptr(t):
    return c_void_p(0 if t is None else t.data_ptr())


# ------------------------------------------------------------------ same names as the C ABI

def tfdp_last_error() -> str:
    msg = load_library().tfdp_last_error()
    return msg.decode() if msg else ""


def tfdp_params_default(**overrides) -> TfdpParams:
    p = TfdpParams()
    load_library().tfdp_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def tfdp_params_validate(p: TfdpParams, n: int, nnz: int) -> int:
    return load_library().tfdp_params_validate(ctypes.byref(p), n, nnz)


def tfdp_workspace_size(n: int, nnz: int, p: TfdpParams) -> int:
    return int(load_library().tfdp_workspace_size(n, nnz, ctypes.byref(p)))


def tfdp_layout_init(n, nnz, row_ptr, col_idx, pos, workspace, params, stream=None):
    h = c_void_p()
    _check(load_library().tfdp_layout_init(ctypes.byref(h), n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(pos),
                                           _ptr(workspace), workspace.numel() * workspace.element_size(),
                                           ctypes.byref(params), _stream(stream)))
    return h


def tfdp_layout_step(h, iters, stream=None):
    return _check(load_library().tfdp_layout_step(h, iters, _stream(stream)))


def tfdp_layout_forces(h, pos_in, k, f_rep=None, f_att=None, f_tot=None, stream=None):
    return _check(load_library().tfdp_layout_forces(h, _ptr(pos_in), k, _ptr(f_rep), _ptr(f_att), _ptr(f_tot),
                                                     _stream(stream)))


def tfdp_layout_set_params(h, params):
    return _check(load_library().tfdp_layout_set_params(h, ctypes.byref(params)))


def tfdp_layout_set_node_weights(h, rep_w=None, att_w=None):
    return _check(load_library().tfdp_layout_set_node_weights(h, _ptr(rep_w), _ptr(att_w)))


def tfdp_layout_get_params(h) -> TfdpParams:
    p = TfdpParams()
    _check(load_library().tfdp_layout_get_params(h, ctypes.byref(p)))
    return p


def tfdp_layout_get_iter(h) -> int:
    t = c_int32()
    _check(load_library().tfdp_layout_get_iter(h, ctypes.byref(t)))
    return t.value


def tfdp_layout_set_iter(h, t):
    return _check(load_library().tfdp_layout_set_iter(h, t))


def tfdp_layout_sync_status(h, stream=None) -> int:
    """Returns the raw status (TFDP_ERR_NONFINITE is reported, not raised)."""
    st = load_library().tfdp_layout_sync_status(h, _stream(stream))
    if st not in (TFDP_OK, -4):
        raise TfdpError(st, tfdp_last_error())
    return st


def tfdp_layout_destroy(h):
    load_library().tfdp_layout_destroy(h)


def tfdp_layout_set_profiling(h, enable):
    return _check(load_library().tfdp_layout_set_profiling(h, int(bool(enable))))


def tfdp_layout_set_graphs(h, enable):
    return _check(load_library().tfdp_layout_set_graphs(h, int(bool(enable))))


def tfdp_layout_set_overlap(h, mode):
    return _check(load_library().tfdp_layout_set_overlap(h, mode))


def tfdp_phase_count() -> int:
    return load_library().tfdp_phase_count()


def tfdp_phase_name(i) -> str:
    return load_library().tfdp_phase_name(i).decode()


def tfdp_layout_phase_times(h):
    n = tfdp_phase_count()
    ms = (c_double * n)()
    cnt = (c_int64 * n)()
    _check(load_library().tfdp_layout_phase_times(h, ms, cnt, n))
    return {tfdp_phase_name(i): (ms[i], cnt[i]) for i in range(n)}


def tfdp_stress_workspace_size(n, nsrc) -> int:
    return int(load_library().tfdp_stress_workspace_size(n, nsrc))


def _metric_workspace(pos, nsrc):
    n = int(pos.shape[0])
    size = tfdp_stress_workspace_size(n, nsrc)
    if size == 0:
        raise TfdpError(-1, "invalid sizes for the metric workspace")
    work = torch.empty(size + 256, dtype=torch.uint8, device=pos.device)
    off = (-work.data_ptr()) % 256
    return work[off:off + size], size


def tfdp_stress_sampled(row_ptr, col_idx, pos, sources, stream=None):
    """Sampled stress error of the layout `pos` (device tensors: int32 CSR,
    float32 [n, 2] positions, int32 sources). Returns (SE, BFS levels)."""
    n = int(pos.shape[0])
    nsrc = int(sources.numel())
    work, size = _metric_workspace(pos, nsrc)
    se = c_double()
    lv = c_int32()
    nnz = int(col_idx.numel())
    _check(load_library().tfdp_stress_sampled(n, nnz, _ptr(row_ptr), _ptr(col_idx if nnz else None), _ptr(pos),
                                              _ptr(sources), nsrc, _ptr(work), size, ctypes.byref(se),
                                              ctypes.byref(lv), _stream(stream)))
    return se.value, lv.value


def tfdp_quality_sampled(row_ptr, col_idx, pos, sources, stream=None):
    """Sampled stress error and neighbourhood preservation NP_1, NP_2 of the
    layout `pos` over the same sources. Returns (SE, (NP_1, NP_2), BFS levels)."""
    n = int(pos.shape[0])
    nsrc = int(sources.numel())
    work, size = _metric_workspace(pos, nsrc)
    se = c_double()
    np_ = (c_double * 2)()
    lv = c_int32()
    nnz = int(col_idx.numel())
    _check(load_library().tfdp_quality_sampled(n, nnz, _ptr(row_ptr), _ptr(col_idx if nnz else None), _ptr(pos),
                                               _ptr(sources), nsrc, _ptr(work), size, ctypes.byref(se), np_,
                                               ctypes.byref(lv), _stream(stream)))
    return se.value, (np_[0], np_[1]), lv.value


def tfdp_quality_sampled_noalloc(row_ptr, col_idx, pos, sources, stream=None):
    """tfdp_quality_sampled with the library's static scratch instead of a
    workspace (no device allocation). Returns (SE, (NP_1, NP_2), BFS levels)."""
    n = int(pos.shape[0])
    nsrc = int(sources.numel())
    se = c_double()
    np_ = (c_double * 2)()
    lv = c_int32()
    nnz = int(col_idx.numel())
    _check(load_library().tfdp_quality_sampled_noalloc(n, nnz, _ptr(row_ptr), _ptr(col_idx if nnz else None),
                                                       _ptr(pos), _ptr(sources), nsrc, ctypes.byref(se), np_,
                                                       ctypes.byref(lv), _stream(stream)))
    return se.value, (np_[0], np_[1]), lv.value


def tfdp_batch_workspace_size(capacity, map_entries) -> int:
    return int(load_library().tfdp_batch_workspace_size(capacity, map_entries))


def tfdp_batch_create(capacity, workspace):
    b = c_void_p()
    _check(load_library().tfdp_batch_create(ctypes.byref(b), capacity, _ptr(workspace), int(workspace.numel())))
    return b


def tfdp_batch_add(b, h):
    return _check(load_library().tfdp_batch_add(b, h))


def tfdp_batch_remove(b, h):
    return _check(load_library().tfdp_batch_remove(b, h))


def tfdp_batch_count(b) -> int:
    return load_library().tfdp_batch_count(b)


def tfdp_batch_step(b, iters, stream=None):
    return _check(load_library().tfdp_batch_step(b, iters, _stream(stream)))


def tfdp_batch_set_graphs(b, enable):
    return _check(load_library().tfdp_batch_set_graphs(b, int(bool(enable))))


def tfdp_batch_set_tiles(b, fft_length, rows_per_block, column_groups, stream=None):
    return _check(load_library().tfdp_batch_set_tiles(b, fft_length, rows_per_block, column_groups,
                                                      _stream(stream)))


def tfdp_batch_get_tiles(b, fft_length):
    r, g = c_int32(), c_int32()
    _check(load_library().tfdp_batch_get_tiles(b, fft_length, ctypes.byref(r), ctypes.byref(g)))
    return r.value, g.value


def tfdp_batch_destroy(b):
    load_library().tfdp_batch_destroy(b)


# ------------------------------------------------------------------ convenience owners of the buffers

class Layout:
    """Owns the device CSR, positions and workspace of one layout handle.

    row_ptr / col_idx: int32 arrays (numpy or torch); pos: float32 [n, 2].
    Host arrays are copied to ``device``; a device float32 ``pos`` tensor is
    used in place.
    """

    def __init__(self, row_ptr, col_idx, pos, params: TfdpParams | None = None, device="cuda", stream=None,
                 workspace_params: TfdpParams | None = None):
        dev = torch.device(device)
        self.row_ptr = torch.as_tensor(row_ptr, dtype=torch.int32).to(dev).contiguous()
        self.col_idx = torch.as_tensor(col_idx, dtype=torch.int32).to(dev).contiguous()
        pos_t = torch.as_tensor(pos)
        if pos_t.device == dev and pos_t.dtype == torch.float32 and pos_t.is_contiguous():
            self.pos = pos_t
        else:
            self.pos = pos_t.to(dtype=torch.float32).to(dev).contiguous()
        if self.pos.dim() != 2 or self.pos.shape[1] != 2:
            raise ValueError("pos must have shape [n, 2]")
        self.n = int(self.pos.shape[0])
        self.nnz = int(self.col_idx.numel())
        if self.row_ptr.numel() != self.n + 1:
            raise ValueError("row_ptr must have n + 1 entries")
        self.params = params if params is not None else tfdp_params_default()
        # the workspace may be sized for a larger grid than the first one
        # (tfdp_layout_set_params can then move to it)
        sizing = [self.params] + ([workspace_params] if workspace_params is not None else [])
        sizes = [tfdp_workspace_size(self.n, self.nnz, q) for q in sizing]
        if min(sizes) == 0:
            bad = sizing[sizes.index(0)]
            raise TfdpError(tfdp_params_validate(bad, self.n, self.nnz), tfdp_last_error())
        size = max(sizes)
        self.workspace = torch.empty(size + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self.workspace = self.workspace[off:off + size]
        col = self.col_idx if self.nnz > 0 else None
        self.handle = tfdp_layout_init(self.n, self.nnz, self.row_ptr, col, self.pos, self.workspace,
                                       self.params, stream)

    def step(self, iters, stream=None):
        tfdp_layout_step(self.handle, iters, stream)

    def forces(self, pos_in=None, k=0, stream=None):
        pos_in = self.pos if pos_in is None else pos_in
        out = [torch.empty((self.n, 2), dtype=torch.float32, device=self.pos.device) for _ in range(3)]
        tfdp_layout_forces(self.handle, pos_in, k, out[0], out[1], out[2], stream)
        return tuple(out)

    def set_params(self, params: TfdpParams):
        tfdp_layout_set_params(self.handle, params)
        self.params = params

    def set_overlap(self, mode):
        """Edge-pass schedule: 1 overlapped with the grid passes, 0 fused, -1 automatic."""
        tfdp_layout_set_overlap(self.handle, mode)

    def set_node_weights(self, rep_w=None, att_w=None):
        """Local-refinement weights (float32 [n] device tensors or None);
        kept referenced here while the handle uses them."""
        dev = self.pos.device
        self.rep_w = None if rep_w is None else torch.as_tensor(rep_w, dtype=torch.float32).to(dev).contiguous()
        self.att_w = None if att_w is None else torch.as_tensor(att_w, dtype=torch.float32).to(dev).contiguous()
        for w in (self.rep_w, self.att_w):
            if w is not None and w.numel() != self.n:
                raise ValueError("weights must have n entries")
        tfdp_layout_set_node_weights(self.handle, self.rep_w, self.att_w)

    @property
    def iteration(self):
        return tfdp_layout_get_iter(self.handle)

    @iteration.setter
    def iteration(self, t):
        tfdp_layout_set_iter(self.handle, t)

    def sync_status(self, stream=None):
        return tfdp_layout_sync_status(self.handle, stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            tfdp_layout_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A tfdp_batch over Layout objects (kept alive while they are members),
    with its device workspace: slot tables for `capacity` members and an
    arena of `map_entries` block-map entries (8 bytes each)."""

    def __init__(self, capacity, map_entries=1 << 22, device="cuda"):
        size = tfdp_batch_workspace_size(capacity, map_entries)
        if size == 0:
            raise TfdpError(-1, "invalid batch capacity or arena size")
        ws = torch.empty(size + 256, dtype=torch.uint8, device=torch.device(device))
        off = (-ws.data_ptr()) % 256
        self.workspace = ws[off:off + size]
        self.handle = tfdp_batch_create(capacity, self.workspace)
        self.members = []

    def add(self, lay: Layout):
        tfdp_batch_add(self.handle, lay.handle)
        self.members.append(lay)

    def remove(self, lay: Layout):
        tfdp_batch_remove(self.handle, lay.handle)
        self.members.remove(lay)

    def __len__(self):
        return tfdp_batch_count(self.handle)

    def step(self, iters, stream=None):
        tfdp_batch_step(self.handle, iters, stream)

    def set_graphs(self, enable):
        tfdp_batch_set_graphs(self.handle, enable)

    def set_tiles(self, fft_length, rows_per_block, column_groups, stream=None):
        tfdp_batch_set_tiles(self.handle, fft_length, rows_per_block, column_groups, stream)

    def tiles(self, fft_length):
        return tfdp_batch_get_tiles(self.handle, fft_length)

    def close(self):
        if getattr(self, "handle", None) is not None:
            tfdp_batch_destroy(self.handle)
            self.handle = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
