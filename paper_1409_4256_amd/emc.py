"""ctypes binding of libemc.so: the C ABI declared in include/emc.h, same names.

Argument marshalling only: tensors are checked for device, dtype, contiguity and
size on the host, then their device pointers and the current HIP stream are
handed to the library.  Every computation runs in the library's kernels; if
the library is missing, loading fails loudly (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemc.so")

EMC_OK = 0
EMC_ERR_INVALID_ARG = -1
EMC_ERR_RANGE = -2
EMC_ERR_WORKSPACE = -3
EMC_ERR_HIP = -4
EMC_ERR_UNSUPPORTED = -5

EMC_PREC_FP32 = 0
EMC_PREC_BF16 = 1

EMC_RESP_FULL = 0
EMC_RESP_PARTIAL = 1
EMC_RESP_FINALIZE = 2

EXPORTS = ("emc_version", "emc_last_error", "emc_pix_stride", "emc_data_stride", "emc_frames_bytes",
           "emc_slices_bytes", "emc_workspace_bytes", "emc_pack_frames", "emc_expand", "emc_loglik",
           "emc_responsibilities", "emc_compress_workspace_bytes", "emc_compress", "emc_finalize", "emc_iterate",
           "emc_iterate_noalloc", "emc_pack_patterns", "emc_validate",
           "emc_cnn_param_count", "emc_cnn_workspace_bytes", "emc_cnn_preprocess", "emc_cnn_forward",
           "emc_cnn_gradients", "emc_cnn_adam", "emc_cnn_topk", "emc_cell_topk", "emc_topk_union",
           "emc_cell_targets",
           "emc_pack_frames_list", "emc_proposal_bytes", "emc_proposal_build", "emc_proposed_workspace_bytes",
           "emc_iterate_proposed", "emc_proposed_accumulate", "emc_proposed_workspace_view",
           "emc_scatter_plan_min_bytes", "emc_scatter_plan_build",
           "emc_gaussian_workspace_bytes", "emc_iterate_gaussian")


class EmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"emc status {status}: {message}")
        self.status = status
        self.message = message


class Problem(ctypes.Structure):
    _fields_ = [
        ("grid_n", ctypes.c_int32),
        ("n_pix", ctypes.c_int32),
        ("n_rot", ctypes.c_int32),
        ("n_data", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("q", ctypes.c_void_p),
        ("mask", ctypes.c_void_p),
        ("quat", ctypes.c_void_p),
        ("log_w", ctypes.c_void_p),
        ("scatter", ctypes.c_void_p),
    ]


class ScatterPlan(ctypes.Structure):
    _fields_ = [
        ("grid_n", ctypes.c_int32), ("n_pix", ctypes.c_int32), ("n_rot", ctypes.c_int32),
        ("brick", ctypes.c_int32), ("n_bricks", ctypes.c_int32), ("n_groups", ctypes.c_int32),
        ("chunk", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("n_visits", ctypes.c_int64), ("n_items", ctypes.c_int64), ("bytes", ctypes.c_int64),
        ("visits", ctypes.c_void_p), ("items", ctypes.c_void_p), ("rot", ctypes.c_void_p),
        ("q", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("quat", ctypes.c_void_p),
    ]


class Proposal(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int32), ("k_top", ctypes.c_int32), ("n_cand", ctypes.c_int32),
        ("n_audit", ctypes.c_int32), ("words", ctypes.c_int32), ("n_bands", ctypes.c_int32),
        ("n_groups", ctypes.c_int64), ("n_tiles", ctypes.c_int64), ("n_g", ctypes.c_int64),
        ("n_chunks", ctypes.c_int64),
        ("cell_of", ctypes.c_void_p), ("cell_ptr", ctypes.c_void_p), ("cell_rot", ctypes.c_void_p),
        ("pack_of", ctypes.c_void_p), ("cell_first", ctypes.c_void_p), ("pack_rot", ctypes.c_void_p),
        ("rot_local", ctypes.c_void_p),
        ("cand_frames", ctypes.c_void_p), ("audit_frames", ctypes.c_void_p), ("cand_cells", ctypes.c_void_p),
        ("pair_col", ctypes.c_void_p), ("cf_ptr", ctypes.c_void_p), ("cf_frame", ctypes.c_void_p),
        ("cf_mask", ctypes.c_void_p), ("cg_ptr", ctypes.c_void_p), ("groups", ctypes.c_void_p), ("grp_off", ctypes.c_void_p),
        ("tiles", ctypes.c_void_p), ("mask_audit", ctypes.c_void_p),
        ("chunks", ctypes.c_void_p), ("runs", ctypes.c_void_p),
        ("n_dense", ctypes.c_int32), ("n_packs", ctypes.c_int32), ("ld_dense", ctypes.c_int64),
        ("dense_band", ctypes.c_void_p), ("dense_list", ctypes.c_void_p), ("kt_dense", ctypes.c_void_p),
        ("n_rot", ctypes.c_int32), ("n_pix", ctypes.c_int32), ("quat", ctypes.c_void_p), ("mask", ctypes.c_void_p),
    ]


class ProposedView(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in ("G", "P", "b", "L", "S", "Ga", "Pa")]


_lib = None
_P = ctypes.c_void_p
_PB = ctypes.POINTER(Problem)


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libemc.so (built in-tree by paper_1409_4256_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1409_4256_amd.build`")
    lib = ctypes.CDLL(p)
    i32, i64, st = ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    lib.emc_version.restype = ctypes.c_char_p
    lib.emc_last_error.restype = ctypes.c_char_p
    lib.emc_pix_stride.argtypes, lib.emc_pix_stride.restype = [i32], i64
    lib.emc_data_stride.argtypes, lib.emc_data_stride.restype = [i32], i64
    szp = ctypes.POINTER(ctypes.c_size_t)
    for fn in (lib.emc_frames_bytes, lib.emc_slices_bytes, lib.emc_workspace_bytes):
        fn.argtypes, fn.restype = [_PB, szp], st
    lib.emc_pack_frames.argtypes, lib.emc_pack_frames.restype = [_PB, _P, _P, _P], st
    lib.emc_expand.argtypes, lib.emc_expand.restype = [_PB, _P, _P, _P, _P, _P, _P], st
    lib.emc_loglik.argtypes, lib.emc_loglik.restype = [_PB, _P, _P, _P, _P, _P, _P, _P], st
    lib.emc_responsibilities.argtypes = [_PB, _P, _P, _P, i32, _P, _P, _P, _P, _P]
    lib.emc_responsibilities.restype = st
    lib.emc_compress.argtypes = [_PB, _P, _P, _P, _P, _P, _P, i32, _P, ctypes.c_size_t, _P]
    lib.emc_compress.restype = st
    lib.emc_compress_workspace_bytes.argtypes, lib.emc_compress_workspace_bytes.restype = [_PB, szp], st
    lib.emc_finalize.argtypes, lib.emc_finalize.restype = [_PB, _P, _P, _P, _P, _P, i64, _P, _P], st
    lib.emc_iterate.argtypes = [_PB, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    lib.emc_iterate.restype = st
    lib.emc_iterate_noalloc.argtypes = [_PB, _P, _P, _P, _P, _P, _P]
    lib.emc_iterate_noalloc.restype = st
    lib.emc_pack_patterns.argtypes, lib.emc_pack_patterns.restype = [_PB, _P, _P, _P], st
    lib.emc_validate.argtypes, lib.emc_validate.restype = [_PB, _P, _P, _P], st
    lib.emc_cnn_param_count.argtypes, lib.emc_cnn_param_count.restype = [i32], i64
    lib.emc_cnn_workspace_bytes.argtypes, lib.emc_cnn_workspace_bytes.restype = [i32, i32, szp], st
    lib.emc_cnn_preprocess.argtypes, lib.emc_cnn_preprocess.restype = [_PB, _P, _P, _P, i32, _P, _P], st
    lib.emc_cnn_forward.argtypes = [i32, _P, _P, i32, _P, _P, ctypes.c_size_t, _P]
    lib.emc_cnn_forward.restype = st
    lib.emc_cnn_gradients.argtypes = [i32, _P, _P, _P, i32, _P, _P, _P, ctypes.c_size_t, _P]
    lib.emc_cnn_gradients.restype = st
    lib.emc_cnn_adam.argtypes = [i32, _P, _P, _P, _P, i32, ctypes.c_float, _P]
    lib.emc_cnn_adam.restype = st
    lib.emc_cnn_topk.argtypes, lib.emc_cnn_topk.restype = [_P, i64, i32, i32, _P, _P], st
    lib.emc_cell_topk.argtypes, lib.emc_cell_topk.restype = [_P, i64, i32, i32, _P, _P], st
    lib.emc_topk_union.argtypes, lib.emc_topk_union.restype = [_P, i32, _P, i32, i64, i32, _P, _P], st
    lib.emc_cell_targets.argtypes, lib.emc_cell_targets.restype = [_PB, _P, _P, _P, i32, _P, _P], st
    _PP = ctypes.POINTER(Proposal)
    lib.emc_pack_frames_list.argtypes, lib.emc_pack_frames_list.restype = [_PB, _P, _P, _P, _P], st
    lib.emc_proposal_bytes.argtypes, lib.emc_proposal_bytes.restype = [_PB, i32, i32, i32, i64, szp], st
    lib.emc_proposal_build.argtypes = [_PB, _P, i32, _P, i32, _P, i32, _P, i64, _P, ctypes.c_size_t, _PP, _P]
    lib.emc_proposal_build.restype = st
    lib.emc_proposed_workspace_bytes.argtypes = [_PB, _PP, szp]
    lib.emc_proposed_workspace_bytes.restype = st
    lib.emc_iterate_proposed.argtypes = [_PB, _PP, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P, _P]
    lib.emc_iterate_proposed.restype = st
    lib.emc_proposed_accumulate.argtypes = [_PB, _PP, _P, _P, _P, _P, i32, ctypes.c_double, _P, _P, _P,
                                            ctypes.c_size_t, _P, _P]
    lib.emc_proposed_accumulate.restype = st
    lib.emc_proposed_workspace_view.argtypes = [_PB, _PP, ctypes.POINTER(ProposedView)]
    lib.emc_proposed_workspace_view.restype = st
    lib.emc_scatter_plan_min_bytes.argtypes, lib.emc_scatter_plan_min_bytes.restype = [_PB, szp], st
    lib.emc_gaussian_workspace_bytes.argtypes, lib.emc_gaussian_workspace_bytes.restype = [_PB, szp], st
    lib.emc_iterate_gaussian.argtypes = [_PB, ctypes.c_double, _P, _P, _P, i32, _P, _P, _P, _P, ctypes.c_size_t, _P]
    lib.emc_iterate_gaussian.restype = st
    lib.emc_scatter_plan_build.argtypes = [_PB, i32, _P, ctypes.c_size_t, ctypes.POINTER(ScatterPlan), _P]
    lib.emc_scatter_plan_build.restype = st
    _lib = lib
    return lib


def _check(status: int):
    if status != EMC_OK:
        raise EmcError(status, load().emc_last_error().decode())


def _ptr(t, dtype=None, numel=None, name="tensor", allow_none=False, nbytes=None):
    """Device pointer of a contiguous GPU tensor (checked), or None."""
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    import torch

    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} has {t.numel() * t.element_size()} bytes, needs {nbytes}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Geometry:
    """Device-resident problem description (keeps the tensors alive)."""

    def __init__(self, grid_n, q, mask, quat, log_w, n_data, precision=EMC_PREC_FP32):
        import torch

        self.q = q.to(device="cuda", dtype=torch.float32).contiguous()
        self.mask = mask.to(device="cuda", dtype=torch.uint8).contiguous()
        self.quat = quat.to(device="cuda", dtype=torch.float32).contiguous()
        self.log_w = log_w.to(device="cuda", dtype=torch.float64).contiguous()
        self.pb = Problem(int(grid_n), int(self.q.shape[0]), int(self.quat.shape[0]), int(n_data),
                          int(precision), 0, self.q.data_ptr(), self.mask.data_ptr(), self.quat.data_ptr(),
                          self.log_w.data_ptr(), None)
        self.scatter_plan = None   # (ScatterPlan, its device buffer) once built
        self.scatter_buf = None

    def with_frames(self, n_data):
        g = object.__new__(Geometry)
        g.q, g.mask, g.quat, g.log_w = self.q, self.mask, self.quat, self.log_w
        g.scatter_plan, g.scatter_buf = self.scatter_plan, self.scatter_buf
        g.pb = Problem(self.pb.grid_n, self.pb.n_pix, self.pb.n_rot, int(n_data), self.pb.precision, 0,
                       self.pb.q, self.pb.mask, self.pb.quat, self.pb.log_w, self.pb.scatter)
        return g

    def use_brick_scatter(self, chunk=0, stream=None):
        """Build the brick-major c-step plan for this geometry and use it in every
        later call (see emc_scatter_plan_build); returns the plan."""
        plan, buf = emc_scatter_plan_build(self, chunk, stream)
        self.scatter_plan, self.scatter_buf = plan, buf
        self.pb.scatter = ctypes.cast(ctypes.pointer(plan), ctypes.c_void_p)
        return plan

    @property
    def n_pix(self):
        return self.pb.n_pix

    @property
    def n_rot(self):
        return self.pb.n_rot

    @property
    def n_data(self):
        return self.pb.n_data

    @property
    def grid_n(self):
        return self.pb.grid_n

    @property
    def pix_stride(self):
        return emc_pix_stride(self.pb.n_pix)

    @property
    def data_stride(self):
        return emc_data_stride(self.pb.n_data)

    @property
    def bf16(self):
        return self.pb.precision == EMC_PREC_BF16

    @property
    def p_dtype(self):
        """torch dtype of packed frames and responsibilities in this precision."""
        import torch

        return torch.bfloat16 if self.bf16 else torch.float32

    def with_precision(self, precision):
        g = self.with_frames(self.n_data)
        g.pb.precision = int(precision)
        return g


# ------------------------------------------------------------------------- entry points
def emc_version() -> str:
    return load().emc_version().decode()


def emc_pix_stride(n_pix: int) -> int:
    return int(load().emc_pix_stride(int(n_pix)))


def emc_data_stride(n_data: int) -> int:
    return int(load().emc_data_stride(int(n_data)))


def _size_query(fn, geo):
    n = ctypes.c_size_t(0)
    _check(fn(ctypes.byref(geo.pb), ctypes.byref(n)))
    return int(n.value)


def emc_frames_bytes(geo: Geometry) -> int:
    return _size_query(load().emc_frames_bytes, geo)


def emc_slices_bytes(geo: Geometry) -> int:
    return _size_query(load().emc_slices_bytes, geo)


def emc_workspace_bytes(geo: Geometry) -> int:
    return _size_query(load().emc_workspace_bytes, geo)


def frames_tensor(geo: Geometry):
    """An uninitialised device tensor sized for emc_pack_frames' output."""
    import torch

    n = emc_frames_bytes(geo) // (2 if geo.bf16 else 4)
    return torch.empty(max(n, 8), dtype=geo.p_dtype, device="cuda")


def slices_tensor(geo: Geometry):
    import torch

    return torch.empty(max(emc_slices_bytes(geo) // 4, 4), dtype=torch.float32, device="cuda")


def emc_pack_frames(geo: Geometry, counts, K_packed, stream=None):
    import torch

    n = geo.n_data
    _check(load().emc_pack_frames(ctypes.byref(geo.pb),
                                  _ptr(counts, torch.uint16, n * geo.n_pix, "counts") if n else None,
                                  _ptr(K_packed, None, None, "K_packed", nbytes=emc_frames_bytes(geo)) if n else None,
                                  _stream(stream)))


def emc_expand(geo: Geometry, model, c, slices, S, scale=None, stream=None):
    import torch

    _check(load().emc_expand(ctypes.byref(geo.pb), _ptr(model, torch.float32, geo.grid_n ** 3, "model"),
                             _ptr(c, torch.float64, geo.pix_stride, "c"),
                             _ptr(slices, None, None, "slices", nbytes=emc_slices_bytes(geo)),
                             _ptr(S, torch.float64, geo.n_rot, "S"),
                             _ptr(scale, torch.float32, geo.n_rot, "scale", allow_none=not geo.bf16),
                             _stream(stream)))


def emc_loglik(geo: Geometry, K_packed, slices, scale, c, G, b, stream=None):
    import torch

    n = geo.n_data
    if n == 0:
        return
    _check(load().emc_loglik(ctypes.byref(geo.pb), _ptr(K_packed, None, None, "K_packed", nbytes=emc_frames_bytes(geo)),
                             _ptr(slices, None, None, "slices", nbytes=emc_slices_bytes(geo)),
                             _ptr(scale, torch.float32, geo.n_rot, "scale", allow_none=not geo.bf16),
                             _ptr(c, torch.float64, geo.pix_stride, "c"),
                             _ptr(G, torch.float32, geo.n_rot * geo.data_stride, "G"),
                             _ptr(b, torch.float64, n, "b"), _stream(stream)))


def emc_responsibilities(geo: Geometry, G, S, b, mode, stats, P=None, L=None, rho=None, stream=None):
    import torch

    n = geo.n_data
    full = mode != EMC_RESP_PARTIAL
    _check(load().emc_responsibilities(
        ctypes.byref(geo.pb),
        _ptr(G, torch.float32, geo.n_rot * geo.data_stride, "G") if n else None,
        _ptr(S, torch.float64, geo.n_rot, "S"),
        _ptr(b, torch.float64, n, "b") if n else None,
        int(mode),
        _ptr(stats, torch.float64, 2 * n, "stats") if n else None,
        _ptr(P, geo.p_dtype, geo.n_rot * geo.data_stride, "P", allow_none=not full) if n else None,
        _ptr(L, torch.float64, n, "L", allow_none=not full) if n else None,
        _ptr(rho, torch.float64, geo.n_rot, "rho", allow_none=not full),
        _stream(stream)))


def emc_compress_workspace_bytes(geo: Geometry) -> int:
    n = ctypes.c_size_t(0)
    _check(load().emc_compress_workspace_bytes(ctypes.byref(geo.pb), ctypes.byref(n)))
    return int(n.value)


def emc_compress(geo: Geometry, P, K_packed, rho, Wp, num, den, accumulate=False, ws=None, stream=None):
    """ws: None (atomics to num/den) or a uint8 tensor of emc_compress_workspace_bytes (per-XCD grid copies)."""
    import torch

    n = geo.n_data
    M = geo.grid_n ** 3
    _check(load().emc_compress(
        ctypes.byref(geo.pb),
        _ptr(P, geo.p_dtype, geo.n_rot * geo.data_stride, "P") if n else None,
        _ptr(K_packed, None, None, "K_packed", nbytes=emc_frames_bytes(geo)) if n else None,
        _ptr(rho, torch.float64, geo.n_rot, "rho") if n else None,
        _ptr(Wp, torch.float32, geo.n_rot * geo.pix_stride, "Wp") if n else None,
        _ptr(num, torch.float64, M, "num"), _ptr(den, torch.float64, M, "den"), int(bool(accumulate)),
        _ptr(ws, torch.uint8, emc_compress_workspace_bytes(geo), "ws") if ws is not None else None,
        ctypes.c_size_t(ws.numel() if ws is not None else 0), _stream(stream)))


def emc_finalize(geo: Geometry, num, den, model_prev, model_out, L, n_L, loglik, stream=None):
    import torch

    M = geo.grid_n ** 3
    _check(load().emc_finalize(ctypes.byref(geo.pb), _ptr(num, torch.float64, M, "num"),
                               _ptr(den, torch.float64, M, "den"),
                               _ptr(model_prev, torch.float32, M, "model_prev"),
                               _ptr(model_out, torch.float32, M, "model_out"),
                               _ptr(L, torch.float64, n_L, "L") if n_L else None, int(n_L),
                               _ptr(loglik, torch.float64, 1, "loglik"), _stream(stream)))


def emc_iterate(geo: Geometry, model_in, K_packed, model_out, loglik, P_out=None, ws=None, stream=None):
    import torch

    n = geo.n_data
    M = geo.grid_n ** 3
    need = emc_workspace_bytes(geo)
    if ws is None:
        raise ValueError("workspace tensor required (emc_workspace_bytes bytes, uint8)")
    _check(load().emc_iterate(
        ctypes.byref(geo.pb), _ptr(model_in, torch.float32, M, "model_in"),
        _ptr(K_packed, None, None, "K_packed", nbytes=emc_frames_bytes(geo)) if n else None,
        _ptr(model_out, torch.float32, M, "model_out"), _ptr(loglik, torch.float64, 1, "loglik"),
        _ptr(P_out, geo.p_dtype, geo.n_rot * geo.data_stride, "P_out", allow_none=True),
        _ptr(ws, torch.uint8, need, "ws"), ctypes.c_size_t(ws.numel()), _stream(stream)))


def emc_validate(geo: Geometry, model=None, stream=None):
    """Contents check of the geometry (and model): raises EmcError when a quaternion is not
    of unit norm, a weight or used pixel coordinate is not finite, or the model has a
    negative or non-finite value."""
    import torch

    flags = torch.empty(1, dtype=torch.int32, device="cuda")
    _check(load().emc_validate(ctypes.byref(geo.pb),
                               _ptr(model, torch.float32, geo.grid_n ** 3, "model", allow_none=True),
                               _ptr(flags, torch.int32, 1, "flags"), _stream(stream)))


EMC_SCRATCH_MAX_BYTES = 64 << 20    # the static device buffer of emc_iterate_noalloc


def emc_iterate_noalloc(geo: Geometry, model_in, K_packed, model_out, loglik, P_out=None, stream=None):
    """emc_iterate with the library's static device buffer as workspace (no allocation)."""
    import torch

    n = geo.n_data
    M = geo.grid_n ** 3
    _check(load().emc_iterate_noalloc(
        ctypes.byref(geo.pb), _ptr(model_in, torch.float32, M, "model_in"),
        _ptr(K_packed, None, None, "K_packed", nbytes=emc_frames_bytes(geo)) if n else None,
        _ptr(model_out, torch.float32, M, "model_out"), _ptr(loglik, torch.float64, 1, "loglik"),
        _ptr(P_out, geo.p_dtype, geo.n_rot * geo.data_stride, "P_out", allow_none=True), _stream(stream)))


# ------------------------------------------------------------------------- proposal network
def emc_cnn_param_count(n_cells: int) -> int:
    return int(load().emc_cnn_param_count(int(n_cells)))


def emc_cnn_workspace_bytes(n_cells: int, max_batch: int) -> int:
    n = ctypes.c_size_t(0)
    _check(load().emc_cnn_workspace_bytes(int(n_cells), int(max_batch), ctypes.byref(n)))
    return int(n.value)


def emc_cnn_preprocess(geo: Geometry, K_packed, bins, frames, B, x, stream=None):
    import torch

    _check(load().emc_cnn_preprocess(ctypes.byref(geo.pb), _ptr(K_packed, None, None, "K_packed"),
                                     _ptr(bins, torch.int32, geo.n_pix, "bins"),
                                     _ptr(frames, torch.int32, B, "frames", allow_none=True), int(B),
                                     _ptr(x, torch.float32, B * 4096, "x"), _stream(stream)))


def emc_cnn_forward(n_cells, params, x, B, logits, ws, stream=None):
    import torch

    _check(load().emc_cnn_forward(int(n_cells), _ptr(params, torch.float32, emc_cnn_param_count(n_cells), "params"),
                                  _ptr(x, torch.float32, B * 4096, "x"), int(B),
                                  _ptr(logits, torch.float32, B * n_cells, "logits"),
                                  _ptr(ws, torch.uint8, None, "ws"), ctypes.c_size_t(ws.numel()), _stream(stream)))


def emc_cnn_gradients(n_cells, params, x, T, B, grads, loss, ws, stream=None):
    import torch

    n_par = emc_cnn_param_count(n_cells)
    _check(load().emc_cnn_gradients(int(n_cells), _ptr(params, torch.float32, n_par, "params"),
                                    _ptr(x, torch.float32, B * 4096, "x"), _ptr(T, torch.float32, B * n_cells, "T"),
                                    int(B), _ptr(grads, torch.float32, n_par, "grads"),
                                    _ptr(loss, torch.float64, 1, "loss"), _ptr(ws, torch.uint8, None, "ws"),
                                    ctypes.c_size_t(ws.numel()), _stream(stream)))


def emc_cnn_adam(n_cells, params, grads, m, v, step, lr, stream=None):
    import torch

    n_par = emc_cnn_param_count(n_cells)
    _check(load().emc_cnn_adam(int(n_cells), _ptr(params, torch.float32, n_par, "params"),
                               _ptr(grads, torch.float32, n_par, "grads"), _ptr(m, torch.float32, n_par, "m"),
                               _ptr(v, torch.float32, n_par, "v"), int(step), ctypes.c_float(lr), _stream(stream)))


def emc_cnn_topk(logits, rows, n_cells, k, out, stream=None):
    import torch

    _check(load().emc_cnn_topk(_ptr(logits, torch.float32, rows * n_cells, "logits"), int(rows), int(n_cells),
                               int(k), _ptr(out, torch.int32, rows * k, "out"), _stream(stream)))


def emc_cell_topk(T, rows, n_cells, k, out, stream=None):
    import torch

    _check(load().emc_cell_topk(_ptr(T, torch.float32, rows * n_cells, "T"), int(rows), int(n_cells), int(k),
                                _ptr(out, torch.int32, rows * k, "out"), _stream(stream)))


def emc_topk_union(a, ka, b, kb, rows, n_cells, out, stream=None):
    import torch

    _check(load().emc_topk_union(_ptr(a, torch.int32, rows * ka, "a") if ka else None, int(ka),
                                 _ptr(b, torch.int32, rows * kb, "b") if kb else None, int(kb), int(rows),
                                 int(n_cells), _ptr(out, torch.int32, rows * (ka + kb), "out"), _stream(stream)))


def emc_cell_targets(geo: Geometry, P, cell_ptr, cell_rot, n_cells, T, stream=None):
    import torch

    _check(load().emc_cell_targets(ctypes.byref(geo.pb), _ptr(P, geo.p_dtype, geo.n_rot * geo.data_stride, "P"),
                                   _ptr(cell_ptr, torch.int32, n_cells + 1, "cell_ptr"),
                                   _ptr(cell_rot, torch.int32, geo.n_rot, "cell_rot"), int(n_cells),
                                   _ptr(T, torch.float32, geo.n_data * n_cells, "T"), _stream(stream)))


# ------------------------------------------------------------------------- learned-proposal iteration
def emc_pack_frames_list(geo: Geometry, counts, frames, K_packed, stream=None):
    """geo.n_data = number of listed frames; counts is the full [frames][n_pix] array."""
    import torch

    n = geo.n_data
    _check(load().emc_pack_frames_list(ctypes.byref(geo.pb), _ptr(counts, torch.uint16, None, "counts") if n else None,
                                       _ptr(frames, torch.int32, n, "frames") if n else None,
                                       _ptr(K_packed, None, None, "K_packed", nbytes=emc_frames_bytes(geo)) if n else None,
                                       _stream(stream)))


def emc_proposal_bytes(geo: Geometry, n_cells: int, k_top: int, n_audit: int, nz_cap: int) -> int:
    n = ctypes.c_size_t(0)
    _check(load().emc_proposal_bytes(ctypes.byref(geo.pb), int(n_cells), int(k_top), int(n_audit), int(nz_cap),
                                     ctypes.byref(n)))
    return int(n.value)


def emc_proposal_build(geo: Geometry, coarse, n_cells, topk, k_top, audit, counts, nz_cap, buf,
                       stream=None) -> Proposal:
    import torch

    plan = Proposal()
    n_audit = 0 if audit is None else int(audit.numel())
    _check(load().emc_proposal_build(
        ctypes.byref(geo.pb), _ptr(coarse, torch.float32, 4 * n_cells, "coarse"), int(n_cells),
        _ptr(topk, torch.int32, geo.n_data * k_top, "topk"), int(k_top),
        _ptr(audit, torch.int32, n_audit, "audit") if n_audit else None, n_audit,
        _ptr(counts, torch.uint16, geo.n_data * geo.n_pix, "counts"), int(nz_cap),
        _ptr(buf, torch.uint8, emc_proposal_bytes(geo, n_cells, k_top, n_audit, nz_cap), "buf"),
        ctypes.c_size_t(buf.numel()), ctypes.byref(plan), _stream(stream)))
    return plan


def emc_gaussian_workspace_bytes(geo: Geometry) -> int:
    n = ctypes.c_size_t(0)
    _check(load().emc_gaussian_workspace_bytes(ctypes.byref(geo.pb), ctypes.byref(n)))
    return int(n.value)


def emc_iterate_gaussian(geo: Geometry, sigma, model_in, K_packed, phi, phi_from_model, model_out, loglik,
                         P_out=None, ws=None, stream=None):
    """One iteration under the Gaussian model with fluence (FP32 form).  phi: float
    [n_rot * data_stride], read as phi^(n) unless phi_from_model, overwritten with
    phi^(n+1)."""
    import torch

    n = geo.n_data
    M = geo.grid_n ** 3
    nrd = geo.n_rot * geo.data_stride
    _check(load().emc_iterate_gaussian(
        ctypes.byref(geo.pb), ctypes.c_double(float(sigma)), _ptr(model_in, torch.float32, M, "model_in"),
        _ptr(K_packed, None, None, "K_packed", nbytes=emc_frames_bytes(geo)) if n else None,
        _ptr(phi, torch.float32, nrd, "phi") if n else None, int(bool(phi_from_model)),
        _ptr(model_out, torch.float32, M, "model_out"), _ptr(loglik, torch.float64, 1, "loglik"),
        _ptr(P_out, torch.float32, nrd, "P_out", allow_none=True),
        _ptr(ws, torch.uint8, emc_gaussian_workspace_bytes(geo), "ws"), ctypes.c_size_t(ws.numel()),
        _stream(stream)))


def emc_scatter_plan_min_bytes(geo: Geometry) -> int:
    n = ctypes.c_size_t(0)
    _check(load().emc_scatter_plan_min_bytes(ctypes.byref(geo.pb), ctypes.byref(n)))
    return int(n.value)


def emc_scatter_plan_build(geo: Geometry, chunk=0, stream=None):
    """(plan, buf): the brick-major c-step plan for geo's geometry in a device
    buffer sized by a first call that counts the visits."""
    import torch

    lib = load()
    plan = ScatterPlan()
    buf = torch.empty(emc_scatter_plan_min_bytes(geo), dtype=torch.uint8, device="cuda")
    for attempt in range(2):
        status = lib.emc_scatter_plan_build(ctypes.byref(geo.pb), int(chunk), _ptr(buf, torch.uint8, name="buf"),
                                            ctypes.c_size_t(buf.numel()), ctypes.byref(plan), _stream(stream))
        if status == EMC_ERR_WORKSPACE and attempt == 0 and plan.bytes > buf.numel():
            buf = torch.empty(int(plan.bytes), dtype=torch.uint8, device="cuda")
            continue
        _check(status)
        return plan, buf
    raise AssertionError("unreachable")


def emc_proposed_workspace_bytes(geo: Geometry, plan: Proposal) -> int:
    n = ctypes.c_size_t(0)
    _check(load().emc_proposed_workspace_bytes(ctypes.byref(geo.pb), ctypes.byref(plan), ctypes.byref(n)))
    return int(n.value)


EMC_PROPOSED_STAGES = 7
PROPOSED_STAGE_NAMES = ("expand", "cand_loglik", "cand_estep", "audit", "cand_mstep", "dense_mstep", "compress")


def emc_iterate_proposed(geo: Geometry, plan: Proposal, K_audit, model_in, model_out, loglik, recall_mean, ws,
                         stage_events=None, stream=None):
    """stage_events: None or EMC_PROPOSED_STAGES + 1 torch.cuda.Event(enable_timing=True) objects."""
    import torch

    M = geo.grid_n ** 3
    evs = _events(stage_events)
    _check(load().emc_iterate_proposed(
        ctypes.byref(geo.pb), ctypes.byref(plan),
        _ptr(K_audit, None, None, "K_audit") if plan.n_audit else None,
        _ptr(model_in, torch.float32, M, "model_in"), _ptr(model_out, torch.float32, M, "model_out"),
        _ptr(loglik, torch.float64, 1, "loglik"), _ptr(recall_mean, torch.float64, 1, "recall_mean"),
        _ptr(ws, torch.uint8, emc_proposed_workspace_bytes(geo, plan), "ws"),
        ctypes.c_size_t(ws.numel()), evs, _stream(stream)))


def _events(stage_events):
    if stage_events is None:
        return None
    if len(stage_events) != EMC_PROPOSED_STAGES + 1:
        raise ValueError(f"need {EMC_PROPOSED_STAGES + 1} stage events")
    for ev in stage_events:
        if not ev.cuda_event:            # the event is created on its first record
            ev.record()
    return (ctypes.c_void_p * len(stage_events))(*[ctypes.c_void_p(ev.cuda_event) for ev in stage_events])


def emc_proposed_accumulate(geo: Geometry, plan: Proposal, K_audit, model_in, num, den, accumulate, recall_min, L,
                            recall_mean, ws, stage_events=None, stream=None):
    """One frame chunk of the restricted iteration into num/den (added only when the
    chunk's audit recall reaches recall_min); L [n_data] per-frame log-evidence."""
    import torch

    M = geo.grid_n ** 3
    _check(load().emc_proposed_accumulate(
        ctypes.byref(geo.pb), ctypes.byref(plan),
        _ptr(K_audit, None, None, "K_audit") if plan.n_audit else None,
        _ptr(model_in, torch.float32, M, "model_in"), _ptr(num, torch.float64, M, "num"),
        _ptr(den, torch.float64, M, "den"), int(bool(accumulate)), ctypes.c_double(float(recall_min)),
        _ptr(L, torch.float64, geo.n_data, "L"), _ptr(recall_mean, torch.float64, 1, "recall_mean"),
        _ptr(ws, torch.uint8, emc_proposed_workspace_bytes(geo, plan), "ws"), ctypes.c_size_t(ws.numel()),
        _events(stage_events), _stream(stream)))


def emc_proposed_workspace_view(geo: Geometry, plan: Proposal) -> ProposedView:
    v = ProposedView()
    _check(load().emc_proposed_workspace_view(ctypes.byref(geo.pb), ctypes.byref(plan), ctypes.byref(v)))
    return v


def plan_array(buf, address: int, n: int, dtype):
    """A tensor view of n elements of a plan array (device address inside `buf`)."""
    import torch

    off = int(address) - buf.data_ptr()
    size = torch.empty(0, dtype=dtype).element_size()
    return buf[off:off + n * size].view(dtype)
