"""ctypes binding of libekm (include/ekm.h): argument marshalling only.

Every function takes torch tensors that already live on the GPU, passes their
device pointers and the current HIP stream to the C ABI, and raises
``EKMError`` with ``kmeans_last_error()`` on a non-OK status.  No step of the
computation runs here; if the library is missing this module raises instead
of falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libekm.so")

KM_OK, KM_ERR_INVALID, KM_ERR_OOM, KM_ERR_HIP, KM_ERR_UNSUPPORTED, KM_ERR_NOT_EXACT = range(6)
KM_F64, KM_F32 = 0, 1
KM_BRUTE, KM_INDEXED = 0, 1
KM_FLAG_SSE = 1
KM_FLAG_TIMING = 2
KM_FLAG_SMALL_LISTS = 4
KM_FLAG_CELL_LEAVES = 8
PHASES = ("tree", "assign", "deferred", "update")

EXPORTED = ("kmeans_workspace_bytes", "kmeans_context_info", "kmeans_context_features", "kmeans_predictor_create",
            "kmeans_predictor_destroy", "kmeans_predictor_add_run", "kmeans_predictor_fit",
            "kmeans_predictor_predict", "kmeans_predictor_begin", "kmeans_predictor_observe", "kmeans_init", "kmeans_init_batched", "kmeans_step", "kmeans_run",
            "kmeans_run_batched", "kmeans_destroy", "kmeans_phase_times", "kmeans_step_times", "distortion_fwd", "distortion_bwd", "distortion_bwd_noalloc",
            "kmeans_last_error")


class EKMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ekm status {status}: {msg}")
        self.status = status


class KmConfig(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("point_dtype", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("cand_tile", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("workspace_limit_bytes", ctypes.c_int64)]


class KmCtxInfo(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_int64), ("model_bytes", ctypes.c_int64),
                ("model_bytes_actual_counts", ctypes.c_int64), ("leaves", ctypes.c_int64),
                ("groups", ctypes.c_int64), ("allocations", ctypes.c_int64), ("leaf_size", ctypes.c_int32),
                ("leaves_per_group", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class KmIterStats(ctypes.Structure):
    _fields_ = [("n_changed", ctypes.c_int64), ("dist_evals", ctypes.c_int64), ("brute_evals", ctypes.c_int64),
                ("single_cand_points", ctypes.c_int64), ("rechecked", ctypes.c_int64),
                ("cand_total", ctypes.c_int64), ("leaves", ctypes.c_int64), ("sse", ctypes.c_double),
                ("inter_leaf_points", ctypes.c_int64), ("inter_points", ctypes.c_int64),
                ("fallback_points", ctypes.c_int64), ("deferred_leaves", ctypes.c_int64),
                ("group_overflows", ctypes.c_int64), ("groups_skipped", ctypes.c_int64),
                ("region_points", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libekm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2412_02244_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.kmeans_workspace_bytes.argtypes = [ctypes.POINTER(KmConfig), I64, I64]
    lib.kmeans_workspace_bytes.restype = ctypes.c_size_t
    lib.kmeans_context_info.argtypes = [P, ctypes.POINTER(KmCtxInfo)]
    D, DP = ctypes.c_double, ctypes.POINTER(ctypes.c_double)
    lib.kmeans_context_features.argtypes = [P, DP, I32, ctypes.POINTER(I32)]
    lib.kmeans_predictor_create.argtypes = [ctypes.POINTER(P), I32, I32, I32, D, D]
    lib.kmeans_predictor_destroy.argtypes = [P]
    lib.kmeans_predictor_add_run.argtypes = [P, DP, DP, I32]
    lib.kmeans_predictor_fit.argtypes = [P]
    lib.kmeans_predictor_predict.argtypes = [P, DP, ctypes.POINTER(I32), DP, DP]
    lib.kmeans_predictor_begin.argtypes = [P, DP]
    lib.kmeans_predictor_observe.argtypes = [P, I32, D, DP, DP]
    lib.kmeans_init.argtypes = [ctypes.POINTER(P), ctypes.POINTER(KmConfig), P, I64, I64, P]
    lib.kmeans_init_batched.argtypes = [ctypes.POINTER(P), ctypes.POINTER(KmConfig), P, ctypes.POINTER(I64),
                                        ctypes.POINTER(I64), I32, P]
    lib.kmeans_run_batched.argtypes = [P, ctypes.POINTER(I64), P, ctypes.POINTER(I64), P, I32,
                                       ctypes.POINTER(KmConfig), I32, P, ctypes.POINTER(I32)]
    lib.kmeans_step.argtypes = [P, P, P, P, ctypes.POINTER(KmIterStats)]
    lib.kmeans_run.argtypes = [P, P, P, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(KmIterStats)]
    lib.kmeans_destroy.argtypes = [P]
    lib.kmeans_phase_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
    lib.kmeans_step_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), I64, ctypes.POINTER(I64)]
    lib.distortion_fwd.argtypes = [P, P, I32, I64, I64, I64, I32, P, P, P]
    lib.distortion_bwd.argtypes = [P, P, P, P, I32, I64, I64, I64, I32, P, P, P]
    lib.distortion_bwd_noalloc.argtypes = [P, P, P, P, I32, I64, I64, I64, I32, P, P, P]
    lib.kmeans_last_error.restype = ctypes.c_char_p
    for name in ("kmeans_context_info", "kmeans_context_features", "kmeans_predictor_create",
                 "kmeans_predictor_destroy", "kmeans_predictor_add_run", "kmeans_predictor_fit",
                 "kmeans_predictor_predict", "kmeans_predictor_begin", "kmeans_predictor_observe", "kmeans_init", "kmeans_init_batched", "kmeans_run_batched", "kmeans_step", "kmeans_run",
                 "kmeans_destroy", "kmeans_phase_times", "kmeans_step_times", "distortion_fwd", "distortion_bwd",
                 "distortion_bwd_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def kmeans_last_error() -> str:
    return load_library().kmeans_last_error().decode()


def _check(status: int):
    if status != KM_OK:
        raise EKMError(status, kmeans_last_error())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, name: str, dtype=None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _pt_dtype(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return KM_F32
    if t.dtype == torch.float64:
        return KM_F64
    raise ValueError(f"points must be float32 or float64, got {t.dtype}")


def kmeans_workspace_bytes(n: int, k: int, d: int, point_dtype: int = KM_F32, algo: int = KM_INDEXED,
                           leaf_size: int = 0, cand_tile: int = 0, flags: int = 0,
                           workspace_limit_bytes: int = 0) -> int:
    """Modelled device workspace of kmeans_init (0 for an invalid configuration)."""
    cfg = KmConfig(d, point_dtype, algo, leaf_size, cand_tile, flags, workspace_limit_bytes)
    return int(load_library().kmeans_workspace_bytes(ctypes.byref(cfg), n, k))


def kmeans_context_info(ctx: "Context") -> dict:
    """Device bytes held, the model's prediction, leaf size and counts of a context."""
    info = KmCtxInfo()
    _check(load_library().kmeans_context_info(ctypes.c_void_p(ctx.handle), ctypes.byref(info)))
    return info.as_dict()


class Context:
    """Owns a km_ctx; released by ``kmeans_destroy`` (or when collected).

    The library launches a context's work on the stream that was current at
    ``kmeans_init``; the step calls check that it is still torch's current
    stream, so that their inputs and outputs stay ordered with the caller's
    work."""

    def __init__(self, handle: int, n: int, k: int, d: int):
        self.handle, self.n, self.k, self.d = handle, n, k, d
        self.stream = _stream()

    def check_stream(self):
        if _stream() != self.stream:
            raise ValueError("the current stream differs from the one this context was created on; "
                             "switch back to it (torch.cuda.stream) before stepping the context")

    def close(self):
        if self.handle:
            _check(load_library().kmeans_destroy(ctypes.c_void_p(self.handle)))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kmeans_init(points: torch.Tensor, k: int, algo: int = KM_INDEXED, leaf_size: int = 0, cand_tile: int = 0,
                flags: int = 0, workspace_limit_bytes: int = 0) -> Context:
    """Create a context over ``points`` ([n, d] float32/float64 on the GPU)."""
    if points.dim() != 2:
        raise ValueError("points must be [n, d]")
    n, d = points.shape
    cfg = KmConfig(d, _pt_dtype(points), algo, leaf_size, cand_tile, flags, workspace_limit_bytes)
    h = ctypes.c_void_p()
    _check(load_library().kmeans_init(ctypes.byref(h), ctypes.byref(cfg), _dev(points, "points"), n, k,
                                      _stream()))
    return Context(h.value, n, k, d)


def _offsets(offs, name: str, B: int):
    """Host int64 array of B + 1 offsets (a list, a tuple or a CPU tensor)."""
    if isinstance(offs, torch.Tensor):
        if offs.is_cuda:
            raise ValueError(f"{name} must be host memory")
        offs = offs.tolist()
    offs = [int(v) for v in offs]
    if len(offs) != B + 1:
        raise ValueError(f"{name} must hold B + 1 = {B + 1} offsets, got {len(offs)}")
    return (ctypes.c_int64 * len(offs))(*offs)


def kmeans_init_batched(points: torch.Tensor, pt_offs, c_offs, algo: int = KM_INDEXED, leaf_size: int = 0,
                        cand_tile: int = 0, flags: int = 0, workspace_limit_bytes: int = 0) -> Context:
    """One context over B clouds: cloud b owns points ``pt_offs[b]:pt_offs[b+1]`` of ``points``
    ([n, d] on the GPU) and centroids ``c_offs[b]:c_offs[b+1]`` of the centroid array."""
    if points.dim() != 2:
        raise ValueError("points must be [n, d]")
    n, d = points.shape
    B = len(pt_offs) - 1
    po, co = _offsets(pt_offs, "pt_offs", B), _offsets(c_offs, "c_offs", B)
    cfg = KmConfig(d, _pt_dtype(points), algo, leaf_size, cand_tile, flags, workspace_limit_bytes)
    h = ctypes.c_void_p()
    _check(load_library().kmeans_init_batched(ctypes.byref(h), ctypes.byref(cfg), _dev(points, "points"), po, co, B,
                                              _stream()))
    return Context(h.value, n, co[B], d)


def kmeans_run_batched(points: torch.Tensor, pt_offs, c_inout: torch.Tensor, c_offs, iters: int,
                       algo: int = KM_INDEXED, leaf_size: int = 0, cand_tile: int = 0,
                       assign_out: torch.Tensor | None = None):
    """``iters`` Lloyd iterations of every cloud, in place on ``c_inout``; returns the (f, G) used
    (the tuned ones where ``leaf_size`` / ``cand_tile`` are 0)."""
    if points.dim() != 2:
        raise ValueError("points must be [n, d]")
    d = points.shape[1]
    B = len(pt_offs) - 1
    po, co = _offsets(pt_offs, "pt_offs", B), _offsets(c_offs, "c_offs", B)
    cfg = KmConfig(d, _pt_dtype(points), algo, leaf_size, cand_tile, 0, 0)
    tuned = (ctypes.c_int32 * 2)()
    _check(load_library().kmeans_run_batched(
        _dev(points, "points"), po, _dev(c_inout, "c_inout", torch.float64), co,
        None if assign_out is None else _dev(assign_out, "assign_out", torch.int32), B, ctypes.byref(cfg), iters,
        _stream(), tuned))
    return tuned[0], tuned[1]


def kmeans_context_features(ctx: Context) -> list:
    """Meta-features of a context: ln n, ln k, d, ln f, ln(points per leaf), ln(leaves), ln(groups),
    centroid-tree levels."""
    buf = (ctypes.c_double * 16)()
    nf = ctypes.c_int32(0)
    _check(load_library().kmeans_context_features(ctypes.c_void_p(ctx.handle), buf, 16, ctypes.byref(nf)))
    return [buf[i] for i in range(nf.value)]


def _dvec(v):
    v = [float(x) for x in v]
    return (ctypes.c_double * max(1, len(v)))(*v)


class Predictor:
    """Runtime predictor (iteration-number regressor, per-iteration polynomial regressor,
    asymmetric-kernel GP adjustment); host-side, in the library."""

    def __init__(self, q: int, nfeat: int, order: int = 2, sigma: float = 2.0, noise: float = 1e-2):
        self.q, self.nfeat = q, nfeat
        h = ctypes.c_void_p()
        _check(load_library().kmeans_predictor_create(ctypes.byref(h), q, nfeat, order, sigma, noise))
        self.handle = h.value

    def close(self):
        if self.handle:
            load_library().kmeans_predictor_destroy(ctypes.c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_run(self, feat, iter_ms):
        _check(load_library().kmeans_predictor_add_run(ctypes.c_void_p(self.handle), _dvec(feat), _dvec(iter_ms),
                                                       len(iter_ms)))

    def fit(self):
        _check(load_library().kmeans_predictor_fit(ctypes.c_void_p(self.handle)))

    def predict(self, feat):
        """-> (iterations, per-iteration ms [q], total ms)"""
        it = ctypes.c_int32(0)
        per = (ctypes.c_double * self.q)()
        tot = ctypes.c_double(0.0)
        _check(load_library().kmeans_predictor_predict(ctypes.c_void_p(self.handle), _dvec(feat), ctypes.byref(it),
                                                       per, ctypes.byref(tot)))
        return it.value, list(per), tot.value

    def begin(self, feat):
        _check(load_library().kmeans_predictor_begin(ctypes.c_void_p(self.handle), _dvec(feat)))

    def observe(self, iteration: int, ms: float):
        """-> (remaining ms, total ms)"""
        rem, tot = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(load_library().kmeans_predictor_observe(ctypes.c_void_p(self.handle), iteration, ms,
                                                       ctypes.byref(rem), ctypes.byref(tot)))
        return rem.value, tot.value


def kmeans_step(ctx: Context, c_in: torch.Tensor, c_out: torch.Tensor | None = None,
                assign_out: torch.Tensor | None = None, stats: bool = False):
    """One Lloyd iteration; returns ``c_out`` (and a stats dict when ``stats``)."""
    ctx.check_stream()
    if c_out is None:
        c_out = torch.empty_like(c_in)
    st = KmIterStats()
    _check(load_library().kmeans_step(
        ctypes.c_void_p(ctx.handle), _dev(c_in, "c_in", torch.float64), _dev(c_out, "c_out", torch.float64),
        None if assign_out is None else _dev(assign_out, "assign_out", torch.int32),
        ctypes.byref(st) if stats else None))
    return (c_out, st.as_dict()) if stats else c_out


def kmeans_run(ctx: Context, c_inout: torch.Tensor, max_iter: int, stop_when_stable: bool = False,
               assign_out: torch.Tensor | None = None, per_iter: bool = False):
    """Up to ``max_iter`` iterations in place on ``c_inout``; returns (iterations, [stats])."""
    ctx.check_stream()
    arr = (KmIterStats * max(1, max_iter))() if per_iter else None
    it = ctypes.c_int32(0)
    _check(load_library().kmeans_run(
        ctypes.c_void_p(ctx.handle), _dev(c_inout, "c_inout", torch.float64),
        None if assign_out is None else _dev(assign_out, "assign_out", torch.int32),
        max_iter, int(bool(stop_when_stable)), ctypes.byref(it), arr))
    stats = [arr[i].as_dict() for i in range(it.value)] if per_iter else None
    return it.value, stats


def kmeans_destroy(ctx: Context):
    ctx.close()


def kmeans_phase_times(ctx: Context):
    """GPU milliseconds per phase summed since the last call -> (dict, steps)."""
    ms = (ctypes.c_double * len(PHASES))()
    steps = ctypes.c_int64(0)
    _check(load_library().kmeans_phase_times(ctypes.c_void_p(ctx.handle), ms, ctypes.byref(steps)))
    return {name: ms[i] for i, name in enumerate(PHASES)}, steps.value


def kmeans_step_times(ctx: Context, cap: int = 4096):
    """GPU milliseconds per phase of each recorded step -> list of dicts (oldest first)."""
    ms = (ctypes.c_double * (max(1, cap) * len(PHASES)))()
    steps = ctypes.c_int64(0)
    _check(load_library().kmeans_step_times(ctypes.c_void_p(ctx.handle), ms, cap, ctypes.byref(steps)))
    n = min(steps.value, cap)
    return [{name: ms[s * len(PHASES) + i] for i, name in enumerate(PHASES)} for s in range(n)]


def distortion_fwd(x: torch.Tensor, c: torch.Tensor):
    """``x [B,n,d]``, ``c [B,k,d]`` -> ``(assign int32 [B,n], loss float64 [B])``."""
    if x.dim() != 3 or c.dim() != 3 or x.shape[0] != c.shape[0] or x.shape[2] != c.shape[2]:
        raise ValueError("x must be [B,n,d] and c [B,k,d]")
    if x.dtype != c.dtype:
        raise ValueError("x and c must have the same dtype")
    B, n, d = x.shape
    k = c.shape[1]
    a = torch.empty((B, n), dtype=torch.int32, device=x.device)
    loss = torch.empty(B, dtype=torch.float64, device=x.device)
    _check(load_library().distortion_fwd(_dev(x, "x"), _dev(c, "c"), _pt_dtype(x), B, n, k, d, a.data_ptr(),
                                         loss.data_ptr(), _stream()))
    return a, loss


def distortion_bwd(x: torch.Tensor, c: torch.Tensor, assign: torch.Tensor, grad_loss: torch.Tensor,
                   need_x: bool = True, need_c: bool = True):
    """Gradients of ``sum_b grad_loss[b] * L_b`` -> ``(grad_x or None, grad_c or None)``."""
    B, n, d = x.shape
    k = c.shape[1]
    gx = torch.empty_like(x) if need_x else None
    gc = torch.empty_like(c) if need_c else None
    _check(load_library().distortion_bwd(
        _dev(x, "x"), _dev(c, "c"), _dev(assign, "assign", torch.int32), _dev(grad_loss, "grad_loss", torch.float64),
        _pt_dtype(x), B, n, k, d, None if gx is None else gx.data_ptr(), None if gc is None else gc.data_ptr(),
        _stream()))
    return gx, gc


def distortion_bwd_noalloc(x: torch.Tensor, c: torch.Tensor, assign: torch.Tensor, grad_loss: torch.Tensor,
                           grad_x: torch.Tensor | None, grad_c: torch.Tensor | None):
    """``distortion_bwd`` into caller-provided outputs, with no allocation in the library."""
    B, n, d = x.shape
    k = c.shape[1]
    _check(load_library().distortion_bwd_noalloc(
        _dev(x, "x"), _dev(c, "c"), _dev(assign, "assign", torch.int32), _dev(grad_loss, "grad_loss", torch.float64),
        _pt_dtype(x), B, n, k, d, None if grad_x is None else _dev(grad_x, "grad_x", x.dtype),
        None if grad_c is None else _dev(grad_c, "grad_c", c.dtype), _stream()))
    return grad_x, grad_c


class Distortion(torch.autograd.Function):
    """Per-cloud distortion ``L_b = sum_i ||x_i - c_a(i)||^2`` (FP64 values, Eq. (1)).

    ``forward(x [B,n,d], c [B,k,d]) -> loss [B] float64``; the nearest-centroid
    assignment is saved and held fixed in backward.
    """

    @staticmethod
    def forward(ctx, x, c):
        x = x.contiguous()
        c = c.contiguous()
        a, loss = distortion_fwd(x, c)
        ctx.save_for_backward(x, c, a)
        ctx.mark_non_differentiable(a)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        x, c, a = ctx.saved_tensors
        g = grad_loss.to(torch.float64).contiguous()
        gx, gc = distortion_bwd(x, c, a, g, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return gx, gc
