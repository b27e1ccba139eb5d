"""Python binding of the GridShift HIP library (``libgridshift.so``).

Argument marshalling only: every step of the fit runs in the library's
kernels on the GPU.  PyTorch supplies device memory (tensors) and the stream
(``torch.cuda.current_stream()``).  The C ABI is declared in
``include/gridshift.h``; the method is GridShift (arXiv 2206.02200,
Section 2.1, Algorithm 1, parallel update Eq. 6).

If the library has not been built, every call raises ``RuntimeError``: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgridshift.so")

GS_F32, GS_F64 = 0, 1
CONVERGED, STATIONARY, CAPPED = 1, 2, 4
STATUS = {
    0: "GS_OK", 1: "GS_ERR_INVALID_ARG", 2: "GS_ERR_NONFINITE", 3: "GS_ERR_KEY_RANGE",
    4: "GS_ERR_ALLOC", 5: "GS_ERR_DEVICE", 6: "GS_ERR_UNSUPPORTED", 7: "GS_ERR_STATE",
}
EXPORTED = [
    "gs_abi_version", "gs_last_error", "gs_context_create", "gs_context_destroy",
    "gs_ctx_fit", "gs_ctx_fit_batched", "gs_copy_modes", "gs_copy_keys",
    "gs_fit", "gs_fit_batched", "gs_result_info", "gs_result_offsets", "gs_result_copy", "gs_backward",
    "gs_point_mode_loss", "gs_point_mode_loss_backward", "gs_result_free",
    "gs_profile_enable", "gs_profile_reset", "gs_profile_count", "gs_profile_entry",
    "gs_context_set_tape", "gs_ctx_backward", "gs_ctx_point_mode_loss", "gs_ctx_point_mode_loss_backward",
    "gs_context_set_config", "gs_context_get_config", "gs_autotune",
    "gs_context_set_update", "gs_context_get_update", "gs_fit_hsweep", "gs_track",
    "gs_track_batched", "gs_fit_noalloc",
]
CFG_MERGE_SMALL, CFG_TILE_CHUNKS, CFG_DENSE_TABLE, CFG_SORT_DIGIT10, CFG_SORT_TILE = 0, 1, 2, 3, 4
CONFIG_KEYS = {"merge_small": CFG_MERGE_SMALL, "tile_chunks": CFG_TILE_CHUNKS, "dense_table": CFG_DENSE_TABLE,
               "sort_digit10": CFG_SORT_DIGIT10, "sort_tile": CFG_SORT_TILE}
UPDATE_RULES = {"parallel": 0, "sequential": 1}  # gs_context_set_update


class GridShiftError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """gs_allocator"""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    """gs_problem"""
    _fields_ = [("points", ctypes.c_void_p), ("dtype", ctypes.c_int), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("ld", ctypes.c_int64), ("h", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32)]


# device memory of results from torch's caching allocator (counted, for tests)
ALLOC_STATS = {"allocs": 0, "frees": 0, "bytes": 0}


def _torch_alloc(ctx, nbytes, stream):
    try:
        p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # out of memory: the library reports GS_ERR_ALLOC
        return None
    ALLOC_STATS["allocs"] += 1
    ALLOC_STATS["bytes"] += int(nbytes)
    return p


def _torch_free(ctx, p, stream):
    torch.cuda.caching_allocator_delete(int(p))
    ALLOC_STATS["frees"] += 1


TORCH_ALLOCATOR = Allocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)


class Info(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_int64),
        ("n_cells0", ctypes.c_int64),
        ("n_clusters", ctypes.c_int64),
        ("n_iter", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {"n_points": self.n_points, "n_cells0": self.n_cells0, "n_clusters": self.n_clusters,
                "n_iter": self.n_iter, "flags": self.flags}


_lib = None
_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:  # loaded once per process
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(
                f"GridShift HIP library not found at {path}; build it with "
                "`python paper_2206_02200_amd/build.py` (no CPU fallback exists)")
        lib = ctypes.CDLL(path)
        V, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.gs_abi_version.restype = I32
        lib.gs_last_error.restype = ctypes.c_char_p
        lib.gs_context_create.argtypes = [ctypes.POINTER(V)]
        lib.gs_context_create.restype = ctypes.c_int
        lib.gs_context_destroy.argtypes = [V]
        lib.gs_context_destroy.restype = None
        lib.gs_fit.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Allocator), V, V, ctypes.POINTER(V)]
        lib.gs_fit.restype = ctypes.c_int
        lib.gs_fit_batched.argtypes = [V, ctypes.c_int, I32, I32, V, V, I32, I32, ctypes.POINTER(Allocator), V, V,
                                       ctypes.POINTER(V)]
        lib.gs_fit_batched.restype = ctypes.c_int
        lib.gs_result_info.argtypes = [V, I32, ctypes.POINTER(Info)]
        lib.gs_result_info.restype = ctypes.c_int
        lib.gs_result_offsets.argtypes = [V, V]
        lib.gs_result_offsets.restype = ctypes.c_int
        lib.gs_result_copy.argtypes = [V, V, V, V]
        lib.gs_result_copy.restype = ctypes.c_int
        lib.gs_backward.argtypes = [V, V, V, V]
        lib.gs_backward.restype = ctypes.c_int
        lib.gs_point_mode_loss.argtypes = [V, V, V, V]
        lib.gs_point_mode_loss.restype = ctypes.c_int
        lib.gs_point_mode_loss_backward.argtypes = [V, V, V, V, V]
        lib.gs_point_mode_loss_backward.restype = ctypes.c_int
        lib.gs_result_free.argtypes = [V]
        lib.gs_fit_noalloc.restype = ctypes.c_int
        lib.gs_fit_noalloc.argtypes = [ctypes.POINTER(Problem), V, V, V, V, I64, ctypes.POINTER(Info)]
        lib.gs_result_free.restype = None
        lib.gs_ctx_fit.argtypes = [V, V, ctypes.c_int, I64, I32, I64, D, I32, V, ctypes.POINTER(Info), V]
        lib.gs_ctx_fit.restype = ctypes.c_int
        lib.gs_ctx_fit_batched.argtypes = [V, V, ctypes.c_int, I32, I64, I32, V, V, I32, V, V, V]
        lib.gs_ctx_fit_batched.restype = ctypes.c_int
        lib.gs_fit_hsweep.argtypes = [V, V, ctypes.c_int, I64, I32, I64, I32, V, I32, V, V, V]
        lib.gs_fit_hsweep.restype = ctypes.c_int
        lib.gs_track.argtypes = [V, V, ctypes.c_int, I32, I32, I32, I32, V, D, D, D, D, D, I32, I32, I32, V, V]
        lib.gs_track.restype = ctypes.c_int
        lib.gs_track_batched.argtypes = [V, V, ctypes.c_int, I32, I32, I32, I32, I32, V, V, V, D, D, D, I32, I32, I32,
                                         V, V]
        lib.gs_track_batched.restype = ctypes.c_int
        lib.gs_copy_modes.argtypes = [V, V, V, V, V]
        lib.gs_copy_modes.restype = ctypes.c_int
        lib.gs_copy_keys.argtypes = [V, V, V]
        lib.gs_copy_keys.restype = ctypes.c_int
        lib.gs_profile_enable.argtypes = [V, ctypes.c_char_p]
        lib.gs_profile_enable.restype = ctypes.c_int
        lib.gs_profile_reset.argtypes = [V]
        lib.gs_profile_reset.restype = ctypes.c_int
        lib.gs_profile_count.argtypes = [V]
        lib.gs_profile_count.restype = I32
        lib.gs_profile_entry.argtypes = [V, I32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(D),
                                         ctypes.POINTER(I64), ctypes.POINTER(D)]
        lib.gs_profile_entry.restype = ctypes.c_int
        lib.gs_context_set_tape.argtypes = [V, I32]
        lib.gs_context_set_tape.restype = ctypes.c_int
        lib.gs_ctx_backward.argtypes = [V, V, V, V]
        lib.gs_ctx_backward.restype = ctypes.c_int
        lib.gs_ctx_point_mode_loss.argtypes = [V, V, V, V, V]
        lib.gs_ctx_point_mode_loss.restype = ctypes.c_int
        lib.gs_ctx_point_mode_loss_backward.argtypes = [V, V, V, V, V, V]
        lib.gs_ctx_point_mode_loss_backward.restype = ctypes.c_int
        lib.gs_context_set_update.argtypes = [V, I32]
        lib.gs_context_set_update.restype = ctypes.c_int
        lib.gs_context_get_update.argtypes = [V, ctypes.POINTER(I32)]
        lib.gs_context_get_update.restype = ctypes.c_int
        lib.gs_context_set_config.argtypes = [V, I32, I32]
        lib.gs_context_set_config.restype = ctypes.c_int
        lib.gs_context_get_config.argtypes = [V, I32, ctypes.POINTER(I32)]
        lib.gs_context_get_config.restype = ctypes.c_int
        lib.gs_autotune.argtypes = [V, V, ctypes.c_int, I32, I64, I32, V, V, I32, I32, V]
        lib.gs_autotune.restype = ctypes.c_int
        _lib = lib
        return lib


def _check(rc: int):
    if rc != 0:
        raise GridShiftError(rc, _lib.gs_last_error().decode())


class Context:
    """Owns a ``gs_context`` (device scratch memory reused across fits)."""

    def __init__(self, device: int | None = None):
        lib = load_library()
        self.device = torch.cuda.current_device() if device is None else device
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            _check(lib.gs_context_create(ctypes.byref(h)))
        self.handle = h

    def set_tape(self, on: bool | int = True):
        """Record the trajectory of later fits (needed by the backward calls).

        True or 1 records every round; an integer k > 1 saves the tail's cell
        table every k rounds instead and recomputes each k-round segment
        during the backward pass; False or 0 records nothing."""
        _check(_lib.gs_context_set_tape(self.handle, int(on)))

    def set_update(self, rule: str = "parallel"):
        """Update rule of later fits: "parallel" (Eq. 6, the default) or
        "sequential" (Eq. 5, cells moved colour by colour, each colour reading
        the centroids the earlier colours just moved)."""
        if rule not in UPDATE_RULES:
            raise ValueError(f"unknown update rule {rule!r}")
        _check(_lib.gs_context_set_update(self.handle, UPDATE_RULES[rule]))

    def update_rule(self) -> str:
        v = ctypes.c_int32()
        _check(_lib.gs_context_get_update(self.handle, ctypes.byref(v)))
        return {i: k for k, i in UPDATE_RULES.items()}[v.value]

    def set_config(self, **kv):
        """Launch choices (merge_small=0/1, tile_chunks=1..64, dense_table=0/1, sort_digit10=0/1,
        sort_tile=8192/4096); results never depend on them."""
        for k, v in kv.items():
            _check(_lib.gs_context_set_config(self.handle, CONFIG_KEYS[k], int(v)))

    def config(self) -> dict:
        out = {}
        for k, key in CONFIG_KEYS.items():
            v = ctypes.c_int32()
            _check(_lib.gs_context_get_config(self.handle, key, ctypes.byref(v)))
            out[k] = v.value
        return out

    def autotune(self, x: torch.Tensor, h, max_iter: int = 100, offsets=None, reps: int = 3, stream=None) -> dict:
        """Time every candidate configuration on this input and keep the fastest."""
        x, dt, ld = _points(x)
        n, d = x.shape
        off = np.ascontiguousarray(np.asarray([0, n] if offsets is None else offsets, dtype=np.int64))
        B = off.size - 1
        hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (B,)))
        _check(_lib.gs_autotune(self.handle, ctypes.c_void_p(x.data_ptr()), dt, d, ld, B,
                                off.ctypes.data_as(ctypes.c_void_p), hs.ctypes.data_as(ctypes.c_void_p),
                                int(max_iter), int(reps), _stream_ptr(stream)))
        return self.config()

    def profile(self, prefix: str | None = ""):
        """Time later fits' kernels whose name starts with ``prefix`` (None: off)."""
        _check(_lib.gs_profile_enable(self.handle, None if prefix is None else prefix.encode()))

    def profile_reset(self):
        _check(_lib.gs_profile_reset(self.handle))

    def profile_table(self) -> dict:
        """{kernel: {"ms": total, "launches": n, "bytes": algorithmic bytes}}"""
        out = {}
        for i in range(_lib.gs_profile_count(self.handle)):
            name, ms, nl, by = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
            _check(_lib.gs_profile_entry(self.handle, i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(nl),
                                         ctypes.byref(by)))
            out[name.value.decode()] = {"ms": ms.value, "launches": nl.value, "bytes": by.value}
        return out

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib.gs_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict[int, Context] = {}


def default_context(device: int | None = None) -> Context:
    dev = torch.cuda.current_device() if device is None else device
    ctx = _contexts.get(dev)
    if ctx is None:
        ctx = Context(dev)
        _contexts[dev] = ctx
    return ctx


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        if _raw_stream is not None:  # the current stream's handle, without building a Stream object
            return ctypes.c_void_p(_raw_stream(torch.cuda.current_device()))
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _points(x: torch.Tensor) -> tuple[torch.Tensor, int, int]:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("points must be a CUDA (HIP) tensor")
    if x.dim() != 2:
        raise ValueError("points must be [n, d]")
    if x.dtype == torch.float32:
        dt = GS_F32
    elif x.dtype == torch.float64:
        dt = GS_F64
    else:
        raise TypeError("points must be float32 or float64")
    if x.stride(1) != 1:
        x = x.contiguous()
    ld = x.stride(0) if x.shape[0] > 1 else x.shape[1]
    return x, dt, max(ld, x.shape[1])


@dataclass
class FitResult:
    labels: torch.Tensor  # int32 [n]
    modes: torch.Tensor  # float64 [K, d]
    counts: torch.Tensor  # int64 [K]
    info: dict
    sums: torch.Tensor | None = None  # float64 [K, d]
    keys: torch.Tensor | None = None  # int64 [K, d]


def fit(x: torch.Tensor, h: float, max_iter: int = 100, *, with_sums: bool = False, with_keys: bool = False,
        ctx: Context | None = None, stream=None) -> FitResult:
    """GridShift of one point set ``x`` ([n, d] float32/float64 on the GPU)."""
    lib = load_library()
    x, dt, ld = _points(x)
    n, d = x.shape
    ctx = ctx or default_context(x.device.index)
    sp = _stream_ptr(stream)
    labels = torch.empty(n, dtype=torch.int32, device=x.device)
    info = Info()
    _check(lib.gs_ctx_fit(ctx.handle, ctypes.c_void_p(x.data_ptr()), dt, n, d, ld, float(h), int(max_iter),
                      ctypes.c_void_p(labels.data_ptr()), ctypes.byref(info), sp))
    K = info.n_clusters
    modes = torch.empty((K, d), dtype=torch.float64, device=x.device)
    counts = torch.empty(K, dtype=torch.int64, device=x.device)
    sums = torch.empty((K, d), dtype=torch.float64, device=x.device) if with_sums else None
    _check(lib.gs_copy_modes(ctx.handle, ctypes.c_void_p(modes.data_ptr()), ctypes.c_void_p(counts.data_ptr()),
                             ctypes.c_void_p(sums.data_ptr() if sums is not None else 0), sp))
    keys = None
    if with_keys:
        keys = torch.empty((K, d), dtype=torch.int64, device=x.device)
        _check(lib.gs_copy_keys(ctx.handle, ctypes.c_void_p(keys.data_ptr()), sp))
    return FitResult(labels, modes, counts, info.as_dict(), sums, keys)


@dataclass
class BatchedResult:
    labels: torch.Tensor  # int32 [N], per-instance ids
    modes: torch.Tensor  # float64 [sum K, d]
    counts: torch.Tensor  # int64 [sum K]
    k_offsets: np.ndarray  # int64 [B+1]
    infos: list
    sums: torch.Tensor | None = None


def fit_batched(x: torch.Tensor, offsets, h, max_iter: int = 100, *, with_sums: bool = False,
                ctx: Context | None = None, stream=None) -> BatchedResult:
    """GridShift of B independent point sets concatenated in ``x``; instance b
    owns rows offsets[b]..offsets[b+1]-1 and uses bandwidth h[b]."""
    lib = load_library()
    x, dt, ld = _points(x)
    d = x.shape[1]
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    B = off.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (B,)))
    if off[-1] != x.shape[0]:
        raise ValueError("offsets[-1] must equal the number of rows")
    ctx = ctx or default_context(x.device.index)
    sp = _stream_ptr(stream)
    labels = torch.empty(x.shape[0], dtype=torch.int32, device=x.device)
    infos = (Info * B)()
    _check(lib.gs_ctx_fit_batched(ctx.handle, ctypes.c_void_p(x.data_ptr()), dt, d, ld, B,
                              off.ctypes.data_as(ctypes.c_void_p), hs.ctypes.data_as(ctypes.c_void_p), int(max_iter),
                              ctypes.c_void_p(labels.data_ptr()), ctypes.cast(infos, ctypes.c_void_p), sp))
    ks = np.array([infos[b].n_clusters for b in range(B)], dtype=np.int64)
    koff = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    tot = int(koff[-1])
    modes = torch.empty((tot, d), dtype=torch.float64, device=x.device)
    counts = torch.empty(tot, dtype=torch.int64, device=x.device)
    sums = torch.empty((tot, d), dtype=torch.float64, device=x.device) if with_sums else None
    _check(lib.gs_copy_modes(ctx.handle, ctypes.c_void_p(modes.data_ptr()), ctypes.c_void_p(counts.data_ptr()),
                             ctypes.c_void_p(sums.data_ptr() if sums is not None else 0), sp))
    return BatchedResult(labels, modes, counts, koff, [infos[b].as_dict() for b in range(B)], sums)


def fit_hsweep(x: torch.Tensor, hs, max_iter: int = 100, *, with_sums: bool = False,
               ctx: Context | None = None, stream=None) -> BatchedResult:
    """The point set ``x`` fitted once per bandwidth in ``hs``, all in one
    batched pass; labels come back as [H, n], the cluster rows of bandwidth j
    at k_offsets[j]..k_offsets[j+1]-1."""
    lib = load_library()
    x, dt, ld = _points(x)
    n, d = x.shape
    hv = np.ascontiguousarray(np.asarray(hs, dtype=np.float64).ravel())
    H = hv.size
    ctx = ctx or default_context(x.device.index)
    sp = _stream_ptr(stream)
    labels = torch.empty((H, n), dtype=torch.int32, device=x.device)
    infos = (Info * H)()
    _check(lib.gs_fit_hsweep(ctx.handle, ctypes.c_void_p(x.data_ptr()), dt, n, d, ld, H,
                             hv.ctypes.data_as(ctypes.c_void_p), int(max_iter), ctypes.c_void_p(labels.data_ptr()),
                             ctypes.cast(infos, ctypes.c_void_p), sp))
    ks = np.array([infos[j].n_clusters for j in range(H)], dtype=np.int64)
    koff = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    tot = int(koff[-1])
    modes = torch.empty((tot, d), dtype=torch.float64, device=x.device)
    counts = torch.empty(tot, dtype=torch.int64, device=x.device)
    sums = torch.empty((tot, d), dtype=torch.float64, device=x.device) if with_sums else None
    _check(lib.gs_copy_modes(ctx.handle, ctypes.c_void_p(modes.data_ptr()), ctypes.c_void_p(counts.data_ptr()),
                             ctypes.c_void_p(sums.data_ptr() if sums is not None else 0), sp))
    return BatchedResult(labels, modes, counts, koff, [infos[j].as_dict() for j in range(H)], sums)


def track(frames: torch.Tensor, o0, l0: float, w0: float, f: float, h: float, eta: float, max_inner: int = 20,
          n_select: int = 1, max_iter: int = 100, *, ctx: Context | None = None, stream=None) -> np.ndarray:
    """Object tracking (Algorithm 2) through ``frames`` ([T, H, W, dc] float32
    or float64 colour features on the GPU); returns the windows
    (o_x, o_y, l, w) of every frame as a float64 [T, 4] array."""
    lib = load_library()
    if frames.dim() != 4 or not frames.is_cuda:
        raise ValueError("frames must be a [T, H, W, dc] GPU tensor")
    if frames.dtype == torch.float32:
        dt = GS_F32
    elif frames.dtype == torch.float64:
        dt = GS_F64
    else:
        raise TypeError("frames must be float32 or float64")
    frames = frames.contiguous()
    T, H, W, dc = frames.shape
    ctx = ctx or default_context(frames.device.index)
    o = np.ascontiguousarray(np.asarray(o0, dtype=np.float64).ravel()[:2])
    out = np.empty((T, 4), np.float64)
    _check(lib.gs_track(ctx.handle, ctypes.c_void_p(frames.data_ptr()), dt, T, H, W, dc,
                        o.ctypes.data_as(ctypes.c_void_p), float(l0), float(w0), float(f), float(h), float(eta),
                        int(max_inner), int(n_select), int(max_iter), out.ctypes.data_as(ctypes.c_void_p),
                        _stream_ptr(stream)))
    return out


def track_batched(frames: torch.Tensor, o0, l0, w0, f: float, h: float, eta: float, max_inner: int = 20,
                  n_select: int = 1, max_iter: int = 100, *, ctx: Context | None = None, stream=None) -> np.ndarray:
    """Several objects tracked through the same ``frames`` at once (one
    workgroup per track): ``o0`` [ntracks, 2], ``l0`` and ``w0`` [ntracks];
    returns the windows as a float64 [ntracks, T, 4] array, bitwise those of
    ``track`` run per object."""
    lib = load_library()
    if frames.dim() != 4 or not frames.is_cuda:
        raise ValueError("frames must be a [T, H, W, dc] GPU tensor")
    if frames.dtype == torch.float32:
        dt = GS_F32
    elif frames.dtype == torch.float64:
        dt = GS_F64
    else:
        raise TypeError("frames must be float32 or float64")
    frames = frames.contiguous()
    T, H, W, dc = frames.shape
    o = np.ascontiguousarray(np.asarray(o0, dtype=np.float64).reshape(-1, 2))
    nt = o.shape[0]
    lv = np.ascontiguousarray(np.broadcast_to(np.asarray(l0, dtype=np.float64), (nt,)))
    wv = np.ascontiguousarray(np.broadcast_to(np.asarray(w0, dtype=np.float64), (nt,)))
    ctx = ctx or default_context(frames.device.index)
    out = np.empty((nt, T, 4), np.float64)
    _check(lib.gs_track_batched(ctx.handle, ctypes.c_void_p(frames.data_ptr()), dt, T, H, W, dc, nt,
                                o.ctypes.data_as(ctypes.c_void_p), lv.ctypes.data_as(ctypes.c_void_p),
                                wv.ctypes.data_as(ctypes.c_void_p), float(f), float(h), float(eta), int(max_inner),
                                int(n_select), int(max_iter), out.ctypes.data_as(ctypes.c_void_p),
                                _stream_ptr(stream)))
    return out


class Result:
    """A gs_result: one fit's (or one batched fit's) cluster tables and, when
    recorded, its trajectory; its device memory comes from torch's caching
    allocator (or hipMalloc with ``allocator=None``) until ``close``."""

    def __init__(self, handle, B: int, d: int, labels: torch.Tensor, stream, dtype: int, ld: int):
        self.handle, self.B, self.d, self.labels, self._stream = handle, B, d, labels, stream
        # the loss calls read the points with the fit's row stride and type
        self._dtype, self._ld = dtype, ld

    def _same_points(self, x: torch.Tensor) -> torch.Tensor:
        x, dt, ld = _points(x)
        if dt != self._dtype or ld != self._ld or x.shape != (self.labels.numel(), self.d):
            raise ValueError(f"the loss needs the points in the fit's layout: [{self.labels.numel()}, {self.d}] "
                             f"rows of stride {self._ld}, dtype code {self._dtype} (got {tuple(x.shape)}, "
                             f"stride {ld}, dtype code {dt})")
        return x

    def info(self, b: int = 0) -> dict:
        out = Info()
        _check(_lib.gs_result_info(self.handle, int(b), ctypes.byref(out)))
        return out.as_dict()

    def offsets(self) -> np.ndarray:
        k = np.empty(self.B + 1, np.int64)
        _check(_lib.gs_result_offsets(self.handle, k.ctypes.data_as(ctypes.c_void_p)))
        return k

    def copy(self):
        """(modes float64 [sum K, d], counts int64 [sum K])"""
        tot = int(self.offsets()[-1])
        dev = self.labels.device
        modes = torch.empty((tot, self.d), dtype=torch.float64, device=dev)
        counts = torch.empty(tot, dtype=torch.int64, device=dev)
        _check(_lib.gs_result_copy(self.handle, _vp(modes), _vp(counts), self._stream))
        return modes, counts

    def backward(self, grad_modes: torch.Tensor) -> torch.Tensor:
        g = grad_modes.to(torch.float64).contiguous()
        out = torch.empty((self.labels.numel(), self.d), dtype=torch.float64, device=g.device)
        _check(_lib.gs_backward(self.handle, _vp(g), _vp(out), self._stream))
        return out

    def loss(self, x: torch.Tensor) -> torch.Tensor:
        x = self._same_points(x)
        out = torch.empty(self.B, dtype=torch.float64, device=x.device)
        _check(_lib.gs_point_mode_loss(self.handle, _vp(x), _vp(out), self._stream))
        return out

    def loss_backward(self, x: torch.Tensor, grad_loss: torch.Tensor) -> torch.Tensor:
        x = self._same_points(x)
        gl = grad_loss.to(torch.float64).contiguous()
        out = torch.empty((self.labels.numel(), self.d), dtype=torch.float64, device=x.device)
        _check(_lib.gs_point_mode_loss_backward(self.handle, _vp(x), _vp(gl), _vp(out), self._stream))
        return out

    def close(self):
        if self.handle:
            _lib.gs_result_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit_result(x: torch.Tensor, h: float, max_iter: int = 100, ckpt_every: int = 0, *, allocator="torch",
               stream=None) -> Result:
    """gs_fit: one point set, its result object owning the fit's memory."""
    lib = load_library()
    x, dt, ld = _points(x)
    n, d = x.shape
    labels = torch.empty(n, dtype=torch.int32, device=x.device)
    p = Problem(ctypes.c_void_p(x.data_ptr()), dt, n, d, ld, float(h), int(max_iter), int(ckpt_every))
    out = ctypes.c_void_p()
    al = ctypes.byref(TORCH_ALLOCATOR) if allocator == "torch" else None
    sp = _stream_ptr(stream)
    _check(lib.gs_fit(ctypes.byref(p), al, sp, ctypes.c_void_p(labels.data_ptr()), ctypes.byref(out)))
    return Result(out, 1, d, labels, sp, dt, ld)


def fit_batched_result(x: torch.Tensor, offsets, h, max_iter: int = 100, ckpt_every: int = 0, *,
                       allocator="torch", stream=None) -> Result:
    """gs_fit_batched: B concatenated dense point sets, one result object."""
    lib = load_library()
    x, dt, ld = _points(x)
    d = x.shape[1]
    if ld != d:
        raise ValueError("gs_fit_batched takes dense rows")
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    B = off.size - 1
    hs = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (B,)))
    labels = torch.empty(x.shape[0], dtype=torch.int32, device=x.device)
    out = ctypes.c_void_p()
    al = ctypes.byref(TORCH_ALLOCATOR) if allocator == "torch" else None
    sp = _stream_ptr(stream)
    _check(lib.gs_fit_batched(ctypes.c_void_p(x.data_ptr()), dt, d, B, off.ctypes.data_as(ctypes.c_void_p),
                              hs.ctypes.data_as(ctypes.c_void_p), int(max_iter), int(ckpt_every), al, sp,
                              ctypes.c_void_p(labels.data_ptr()), ctypes.byref(out)))
    return Result(out, B, d, labels, sp, dt, ld)


NOALLOC_MAX_POINTS = 131072  # GS_NOALLOC_MAX_POINTS


def fit_noalloc(x: torch.Tensor, h: float, max_iter: int = 100, *, labels: torch.Tensor | None = None,
                modes: torch.Tensor | None = None, counts: torch.Tensor | None = None, stream=None) -> FitResult:
    """gs_fit_noalloc: a plain fit whose device scratch is the library's fixed
    array (no allocation inside the call).  The output tensors may be passed
    in (labels int32 [n], modes float64 [k, d], counts int64 [k]); missing ones
    are created here, with room for n clusters.  Returns views of the K rows."""
    lib = load_library()
    x, dt, ld = _points(x)
    n, d = x.shape
    dev = x.device
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
    if modes is None:
        modes = torch.empty((max(n, 1), d), dtype=torch.float64, device=dev)
    if counts is None:
        counts = torch.empty(modes.shape[0], dtype=torch.int64, device=dev)
    kcap = min(modes.shape[0], counts.shape[0])
    p = Problem(ctypes.c_void_p(x.data_ptr()), dt, n, d, ld, float(h), int(max_iter), 0)
    info = Info()
    _check(lib.gs_fit_noalloc(ctypes.byref(p), _stream_ptr(stream), _vp(labels), _vp(modes), _vp(counts), kcap,
                              ctypes.byref(info)))
    K = info.n_clusters
    return FitResult(labels, modes[:K], counts[:K], info.as_dict())


# ---------------------------------------------------------------------------
# differentiable form
# ---------------------------------------------------------------------------
def _vp(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def backward_modes(ctx: Context, grad_modes: torch.Tensor, n: int, d: int, stream=None) -> torch.Tensor:
    """Gradient of sum(grad_modes * modes) with respect to the points of the
    context's last (recorded) fit; float64 [n, d]."""
    g = grad_modes.to(torch.float64).contiguous()
    out = torch.empty((n, d), dtype=torch.float64, device=g.device)
    _check(_lib.gs_ctx_backward(ctx.handle, _vp(g), _vp(out), _stream_ptr(stream)))
    return out


def point_mode_loss_values(ctx: Context, x: torch.Tensor, labels: torch.Tensor, B: int, stream=None) -> torch.Tensor:
    """Per-instance loss sum_i ||x_i - mode(label_i)||^2 of the last recorded fit."""
    x, _, _ = _points(x)
    loss = torch.empty(B, dtype=torch.float64, device=x.device)
    _check(_lib.gs_ctx_point_mode_loss(ctx.handle, _vp(x), _vp(labels), _vp(loss), _stream_ptr(stream)))
    return loss


def point_mode_loss_grad(ctx: Context, x: torch.Tensor, labels: torch.Tensor, grad_loss: torch.Tensor,
                         stream=None) -> torch.Tensor:
    """Gradient of sum_b grad_loss[b] * L_b with respect to the points (float64)."""
    x, _, _ = _points(x)
    gl = grad_loss.to(torch.float64).contiguous()
    out = torch.empty(x.shape, dtype=torch.float64, device=x.device)
    _check(_lib.gs_ctx_point_mode_loss_backward(ctx.handle, _vp(x), _vp(labels), _vp(gl), _vp(out),
                                            _stream_ptr(stream)))
    return out


def _fit_any(x, offsets, h, max_iter, ctx):
    if offsets is None:
        r = fit(x, h, max_iter, ctx=ctx)
        return r.labels, r.modes, r.counts, np.array([0, r.modes.shape[0]], dtype=np.int64), [r.info]
    r = fit_batched(x, offsets, h, max_iter, ctx=ctx)
    return r.labels, r.modes, r.counts, r.k_offsets, r.infos


class GridShiftModes(torch.autograd.Function):
    """modes, labels, counts = GridShiftModes.apply(x, h, max_iter, offsets, ctx)

    Forward: the GridShift fit of x (one point set, or B concatenated ones when
    ``offsets`` is given), recording its trajectory.  Backward: the adjoint of
    the shift-and-merge rounds with that trajectory held fixed.  labels and
    counts are not differentiable.  A context, if given, must not run another
    fit before the backward pass."""

    @staticmethod
    def forward(actx, x, h, max_iter=100, offsets=None, ctx=None, ckpt_every=1):
        gctx = ctx or Context(x.device.index)
        gctx.set_tape(ckpt_every)
        labels, modes, counts, koff, infos = _fit_any(x, offsets, h, max_iter, gctx)
        actx.gctx = gctx
        actx.shape = tuple(x.shape)
        actx.x_dtype = x.dtype
        actx.mark_non_differentiable(labels, counts)
        return modes, labels, counts

    @staticmethod
    def backward(actx, g_modes, g_labels, g_counts):
        n, d = actx.shape
        grad = backward_modes(actx.gctx, g_modes, n, d)
        return grad.to(actx.x_dtype), None, None, None, None, None


class PointModeLoss(torch.autograd.Function):
    """loss = PointModeLoss.apply(x, h, max_iter, offsets, ctx)

    loss[b] = sum over the points of instance b of ||x_i - mode(label_i)||^2
    after a GridShift fit; the gradient holds the fit's trajectory fixed (the
    direct term 2 (x_i - mode) plus the adjoint of the modes)."""

    @staticmethod
    def forward(actx, x, h, max_iter=100, offsets=None, ctx=None, ckpt_every=1):
        gctx = ctx or Context(x.device.index)
        gctx.set_tape(ckpt_every)
        labels, modes, counts, koff, infos = _fit_any(x, offsets, h, max_iter, gctx)
        B = 1 if offsets is None else len(offsets) - 1
        loss = point_mode_loss_values(gctx, x, labels, B)
        actx.gctx = gctx
        actx.save_for_backward(x, labels)
        actx.x_dtype = x.dtype
        return loss

    @staticmethod
    def backward(actx, g_loss):
        x, labels = actx.saved_tensors
        grad = point_mode_loss_grad(actx.gctx, x, labels, g_loss)
        return grad.to(actx.x_dtype), None, None, None, None, None


def point_mode_loss(x, h, max_iter=100, offsets=None, ctx=None, ckpt_every=1):
    """Differentiable point-to-mode loss (per instance, float64).  ckpt_every
    > 1 keeps tail checkpoints every that many rounds instead of the whole
    trajectory (same gradient, recomputed segment by segment)."""
    return PointModeLoss.apply(x, h, max_iter, offsets, ctx, ckpt_every)


def gridshift_modes(x, h, max_iter=100, offsets=None, ctx=None, ckpt_every=1):
    """Differentiable modes (float64) with labels and counts."""
    return GridShiftModes.apply(x, h, max_iter, offsets, ctx, ckpt_every)
