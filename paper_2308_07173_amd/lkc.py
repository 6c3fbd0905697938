"""Thin Python binding of ``liblkc.so`` (the C ABI in ``include/lkc.h``).

Argument marshalling only: every step of the search and covariance runs in
the HIP kernels of the library.  Torch is used for device memory and
streams -- tensors are passed by ``data_ptr()`` and every call is enqueued
on ``torch.cuda.current_stream()``.  If the library is not built, or no
gfx950 device is present, the calls raise; there is no CPU fallback.

The functions keep the C names (``lkc_build_target``, ``lkc_knn_query``,
``lkc_covariances``, ``lkc_knn_cov``, ``lkc_knn_cov_batched`` ...); the
``Context`` / ``Target`` / ``TargetSet`` classes own the C objects.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading
from dataclasses import dataclass
from typing import Dict, Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblkc.so")

LKC_OK = 0
LKC_ERR_INVALID_ARG = -1
LKC_ERR_OOM = -2
LKC_ERR_HIP = -3
LKC_ERR_BUDGET = -4
LKC_ERR_NONFINITE = -5
LKC_ERR_UNSUPPORTED = -6
LKC_MAX_K = 64

_STATUS_NAMES = {0: "LKC_OK", -1: "LKC_ERR_INVALID_ARG", -2: "LKC_ERR_OOM", -3: "LKC_ERR_HIP",
                 -4: "LKC_ERR_BUDGET", -5: "LKC_ERR_NONFINITE", -6: "LKC_ERR_UNSUPPORTED",
                 -7: "LKC_ERR_DEGENERATE"}

# every symbol include/lkc.h declares
EXPORTED_SYMBOLS = (
    "lkc_version", "lkc_ctx_create", "lkc_ctx_destroy", "lkc_ctx_set_stream", "lkc_last_error",
    "lkc_synchronize", "lkc_build_target", "lkc_target_rebuild", "lkc_target_rebuild_async",
    "lkc_target_free",
    "lkc_target_get_info", "lkc_target_arrays", "lkc_knn_query", "lkc_covariances",
    "lkc_knn_cov", "lkc_target_set_create", "lkc_target_set_free", "lkc_target_set_stage",
    "lkc_knn_cov_batched", "lkc_knn_cov_self", "lkc_ctx_reserve", "lkc_ctx_search_stats",
    "lkc_ctx_set_timing", "lkc_ctx_set_profile", "lkc_covariances_weighted",
    "lkc_knn_cov_weighted", "lkc_gicp_linearize", "lkc_gicp_align", "lkc_voxel_filter",
    "lkc_submap_extract", "lkc_submap_build", "lkc_zvote", "lkc_euclid_cluster",
    "lkc_target_status", "lkc_autotune", "lkc_knn_cov_noalloc", "lkc_raceline_build",
    "lkc_raceline_free", "lkc_raceline_get_info", "lkc_raceline_bins", "lkc_submap_window",
    "lkc_submap_window_build", "lkc_voxel_filter_async", "lkc_euclid_cluster_async",
    "lkc_calib_gather",
)

# window statuses (info[2] of lkc_submap_window)
LKC_WINDOW_OK = 0
LKC_WINDOW_NO_BIN = 1
LKC_WINDOW_UNCOVERED = 2
LKC_WINDOW_OVERFLOW = 3

# neighbour weight kernels of lkc_covariances_weighted / lkc_knn_cov_weighted
WEIGHT_KERNELS = {"none": 0, "rbf": 1, "gaussian": 2, "laplacian": 3}


class LkcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class LaunchCfg(ctypes.Structure):
    _fields_ = [("algorithm", ctypes.c_int32), ("group_reach", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("merge_min", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("group_split", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TargetInfo(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_cells", ctypes.c_int64),
                ("hash_capacity", ctypes.c_int64), ("cell_min", ctypes.c_int32 * 3),
                ("cell_max", ctypes.c_int32 * 3), ("key_bits", ctypes.c_int32),
                ("sort_passes", ctypes.c_int32), ("cell_size", ctypes.c_float),
                ("device_bytes", ctypes.c_int64)]


class SearchStats(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_int64), ("fallback_queries", ctypes.c_int64),
                ("sort_ms", ctypes.c_float), ("group_ms", ctypes.c_float),
                ("fallback_ms", ctypes.c_float), ("reduce_ms", ctypes.c_float)]


class AutotuneResult(ctypes.Structure):
    _fields_ = [("cell_size", ctypes.c_float), ("cfg_index", ctypes.c_int32),
                ("cfg", LaunchCfg), ("ms", ctypes.c_float), ("reserved", ctypes.c_int32),
                ("sample", ctypes.c_int64)]


class RaceLineInfo(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int64), ("n_ranges", ctypes.c_int64),
                ("pose_cells", ctypes.c_int64), ("max_bin_points", ctypes.c_int64),
                ("sum_bin_points", ctypes.c_int64), ("bin_length", ctypes.c_float),
                ("pose_grid", ctypes.c_float), ("radius", ctypes.c_float),
                ("lateral", ctypes.c_float), ("cover_radius", ctypes.c_float),
                ("reserved", ctypes.c_int32), ("device_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class ScanDesc(ctypes.Structure):
    _fields_ = [("q_offset", ctypes.c_int64), ("q_count", ctypes.c_int64),
                ("target_index", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GicpStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("correspondences", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("error", ctypes.c_double), ("last_step", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


GICP_SYSTEM_WORDS = 45

_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``liblkc.so``; raises if it has not been built."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run `python __graft_entry__.py build` "
                               "(or paper_2308_07173_amd/build_lib.py) first")
        lib = ctypes.CDLL(path)
        P, I32, I64, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        PP = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "lkc_version": ([], I32),
            "lkc_ctx_create": ([P, PP], I32),
            "lkc_ctx_destroy": ([P], I32),
            "lkc_ctx_set_stream": ([P, P], I32),
            "lkc_last_error": ([P], ctypes.c_char_p),
            "lkc_synchronize": ([P], I32),
            "lkc_build_target": ([P, P, I64, F, PP], I32),
            "lkc_target_rebuild": ([P, P, P, I64], I32),
            "lkc_target_rebuild_async": ([P, P, P, I64], I32),
            "lkc_target_free": ([P, P], I32),
            "lkc_target_get_info": ([P, ctypes.POINTER(TargetInfo)], I32),
            "lkc_target_arrays": ([P, PP, PP, PP], I32),
            "lkc_knn_query": ([P, P, P, I64, I32, F, P, P, P, P], I32),
            "lkc_covariances": ([P, P, P, P, P, I64, I32, F, P, P, P, P], I32),
            "lkc_knn_cov": ([P, P, P, I64, I32, F, F, P, P, P, P, P, P, P, P], I32),
            "lkc_knn_cov_noalloc": ([P, P, P, I64, I32, F, F, P, P, P, P, P, P, P, P], I32),
            "lkc_target_set_create": ([P, P, I32, I32, PP], I32),
            "lkc_target_set_free": ([P, P], I32),
            "lkc_target_set_stage": ([P, P, P, I32], I32),
            "lkc_knn_cov_batched": ([P, P, P, I64, I32, F, F, P, P, P, P, P, P, P, P], I32),
            "lkc_knn_cov_self": ([P, P, I32, F, F, P, P, P, P, P, P, P, P], I32),
            "lkc_ctx_reserve": ([P, I64], I32),
            "lkc_ctx_search_stats": ([P, P], I32),
            "lkc_ctx_set_timing": ([P, I32], I32),
            "lkc_calib_gather": ([P, P, I64, P, I64, P], I32),
            "lkc_ctx_set_profile": ([P, P, I64], I32),
            "lkc_covariances_weighted": ([P, P, P, P, P, I64, I32, I32, F, F, P, P, P, P], I32),
            "lkc_knn_cov_weighted": ([P, P, P, I64, I32, F, I32, F, F, P, P, P, P, P, P, P, P],
                                     I32),
            "lkc_gicp_linearize": ([P, P, P, P, P, I64, P, F, P, P, P], I32),
            "lkc_gicp_align": ([P, P, P, P, P, I64, P, F, I32, ctypes.c_double, P,
                                ctypes.POINTER(GicpStats), P], I32),
            "lkc_voxel_filter": ([P, P, I64, P, F, P, P, P, I64, ctypes.POINTER(ctypes.c_int64)],
                                 I32),
            "lkc_voxel_filter_async": ([P, P, I64, P, F, I32, P, P, P, I64, P, P], I32),
            "lkc_euclid_cluster_async": ([P, P, I64, F, P, P, P, P], I32),
            "lkc_submap_extract": ([P, P, P, F, P, I64, ctypes.POINTER(ctypes.c_int64)], I32),
            "lkc_submap_build": ([P, P, P, F, P, I64, ctypes.POINTER(ctypes.c_int64), PP], I32),
            "lkc_zvote": ([P, P, I64, F, I32, P, P], I32),
            "lkc_euclid_cluster": ([P, P, I64, F, P, P, ctypes.POINTER(ctypes.c_int64)], I32),
            "lkc_target_status": ([P, P], I32),
            "lkc_raceline_build": ([P, P, P, I64, F, F, F, PP], I32),
            "lkc_raceline_free": ([P, P], I32),
            "lkc_raceline_get_info": ([P, ctypes.POINTER(RaceLineInfo)], I32),
            "lkc_raceline_bins": ([P, P, P], I32),
            "lkc_submap_window": ([P, P, P, F, P, P, I64, P], I32),
            "lkc_submap_window_build": ([P, P, P, F, P, I64, ctypes.POINTER(ctypes.c_int64),
                                         PP], I32),
            "lkc_autotune": ([P, P, I64, P, I64, I32, F, F, P, I32, P, I32, I64,
                              ctypes.c_uint64, I32, P, ctypes.POINTER(AutotuneResult)], I32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_dev(t, name, dtype=None, shape_tail=None):
    torch = _torch()
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [*, {shape_tail}], got {tuple(t.shape)}")
    del torch


def _cfg_ptr(cfg) -> Optional[ctypes.POINTER(LaunchCfg)]:
    if cfg is None:
        return None
    if isinstance(cfg, dict):
        c = LaunchCfg(**{k: int(v) for k, v in cfg.items()})
    else:
        c = cfg
    return ctypes.byref(c)


class Context:
    """Owns an ``lkc_ctx``; every call rebinds it to torch's current stream."""

    def __init__(self):
        torch = _torch()
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.lkc_ctx_create(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                     ctypes.byref(h))
        if st != LKC_OK:
            raise LkcError(st, self.lib.lkc_last_error(None).decode())
        self.handle = h

    def _bind(self):
        torch = _torch()
        self.lib.lkc_ctx_set_stream(self.handle,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))

    def check(self, st: int):
        if st != LKC_OK:
            raise LkcError(st, self.lib.lkc_last_error(self.handle).decode())

    def reserve(self, max_queries: int):
        self._bind()
        self.check(self.lib.lkc_ctx_reserve(self.handle, int(max_queries)))

    def search_stats(self) -> Dict:
        """Queries, fallback queries and (with timing on) phase GPU times of
        the last search (synchronises)."""
        st = SearchStats()
        self._bind()
        self.check(self.lib.lkc_ctx_search_stats(self.handle, ctypes.byref(st)))
        return {"queries": st.queries, "fallback_queries": st.fallback_queries,
                "sort_ms": st.sort_ms, "group_ms": st.group_ms, "fallback_ms": st.fallback_ms,
                "reduce_ms": st.reduce_ms}

    def set_profile(self, buf=None):
        """Per-group counters of the group search into `buf` (device int32
        tensor [groups, 25]) or off (None)."""
        if buf is None:
            self.check(self.lib.lkc_ctx_set_profile(self.handle, None, 0))
        else:
            self.check(self.lib.lkc_ctx_set_profile(self.handle, ctypes.c_void_p(buf.data_ptr()),
                                                    buf.shape[0]))

    def set_timing(self, on: bool):
        self.check(self.lib.lkc_ctx_set_timing(self.handle, 1 if on else 0))

    def calib_gather(self, src, idx, dst):
        """dst[i] = src[idx[i]] over float32 [*, 4] rows (device tensors;
        idx int32 holding row numbers), on the context's stream."""
        self._bind()
        assert src.dim() == 2 and src.shape[1] == 4 and dst.shape == (idx.shape[0], 4)
        self.check(self.lib.lkc_calib_gather(
            self.handle, ctypes.c_void_p(src.data_ptr()), src.shape[0],
            ctypes.c_void_p(idx.data_ptr()), idx.shape[0], ctypes.c_void_p(dst.data_ptr())))

    def synchronize(self):
        self._bind()
        self.check(self.lib.lkc_synchronize(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lkc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass


class Target:
    """A built ``lkc_target`` (device-resident hashed voxel grid)."""

    def __init__(self, ctx: Context, handle: ctypes.c_void_p):
        self.ctx = ctx
        self.handle = handle

    def info(self) -> Dict:
        inf = TargetInfo()
        self.ctx.check(self.ctx.lib.lkc_target_get_info(self.handle, ctypes.byref(inf)))
        return dict(n_points=inf.n_points, n_cells=inf.n_cells,
                    hash_capacity=inf.hash_capacity, cell_min=list(inf.cell_min),
                    cell_max=list(inf.cell_max), key_bits=inf.key_bits,
                    sort_passes=inf.sort_passes, cell_size=inf.cell_size,
                    device_bytes=inf.device_bytes)

    def arrays(self):
        """(pts float4 [n,4], cell_start int32 [C+1], cell_keys int64 [C]) copied to host."""
        torch = _torch()
        a, b, c = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        self.ctx.check(self.ctx.lib.lkc_target_arrays(self.handle, ctypes.byref(a),
                                                      ctypes.byref(b), ctypes.byref(c)))
        inf = self.info()
        n, C = inf["n_points"], inf["n_cells"]
        self.ctx.synchronize()
        pts = _copy_device(a.value, 16 * n, torch.float32).view(n, 4) if n else \
            torch.zeros(0, 4)
        cs = _copy_device(b.value, 4 * (C + 1), torch.int32)
        ck = _copy_device(c.value, 8 * C, torch.int64) if C else torch.zeros(0, dtype=torch.int64)
        return pts, cs, ck

    def rebuild(self, points, sync: bool = True):
        """lkc_target_rebuild, or with sync=False lkc_target_rebuild_async
        (no host round trip; errors surface at status() or the next call
        that needs the host-side layout)."""
        _check_dev(points, "points", _torch().float32, (3,))
        self.ctx._bind()
        fn = self.ctx.lib.lkc_target_rebuild if sync else self.ctx.lib.lkc_target_rebuild_async
        self.ctx.check(fn(self.ctx.handle, self.handle, ctypes.c_void_p(_ptr(points)),
                          points.shape[0]))

    def status(self) -> int:
        """lkc_target_status: LKC_OK, or the error of the last (re)build
        that left the target empty (synchronises)."""
        self.ctx._bind()
        return int(self.ctx.lib.lkc_target_status(self.ctx.handle, self.handle))

    def free(self):
        if self.handle:
            self.ctx._bind()
            self.ctx.lib.lkc_target_free(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                self.free()
        except Exception:  # pragma: no cover
            pass


def _copy_device(addr: int, nbytes: int, dtype):
    """Copy raw device memory into a host tensor (hipMemcpy via torch)."""
    torch = _torch()
    out = torch.empty(nbytes // torch.empty(0, dtype=dtype).element_size(), dtype=dtype)
    if nbytes == 0:
        return out
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(addr), nbytes, 2)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out


# ------------------------------------------------------------------ calls --

def lkc_build_target(ctx: Context, points, cell_size: float) -> Target:
    torch = _torch()
    _check_dev(points, "points", torch.float32, (3,))
    ctx._bind()
    h = ctypes.c_void_p()
    ctx.check(ctx.lib.lkc_build_target(ctx.handle, ctypes.c_void_p(_ptr(points)),
                                       points.shape[0], float(cell_size), ctypes.byref(h)))
    return Target(ctx, h)


def lkc_knn_query(ctx: Context, target: Target, queries, k: int,
                  radius: float = math.inf, out=None, cfg=None):
    """Returns (idx int32 [q,k], d2 float32 [q,k], count int32 [q])."""
    torch = _torch()
    _check_dev(queries, "queries", torch.float32, (3,))
    q = queries.shape[0]
    if out is None:
        dev = queries.device
        out = (torch.empty(q, k, dtype=torch.int32, device=dev),
               torch.empty(q, k, dtype=torch.float32, device=dev),
               torch.empty(q, dtype=torch.int32, device=dev))
    idx, d2, cnt = out
    ctx._bind()
    ctx.check(ctx.lib.lkc_knn_query(ctx.handle, target.handle, ctypes.c_void_p(_ptr(queries)),
                                    q, int(k), float(radius), ctypes.c_void_p(_ptr(idx)),
                                    ctypes.c_void_p(_ptr(d2)), ctypes.c_void_p(_ptr(cnt)),
                                    _cfg_ptr(cfg)))
    return idx, d2, cnt


def _cov_out(q, dev):
    torch = _torch()
    return dict(mean=torch.empty(q, 3, dtype=torch.float32, device=dev),
                cov=torch.empty(q, 3, 3, dtype=torch.float32, device=dev),
                reg=torch.empty(q, 3, 3, dtype=torch.float32, device=dev),
                valid=torch.empty(q, dtype=torch.uint8, device=dev))


def lkc_covariances(ctx: Context, target: Target, idx, count, queries=None,
                    plane_eps: float = 1e-3, out: Optional[Dict] = None):
    torch = _torch()
    _check_dev(idx, "idx", torch.int32)
    _check_dev(count, "count", torch.int32)
    _check_dev(queries, "queries", torch.float32, (3,))
    q, k = idx.shape
    out = out or _cov_out(q, idx.device)
    ctx._bind()
    ctx.check(ctx.lib.lkc_covariances(
        ctx.handle, target.handle, ctypes.c_void_p(_ptr(queries)), ctypes.c_void_p(_ptr(idx)),
        ctypes.c_void_p(_ptr(count)), q, int(k), float(plane_eps),
        ctypes.c_void_p(_ptr(out.get("mean"))), ctypes.c_void_p(_ptr(out.get("cov"))),
        ctypes.c_void_p(_ptr(out.get("reg"))), ctypes.c_void_p(_ptr(out["valid"]))))
    return out


def lkc_knn_cov(ctx: Context, target: Target, queries, k: int, radius: float = math.inf,
                plane_eps: float = 1e-3, out: Optional[Dict] = None, cfg=None,
                noalloc: bool = False):
    """noalloc: call lkc_knn_cov_noalloc (static scratch, no device
    allocation, q <= 131,072); the outputs must then be allocated already
    (pass `out`) for the call itself to allocate nothing."""
    torch = _torch()
    _check_dev(queries, "queries", torch.float32, (3,))
    q = queries.shape[0]
    if out is None:
        out = _cov_out(q, queries.device)
        out.update(idx=torch.empty(q, k, dtype=torch.int32, device=queries.device),
                   d2=torch.empty(q, k, dtype=torch.float32, device=queries.device),
                   count=torch.empty(q, dtype=torch.int32, device=queries.device))
    ctx._bind()
    fn = ctx.lib.lkc_knn_cov_noalloc if noalloc else ctx.lib.lkc_knn_cov
    ctx.check(fn(
        ctx.handle, target.handle, ctypes.c_void_p(_ptr(queries)), q, int(k), float(radius),
        float(plane_eps), ctypes.c_void_p(_ptr(out["idx"])), ctypes.c_void_p(_ptr(out["d2"])),
        ctypes.c_void_p(_ptr(out["count"])), ctypes.c_void_p(_ptr(out.get("mean"))),
        ctypes.c_void_p(_ptr(out.get("cov"))), ctypes.c_void_p(_ptr(out.get("reg"))),
        ctypes.c_void_p(_ptr(out["valid"])), _cfg_ptr(cfg)))
    return out


def _weight_kernel(kernel) -> int:
    if isinstance(kernel, str):
        return WEIGHT_KERNELS[kernel]
    return int(kernel)


def lkc_covariances_weighted(ctx: Context, target: Target, idx, count, kernel, sigma: float,
                             queries=None, plane_eps: float = 1e-3, out: Optional[Dict] = None):
    """Kernel-descriptor weighted mean / covariance; ``kernel`` is a name of
    ``WEIGHT_KERNELS`` or its code."""
    torch = _torch()
    _check_dev(idx, "idx", torch.int32)
    _check_dev(count, "count", torch.int32)
    _check_dev(queries, "queries", torch.float32, (3,))
    q, k = idx.shape
    out = out or _cov_out(q, idx.device)
    ctx._bind()
    ctx.check(ctx.lib.lkc_covariances_weighted(
        ctx.handle, target.handle, ctypes.c_void_p(_ptr(queries)), ctypes.c_void_p(_ptr(idx)),
        ctypes.c_void_p(_ptr(count)), q, int(k), _weight_kernel(kernel), float(sigma),
        float(plane_eps), ctypes.c_void_p(_ptr(out.get("mean"))),
        ctypes.c_void_p(_ptr(out.get("cov"))), ctypes.c_void_p(_ptr(out.get("reg"))),
        ctypes.c_void_p(_ptr(out["valid"]))))
    return out


def lkc_knn_cov_weighted(ctx: Context, target: Target, queries, k: int, kernel, sigma: float,
                         radius: float = math.inf, plane_eps: float = 1e-3,
                         out: Optional[Dict] = None, cfg=None):
    torch = _torch()
    _check_dev(queries, "queries", torch.float32, (3,))
    q = queries.shape[0]
    if out is None:
        out = _cov_out(q, queries.device)
        out.update(idx=torch.empty(q, k, dtype=torch.int32, device=queries.device),
                   d2=torch.empty(q, k, dtype=torch.float32, device=queries.device),
                   count=torch.empty(q, dtype=torch.int32, device=queries.device))
    ctx._bind()
    ctx.check(ctx.lib.lkc_knn_cov_weighted(
        ctx.handle, target.handle, ctypes.c_void_p(_ptr(queries)), q, int(k), float(radius),
        _weight_kernel(kernel), float(sigma), float(plane_eps),
        ctypes.c_void_p(_ptr(out["idx"])), ctypes.c_void_p(_ptr(out["d2"])),
        ctypes.c_void_p(_ptr(out["count"])), ctypes.c_void_p(_ptr(out.get("mean"))),
        ctypes.c_void_p(_ptr(out.get("cov"))), ctypes.c_void_p(_ptr(out.get("reg"))),
        ctypes.c_void_p(_ptr(out["valid"])), _cfg_ptr(cfg)))
    return out


def _host_T(T):
    import numpy as np
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float64))
    if T.shape != (4, 4):
        raise ValueError("T must be a 4x4 transform")
    return T


def lkc_gicp_linearize(ctx: Context, target: Target, target_cov, source, source_cov, T,
                       max_corr_dist: float = math.inf, corr=None, system=None, cfg=None):
    """One GICP linearisation at T (host 4x4).  Returns (system, corr) device
    tensors: system float64 [45] = H (36, row-major), b (6), E, count, rejected."""
    torch = _torch()
    _check_dev(target_cov, "target_cov", torch.float32, (3, 3))
    _check_dev(source, "source", torch.float32, (3,))
    _check_dev(source_cov, "source_cov", torch.float32, (3, 3))
    n = source.shape[0]
    if source_cov.shape[0] != n:
        raise ValueError("source_cov must have one row per source point")
    if target_cov.shape[0] != target.info()["n_points"]:
        raise ValueError("target_cov must have one row per target point")
    if corr is None:
        corr = torch.empty(n, dtype=torch.int32, device=source.device)
    if system is None:
        system = torch.empty(GICP_SYSTEM_WORDS, dtype=torch.float64, device=source.device)
    _check_dev(corr, "corr", torch.int32)
    _check_dev(system, "system", torch.float64)
    Th = _host_T(T)
    ctx._bind()
    ctx.check(ctx.lib.lkc_gicp_linearize(
        ctx.handle, target.handle, ctypes.c_void_p(_ptr(target_cov)),
        ctypes.c_void_p(_ptr(source)), ctypes.c_void_p(_ptr(source_cov)), n,
        Th.ctypes.data_as(ctypes.c_void_p), float(max_corr_dist),
        ctypes.c_void_p(_ptr(corr)), ctypes.c_void_p(_ptr(system)), _cfg_ptr(cfg)))
    return system, corr


def split_system(system):
    """Host view of a system vector: dict H [6,6], b [6], E, count, rejected."""
    import numpy as np
    v = np.asarray(system.cpu().numpy() if hasattr(system, "cpu") else system, np.float64)
    return dict(H=v[:36].reshape(6, 6), b=v[36:42], E=float(v[42]), count=int(v[43]),
                rejected=int(v[44]))


def lkc_gicp_align(ctx: Context, target: Target, target_cov, source, source_cov, T_init,
                   max_corr_dist: float = math.inf, max_iters: int = 30, tol: float = 1e-6,
                   cfg=None):
    """Gauss-Newton GICP iterations; returns (T 4x4 numpy, stats dict)."""
    import numpy as np
    torch = _torch()
    _check_dev(target_cov, "target_cov", torch.float32, (3, 3))
    _check_dev(source, "source", torch.float32, (3,))
    _check_dev(source_cov, "source_cov", torch.float32, (3, 3))
    n = source.shape[0]
    if source_cov.shape[0] != n:
        raise ValueError("source_cov must have one row per source point")
    if target_cov.shape[0] != target.info()["n_points"]:
        raise ValueError("target_cov must have one row per target point")
    T0 = _host_T(T_init)
    Tout = np.empty((4, 4))
    st = GicpStats()
    ctx._bind()
    ctx.check(ctx.lib.lkc_gicp_align(
        ctx.handle, target.handle, ctypes.c_void_p(_ptr(target_cov)),
        ctypes.c_void_p(_ptr(source)), ctypes.c_void_p(_ptr(source_cov)), n,
        T0.ctypes.data_as(ctypes.c_void_p), float(max_corr_dist), int(max_iters), float(tol),
        Tout.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st), _cfg_ptr(cfg)))
    return Tout, st.as_dict()


def lkc_voxel_filter(ctx: Context, points, leaf: float, origin=None, capacity=None):
    """Voxel centroids of a device cloud.  Returns dict centroid float32
    [m, 3], count int32 [m], voxel int32 [m, 3] (device tensors)."""
    import numpy as np
    torch = _torch()
    _check_dev(points, "points", torch.float32, (3,))
    n = points.shape[0]
    cap = n if capacity is None else int(capacity)
    dev = points.device
    cen = torch.empty(max(cap, 1), 3, dtype=torch.float32, device=dev)
    cnt = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    vox = torch.empty(max(cap, 1), 3, dtype=torch.int32, device=dev)
    o = None if origin is None else np.ascontiguousarray(origin, np.float32)
    m = ctypes.c_int64(0)
    ctx._bind()
    ctx.check(ctx.lib.lkc_voxel_filter(
        ctx.handle, ctypes.c_void_p(_ptr(points)), n,
        None if o is None else o.ctypes.data_as(ctypes.c_void_p), float(leaf),
        ctypes.c_void_p(_ptr(cen)), ctypes.c_void_p(_ptr(cnt)), ctypes.c_void_p(_ptr(vox)), cap,
        ctypes.byref(m)))
    k = m.value
    return dict(centroid=cen[:k], count=cnt[:k], voxel=vox[:k])


def lkc_voxel_filter_async(ctx: Context, points, leaf: float, axis_bits: int, origin=None,
                           capacity=None, out: Optional[Dict] = None):
    """lkc_voxel_filter with no host wait: dict of device tensors centroid
    [capacity, 3], count [capacity], voxel [capacity, 3], n_out int64 [1]
    and status int32 [1] (rows past n_out are untouched).  Pass `out` (a
    dict from an earlier call of the same capacity) to reuse its tensors,
    e.g. in a captured graph."""
    import numpy as np
    torch = _torch()
    _check_dev(points, "points", torch.float32, (3,))
    n = points.shape[0]
    dev = points.device
    if out is None:
        cap = n if capacity is None else int(capacity)
        out = dict(centroid=torch.empty(max(cap, 1), 3, dtype=torch.float32, device=dev),
                   count=torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                   voxel=torch.empty(max(cap, 1), 3, dtype=torch.int32, device=dev),
                   n_out=torch.zeros(1, dtype=torch.int64, device=dev),
                   status=torch.zeros(1, dtype=torch.int32, device=dev), capacity=cap)
    o = None if origin is None else np.ascontiguousarray(origin, np.float32)
    ctx._bind()
    ctx.check(ctx.lib.lkc_voxel_filter_async(
        ctx.handle, ctypes.c_void_p(_ptr(points)), n,
        None if o is None else o.ctypes.data_as(ctypes.c_void_p), float(leaf), int(axis_bits),
        ctypes.c_void_p(_ptr(out["centroid"])), ctypes.c_void_p(_ptr(out["count"])),
        ctypes.c_void_p(_ptr(out["voxel"])), int(out["capacity"]),
        ctypes.c_void_p(_ptr(out["n_out"])), ctypes.c_void_p(_ptr(out["status"]))))
    return out


def lkc_submap_extract(ctx: Context, target: Target, center, radius: float, capacity=None):
    """Ascending indices (device int32) of the target points within radius of center."""
    import numpy as np
    torch = _torch()
    n = target.info()["n_points"]
    cap = n if capacity is None else int(capacity)
    dev = torch.device("cuda", torch.cuda.current_device())
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    c = np.ascontiguousarray(center, np.float32)
    m = ctypes.c_int64(0)
    ctx._bind()
    ctx.check(ctx.lib.lkc_submap_extract(ctx.handle, target.handle,
                                         c.ctypes.data_as(ctypes.c_void_p), float(radius),
                                         ctypes.c_void_p(_ptr(idx)), cap, ctypes.byref(m)))
    return idx[:m.value]


def lkc_submap_build(ctx: Context, target: Target, center, radius: float, with_idx: bool = True):
    """Build the window around center into a new Target; returns (Target, idx)."""
    import numpy as np
    torch = _torch()
    n = target.info()["n_points"]
    dev = torch.device("cuda", torch.cuda.current_device())
    idx = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if with_idx else None
    c = np.ascontiguousarray(center, np.float32)
    m = ctypes.c_int64(0)
    h = ctypes.c_void_p()
    ctx._bind()
    ctx.check(ctx.lib.lkc_submap_build(ctx.handle, target.handle,
                                       c.ctypes.data_as(ctypes.c_void_p), float(radius),
                                       ctypes.c_void_p(_ptr(idx)), n if with_idx else 0,
                                       ctypes.byref(m), ctypes.byref(h)))
    return Target(ctx, h), (idx[:m.value] if with_idx else None)


class RaceLine:
    """A race-line keyed index of a map target (``lkc_raceline``)."""

    def __init__(self, ctx: Context, handle: ctypes.c_void_p, target: Target):
        self.ctx = ctx
        self.handle = handle
        self.target = target      # the map must outlive the index

    def info(self) -> Dict:
        inf = RaceLineInfo()
        self.ctx.check(self.ctx.lib.lkc_raceline_get_info(self.handle, ctypes.byref(inf)))
        return inf.as_dict()

    def bins(self):
        """(anchors float32 [bins, 3], points per bin int64 [bins]) on the host."""
        import numpy as np
        b = self.info()["n_bins"]
        a = np.empty((b, 3), np.float32)
        c = np.empty(b, np.int64)
        self.ctx.check(self.ctx.lib.lkc_raceline_bins(self.handle,
                                                      a.ctypes.data_as(ctypes.c_void_p),
                                                      c.ctypes.data_as(ctypes.c_void_p)))
        return a, c

    def free(self):
        if self.handle:
            self.ctx._bind()
            self.ctx.lib.lkc_raceline_free(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                self.free()
        except Exception:  # pragma: no cover
            pass


def lkc_raceline_build(ctx: Context, target: Target, line, bin_length: float, radius: float,
                       lateral: float) -> RaceLine:
    """Race-line index of ``target``: ``line`` is the closed race line, host
    float [m, 3] in driving order."""
    import numpy as np
    ln = np.ascontiguousarray(line, np.float32)
    if ln.ndim != 2 or ln.shape[1] != 3:
        raise ValueError("line must be [m, 3]")
    h = ctypes.c_void_p()
    ctx._bind()
    ctx.check(ctx.lib.lkc_raceline_build(ctx.handle, target.handle,
                                         ln.ctypes.data_as(ctypes.c_void_p), ln.shape[0],
                                         float(bin_length), float(radius), float(lateral),
                                         ctypes.byref(h)))
    return RaceLine(ctx, h, target)


def _pose_dev(pose):
    torch = _torch()
    if isinstance(pose, torch.Tensor) and pose.is_cuda:
        _check_dev(pose, "pose", torch.float32)
        if pose.numel() != 3:
            raise ValueError("pose must hold 3 floats")
        return pose
    import numpy as np
    p = np.ascontiguousarray(pose, np.float32).reshape(3)
    return torch.from_numpy(p).to(torch.device("cuda", torch.cuda.current_device()))


def lkc_submap_window(ctx: Context, rl: RaceLine, pose, radius: float, capacity=None,
                      with_points: bool = False, out=None):
    """Enqueue the window of ``pose`` (no synchronisation).  Returns device
    tensors (idx int32 [capacity], points float32 [capacity, 3] or None,
    info int64 [3] = count, bin, status); ``out`` may pass those three
    buffers in (for graph capture).  The first ``info[0]`` entries of idx
    are the window."""
    torch = _torch()
    pose = _pose_dev(pose)
    if out is None:
        cap = rl.info()["max_bin_points"] if capacity is None else int(capacity)
        dev = pose.device
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        pts = torch.empty(max(cap, 1), 3, dtype=torch.float32, device=dev) if with_points \
            else None
        info = torch.empty(3, dtype=torch.int64, device=dev)
    else:
        idx, pts, info = out
        cap = idx.shape[0] if capacity is None else int(capacity)
        if cap > idx.shape[0] or (pts is not None and cap > pts.shape[0]):
            raise ValueError("capacity exceeds the output buffers")
    ctx._bind()
    ctx.check(ctx.lib.lkc_submap_window(ctx.handle, rl.handle, ctypes.c_void_p(_ptr(pose)),
                                        float(radius), ctypes.c_void_p(_ptr(idx)),
                                        ctypes.c_void_p(_ptr(pts)), cap,
                                        ctypes.c_void_p(_ptr(info))))
    return idx, pts, info


def lkc_submap_window_build(ctx: Context, rl: RaceLine, pose, radius: float,
                            with_idx: bool = True):
    """The window of ``pose`` built into a new Target; returns (Target, idx)."""
    torch = _torch()
    pose = _pose_dev(pose)
    cap = rl.info()["max_bin_points"]
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=pose.device) if with_idx else None
    m = ctypes.c_int64(0)
    h = ctypes.c_void_p()
    ctx._bind()
    ctx.check(ctx.lib.lkc_submap_window_build(ctx.handle, rl.handle, ctypes.c_void_p(_ptr(pose)),
                                              float(radius), ctypes.c_void_p(_ptr(idx)),
                                              cap if with_idx else 0, ctypes.byref(m),
                                              ctypes.byref(h)))
    return Target(ctx, h), (idx[:m.value] if with_idx else None)


def lkc_zvote(ctx: Context, points, cell: float, tau: int, with_votes: bool = True):
    """z-vote filter: (keep uint8 [n], votes int32 [n] or None), device tensors."""
    torch = _torch()
    _check_dev(points, "points", torch.float32, (3,))
    n = points.shape[0]
    keep = torch.empty(n, dtype=torch.uint8, device=points.device)
    votes = torch.empty(n, dtype=torch.int32, device=points.device) if with_votes else None
    ctx._bind()
    ctx.check(ctx.lib.lkc_zvote(ctx.handle, ctypes.c_void_p(_ptr(points)), n, float(cell),
                                int(tau), ctypes.c_void_p(_ptr(keep)),
                                ctypes.c_void_p(_ptr(votes))))
    return keep, votes


def lkc_euclid_cluster(ctx: Context, points, eps: float, mask=None):
    """Distance clustering: (labels int32 [n] device, number of clusters);
    ``mask`` (device uint8 [n]) selects the points, the others get -1."""
    torch = _torch()
    _check_dev(points, "points", torch.float32, (3,))
    _check_dev(mask, "mask", torch.uint8)
    n = points.shape[0]
    if mask is not None and mask.shape[0] != n:
        raise ValueError("mask must have one entry per point")
    labels = torch.empty(n, dtype=torch.int32, device=points.device)
    k = ctypes.c_int64(0)
    ctx._bind()
    ctx.check(ctx.lib.lkc_euclid_cluster(ctx.handle, ctypes.c_void_p(_ptr(points)), n,
                                         float(eps), ctypes.c_void_p(_ptr(mask)),
                                         ctypes.c_void_p(_ptr(labels)), ctypes.byref(k)))
    return labels, k.value


def lkc_euclid_cluster_async(ctx: Context, points, eps: float, mask=None,
                             out: Optional[Dict] = None):
    """lkc_euclid_cluster with no host wait: dict of device tensors labels
    int32 [n], n_clusters int64 [1], status int32 [1].  Pass `out` (from an
    earlier call on as many points) to reuse its tensors, e.g. in a
    captured graph."""
    torch = _torch()
    _check_dev(points, "points", torch.float32, (3,))
    _check_dev(mask, "mask", torch.uint8)
    n = points.shape[0]
    if mask is not None and mask.shape[0] != n:
        raise ValueError("mask must have one entry per point")
    if out is None:
        out = dict(labels=torch.empty(n, dtype=torch.int32, device=points.device),
                   n_clusters=torch.zeros(1, dtype=torch.int64, device=points.device),
                   status=torch.zeros(1, dtype=torch.int32, device=points.device))
    ctx._bind()
    ctx.check(ctx.lib.lkc_euclid_cluster_async(
        ctx.handle, ctypes.c_void_p(_ptr(points)), n, float(eps), ctypes.c_void_p(_ptr(mask)),
        ctypes.c_void_p(_ptr(out["labels"])), ctypes.c_void_p(_ptr(out["n_clusters"])),
        ctypes.c_void_p(_ptr(out["status"]))))
    return out


def lkc_knn_cov_self(ctx: Context, target: Target, k: int, radius: float = math.inf,
                     plane_eps: float = 1e-3, out: Optional[Dict] = None, cfg=None,
                     with_cov: bool = True):
    """k nearest neighbours (+ covariances) of every point of the target itself;
    rows in the target's original point order."""
    torch = _torch()
    n = target.info()["n_points"] if out is None else out["count"].shape[0]
    if out is None:
        dev = torch.device("cuda", torch.cuda.current_device())
        out = _cov_out(n, dev) if with_cov else {}
        out.update(idx=torch.empty(n, k, dtype=torch.int32, device=dev),
                   d2=torch.empty(n, k, dtype=torch.float32, device=dev),
                   count=torch.empty(n, dtype=torch.int32, device=dev))
    ctx._bind()
    ctx.check(ctx.lib.lkc_knn_cov_self(
        ctx.handle, target.handle, int(k), float(radius), float(plane_eps),
        ctypes.c_void_p(_ptr(out["idx"])), ctypes.c_void_p(_ptr(out["d2"])),
        ctypes.c_void_p(_ptr(out["count"])), ctypes.c_void_p(_ptr(out.get("mean"))),
        ctypes.c_void_p(_ptr(out.get("cov"))), ctypes.c_void_p(_ptr(out.get("reg"))),
        ctypes.c_void_p(_ptr(out.get("valid"))), _cfg_ptr(cfg)))
    return out


class TargetSet:
    """``lkc_target_set``: several targets + a staged scan table for batching."""

    def __init__(self, ctx: Context, targets: Sequence[Target], max_scans: int):
        self.ctx = ctx
        self.targets = list(targets)
        arr = (ctypes.c_void_p * len(self.targets))(*[t.handle.value for t in self.targets])
        h = ctypes.c_void_p()
        ctx._bind()
        ctx.check(ctx.lib.lkc_target_set_create(ctx.handle, arr, len(self.targets),
                                                int(max_scans), ctypes.byref(h)))
        self.handle = h
        self.max_scans = max_scans

    def stage(self, scans: Sequence[Tuple[int, int, int]]):
        """scans: (q_offset, q_count, target_index) per scan."""
        arr = (ScanDesc * max(1, len(scans)))()
        for i, (o, c, t) in enumerate(scans):
            arr[i].q_offset, arr[i].q_count, arr[i].target_index = int(o), int(c), int(t)
        self.ctx._bind()
        self.ctx.check(self.ctx.lib.lkc_target_set_stage(self.ctx.handle, self.handle, arr,
                                                         len(scans)))

    def free(self):
        if self.handle:
            self.ctx._bind()
            self.ctx.lib.lkc_target_set_free(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                self.free()
        except Exception:  # pragma: no cover
            pass


def lkc_knn_cov_batched(ctx: Context, tset: TargetSet, queries, k: int,
                        radius: float = math.inf, plane_eps: float = 1e-3,
                        out: Optional[Dict] = None, cfg=None):
    torch = _torch()
    _check_dev(queries, "queries", torch.float32, (3,))
    q = queries.shape[0]
    if out is None:
        out = _cov_out(q, queries.device)
        out.update(idx=torch.empty(q, k, dtype=torch.int32, device=queries.device),
                   d2=torch.empty(q, k, dtype=torch.float32, device=queries.device),
                   count=torch.empty(q, dtype=torch.int32, device=queries.device))
    ctx._bind()
    ctx.check(ctx.lib.lkc_knn_cov_batched(
        ctx.handle, tset.handle, ctypes.c_void_p(_ptr(queries)), q, int(k), float(radius),
        float(plane_eps), ctypes.c_void_p(_ptr(out["idx"])), ctypes.c_void_p(_ptr(out["d2"])),
        ctypes.c_void_p(_ptr(out["count"])), ctypes.c_void_p(_ptr(out.get("mean"))),
        ctypes.c_void_p(_ptr(out.get("cov"))), ctypes.c_void_p(_ptr(out.get("reg"))),
        ctypes.c_void_p(_ptr(out["valid"])), _cfg_ptr(cfg)))
    return out


# pythonic aliases
build_target = lkc_build_target
knn_query = lkc_knn_query
covariances = lkc_covariances
knn_cov = lkc_knn_cov
knn_cov_batched = lkc_knn_cov_batched
knn_cov_self = lkc_knn_cov_self
