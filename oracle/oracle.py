"""FP64 CPU oracle for nearest-points search + per-point covariance.

TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does, and nothing here imports
the GPU package.

Two independent implementations live here:

* ``knn`` / ``covariances`` -- ctypes wrappers over ``lkc_oracle.c`` (plain
  C, FP64 loops, pthreads over query chunks), used at every size;
* ``knn_np`` / ``covariances_np`` -- a NumPy twin for tiny inputs (a full
  lexicographic sort per query and ``numpy.linalg.eigh``), used only to
  cross-check the C oracle.

What both compute follows the paper's registration section (Sec. III-C.1:
each point is a Gaussian whose covariance comes from its corresponding
nearest points; that search and covariance are the GPU step).  The readings
of what the paper leaves open -- lower-index tie-break, inclusive radius,
1/n normalisation, ``C_reg = I - (1 - eps) v0 v0^T`` with ``valid = n >= 3``
-- are stated in ``lkc_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lkc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblkc_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile ``lkc_oracle.c`` with gcc into ``liblkc_oracle.so`` (in-tree)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lpthread", "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    P = ctypes.c_void_p
    lib.oracle_knn.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_int32, P, P, P]
    lib.oracle_knn.restype = ctypes.c_int
    lib.oracle_covariances.argtypes = [P, ctypes.c_int64, P, P, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                       P, P, P, P, P, P]
    lib.oracle_covariances.restype = ctypes.c_int
    lib.oracle_sym3_eig.argtypes = [P, P, P]
    lib.oracle_sym3_eig.restype = None
    if hasattr(lib, "oracle_covariances_weighted"):
        lib.oracle_covariances_weighted.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int64,
                                                    ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_double, ctypes.c_double,
                                                    P, P, P, P]
        lib.oracle_covariances_weighted.restype = ctypes.c_int
    if hasattr(lib, "oracle_voxel_filter"):
        lib.oracle_voxel_filter.argtypes = [P, ctypes.c_int64, P, ctypes.c_float, P, P, P]
        lib.oracle_voxel_filter.restype = ctypes.c_int64
        lib.oracle_submap.argtypes = [P, ctypes.c_int64, P, ctypes.c_float, P]
        lib.oracle_submap.restype = ctypes.c_int64
    if hasattr(lib, "oracle_zvote"):
        lib.oracle_zvote.argtypes = [P, ctypes.c_int64, ctypes.c_float, ctypes.c_int32, P, P]
        lib.oracle_zvote.restype = ctypes.c_int
        lib.oracle_euclid_cluster.argtypes = [P, ctypes.c_int64, ctypes.c_float, P]
        lib.oracle_euclid_cluster.restype = ctypes.c_int64
    if hasattr(lib, "oracle_gicp_linearize"):
        lib.oracle_gicp_correspond.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P,
                                               ctypes.c_double, ctypes.c_int32, P, P]
        lib.oracle_gicp_correspond.restype = ctypes.c_int
        lib.oracle_gicp_linearize.argtypes = [P, P, ctypes.c_int64, P, P, ctypes.c_int64, P, P,
                                              P, P, P, P]
        lib.oracle_gicp_linearize.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            _lib = configure(ctypes.CDLL(build()))
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1, 3))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def knn(target, queries, k: int, radius: float = float("inf"), threads: int | None = None):
    """Brute-force kNN.  Returns (idx int32 [q,k], d2 float64 [q,k], count int32 [q])."""
    t = _f32(target)
    q = _f32(queries)
    nq = q.shape[0]
    idx = np.empty((nq, k), np.int32)
    d2 = np.empty((nq, k), np.float64)
    cnt = np.empty(nq, np.int32)
    rc = _load().oracle_knn(_ptr(t), t.shape[0], _ptr(q), nq, int(k), float(radius),
                            int(threads or default_threads()), _ptr(idx), _ptr(d2), _ptr(cnt))
    if rc != 0:
        raise ValueError("oracle_knn: invalid arguments")
    return idx, d2, cnt


def covariances(target, idx, count, eps: float = 1e-3, threads: int | None = None,
                with_eig: bool = False):
    """Two-pass FP64 mean / covariance / regularised covariance per query.

    Returns a dict with mean [q,3], cov [q,3,3], reg [q,3,3] (float64),
    valid [q] (uint8) and, if ``with_eig``, evals [q,3] (ascending) and
    evec0 [q,3] (unit eigenvector of the smallest eigenvalue).
    """
    t = _f32(target)
    idx = np.ascontiguousarray(idx, np.int32)
    count = np.ascontiguousarray(count, np.int32)
    nq, k = idx.shape
    mean = np.empty((nq, 3))
    cov = np.empty((nq, 3, 3))
    reg = np.empty((nq, 3, 3))
    valid = np.empty(nq, np.uint8)
    evals = np.empty((nq, 3)) if with_eig else None
    evec0 = np.empty((nq, 3)) if with_eig else None
    rc = _load().oracle_covariances(
        _ptr(t), t.shape[0], _ptr(idx), _ptr(count), nq, int(k), float(eps),
        int(threads or default_threads()), _ptr(mean), _ptr(cov), _ptr(reg), _ptr(valid),
        _ptr(evals) if with_eig else None, _ptr(evec0) if with_eig else None)
    if rc != 0:
        raise ValueError("oracle_covariances: invalid arguments or neighbour index")
    out = dict(mean=mean, cov=cov, reg=reg, valid=valid)
    if with_eig:
        out.update(evals=evals, evec0=evec0)
    return out


WEIGHT_KINDS = {"rbf": 1, "gaussian": 2, "laplacian": 3}


def covariances_weighted(target, idx, count, kind: str, sigma: float, queries=None,
                         eps: float = 1e-3):
    """Kernel-descriptor weighted mean / covariance (FP64); see lkc_oracle.c."""
    t = _f32(target)
    idx = np.ascontiguousarray(idx, np.int32)
    count = np.ascontiguousarray(count, np.int32)
    nq, k = idx.shape
    qa = None if queries is None else _f32(queries)
    mean = np.empty((nq, 3))
    cov = np.empty((nq, 3, 3))
    reg = np.empty((nq, 3, 3))
    valid = np.empty(nq, np.uint8)
    rc = _load().oracle_covariances_weighted(
        _ptr(t), t.shape[0], None if qa is None else _ptr(qa), _ptr(idx), _ptr(count), nq, int(k),
        WEIGHT_KINDS[kind], float(sigma), float(eps), _ptr(mean), _ptr(cov), _ptr(reg),
        _ptr(valid))
    if rc != 0:
        raise ValueError("oracle_covariances_weighted: invalid arguments")
    return dict(mean=mean, cov=cov, reg=reg, valid=valid)


def _T(T):
    T = np.ascontiguousarray(T, np.float64)
    assert T.shape == (4, 4)
    return T


def gicp_correspond(source, target, T, max_dist: float = float("inf"),
                    threads: int | None = None):
    """Nearest target point of T p_i (FP64 brute force).  Returns (corr int32, d2 float64)."""
    s, t, T = _f32(source), _f32(target), _T(T)
    n = s.shape[0]
    corr = np.empty(n, np.int32)
    d2 = np.empty(n)
    rc = _load().oracle_gicp_correspond(_ptr(s), n, _ptr(t), t.shape[0], _ptr(T),
                                        float(max_dist), int(threads or default_threads()),
                                        _ptr(corr), _ptr(d2))
    if rc != 0:
        raise ValueError("oracle_gicp_correspond: invalid arguments")
    return corr, d2


def gicp_linearize(source, source_cov, target, target_cov, T, corr):
    """Gauss-Newton system of the GICP cost at T.  Returns dict H [6,6], b [6],
    E, count."""
    s, t, T = _f32(source), _f32(target), _T(T)
    sc = np.ascontiguousarray(np.asarray(source_cov, np.float32).reshape(-1, 9))
    tc = np.ascontiguousarray(np.asarray(target_cov, np.float32).reshape(-1, 9))
    corr = np.ascontiguousarray(corr, np.int32)
    H = np.empty((6, 6))
    b = np.empty(6)
    E = np.empty(1)
    cnt = np.empty(1, np.int64)
    rc = _load().oracle_gicp_linearize(_ptr(s), _ptr(sc), s.shape[0], _ptr(t), _ptr(tc),
                                       t.shape[0], _ptr(T), _ptr(corr), _ptr(H), _ptr(b),
                                       _ptr(E), _ptr(cnt))
    if rc != 0:
        raise ValueError("oracle_gicp_linearize: bad correspondence or covariance")
    return dict(H=H, b=b, E=float(E[0]), count=int(cnt[0]))


def voxel_filter(points, leaf: float, origin=(0.0, 0.0, 0.0)):
    """Voxel centroids (FP64), voxel coordinates (int64) and counts, voxels
    ordered by (vz, vy, vx)."""
    p = _f32(points)
    n = p.shape[0]
    o = np.ascontiguousarray(origin, np.float32)
    vox = np.empty((max(n, 1), 3), np.int64)
    cen = np.empty((max(n, 1), 3))
    cnt = np.empty(max(n, 1), np.int32)
    m = _load().oracle_voxel_filter(_ptr(p), n, _ptr(o), float(np.float32(leaf)), _ptr(vox),
                                    _ptr(cen), _ptr(cnt))
    if m < 0:
        raise ValueError("oracle_voxel_filter: invalid leaf or voxel coordinate out of range")
    return dict(voxel=vox[:m], centroid=cen[:m], count=cnt[:m])


def submap(points, center, radius: float):
    """Ascending indices of the points within radius of center (FP64 decision)."""
    p = _f32(points)
    c = np.ascontiguousarray(center, np.float32)
    out = np.empty(max(p.shape[0], 1), np.int32)
    m = _load().oracle_submap(_ptr(p), p.shape[0], _ptr(c), float(np.float32(radius)),
                              _ptr(out))
    if m < 0:
        raise ValueError("oracle_submap: invalid radius")
    return out[:m]


def zvote(points, cell: float, tau: int):
    """z-axis voting: (keep uint8 [n], votes int32 [n])."""
    p = _f32(points)
    n = p.shape[0]
    keep = np.empty(max(n, 1), np.uint8)
    votes = np.empty(max(n, 1), np.int32)
    rc = _load().oracle_zvote(_ptr(p), n, float(np.float32(cell)), int(tau), _ptr(keep),
                              _ptr(votes))
    if rc != 0:
        raise ValueError("oracle_zvote: invalid arguments")
    return keep[:n], votes[:n]


def euclid_cluster(points, eps: float):
    """Connected components under d2 <= eps^2: (label int32 [n], n_clusters)."""
    p = _f32(points)
    n = p.shape[0]
    label = np.empty(max(n, 1), np.int32)
    k = _load().oracle_euclid_cluster(_ptr(p), n, float(np.float32(eps)), _ptr(label))
    if k < 0:
        raise ValueError("oracle_euclid_cluster: invalid arguments")
    return label[:n], int(k)


def sym3_eig(a):
    """Jacobi eigen-decomposition of one symmetric 3x3 (evals ascending, evecs columns)."""
    a = np.ascontiguousarray(a, np.float64).reshape(3, 3)
    ev = np.empty(3)
    V = np.empty((3, 3))
    _load().oracle_sym3_eig(_ptr(a), _ptr(ev), _ptr(V))
    return ev, V


# ----------------------------------------------------------- NumPy twin ---

def knn_np(target, queries, k: int, radius: float = float("inf")):
    """Tiny-input twin: full lexicographic sort of every candidate per query."""
    t = _f32(target).astype(np.float64)
    q = _f32(queries).astype(np.float64)
    nq = q.shape[0]
    idx = np.full((nq, k), -1, np.int32)
    d2 = np.full((nq, k), np.inf)
    cnt = np.zeros(nq, np.int32)
    r2 = np.inf if np.isinf(radius) else radius * radius
    j = np.arange(t.shape[0])
    for i in range(nq):
        if not np.all(np.isfinite(q[i])):
            continue
        d = ((q[i] - t) ** 2).sum(axis=1)
        keep = d <= r2
        order = np.lexsort((j[keep], d[keep]))[:k]
        m = order.size
        idx[i, :m] = j[keep][order]
        d2[i, :m] = d[keep][order]
        cnt[i] = m
    return idx, d2, cnt


def covariances_np(target, idx, count, eps: float = 1e-3):
    """Tiny-input twin using numpy.cov(bias=True) and numpy.linalg.eigh."""
    t = _f32(target).astype(np.float64)
    nq = idx.shape[0]
    mean = np.zeros((nq, 3))
    cov = np.zeros((nq, 3, 3))
    reg = np.tile(np.eye(3), (nq, 1, 1))
    valid = np.zeros(nq, np.uint8)
    for i in range(nq):
        n = int(count[i])
        if n == 0:
            continue
        p = t[idx[i, :n]]
        mean[i] = p.mean(axis=0)
        cov[i] = np.cov(p.T, bias=True) if n > 1 else np.zeros((3, 3))
        if n >= 3:
            w, V = np.linalg.eigh(cov[i])
            v0 = V[:, 0]
            reg[i] = np.eye(3) - (1.0 - eps) * np.outer(v0, v0)
            valid[i] = 1
    return dict(mean=mean, cov=cov, reg=reg, valid=valid)
