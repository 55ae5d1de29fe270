"""FP64 CPU reference ("oracle") of the SSLIC per-iteration path.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the HIP library and
its Python binding never do, and nothing here imports them.

The arithmetic lives in ``sslic_oracle.c`` (plain C, FP64, no fused
multiply-add); this module only marshals numpy arrays through ctypes.  Each
function names the part of the paper it follows:

* ``seed``          Sec. 2.2 / 3.1 stage 1 -- grid sampling, move to the lowest
                    gradient magnitude in the 3^n neighbourhood
* ``assign``        Sec. 2.1 distance (per-axis weights of Sec. 3.3), Sec. 3.1
                    stage 2 -- one assignment step over every centre's window
* ``update``        Sec. 3.1 stage 2 -- centres become member means; residual
                    of Sec. 3.2
* ``connectivity``  Sec. 3.1 stage 3 -- marker image, first pass per centre,
                    raster scan of the rest
* ``run``           the whole filter
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sslic_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsslic_oracle.so")

U8, U16, F32 = 0, 1, 2
_DTYPES = {np.dtype(np.uint8): U8, np.dtype(np.uint16): U16, np.dtype(np.float32): F32}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, -ffp-contract=off)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.or_num_clusters.argtypes = [I, P, P, P, P]
        lib.or_grid_labels.argtypes = [I, P, P, P]
        lib.or_seed.argtypes = [P, I, P, I, I, P, P]
        lib.or_assign.argtypes = [P, I, P, I, I, P, D, P, I64, P]
        lib.or_assign_points.argtypes = [P, I, P, I, I, P, D, P, I64, P, I64, P, P]
        lib.or_update.argtypes = [P, I, P, I, I, P, D, P, I64, P, P, P]
        lib.or_connectivity.argtypes = [I, P, P, P, I, I64, P, P]
        lib.or_assign_persist.argtypes = [P, I, P, I, I, P, D, P, I64, P, P]
        lib.or_run.argtypes = [P, I, P, I, I, P, D, I, D, I, I, P, P, P, P, P, P, P]
        lib.or_mask_contours.argtypes = [P, I, P, I, I, P, P]
        lib.or_rgb_to_lab.argtypes = [P, I64, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _geom(img: np.ndarray, ndim: int):
    """Split an array of shape (dims reversed..., C) into (dims, C).

    Arrays are indexed [z, y, x, c] (C order), so axis 0 (x) is fastest, as
    the C side expects.
    """
    img = np.ascontiguousarray(img)
    if img.dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {img.dtype}")
    if img.ndim != ndim + 1:
        raise ValueError("image must have shape (*reversed(dims), C)")
    dims = np.array(img.shape[:ndim][::-1], dtype=np.int64)
    return img, dims, int(img.shape[-1]), _DTYPES[img.dtype]


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle returned {rc}")


def num_clusters(dims, S):
    dims = np.asarray(dims, dtype=np.int64)
    S = np.asarray(S, dtype=np.int32)
    ka = np.zeros(len(dims), dtype=np.int64)
    k = np.zeros(1, dtype=np.int64)
    _check(_load().or_num_clusters(len(dims), _ptr(dims), _ptr(S), _ptr(ka), _ptr(k)))
    return int(k[0]), ka


def grid_labels(dims, S):
    dims = np.asarray(dims, dtype=np.int64)
    S = np.asarray(S, dtype=np.int32)
    out = np.empty(int(np.prod(dims)), dtype=np.int32)
    _check(_load().or_grid_labels(len(dims), _ptr(dims), _ptr(S), _ptr(out)))
    return out


def seed(img, ndim, S):
    img, dims, C, dt = _geom(img, ndim)
    S = np.asarray(S, dtype=np.int32)
    K, _ = num_clusters(dims, S)
    cen = np.zeros((K, C + ndim), dtype=np.float64)
    _check(_load().or_seed(_ptr(img), ndim, _ptr(dims), C, dt, _ptr(S), _ptr(cen)))
    return cen


def assign(img, ndim, S, m, centres, labels):
    """One assignment step; ``labels`` (int32, N) is updated in place for every
    covered voxel and kept where no window reaches."""
    img, dims, C, dt = _geom(img, ndim)
    S = np.asarray(S, dtype=np.int32)
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    assert labels.dtype == np.int32 and labels.flags.c_contiguous
    _check(_load().or_assign(_ptr(img), ndim, _ptr(dims), C, dt, _ptr(S), float(m),
                             _ptr(centres), centres.shape[0], _ptr(labels)))
    return labels


def assign_persist(img, ndim, S, m, centres, labels, dist):
    """One assignment step on a distance image kept between iterations:
    ``labels`` (int32, N) and ``dist`` (float64 squared distances, N, +inf
    where no centre has reached yet) are updated in place."""
    img, dims, C, dt = _geom(img, ndim)
    S = np.asarray(S, dtype=np.int32)
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    assert labels.dtype == np.int32 and labels.flags.c_contiguous
    assert dist.dtype == np.float64 and dist.flags.c_contiguous and dist.size == labels.size
    _check(_load().or_assign_persist(_ptr(img), ndim, _ptr(dims), C, dt, _ptr(S), float(m),
                                     _ptr(centres), centres.shape[0], _ptr(labels),
                                     _ptr(dist)))
    return labels, dist


def assign_points(img, ndim, S, m, centres, points):
    """Labels (int32, -1 where no window holds the voxel) and least distances
    of the voxels at linear indices ``points``, each computed on its own over
    every centre."""
    img, dims, C, dt = _geom(img, ndim)
    S = np.asarray(S, dtype=np.int32)
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    lab = np.empty(pts.shape[0], dtype=np.int32)
    dist = np.empty(pts.shape[0], dtype=np.float64)
    _check(_load().or_assign_points(_ptr(img), ndim, _ptr(dims), C, dt, _ptr(S), float(m),
                                    _ptr(centres), centres.shape[0], _ptr(pts), pts.shape[0],
                                    _ptr(lab), _ptr(dist)))
    return lab, dist


def update(img, ndim, S, m, labels, centres):
    """One update step: returns (new centres, counts, residual)."""
    img, dims, C, dt = _geom(img, ndim)
    S = np.asarray(S, dtype=np.int32)
    cen = np.array(centres, dtype=np.float64, copy=True)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    counts = np.zeros(cen.shape[0], dtype=np.int64)
    res = np.zeros(1, dtype=np.float64)
    _check(_load().or_update(_ptr(img), ndim, _ptr(dims), C, dt, _ptr(S), float(m),
                             _ptr(labels), cen.shape[0], _ptr(cen), _ptr(counts),
                             _ptr(res)))
    return cen, counts, float(res[0])


def connectivity(dims, S, centres, C, labels):
    """Connectivity enforcement in place on ``labels``; returns n_labels."""
    dims = np.asarray(dims, dtype=np.int64)
    S = np.asarray(S, dtype=np.int32)
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    assert labels.dtype == np.int32 and labels.flags.c_contiguous
    nl = np.zeros(1, dtype=np.int32)
    _check(_load().or_connectivity(len(dims), _ptr(dims), _ptr(S), _ptr(centres), C,
                                   centres.shape[0], _ptr(labels), _ptr(nl)))
    return int(nl[0])


def rgb_to_lab(rgb):
    """8-bit RGB (..., 3) to CIE-Lab (FP64, same shape)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    assert rgb.shape[-1] == 3
    out = np.empty(rgb.shape, dtype=np.float64)
    _check(_load().or_rgb_to_lab(_ptr(rgb), rgb.size // 3, _ptr(out)))
    return out


def mask_contours(img, ndim, labels):
    """The image with its label contours set to 0 (same shape and dtype)."""
    img, dims, C, dt = _geom(img, ndim)
    labels = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    assert labels.size == int(np.prod(dims))
    out = np.empty_like(img)
    _check(_load().or_mask_contours(_ptr(img), ndim, _ptr(dims), C, dt, _ptr(labels), _ptr(out)))
    return out


def run(img, ndim, S, m, iterations, tol=0.0, connectivity=True, init_centres=None,
        persist_distance=False):
    """The whole filter.  Returns a dict with labels (flat int32), centres,
    counts, residuals, iterations run and n_labels.  ``persist_distance``
    keeps the distance image across iterations instead of resetting it."""
    img, dims, C, dt = _geom(img, ndim)
    S = np.asarray(S, dtype=np.int32)
    K, _ = num_clusters(dims, S)
    N = int(np.prod(dims))
    labels = np.zeros(N, dtype=np.int32)
    cen = np.zeros((K, C + ndim), dtype=np.float64)
    counts = np.zeros(K, dtype=np.int64)
    res = np.zeros(iterations, dtype=np.float64)
    it = np.zeros(1, dtype=np.int32)
    nl = np.zeros(1, dtype=np.int32)
    init = None
    if init_centres is not None:
        init = np.ascontiguousarray(init_centres, dtype=np.float64)
    _check(_load().or_run(_ptr(img), ndim, _ptr(dims), C, dt, _ptr(S), float(m),
                          int(iterations), float(tol), int(bool(connectivity)),
                          int(bool(persist_distance)), _ptr(init), _ptr(labels), _ptr(cen),
                          _ptr(counts), _ptr(res), _ptr(it), _ptr(nl)))
    return {"labels": labels, "centres": cen, "counts": counts,
            "residuals": res[: int(it[0])], "iterations": int(it[0]),
            "n_labels": int(nl[0])}
