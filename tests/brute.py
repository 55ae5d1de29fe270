"""Independent brute-force checks used to pin the oracle.

Nothing here calls the oracle or the HIP library.  The assignment is written
as plain k-means in the joint (channels, scaled coordinates) space through
``scipy.spatial.distance.cdist``; the update is ``numpy.bincount``; the
connectivity check uses ``scipy.ndimage.label``.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage
from scipy.spatial.distance import cdist


def coords(dims):
    """(N, n) integer coordinates in linear order, axis 0 fastest."""
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    # linear order with axis 0 fastest == Fortran order over (x, y, z)
    return np.stack([g.ravel(order="F") for g in grids], 1)


def features(img, dims):
    """(N, C) float64 channel values in linear order."""
    C = img.shape[-1]
    return np.asarray(img, dtype=np.float64).reshape(-1, C)


def kmeans_assign(img, dims, S, m, centres, window=False, prev=None):
    """Plain k-means assignment in the joint space [I, x*m/S].

    Scaling coordinates by m/S_i turns the paper's weighted distance into an
    ordinary squared Euclidean distance, so the argmin over all centres is
    textbook k-means.  With ``window`` the distance is +inf wherever some
    |x_i - c_i| > S_i and voxels with no finite distance keep ``prev``.
    """
    dims = list(dims)
    n = len(dims)
    C = img.shape[-1]
    X = coords(dims).astype(np.float64)
    scale = np.array([m / s for s in S], dtype=np.float64)
    f = np.concatenate([features(img, dims), X * scale], 1)
    g = np.concatenate([centres[:, :C], centres[:, C:] * scale], 1)
    D = cdist(f, g, "sqeuclidean")
    if window:
        out = np.zeros(D.shape, dtype=bool)
        for i in range(n):
            out |= np.abs(X[:, i:i + 1] - centres[None, :, C + i]) > S[i]
        D[out] = np.inf
    lab = np.argmin(D, 1).astype(np.int32)  # first index among equal minima
    if window:
        none = ~np.isfinite(D).any(1)
        lab[none] = prev[none]
    return lab


def kmeans_assign_persist(img, dims, S, m, centres, prev, dist):
    """The windowed k-means step on a kept distance image: the least windowed
    squared distance of each voxel replaces ``dist`` and its (first) argmin
    replaces ``prev`` only where it is strictly below ``dist``.  Returns new
    (labels, dist)."""
    dims = list(dims)
    n = len(dims)
    C = img.shape[-1]
    X = coords(dims).astype(np.float64)
    scale = np.array([m / s for s in S], dtype=np.float64)
    f = np.concatenate([features(img, dims), X * scale], 1)
    g = np.concatenate([centres[:, :C], centres[:, C:] * scale], 1)
    D = cdist(f, g, "sqeuclidean")
    out = np.zeros(D.shape, dtype=bool)
    for i in range(n):
        out |= np.abs(X[:, i:i + 1] - centres[None, :, C + i]) > S[i]
    D[out] = np.inf
    best = D.min(1)
    arg = np.argmin(D, 1).astype(np.int32)
    take = best < dist
    return np.where(take, arg, prev).astype(np.int32), np.where(take, best, dist)


def bincount_update(img, dims, labels, centres):
    """Member means via numpy.bincount; empty clusters keep their centre."""
    K = centres.shape[0]
    C = img.shape[-1]
    X = coords(dims)
    cnt = np.bincount(labels, minlength=K)
    out = centres.copy()
    nz = cnt > 0
    F = features(img, dims)
    for c in range(C):
        if np.issubdtype(img.dtype, np.integer):
            s = np.zeros(K, dtype=np.int64)
            np.add.at(s, labels, F[:, c].astype(np.int64))
            out[nz, c] = s[nz] / cnt[nz]
        else:
            s = np.bincount(labels, weights=F[:, c], minlength=K)
            out[nz, c] = s[nz] / cnt[nz]
    for i in range(X.shape[1]):
        s = np.zeros(K, dtype=np.int64)
        np.add.at(s, labels, X[:, i])
        out[nz, C + i] = s[nz] / cnt[nz]
    return out, cnt


def grid_cell_labels(dims, K_axis):
    """Label of the grid cell of every voxel: sum_i floor(x_i K_i / N_i) * stride_i."""
    X = coords(dims)
    lab = np.zeros(X.shape[0], dtype=np.int64)
    st = 1
    for i, d in enumerate(dims):
        lab += (X[:, i] * K_axis[i] // d) * st
        st *= K_axis[i]
    return lab.astype(np.int32)


def components(labels, dims):
    """Face-connected components of equal labels (scipy.ndimage.label per label).

    Returns (component id per voxel in linear order, sizes)."""
    arr = labels.reshape(tuple(dims[::-1]))
    comp = np.zeros(arr.shape, dtype=np.int64)
    nxt = 0
    for v in np.unique(arr):
        lab, k = ndimage.label(arr == v)  # default structure = face adjacency
        sel = lab > 0
        comp[sel] = lab[sel] + nxt
        nxt += k
    flat = comp.ravel()
    sizes = np.bincount(flat)
    return flat, sizes
