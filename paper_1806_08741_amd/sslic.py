"""Thin ctypes binding of libsslic.so (include/sslic.h, include/sslic_steps.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback -- a missing library or a missing GPU raises.

Images are torch tensors of shape ``(*reversed(dims), C)`` (C order, so the
channel is fastest, then axis 0), dtype uint8, uint16 or float32, on a CUDA
(HIP) device.  Labels come back as flat int32 tensors in linear order (axis 0
fastest) and centres as float64 ``(K, C + ndim)`` tensors.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsslic.so")

_DT = {torch.uint8: 0, torch.uint16: 1, torch.float32: 2}

P = ctypes.c_void_p
I = ctypes.c_int
I64 = ctypes.c_int64
D = ctypes.c_double


class SslicError(RuntimeError):
    pass


class _Options(ctypes.Structure):
    _fields_ = [("tol", D), ("no_connectivity", I), ("init_centres", P), ("residuals", P),
                ("iters_done_dev", P), ("n_labels_dev", P), ("no_graph", I), ("no_autotune", I),
                ("persist_distance", I)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("image", P), ("ndim", I), ("dims", I64 * 4), ("channels", I), ("dtype", I),
                ("S", ctypes.c_int32 * 4), ("m", D), ("iterations", I), ("labels", P),
                ("centres", P), ("counts", P), ("residuals", P), ("iters_done", P)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load libsslic.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise SslicError(f"{LIB_PATH} is missing: build it first "
                                 "(python -c 'import __graft_entry__ as g; g.build()')")
            L = ctypes.CDLL(LIB_PATH)
            L.sslic_last_error.restype = ctypes.c_char_p
            L.sslic_create.argtypes = [ctypes.POINTER(P), I]
            L.sslic_destroy.argtypes = [P]
            L.sslic_destroy.restype = None
            L.sslic_num_clusters.argtypes = [I, P, P, P, P]
            L.sslic_run.argtypes = [P, P, I, P, I, I, P, D, I, ctypes.POINTER(_Options), P, P, P,
                                    P, P, P]
            L.sslic_run_static.argtypes = [P, I, P, I, I, P, D, I, ctypes.POINTER(_Options), P,
                                           P, P, P]
            L.sslic_run_batch.argtypes = [P, ctypes.POINTER(ImageDesc), I,
                                          ctypes.POINTER(_Options), P, P]
            L.sslic_seed.argtypes = [P, P, I, P, I, I, P, P, P]
            L.sslic_grid_labels.argtypes = [P, I, P, P, P, P]
            L.sslic_assign.argtypes = [P, P, I, P, I, I, P, D, P, I64, P, P]
            L.sslic_assign_persist.argtypes = [P, P, I, P, I, I, P, D, P, I64, P, P, P]
            L.sslic_update.argtypes = [P, P, I, P, I, I, P, D, P, I64, P, P, P, P]
            L.sslic_connectivity.argtypes = [P, I, P, P, I, P, I64, P, P, P, P]
            L.sslic_mask_contours.argtypes = [P, P, I, P, I, I, P, P, P]
            L.sslic_rgb_to_lab.argtypes = [P, P, I64, P, P]
            for name in ("sslic_create", "sslic_num_clusters", "sslic_run", "sslic_run_static",
                         "sslic_run_batch",
                         "sslic_seed", "sslic_grid_labels", "sslic_assign",
                         "sslic_assign_persist", "sslic_update",
                         "sslic_connectivity", "sslic_mask_contours", "sslic_rgb_to_lab"):
                getattr(L, name).restype = I
            _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        msg = lib().sslic_last_error().decode(errors="replace")
        raise SslicError(f"libsslic error {rc}: {msg}")


def _i64(vals):
    return (I64 * len(vals))(*[int(v) for v in vals])


def _i32(vals):
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def _stream(dev: torch.device):
    return P(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else P(t.data_ptr())


def num_clusters(dims: Sequence[int], S: Sequence[int]) -> int:
    k = I64(0)
    _check(lib().sslic_num_clusters(len(dims), _i64(dims), _i32(S), ctypes.byref(k), None))
    return int(k.value)


def _geom(img: torch.Tensor):
    if not img.is_cuda:
        raise SslicError("the image must be on a GPU; there is no CPU path")
    if img.dtype not in _DT:
        raise SslicError(f"unsupported dtype {img.dtype}")
    if not img.is_contiguous():
        raise SslicError("the image must be contiguous")
    nd = img.dim() - 1
    dims = list(img.shape[:nd])[::-1]
    return nd, dims, int(img.shape[-1]), _DT[img.dtype]


class Context:
    """A libsslic context (owns the device workspace) bound to one device."""

    def __init__(self, device: int | torch.device = 0):
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if dev.type != "cuda":
            raise SslicError("libsslic needs a GPU device")
        self.device = dev
        h = P()
        _check(lib().sslic_create(ctypes.byref(h), dev.index or 0))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().sslic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- whole filter -------------------------------------------------------
    def run(self, img: torch.Tensor, S: Sequence[int], m: float, iterations: int, *,
            tol: float = 0.0, connectivity: bool = True,
            init_centres: Optional[torch.Tensor] = None, residuals: bool = False,
            out: Optional[dict] = None, sync: bool = True,
            persist_distance: bool = False) -> dict:
        """Run SSLIC on one image.  ``out`` may hold preallocated ``labels``,
        ``centres``, ``counts`` tensors.  With ``sync`` the label count and the
        iterations run are read back (the call then waits for the stream).
        ``persist_distance`` keeps the distance image across iterations (the
        loop as Sec. 2.2 and Sec. 3.1 write it, d set to infinity once in
        stage 1) instead of resetting it every iteration."""
        nd, dims, C, dt = _geom(img)
        K = num_clusters(dims, S)
        N = int(img.numel() // C)
        dev = img.device
        out = dict(out or {})
        labels = out.get("labels")
        if labels is None:
            labels = torch.empty(N, dtype=torch.int32, device=dev)
        centres = out.get("centres")
        if centres is None:
            centres = torch.empty((K, C + nd), dtype=torch.float64, device=dev)
        counts = out.get("counts")
        if counts is None:
            counts = torch.empty(K, dtype=torch.int64, device=dev)
        res = torch.zeros(iterations, dtype=torch.float64, device=dev) if residuals else None
        o = _Options(float(tol), 0 if connectivity else 1, None, None, None, None, 0, 0,
                     1 if persist_distance else 0)
        if init_centres is not None:
            ic = init_centres.to(device=dev, dtype=torch.float64).contiguous()
            o.init_centres = ic.data_ptr()
        if res is not None:
            o.residuals = res.data_ptr()
        nl = ctypes.c_int32(0)
        it = ctypes.c_int32(0)
        _check(lib().sslic_run(self._h, _ptr(img), nd, _i64(dims), C, dt, _i32(S), float(m),
                               int(iterations), ctypes.byref(o), _ptr(labels), _ptr(centres),
                               _ptr(counts), ctypes.byref(nl) if sync else None,
                               ctypes.byref(it) if sync else None, _stream(dev)))
        r = {"labels": labels, "centres": centres, "counts": counts}
        if res is not None:
            r["residuals"] = res
        if sync:
            r["n_labels"] = int(nl.value)
            r["iterations"] = int(it.value)
            if res is not None:
                r["residuals"] = res[: r["iterations"]]
        return r

    def run_batch(self, items: list, *, tol: float = 0.0, connectivity: bool = False,
                  sync: bool = True, graph: bool = True, autotune: bool = True) -> list:
        """Run many images in one batched call (``sslic_run_batch``).

        ``items`` holds dicts with ``image``, ``S``, ``m``, ``iterations`` and
        optional preallocated ``labels``/``centres``/``counts``/``residuals``/
        ``iters`` (device int32 [1]).  Returns one dict of outputs per item;
        with ``sync`` also ``n_labels``.  Calling again with the same tensors
        and options replays the captured graph."""
        n = len(items)
        descs = (ImageDesc * max(n, 1))()
        outs = []
        for i, itm in enumerate(items):
            img = itm["image"]
            nd, dims, C, dt = _geom(img)
            S = list(itm["S"])
            K = num_clusters(dims, S)
            N = int(img.numel() // C)
            dev = img.device
            lab = itm.get("labels")
            if lab is None:
                lab = torch.empty(N, dtype=torch.int32, device=dev)
            cen = itm.get("centres")
            if cen is None:
                cen = torch.empty((K, C + nd), dtype=torch.float64, device=dev)
            cnt = itm.get("counts")
            if cnt is None:
                cnt = torch.empty(K, dtype=torch.int64, device=dev)
            res = itm.get("residuals")
            if res is None and itm.get("want_residuals"):
                res = torch.zeros(int(itm["iterations"]), dtype=torch.float64, device=dev)
            its = itm.get("iters")
            if its is None:
                its = torch.zeros(1, dtype=torch.int32, device=dev)
            d = descs[i]
            d.image = img.data_ptr()
            d.ndim = nd
            for a in range(4):
                d.dims[a] = int(dims[a]) if a < nd else 1
                d.S[a] = int(S[a]) if a < nd else 1
            d.channels = C
            d.dtype = dt
            d.m = float(itm["m"])
            d.iterations = int(itm["iterations"])
            d.labels = lab.data_ptr()
            d.centres = cen.data_ptr()
            d.counts = cnt.data_ptr()
            d.residuals = res.data_ptr() if res is not None else None
            d.iters_done = its.data_ptr()
            outs.append({"labels": lab, "centres": cen, "counts": cnt, "residuals": res,
                         "iters": its})
        o = _Options(float(tol), 0 if connectivity else 1, None, None, None, None,
                     0 if graph else 1, 0 if autotune else 1)
        nl = (ctypes.c_int32 * max(n, 1))()
        dev = items[0]["image"].device if n else self.device
        _check(lib().sslic_run_batch(self._h, descs, n, ctypes.byref(o), nl if sync else None,
                                     _stream(dev)))
        if sync:
            for i in range(n):
                outs[i]["n_labels"] = int(nl[i])
        return outs

    # -- single steps -------------------------------------------------------
    def seed(self, img: torch.Tensor, S: Sequence[int]) -> torch.Tensor:
        nd, dims, C, dt = _geom(img)
        K = num_clusters(dims, S)
        cen = torch.empty((K, C + nd), dtype=torch.float64, device=img.device)
        _check(lib().sslic_seed(self._h, _ptr(img), nd, _i64(dims), C, dt, _i32(S), _ptr(cen),
                                _stream(img.device)))
        return cen

    def grid_labels(self, dims: Sequence[int], S: Sequence[int]) -> torch.Tensor:
        N = 1
        for d in dims:
            N *= int(d)
        lab = torch.empty(N, dtype=torch.int32, device=self.device)
        _check(lib().sslic_grid_labels(self._h, len(dims), _i64(dims), _i32(S), _ptr(lab),
                                       _stream(self.device)))
        return lab

    def assign(self, img: torch.Tensor, S, m, centres: torch.Tensor, labels: torch.Tensor):
        """One assignment step in place on ``labels`` (kept where no window reaches)."""
        nd, dims, C, dt = _geom(img)
        centres = centres.to(device=img.device, dtype=torch.float64).contiguous()
        assert labels.dtype == torch.int32 and labels.is_contiguous() and labels.is_cuda
        _check(lib().sslic_assign(self._h, _ptr(img), nd, _i64(dims), C, dt, _i32(S), float(m),
                                  _ptr(centres), centres.shape[0], _ptr(labels),
                                  _stream(img.device)))
        return labels

    def assign_persist(self, img: torch.Tensor, S, m, centres: torch.Tensor,
                       labels: torch.Tensor, dist: torch.Tensor):
        """One assignment step on a kept distance image, in place on ``labels``
        (int32) and ``dist`` (float32 squared distances, +inf where no centre
        has reached yet)."""
        nd, dims, C, dt = _geom(img)
        centres = centres.to(device=img.device, dtype=torch.float64).contiguous()
        for t, want in ((labels, torch.int32), (dist, torch.float32)):
            if t.device != img.device or t.dtype != want or not t.is_contiguous():
                raise SslicError(f"expected a contiguous {want} tensor on the image's device")
            if t.numel() != img.numel() // C:
                raise SslicError("labels and dist must hold one value per voxel")
        _check(lib().sslic_assign_persist(self._h, _ptr(img), nd, _i64(dims), C, dt, _i32(S),
                                          float(m), _ptr(centres), centres.shape[0],
                                          _ptr(labels), _ptr(dist), _stream(img.device)))
        return labels, dist

    def update(self, img: torch.Tensor, S, m, labels: torch.Tensor, centres: torch.Tensor):
        """One update step: returns (new centres, counts, residual tensor[1])."""
        nd, dims, C, dt = _geom(img)
        cen = centres.to(device=img.device, dtype=torch.float64).clone().contiguous()
        K = cen.shape[0]
        counts = torch.empty(K, dtype=torch.int64, device=img.device)
        res = torch.zeros(1, dtype=torch.float64, device=img.device)
        _check(lib().sslic_update(self._h, _ptr(img), nd, _i64(dims), C, dt, _i32(S), float(m),
                                  _ptr(labels), K, _ptr(cen), _ptr(counts), _ptr(res),
                                  _stream(img.device)))
        return cen, counts, res

    def mask_contours(self, img: torch.Tensor, labels: torch.Tensor,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The image with its label contours set to 0 (``sslic_mask_contours``)."""
        nd, dims, C, dt = _geom(img)
        if labels.device != img.device or labels.dtype != torch.int32 or not labels.is_contiguous():
            raise SslicError("labels must be a contiguous int32 tensor on the image's device")
        if labels.numel() != img.numel() // C:
            raise SslicError("labels must hold one entry per voxel")
        if out is None:
            out = torch.empty_like(img)
        _check(lib().sslic_mask_contours(self._h, _ptr(img), nd, _i64(dims), C, dt,
                                         _ptr(labels), _ptr(out), _stream(img.device)))
        return out

    def rgb_to_lab(self, rgb: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """8-bit sRGB (..., 3) to CIE-Lab float32 of the same shape
        (``sslic_rgb_to_lab``)."""
        if not rgb.is_cuda or rgb.dtype != torch.uint8 or rgb.shape[-1] != 3 or \
                not rgb.is_contiguous():
            raise SslicError("rgb must be a contiguous uint8 (..., 3) tensor on a GPU")
        if out is None:
            out = torch.empty(rgb.shape, dtype=torch.float32, device=rgb.device)
        _check(lib().sslic_rgb_to_lab(self._h, _ptr(rgb), rgb.numel() // 3, _ptr(out),
                                      _stream(rgb.device)))
        return out

    def connectivity(self, dims, S, centres: torch.Tensor, C: int, labels: torch.Tensor) -> int:
        """Connectivity enforcement in place on ``labels``; returns n_labels."""
        centres = centres.to(device=labels.device, dtype=torch.float64).contiguous()
        nl = ctypes.c_int32(0)
        _check(lib().sslic_connectivity(self._h, len(dims), _i64(dims), _i32(S), int(C),
                                        _ptr(centres), centres.shape[0], _ptr(labels),
                                        ctypes.byref(nl), None, _stream(labels.device)))
        return int(nl.value)


_default: dict = {}


def context(device: int = 0) -> Context:
    """A shared context per device."""
    c = _default.get(device)
    if c is None:
        c = _default[device] = Context(device)
    return c


def run(img: torch.Tensor, S, m, iterations, **kw) -> dict:
    return context(img.device.index or 0).run(img, S, m, iterations, **kw)


STATIC_SCRATCH_BYTES = 64 << 20  # SSLIC_STATIC_SCRATCH_BYTES


def run_static(img: torch.Tensor, S, m, iterations, *, tol: float = 0.0,
               connectivity: bool = True, out: Optional[dict] = None,
               persist_distance: bool = False) -> dict:
    """``sslic_run_static``: the whole filter with no device allocation in
    the library (its workspace is a static device array of 64 MiB per GPU).
    ``out`` must then hold preallocated ``labels`` (int32 [N]), ``centres``
    (float64 [K, C + ndim]), ``counts`` (int64 [K]), ``n_labels`` and
    ``iterations`` (int32 [1] each) on the image's device; without ``out``
    they are allocated here with torch.  Nothing waits for the stream: the
    label count and the iterations run stay in those device tensors."""
    nd, dims, C, dt = _geom(img)
    dev = img.device
    o = dict(out or {})
    if not o:
        K = num_clusters(dims, S)
        N = int(img.numel() // C)
        o = {"labels": torch.empty(N, dtype=torch.int32, device=dev),
             "centres": torch.empty((K, C + nd), dtype=torch.float64, device=dev),
             "counts": torch.empty(K, dtype=torch.int64, device=dev),
             "n_labels": torch.zeros(1, dtype=torch.int32, device=dev),
             "iterations": torch.zeros(1, dtype=torch.int32, device=dev)}
    opt = _Options(float(tol), 0 if connectivity else 1, None, None,
                   o["iterations"].data_ptr(), o["n_labels"].data_ptr(), 0, 0,
                   1 if persist_distance else 0)
    with torch.cuda.device(dev):
        _check(lib().sslic_run_static(_ptr(img), nd, _i64(dims), C, dt, _i32(S), float(m),
                                      int(iterations), ctypes.byref(opt), _ptr(o["labels"]),
                                      _ptr(o["centres"]), _ptr(o["counts"]), _stream(dev)))
    return o
