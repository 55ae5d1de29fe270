"""Seeded synthetic images shaped like the paper's workloads.

This module only *generates inputs*; it holds none of the SLIC arithmetic and
imports neither the HIP binding nor the oracle, so both sides can be fed the
same bytes.  All images are Voronoi partitions plus Gaussian noise:

* slide-like 2D RGB uint8 (whole-slide histology, Sec. 1 of the paper),
* FIB-SEM-like 3D single-channel uint16 with dark 2-voxel membranes,
* confocal-like 3D multi-channel float32,

with the recipe of each workload written out in ``WORKLOADS`` below.

Arrays are laid out as ``(*reversed(dims), C)`` in C order, i.e. channel
fastest, then axis 0 (x), axis 1 (y), ...  Parameters drawn per image (seed
positions, region means) come from ``numpy.random.default_rng([key...])``; the
per-voxel noise comes from a ``torch.Generator`` seeded from the same key on
the device the image is generated on.  Generate once and copy: the same
device and seed always give the same bytes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np
import torch

__all__ = ["Workload", "WORKLOADS", "voronoi", "voronoi_image", "workload_image",
           "batch_specs", "batch_image", "request_trace", "request_image"]


@dataclass(frozen=True)
class Workload:
    """A named synthetic workload: image geometry, content and SLIC parameters."""
    name: str
    dims: tuple          # axis 0 first
    channels: int
    dtype: torch.dtype
    S: tuple
    m: float
    iterations: int
    connectivity: bool
    n_seeds: int
    recipe: str          # human-readable content recipe
    extra: dict = field(default_factory=dict)

    @property
    def voxels(self) -> int:
        return int(np.prod(self.dims))


WORKLOADS = {
    "rgb-256": Workload(
        "rgb-256", (256, 256), 3, torch.uint8, (16, 16), 10.0, 10, True, 64,
        "Voronoi of 64 uniform seeds; region mean U[0,255]^3; noise sigma 8; "
        "rint, clip [0,255]"),
    "slide-16k": Workload(
        "slide-16k", (16384, 16384), 3, torch.uint8, (16, 16), 10.0, 10, False, 20000,
        "Voronoi of 20000 uniform seeds; region mean R~U[150,235], G~U[60,150], "
        "B~U[140,220]; noise sigma 10; every channel + 15 sin(2 pi (x + y/2)/16384); "
        "rint, clip [0,255]",
        {"ranges": ((150, 235), (60, 150), (140, 220)), "sigma": 10.0,
         "ramp": (15.0, 16384.0)}),
    "fibsem-1k": Workload(
        "fibsem-1k", (1024, 1024, 1024), 1, torch.uint16, (8, 8, 8), 20.0, 10, True,
        50000,
        "3D Voronoi of 50000 uniform seeds; cell mean U[2000,50000]; voxels whose "
        "bisector distance to the second-nearest seed is < 1 voxel get mean 600 "
        "(2-voxel membranes); noise sigma 800; rint, clip [0,65535]",
        {"ranges": ((2000, 50000),), "sigma": 800.0, "membrane": 600.0}),
    "lab-2k": Workload(
        "lab-2k", (2048, 1216), 3, torch.float32, (50, 50), 10.0, 5, True, 1000,
        "Voronoi of 1000 uniform seeds; region mean L~U[0,100], a~U[-86.185,98.254], "
        "b~U[-107.863,94.482] (the CIE-Lab ranges of 8-bit sRGB); noise sigma 2; "
        "float32, clip to those ranges",
        {"ranges": ((0.0, 100.0), (-86.185, 98.254), (-107.863, 94.482)), "sigma": 2.0}),
}


# ---------------------------------------------------------------------------
# Voronoi partition with a bucket grid (exact; far voxels fall back to brute force)

def voronoi(dims: Sequence[int], seeds: np.ndarray, device, top2: bool = False,
            chunk_voxels: int = 1 << 24):
    """Index of the nearest seed for every voxel (ties to the lower index).

    ``dims`` is axis-0-first; ``seeds`` is (P, n) float in voxel units.  The
    result is a flat int32 tensor in linear order (axis 0 fastest).  With
    ``top2`` the second-nearest index and both squared distances are returned
    too.  Seeds are bucketed into cells holding about three seeds each; a
    voxel's answer from its 3^n cells is exact whenever the distance found is
    below the cell size, otherwise it is recomputed against every seed.
    """
    dims = [int(d) for d in dims]
    n = len(dims)
    N = int(np.prod(dims))
    P = seeds.shape[0]
    dev = torch.device(device)
    B = max(1.0, (N / P * 3.0) ** (1.0 / n))
    nb = [max(1, math.ceil(d / B)) for d in dims]
    cst = [1] * n
    for i in range(1, n):
        cst[i] = cst[i - 1] * nb[i - 1]
    ncell = cst[-1] * nb[-1]
    sd = torch.as_tensor(seeds, dtype=torch.float32, device=dev)
    scell = torch.zeros(P, dtype=torch.int64, device=dev)
    for i in range(n):
        ci = torch.clamp((sd[:, i] / B).floor().long(), 0, nb[i] - 1)
        scell += ci * cst[i]
    order = torch.argsort(scell, stable=True)
    cnt = torch.bincount(scell, minlength=ncell)
    M = int(cnt.max().item())
    start = torch.cumsum(cnt, 0) - cnt
    sc_sorted = scell[order]
    rank = torch.arange(P, device=dev) - start[sc_sorted]
    table = torch.full((ncell, M), P, dtype=torch.int64, device=dev)
    table[sc_sorted, rank] = order
    far = torch.full((1, n), 1e9, dtype=torch.float32, device=dev)
    sdp = torch.cat([sd, far], 0)

    out1 = torch.empty(N, dtype=torch.int32, device=dev)
    out2 = torch.empty(N, dtype=torch.int32, device=dev) if top2 else None
    od1 = torch.empty(N, dtype=torch.float32, device=dev) if top2 else None
    od2 = torch.empty(N, dtype=torch.float32, device=dev) if top2 else None
    slab = int(np.prod(dims[:-1]))
    rows_per = max(1, chunk_voxels // slab)
    for z0 in range(0, dims[-1], rows_per):
        z1 = min(dims[-1], z0 + rows_per)
        lin = torch.arange(z0 * slab, z1 * slab, device=dev)
        coord = []
        r = lin
        for i in range(n):
            coord.append((r % dims[i]).float())
            r = r // dims[i]
        vcell = []
        for i in range(n):
            vcell.append(torch.clamp((coord[i] / B).floor().long(), 0, nb[i] - 1))
        b1 = torch.full_like(coord[0], float("inf"))
        i1 = torch.full(lin.shape, P, dtype=torch.int64, device=dev)
        b2 = b1.clone() if top2 else None
        i2 = i1.clone() if top2 else None
        for o in range(3 ** n):
            oo = o
            cl = torch.zeros_like(lin)
            ok = torch.ones(lin.shape, dtype=torch.bool, device=dev)
            for i in range(n):
                ci = vcell[i] + (oo % 3) - 1
                oo //= 3
                ok &= (ci >= 0) & (ci < nb[i])
                cl += ci.clamp(0, nb[i] - 1) * cst[i]
            for s in range(M):
                sidx = torch.where(ok, table[cl, s], P)
                sp = sdp[sidx]
                d = torch.zeros_like(b1)
                for i in range(n):
                    d += (coord[i] - sp[:, i]) ** 2
                _top_update(d, sidx, b1, i1, b2, i2)
        # exactness: anything farther than one cell may have been missed
        bad = (b2 if top2 else b1) >= B * B
        if bool(bad.any()):
            bi = torch.nonzero(bad).squeeze(1)
            for c0 in range(0, bi.numel(), 4096):
                sel = bi[c0:c0 + 4096]
                pc = torch.stack([coord[i][sel] for i in range(n)], 1)
                dd = ((pc[:, None, :] - sd[None, :, :]) ** 2).sum(-1)
                # stable sort keeps the lower index first among equal distances
                srt, arg = torch.sort(dd, dim=1, stable=True)
                b1[sel] = srt[:, 0]
                i1[sel] = arg[:, 0]
                if top2:
                    b2[sel] = srt[:, 1] if P > 1 else float("inf")
                    i2[sel] = arg[:, 1] if P > 1 else P
        out1[z0 * slab:z1 * slab] = i1.int()
        if top2:
            out2[z0 * slab:z1 * slab] = i2.int()
            od1[z0 * slab:z1 * slab] = b1
            od2[z0 * slab:z1 * slab] = b2
    if top2:
        return out1, out2, od1, od2
    return out1


def _top_update(d, sidx, b1, i1, b2, i2):
    """Keep the smallest (and second smallest) distance; ties go to the lower index."""
    better1 = (d < b1) | ((d == b1) & (sidx < i1))
    if b2 is not None:
        # candidate displaces the current best into second place, or beats second
        new2_from1 = better1
        better2 = (~better1) & ((d < b2) | ((d == b2) & (sidx < i2))) & (sidx != i1)
        nb2 = torch.where(new2_from1, b1, torch.where(better2, d, b2))
        ni2 = torch.where(new2_from1, i1, torch.where(better2, sidx, i2))
        b2.copy_(nb2)
        i2.copy_(ni2)
    b1.copy_(torch.where(better1, d, b1))
    i1.copy_(torch.where(better1, sidx, i1))


# ---------------------------------------------------------------------------

_TORCH_TO_NP = {torch.uint8: np.uint8, torch.uint16: np.uint16, torch.float32: np.float32}


def _finish(vals: torch.Tensor, dtype: torch.dtype, lo: float, hi: float) -> torch.Tensor:
    vals = vals.clamp_(lo, hi)
    if dtype == torch.float32:
        return vals.to(torch.float32)
    vals = torch.round(vals)  # round half to even == numpy rint
    if dtype == torch.uint16:
        return vals.to(torch.int32).to(torch.uint16)
    return vals.to(dtype)


def voronoi_image(dims: Sequence[int], channels: int, dtype: torch.dtype, n_seeds: int,
                  means: np.ndarray, sigma: float, key: Sequence[int], device,
                  clip=(0.0, 255.0), ramp: Optional[tuple] = None,
                  membrane: Optional[float] = None, seeds: Optional[np.ndarray] = None):
    """Voronoi-plus-noise image of shape (*reversed(dims), C).

    ``means`` is (n_seeds, C); ``ramp=(amp, period)`` adds amp*sin(2 pi (x + y/2)/period)
    to every channel; ``membrane=v`` gives mean v to voxels within one voxel of the
    bisector with the second-nearest seed.
    """
    dims = [int(d) for d in dims]
    n = len(dims)
    dev = torch.device(device)
    if seeds is None:
        rng = np.random.default_rng(list(key) + [1])
        seeds = rng.uniform(0.0, 1.0, size=(n_seeds, n)) * np.asarray(dims, dtype=np.float64)
    if membrane is not None:
        i1, i2, d1, d2 = voronoi(dims, seeds, dev, top2=True)
    else:
        i1 = voronoi(dims, seeds, dev)
    mt = torch.as_tensor(np.asarray(means, dtype=np.float32), device=dev)
    N = int(np.prod(dims))
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(np.random.default_rng(list(key) + [2]).integers(0, 2**62)))
    out = torch.empty((N, channels), dtype=dtype, device=dev)
    chunk = 1 << 24
    sd = torch.as_tensor(seeds, dtype=torch.float32, device=dev)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        idx = i1[a:b].long()
        v = mt[idx].clone()
        if membrane is not None:
            j = i2[a:b].long()
            sep = torch.sqrt(((sd[idx] - sd[j]) ** 2).sum(1)).clamp_min(1e-6)
            bis = (d2[a:b] - d1[a:b]) / (2.0 * sep)
            v[bis < 1.0] = float(membrane)
        if ramp is not None:
            lin = torch.arange(a, b, device=dev)
            x = (lin % dims[0]).float()
            y = ((lin // dims[0]) % dims[1]).float() if n > 1 else torch.zeros_like(x)
            v += (ramp[0] * torch.sin(2.0 * math.pi * (x + 0.5 * y) / ramp[1]))[:, None]
        v += sigma * torch.randn(v.shape, generator=gen, device=dev)
        out[a:b] = _finish(v, dtype, clip[0], clip[1])
    return out.reshape(*dims[::-1], channels)


def workload_image(name: str, device, dims: Optional[Sequence[int]] = None, index: int = 0):
    """The image of a named workload, optionally at other ``dims`` (same recipe,
    seed count scaled with the voxel count, at least 8)."""
    w = WORKLOADS[name]
    full = w.dims
    dims = tuple(full if dims is None else dims)
    scale = float(np.prod(dims)) / float(np.prod(full))
    ns = max(8, int(round(w.n_seeds * scale)))
    key = [sum(ord(c) for c in name), index, *dims]
    rng = np.random.default_rng(key + [3])
    if name == "rgb-256":
        means = rng.uniform(0.0, 255.0, size=(ns, 3))
        return voronoi_image(dims, 3, torch.uint8, ns, means, 8.0, key, device)
    if name == "slide-16k":
        r = w.extra["ranges"]
        means = np.stack([rng.uniform(lo, hi, size=ns) for lo, hi in r], 1)
        return voronoi_image(dims, 3, torch.uint8, ns, means, w.extra["sigma"], key, device,
                             ramp=w.extra["ramp"])
    if name == "fibsem-1k":
        lo, hi = w.extra["ranges"][0]
        means = rng.uniform(lo, hi, size=(ns, 1))
        return voronoi_image(dims, 1, torch.uint16, ns, means, w.extra["sigma"], key, device,
                             clip=(0.0, 65535.0), membrane=w.extra["membrane"])
    if name == "lab-2k":
        r = w.extra["ranges"]
        means = np.stack([rng.uniform(lo, hi, size=ns) for lo, hi in r], 1)
        img = voronoi_image(dims, 3, torch.float32, ns, means, w.extra["sigma"], key, device,
                            clip=(-200.0, 200.0))
        lo = torch.tensor([a for a, _ in r], dtype=torch.float32, device=img.device)
        hi = torch.tensor([b for _, b in r], dtype=torch.float32, device=img.device)
        return torch.maximum(torch.minimum(img, hi), lo)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# Batched workload: 512 images of uneven size, dimensionality and type

@dataclass(frozen=True)
class ImageSpec:
    """One image of a batch or a request stream."""
    index: int
    dims: tuple
    channels: int
    dtype: torch.dtype
    S: tuple
    m: float
    iterations: int
    n_seeds: int
    kind: str

    @property
    def voxels(self) -> int:
        return int(np.prod(self.dims))


def _loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


def batch_specs(n_images: int = 512, key: int = 3) -> list:
    """Half 2D RGB uint8 (sides log-uniform in [96,1024]), half 3D 1-channel
    float32 (sides log-uniform in [32,160]), shuffled; per image S in {8,12,16}
    on every axis, m in {10,20}, 10 iterations; max(8, round(N/1024)) seeds."""
    rng = np.random.default_rng([key, 0])
    kinds = np.array(["rgb2d"] * (n_images // 2) + ["f32-3d"] * (n_images - n_images // 2))
    rng.shuffle(kinds)
    specs = []
    for i, kd in enumerate(kinds):
        if kd == "rgb2d":
            dims = tuple(int(round(v)) for v in _loguniform(rng, 96, 1024, 2))
            C, dt = 3, torch.uint8
        else:
            dims = tuple(int(round(v)) for v in _loguniform(rng, 32, 160, 3))
            C, dt = 1, torch.float32
        s = int(rng.choice([8, 12, 16]))
        m = float(rng.choice([10.0, 20.0]))
        N = int(np.prod(dims))
        specs.append(ImageSpec(i, dims, C, dt, (s,) * len(dims), m, 10,
                               max(8, int(round(N / 1024))), str(kd)))
    return specs


def batch_image(spec: ImageSpec, device, key: int = 3):
    """Content as the 256x256 workload: region means U[0,255]^C, noise sigma 8,
    integer types rounded and clipped, float32 clipped to [0,255]."""
    k = [key, 1, spec.index]
    rng = np.random.default_rng(k + [3])
    means = rng.uniform(0.0, 255.0, size=(spec.n_seeds, spec.channels))
    return voronoi_image(spec.dims, spec.channels, spec.dtype, spec.n_seeds, means, 8.0, k,
                         device)


# ---------------------------------------------------------------------------
# Served stream: Poisson arrivals of a 70/20/10 mix

def request_trace(rate: float, n_requests: int = 2000, key: int = 4,
                  scale: float = 1.0) -> list:
    """(arrival_time_s, ImageSpec) pairs.  70% 2D RGB uint8 with sides
    log-uniform in [256,8192]; 20% 3D 1-channel uint16 with sides in [64,512];
    10% 3D 4-channel float32, x and y in [64,512], z in [32,256].  S in {8,16},
    m = 10, 10 iterations.  ``scale`` shrinks every side (for quick tests)."""
    rng = np.random.default_rng([key, int(rate * 1000), n_requests])
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    out = []
    for i in range(n_requests):
        u = rng.uniform()
        s = int(rng.choice([8, 16]))
        if u < 0.7:
            dims = tuple(max(16, int(round(v * scale))) for v in _loguniform(rng, 256, 8192, 2))
            C, dt, kind, dens = 3, torch.uint8, "rgb2d", 1024
        elif u < 0.9:
            dims = tuple(max(16, int(round(v * scale))) for v in _loguniform(rng, 64, 512, 3))
            C, dt, kind, dens = 1, torch.uint16, "u16-3d", 4096
        else:
            xy = _loguniform(rng, 64, 512, 2)
            z = _loguniform(rng, 32, 256)
            dims = tuple(max(16, int(round(v * scale))) for v in (xy[0], xy[1], z))
            C, dt, kind, dens = 4, torch.float32, "f32x4-3d", 1024
        N = int(np.prod(dims))
        spec = ImageSpec(i, dims, C, dt, (s,) * len(dims), 10.0, 10,
                         max(8, int(round(N / dens))), kind)
        out.append((float(t[i]), spec))
    return out


def request_image(spec: ImageSpec, device, key: int = 4):
    """2D RGB: as the 256x256 workload; 3D uint16: as the FIB-SEM workload;
    3D 4-channel float32: independent channel means U[0,1] per cell, sigma 0.05,
    clipped to [0,1]."""
    k = [key, 1, spec.index]
    rng = np.random.default_rng(k + [3])
    if spec.kind == "rgb2d":
        means = rng.uniform(0.0, 255.0, size=(spec.n_seeds, 3))
        return voronoi_image(spec.dims, 3, torch.uint8, spec.n_seeds, means, 8.0, k, device)
    if spec.kind == "u16-3d":
        means = rng.uniform(2000.0, 50000.0, size=(spec.n_seeds, 1))
        return voronoi_image(spec.dims, 1, torch.uint16, spec.n_seeds, means, 800.0, k, device,
                             clip=(0.0, 65535.0), membrane=600.0)
    means = rng.uniform(0.0, 1.0, size=(spec.n_seeds, 4))
    return voronoi_image(spec.dims, 4, torch.float32, spec.n_seeds, means, 0.05, k, device,
                         clip=(0.0, 1.0))
