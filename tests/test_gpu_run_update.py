"""The update that ``sslic_run`` itself runs (the sweep's map step plus the
reduce step), compared with the oracle's update (Sec. 2.2 and Sec. 3.1 stage
2: each centre becomes the mean position and mean channel vector of the
voxels that took its label).

For every case the GPU runs T and T-1 iterations with connectivity off.  The
oracle's update is fed the GPU's labels after T iterations and the GPU's
centres after T-1, which are exactly the inputs of the GPU's last update, and
its result is compared with the GPU's centres, counts and residual after T.
The cases reach every form of the sweep's map step: the table form (2D, S
>= 12), the hashed form (2D at S = 8), the fast form of 3D integer images
(grey and RGB at S = 8, and at S = (2, 16, 16), where a row of blocks is met
by more than 64 table entries and is walked 64 at a time), the form without
tile slots, whose sums all go through 64-bit atomics (a window wider than a
tile: the paper's own 2D setting S = 50, m = 10 on a 2048 x 1216
three-channel float image with CIE-Lab-range values, and 3D at S = 16), 1D,
4D, five channels and float images with one and two channels.

Bars: counts and coordinate sums are exact integers, so counts are equal and
centres of integer images bit-exact; float channel means within 1e-6
relative (FP64 sums in another order); the residual within 1e-9 relative
(1e-6 for float images).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1806_08741_amd import synth

pytestmark = pytest.mark.gpu

F32_RTOL = 1e-6


@pytest.fixture(scope="module")
def ctx():
    from paper_1806_08741_amd import sslic
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sslic.Context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_image(dims, C, dtype, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(dims[::-1]) + (C,)
    if dtype == np.float32:
        return rng.uniform(0, 255, size=shape).astype(np.float32)
    top = {np.uint8: 255, np.uint16: 65535}[dtype]
    return rng.integers(0, top + 1, size=shape).astype(dtype)


def case_image(name, dims):
    if name in synth.WORKLOADS:
        return synth.workload_image(name, "cpu", dims=dims).numpy()
    kind = name.split("-")
    dt = {"u8": np.uint8, "u16": np.uint16, "f32": np.float32}[kind[1]]
    C = int(kind[2][1:]) if kind[2].startswith("c") else (3 if dt == np.uint8 else 1)
    return rand_image(dims, C, dt, sum(map(ord, name)))


# name, dims, S, m, T, the sweep form the case reaches
CASES = [
    ("slide-16k", (1000, 777), (16, 16), 10.0, 3, "table"),
    ("rgb-256", (256, 256), (16, 16), 10.0, 10, "table"),
    ("rgb-256", (300, 211), (8, 8), 10.0, 3, "hashed"),
    ("fibsem-1k", (90, 77, 65), (8, 8, 8), 20.0, 3, "3D fast"),
    ("rand-u8-3d", (50, 40, 30), (8, 8, 8), 10.0, 3, "3D fast RGB"),
    ("rand-u16-3d", (60, 48, 40), (2, 16, 16), 10.0, 2, "3D fast long rows"),
    ("lab-2k", (2048, 1216), (50, 50), 10.0, 5, "no slots"),
    ("fibsem-1k", (100, 90, 70), (16, 16, 16), 20.0, 3, "no slots"),
    ("rand-u16-1d", (3001,), (16,), 10.0, 3, "1D"),
    ("rand-u8-4d", (13, 11, 9, 7), (4, 4, 3, 3), 8.0, 3, "4D"),
    ("rand-u8-c5", (130, 70), (12, 9), 15.0, 3, "5 channels"),
    ("rand-f32-c2", (67, 45, 19), (7, 6, 5), 5.0, 3, "float, 2 channels"),
    ("rand-f32-c1", (333, 129), (10, 10), 0.5, 3, "float, 1 channel"),
]


@pytest.mark.parametrize("name,dims,S,m,T,form", CASES, ids=[f"{c[0]}-{c[5]}" for c in CASES])
def test_run_update_against_oracle(ctx, name, dims, S, m, T, form):
    img = case_image(name, dims)
    nd = len(dims)
    print(f"[case] {name} {dims} S={S} m={m} T={T} ({form})", flush=True)
    d = dev(img)
    prev = ctx.run(d, S, m, T - 1, connectivity=False)
    last = ctx.run(d, S, m, T, connectivity=False, residuals=True)
    assert last["iterations"] == T
    lab = host(last["labels"])
    cen_prev = host(prev["centres"])
    K = cen_prev.shape[0]
    assert lab.min() >= 0 and lab.max() < K
    exp_c, exp_n, exp_e = oracle.update(img, nd, S, m, lab, cen_prev)
    got_c, got_n = host(last["centres"]), host(last["counts"])
    got_e = float(host(last["residuals"])[T - 1])
    np.testing.assert_array_equal(got_n, exp_n)
    assert int(got_n.sum()) == lab.size
    if img.dtype == np.float32:
        # coordinates are exact integer sums on both sides
        np.testing.assert_array_equal(got_c[:, img.shape[-1]:], exp_c[:, img.shape[-1]:])
        np.testing.assert_allclose(got_c, exp_c, rtol=F32_RTOL, atol=1e-9)
        assert got_e == pytest.approx(exp_e, rel=1e-6)
    else:
        np.testing.assert_array_equal(got_c, exp_c)
        assert got_e == pytest.approx(exp_e, rel=1e-9)


# the first case of the table form, of the 3D fast form and without tile slots
MEANS_CASES = [next(c for c in CASES if c[5] == f) for f in ("table", "3D fast", "no slots")]


@pytest.mark.parametrize("name,dims,S,m,T,form", MEANS_CASES,
                         ids=[f"{c[0]}-{c[5]}" for c in MEANS_CASES])
def test_run_centres_are_member_means(ctx, name, dims, S, m, T, form):
    """With connectivity off every non-empty cluster's centre is the mean of
    its members: the oracle's update of the GPU's final labels, started from
    the GPU's final centres, returns those centres (bit-exact for integer
    images) and the counts of the labels."""
    img = case_image(name, dims)
    nd = len(dims)
    r = ctx.run(dev(img), S, m, T, connectivity=False)
    lab, cen, cnt = host(r["labels"]), host(r["centres"]), host(r["counts"])
    exp_c, exp_n, exp_e = oracle.update(img, nd, S, m, lab, cen)
    np.testing.assert_array_equal(cnt, exp_n)
    np.testing.assert_array_equal(cnt, np.bincount(lab, minlength=cen.shape[0]))
    if img.dtype == np.float32:
        np.testing.assert_allclose(cen, exp_c, rtol=F32_RTOL, atol=1e-9)
        assert exp_e < 1e-6
    else:
        np.testing.assert_array_equal(cen, exp_c)
        assert exp_e == 0.0


def test_lab_run_agrees_with_oracle(ctx):
    """The paper's own 2D setting end to end (S = 50, m = 10, 5 iterations,
    connectivity on) on a Lab-range float image: at least 99% of labels agree
    with the oracle's whole run, every label is valid, and the label count is
    the oracle's within 1%."""
    w = synth.WORKLOADS["lab-2k"]
    img = case_image("lab-2k", w.dims)
    exp = oracle.run(img, 2, w.S, w.m, w.iterations, connectivity=True)
    got = ctx.run(dev(img), w.S, w.m, w.iterations, connectivity=True)
    gl = host(got["labels"])
    agree = float((gl == exp["labels"]).mean())
    assert 0 <= gl.min() and gl.max() < got["n_labels"]
    assert agree >= 0.99, agree
    assert abs(got["n_labels"] - exp["n_labels"]) <= max(1, exp["n_labels"] // 100)


@pytest.mark.parametrize("dims,S", [((1,), (1,)), ((1, 1), (1, 1)), ((1, 1, 1), (1, 1, 1)),
                                    ((3, 1), (5, 5)), ((2, 2, 2, 2), (1, 1, 1, 1)),
                                    ((1, 40), (4, 8)), ((17, 1, 9), (20, 3, 2)), ((64,), (1,))])
def test_run_degenerate_sizes(ctx, dims, S):
    """The reset loop on degenerate geometries: one voxel on 1 to 3 axes, S
    above the axis size (one cluster on that axis), S = 1 (a cluster per
    voxel) and axes of size 1 among larger ones; with connectivity, labels,
    centres and the label count equal the oracle's."""
    img = rand_image(dims, 3, np.uint8, 4)
    nd = len(dims)
    exp = oracle.run(img, nd, S, 10.0, 3)
    got = ctx.run(dev(img), S, 10.0, 3)
    np.testing.assert_array_equal(host(got["labels"]), exp["labels"])
    np.testing.assert_array_equal(host(got["centres"]), exp["centres"])
    np.testing.assert_array_equal(host(got["counts"]), exp["counts"])
    assert got["n_labels"] == exp["n_labels"]
