"""Pins of the oracle's functions beyond the SLIC path proper: the contour
mask of the paper's visualisation (Sec. 4), checked against closed forms of
hand-built label images on 1 to 4 axes; the RGB to CIE-Lab conversion; and
the assignment on a distance image kept across iterations (Sec. 2.2, Sec. 3.1).  CPU
only."""
import json
import os

import numpy as np
import pytest

import oracle

from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

DTYPES = [np.uint8, np.uint16, np.float32]


def image(dims, C, dtype, seed=0):
    rng = np.random.default_rng(seed)
    shape = tuple(dims[::-1]) + (C,)
    if dtype == np.float32:
        return (rng.random(shape) * 100 + 1).astype(np.float32)  # no zeros
    return rng.integers(1, 200, shape).astype(dtype)


SHAPES = [(17,), (9, 7), (6, 5, 4), (5, 4, 3, 3)]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_constant_labels_leave_the_image(dims, dtype):
    img = image(dims, 3, dtype)
    out = oracle.mask_contours(img, len(dims), np.full(int(np.prod(dims)), 7, np.int32))
    np.testing.assert_array_equal(out, img)


@pytest.mark.parametrize("dims", SHAPES)
def test_split_plane_blackens_the_two_layers_beside_it(dims):
    """Labels 0 below x_a = p and 1 from it on: exactly the voxels with
    x_a in {p-1, p} are on the contour."""
    nd = len(dims)
    for a in range(nd):
        if dims[a] < 2:
            continue
        p = dims[a] // 2
        img = image(dims, 2, np.uint16, seed=a)
        coords = np.indices(dims[::-1])[::-1]  # coords[i] is x_i, array in (x_{n-1}, .., x_0)
        lab = (coords[a] >= p).astype(np.int32)
        out = oracle.mask_contours(img, nd, lab.reshape(-1))
        black = (coords[a] == p - 1) | (coords[a] == p)
        exp = img.copy()
        exp[black] = 0
        np.testing.assert_array_equal(out, exp)


@pytest.mark.parametrize("dims", SHAPES[1:])
def test_checkerboard_blackens_everything(dims):
    coords = np.indices(dims[::-1])
    lab = (coords.sum(axis=0) % 2).astype(np.int32)
    img = image(dims, 1, np.float32)
    out = oracle.mask_contours(img, len(dims), lab.reshape(-1))
    assert not out.any()


@pytest.mark.parametrize("dims", SHAPES)
def test_single_voxel_island(dims):
    """One voxel with its own label: it and its face neighbours inside the
    image (2n of them, fewer at a border) turn black, nothing else."""
    nd = len(dims)
    img = image(dims, 3, np.uint8)
    for pos in (tuple(d // 2 for d in dims), tuple(0 for _ in dims)):
        lab = np.zeros(dims[::-1], np.int32)
        lab[pos[::-1]] = 5
        out = oracle.mask_contours(img, nd, lab.reshape(-1))
        black = np.zeros(dims[::-1], bool)
        black[pos[::-1]] = True
        for i in range(nd):
            for s in (-1, 1):
                q = list(pos)
                q[i] += s
                if 0 <= q[i] < dims[i]:
                    black[tuple(q[::-1])] = True
        exp = img.copy()
        exp[black] = 0
        np.testing.assert_array_equal(out, exp)


# ---- RGB to CIE-Lab --------------------------------------------------------

def all_colours_of_red(r):
    g, b = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    return np.stack([np.full(g.size, r), g.reshape(-1), b.reshape(-1)], -1).astype(np.uint8)


def test_lab_ranges_over_all_8bit_colours_are_the_printed_ones():
    """The paper prints L in [0, 100], a in [-86.185, 98.254] and b in
    [-107.863, 94.482] for 8-bit RGB in Lab (Sec. 2.1)."""
    lo = np.full(3, np.inf)
    hi = np.full(3, -np.inf)
    for r in range(256):
        lab = oracle.rgb_to_lab(all_colours_of_red(r))
        lo = np.minimum(lo, lab.min(axis=0))
        hi = np.maximum(hi, lab.max(axis=0))
    np.testing.assert_allclose(lo, [0.0, -86.185, -107.863], atol=1e-3)
    np.testing.assert_allclose(hi, [100.0, 98.254, 94.482], atol=1e-3)


def test_lab_black_white_and_greys():
    lab = oracle.rgb_to_lab(np.repeat(np.arange(256, dtype=np.uint8)[:, None], 3, axis=1))
    np.testing.assert_array_equal(lab[0], [0.0, 0.0, 0.0])
    assert abs(lab[255, 0] - 100.0) < 1e-9
    assert np.abs(lab[:, 1:]).max() < 0.02       # greys are nearly neutral
    assert np.all(np.diff(lab[:, 0]) > 0)        # lightness rises with the grey level


def test_lab_of_pure_red():
    """sRGB red is about (53.24, 80.09, 67.20) in Lab."""
    lab = oracle.rgb_to_lab(np.array([[255, 0, 0]], np.uint8))[0]
    np.testing.assert_allclose(lab, [53.24, 80.09, 67.20], atol=0.05)


# ---- distance image kept across iterations (Sec. 2.2, Sec. 3.1) ------------

def test_persist_golden_1d_separates_the_two_readings():
    with open(os.path.join(GOLDEN, "persist_1d.json")) as fh:
        gd = json.load(fh)
    for dt in (np.uint8, np.float32):
        img = np.array(gd["image"], dtype=dt).reshape(-1, 1)
        init = np.array(gd["init_centres"], dtype=np.float64)
        for mode, persist in (("reset", False), ("persist", True)):
            r = oracle.run(img, 1, gd["S"], gd["m"], gd["iterations"], connectivity=False,
                           init_centres=init, persist_distance=persist)
            np.testing.assert_array_equal(r["labels"], gd[mode]["labels"])
            np.testing.assert_allclose(r["centres"], gd[mode]["centres"], rtol=1e-15, atol=1e-15)
        assert r["residuals"][1] == gd["persist"]["residual_2"]


def _integer_setup(dims, S, C, seed):
    rng = np.random.default_rng(seed)
    n = len(dims)
    img = rng.integers(0, 256, size=tuple(dims[::-1]) + (C,)).astype(np.uint8)
    K, Ka = oracle.num_clusters(dims, S)
    init = np.zeros((K, C + n))
    init[:, :C] = rng.integers(0, 256, (K, C))
    grid = np.stack(np.meshgrid(*[(np.arange(k) + 0.5) * d / k for k, d in zip(Ka, dims)],
                                indexing="ij"), -1).reshape(-1, n, order="F")
    init[:, C:] = np.clip(np.floor(grid) + rng.integers(-1, 2, (K, n)), 0, np.array(dims) - 1)
    return img, init, Ka


@pytest.mark.parametrize("dims,S,m,C", [((40, 24), (8, 8), 8.0, 3), ((20, 16, 12), (4, 4, 4), 8.0, 1),
                                        ((37, 29), (8, 8), 16.0, 2)])
def test_persist_run_equals_brute_force(dims, S, m, C):
    """The whole run with the kept distance image against a NumPy model of
    windowed k-means whose per-voxel minimum persists."""
    img, init, Ka = _integer_setup(dims, S, C, 11)
    T = 5
    r = oracle.run(img, len(dims), S, m, T, connectivity=False, init_centres=init,
                   persist_distance=True)
    lab = brute.grid_cell_labels(dims, Ka)
    dist = np.full(lab.shape, np.inf)
    cen = init.copy()
    for _ in range(T):
        lab, dist = brute.kmeans_assign_persist(img, dims, S, m, cen, lab, dist)
        cen, cnt = brute.bincount_update(img, dims, lab, cen)
    np.testing.assert_array_equal(r["labels"], lab)
    np.testing.assert_array_equal(r["centres"], cen)
    np.testing.assert_array_equal(r["counts"], cnt)
    # the two readings really differ on these inputs
    r0 = oracle.run(img, len(dims), S, m, T, connectivity=False, init_centres=init)
    assert (r0["labels"] != r["labels"]).any()


def test_persist_step_from_infinity_is_the_reset_step():
    img, init, Ka = _integer_setup((33, 21), (6, 6), 3, 5)
    lab0 = brute.grid_cell_labels((33, 21), Ka)
    a = oracle.assign(img, 2, (6, 6), 10.0, init, lab0.copy())
    b, d = oracle.assign_persist(img, 2, (6, 6), 10.0, init, lab0.copy(), np.full(lab0.size, np.inf))
    np.testing.assert_array_equal(a, b)
    _, dist = oracle.assign_points(img, 2, (6, 6), 10.0, init, np.arange(lab0.size))
    np.testing.assert_array_equal(d, dist)


def test_persist_step_invariants():
    """d never grows; a label changes only where d fell; where d fell it is the
    least windowed distance of this step and the label its first argmin."""
    img, init, Ka = _integer_setup((30, 26), (5, 5), 1, 3)
    lab = brute.grid_cell_labels((30, 26), Ka)
    dist = np.full(lab.size, np.inf)
    cen = init.copy()
    for _ in range(4):
        l0, d0 = lab.copy(), dist.copy()
        lab, dist = oracle.assign_persist(img, 2, (5, 5), 6.0, cen, lab, dist)
        assert np.all(dist <= d0)
        fell = dist < d0
        assert np.all(lab[~fell] == l0[~fell])
        pl, pd = oracle.assign_points(img, 2, (5, 5), 6.0, cen, np.nonzero(fell)[0])
        np.testing.assert_array_equal(lab[fell], pl)
        np.testing.assert_array_equal(dist[fell], pd)
        cen, _, _ = oracle.update(img, 2, (5, 5), 6.0, lab, cen)


def test_persist_equals_reset_on_cell_images():
    """On an image that is constant on its S-grid cells with strong contrast,
    every voxel's nearest centre is its own cell's under either reading, so
    the two runs agree."""
    rng = np.random.default_rng(2)
    dims, S = (48, 40), (8, 8)
    K, Ka = oracle.num_clusters(dims, S)
    vals = rng.permutation(K) * (250 // K) + 2
    cell = brute.grid_cell_labels(dims, Ka)
    img = vals[cell].astype(np.uint8).reshape(dims[::-1] + (1,))
    a = oracle.run(img, 2, S, 10.0, 6, connectivity=False)
    b = oracle.run(img, 2, S, 10.0, 6, connectivity=False, persist_distance=True)
    np.testing.assert_array_equal(a["labels"], cell)
    np.testing.assert_array_equal(b["labels"], a["labels"])
    np.testing.assert_array_equal(b["centres"], a["centres"])
