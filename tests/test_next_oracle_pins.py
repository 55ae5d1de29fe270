"""Pins of the oracle's functions beyond the SLIC path proper: the contour
mask of the paper's visualisation (Sec. 4), checked against closed forms of
hand-built label images on 1 to 4 axes.  CPU only."""
import numpy as np
import pytest

import oracle

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
