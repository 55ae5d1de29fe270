"""The batched form (sslic_run_batch) against single-image runs and the oracle.

A batch must give every image the result sslic_run gives it alone:
bit-identical labels, centres and counts for integer images; for float32
images (whose FP64 channel sums are added in a different order) at most 1e-4
of the labels may differ and centres agree to 1e-6 relative.  Graph replays
are checked against an eager run, with the program's own eager work and
synchronisations between replays and new input bytes at the same addresses.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1806_08741_amd import synth

pytestmark = pytest.mark.gpu

LABEL_TOL = 1e-4
F32_RTOL = 1e-6


@pytest.fixture(scope="module")
def sslic_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08741_amd import sslic
    return sslic


@pytest.fixture()
def ctx(sslic_mod):
    return sslic_mod.Context(0)


def rand_image(dims, C, dtype, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    shape = tuple(dims[::-1]) + (C,)
    if dtype == torch.float32:
        t = torch.rand(shape, generator=g) * 255.0
    else:
        top = 256 if dtype == torch.uint8 else 65536
        t = torch.randint(0, top, shape, generator=g).to(dtype)
    return t.cuda()


def mixed_items():
    """Uneven sizes, dimensionalities, channel counts, pixel types, S, m and
    iteration counts."""
    specs = synth.batch_specs(512)
    items = []
    for sp in specs[:6]:  # 2D RGB u8 and 3D f32 from the batched workload recipe
        small = tuple(min(d, 200 if len(sp.dims) == 2 else 40) for d in sp.dims)
        sp2 = synth.ImageSpec(sp.index, small, sp.channels, sp.dtype, sp.S, sp.m, sp.iterations,
                              max(8, int(np.prod(small)) // 1024), sp.kind)
        items.append(dict(image=synth.batch_image(sp2, "cuda"), S=sp.S, m=sp.m, iterations=4))
    items.append(dict(image=rand_image((150, 97), 1, torch.uint16, 1), S=(12, 12), m=10.0,
                      iterations=5))
    items.append(dict(image=rand_image((61, 37, 23), 4, torch.uint8, 2), S=(8, 8, 6), m=20.0,
                      iterations=3))
    items.append(dict(image=rand_image((13, 11, 9, 7), 1, torch.uint8, 3), S=(4, 4, 3, 3),
                      m=8.0, iterations=4))
    items.append(dict(image=rand_image((333, 129), 3, torch.uint8, 4), S=(16, 16), m=10.0,
                      iterations=6))
    items.append(dict(image=rand_image((67, 45, 19), 2, torch.float32, 5), S=(7, 6, 5), m=5.0,
                      iterations=4))
    items.append(dict(image=rand_image((96, 96), 3, torch.uint8, 6), S=(16, 16), m=10.0,
                      iterations=2))
    # 3D integer images with few channels: the sweep's fast form, in the batch as alone
    items.append(dict(image=rand_image((70, 45, 38), 1, torch.uint16, 7), S=(8, 8, 8), m=20.0,
                      iterations=3))
    items.append(dict(image=rand_image((48, 40, 36), 3, torch.uint8, 8), S=(8, 8, 8), m=10.0,
                      iterations=2))
    return items


def solo(ctx, itm, tol=0.0, connectivity=False):
    return ctx.run(itm["image"], itm["S"], itm["m"], itm["iterations"], tol=tol,
                   connectivity=connectivity, residuals=True)


def assert_same(itm, got, ref, what):
    torch.cuda.synchronize()
    lg, lr = got["labels"].cpu().numpy(), ref["labels"].cpu().numpy()
    cg, cr = got["centres"].cpu().numpy(), ref["centres"].cpu().numpy()
    if itm["image"].dtype == torch.float32:
        assert np.mean(lg != lr) <= LABEL_TOL, what
        np.testing.assert_allclose(cg, cr, rtol=F32_RTOL, atol=1e-9, err_msg=what)
    else:
        np.testing.assert_array_equal(lg, lr, err_msg=what)
        np.testing.assert_array_equal(cg, cr, err_msg=what)
        np.testing.assert_array_equal(got["counts"].cpu().numpy(), ref["counts"].cpu().numpy(),
                                      err_msg=what)


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_solo(ctx, graph):
    items = mixed_items()
    outs = ctx.run_batch([dict(it, want_residuals=True) for it in items], graph=graph)
    for i, (itm, o) in enumerate(zip(items, outs)):
        ref = solo(ctx, itm)
        assert_same(itm, o, ref, f"image {i}")
        assert int(o["iters"].item()) == itm["iterations"]
        np.testing.assert_allclose(o["residuals"].cpu().numpy(), ref["residuals"].cpu().numpy(),
                                   rtol=1e-9 if itm["image"].dtype != torch.float32 else 1e-5)


def test_batch_tile_choice_does_not_change_results(ctx):
    items = [it for it in mixed_items() if it["image"].dtype != torch.float32]
    a = ctx.run_batch(items, autotune=True, graph=False)
    b = ctx.run_batch(items, autotune=False, graph=False)
    for i, (itm, x, y) in enumerate(zip(items, a, b)):
        assert_same(itm, x, y, f"image {i}")


def test_batch_graph_replays(ctx, sslic_mod):
    """Replays of the captured graph on new bytes at the same addresses, with
    eager work and synchronisations in between, each equal to an eager run."""
    items = mixed_items()[4:10]
    outs = None
    for rep in range(3):
        for j, itm in enumerate(items):  # new content, same tensors
            fresh = rand_image(tuple(itm["image"].shape[:-1][::-1]), itm["image"].shape[-1],
                               itm["image"].dtype, 100 * rep + j)
            itm["image"].copy_(fresh)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()  # the program's own eager work
        torch.cuda.synchronize()
        if outs is None:
            outs = ctx.run_batch([dict(it) for it in items], graph=True)
        else:  # same tensors as outputs: replay
            outs = ctx.run_batch([dict(it, labels=o["labels"], centres=o["centres"],
                                       counts=o["counts"], iters=o["iters"])
                                  for it, o in zip(items, outs)], graph=True)
        torch.cuda.synchronize()
        eager = sslic_mod.Context(0).run_batch([dict(it) for it in items], graph=False)
        for i, (itm, o, e) in enumerate(zip(items, outs, eager)):
            assert_same(itm, o, e, f"replay {rep} image {i}")


def test_batch_stops_each_image_on_its_own(ctx):
    items = mixed_items()
    for it in items:
        it["iterations"] = 8
    tol = 0.05
    outs = ctx.run_batch([dict(it, want_residuals=True) for it in items], tol=tol, graph=True)
    for i, (itm, o) in enumerate(zip(items, outs)):
        ref = solo(ctx, itm, tol=tol)
        assert int(o["iters"].item()) == ref["iterations"], f"image {i}"
        assert_same(itm, o, ref, f"image {i}")


def test_batch_with_connectivity(ctx):
    items = [it for it in mixed_items() if it["image"].dtype != torch.float32][:5]
    outs = ctx.run_batch(items, connectivity=True, graph=True)
    for i, (itm, o) in enumerate(zip(items, outs)):
        ref = solo(ctx, itm, connectivity=True)
        assert o["n_labels"] == ref["n_labels"], f"image {i}"
        assert_same(itm, o, ref, f"image {i}")


def test_batch_against_oracle(ctx):
    """One 2D RGB and one 3D float image of the batch against the FP64 oracle
    (whole runs: at least 99% of labels agree, as for single images)."""
    items = mixed_items()
    pick = [i for i, it in enumerate(items) if it["image"].dtype == torch.uint8][:1] + \
           [i for i, it in enumerate(items) if it["image"].dtype == torch.float32][:1]
    outs = ctx.run_batch(items, graph=True)
    for i in pick:
        itm = items[i]
        img = itm["image"].cpu().numpy()
        ref = oracle.run(img, len(itm["S"]), itm["S"], itm["m"], itm["iterations"],
                         connectivity=False)
        agree = np.mean(outs[i]["labels"].cpu().numpy() == ref["labels"].reshape(-1))
        assert agree >= 0.99, (i, agree)
