"""sslic_run_static, the entry point that allocates nothing (its workspace is
a static device array), against sslic_run on the same inputs: labels,
centres, counts, label count and iterations run are identical (bit-exact for
integer images; float images within the bars of single runs), on calls in a
row whose second input is smaller than the first, so the second call runs on
scratch the first one left behind."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1806_08741_amd import sslic, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sslic.Context(0)


def _compare(ctx, img, S, m, T, conn, exact):
    print(f"[case] run_static {tuple(img.shape)} {img.dtype} S={S} m={m} T={T} "
          f"connectivity={conn}", flush=True)
    got = sslic.run_static(img, S, m, T, connectivity=conn)
    ref = ctx.run(img, S, m, T, connectivity=conn)
    torch.cuda.synchronize()
    assert int(got["iterations"].item()) == ref["iterations"] == T
    assert int(got["n_labels"].item()) == ref["n_labels"]
    gl, rl = got["labels"].cpu().numpy(), ref["labels"].cpu().numpy()
    gc, rc = got["centres"].cpu().numpy(), ref["centres"].cpu().numpy()
    if exact:
        np.testing.assert_array_equal(gl, rl)
        np.testing.assert_array_equal(gc, rc)
        np.testing.assert_array_equal(got["counts"].cpu().numpy(), ref["counts"].cpu().numpy())
    else:  # FP64 sums of float channels in a run-dependent order
        assert float(np.mean(gl != rl)) <= 1e-4
        np.testing.assert_allclose(gc, rc, rtol=1e-6, atol=1e-9)


def test_static_equals_run_two_calls_second_smaller(ctx):
    big = synth.workload_image("rgb-256", "cuda", dims=(1000, 700))
    small = synth.workload_image("fibsem-1k", "cuda", dims=(40, 36, 30))
    _compare(ctx, big, (16, 16), 10.0, 10, True, True)
    _compare(ctx, small, (8, 8, 8), 20.0, 5, True, True)


def test_static_float_then_smaller_integer(ctx):
    f = synth.workload_image("lab-2k", "cuda", dims=(512, 400))
    u = synth.workload_image("rgb-256", "cuda", dims=(96, 80))
    _compare(ctx, f, (16, 16), 10.0, 5, False, False)
    _compare(ctx, u, (8, 8), 10.0, 3, False, True)


def test_static_rejects_requests_above_the_scratch(ctx):
    img = torch.zeros((3000, 3000, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(sslic.SslicError, match="static scratch"):
        sslic.run_static(img, (16, 16), 10.0, 2)
