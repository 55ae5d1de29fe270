"""Serving loop: host-side admission arithmetic (CPU) and, on the GPU, that
every request's result is the same in the served mix as alone."""
import numpy as np
import pytest
import torch

from paper_1806_08741_amd import serve, synth


def _req(dims, C, dtype, S, i=0, t=0.0):
    img = torch.zeros(tuple(dims[::-1]) + (C,), dtype=dtype)
    return serve.Request(i, t, img, tuple(S), 10.0, 10)


def test_footprint_counts_image_outputs_and_tables():
    r = _req((256, 128), 3, torch.uint8, (16, 16))
    N, K = 256 * 128, 16 * 8
    fp = serve.footprint(r)
    assert fp >= N * 3 + 4 * N + K * (5 * 8 + 8)
    assert fp < N * 3 + 4 * N + K * 1024 + 8192
    # larger image, same kind: larger footprint; float32 4-channel 3D above u16 1-channel
    assert serve.footprint(_req((512, 128), 3, torch.uint8, (16, 16))) > fp
    a = serve.footprint(_req((64, 64, 32), 4, torch.float32, (8, 8, 8)))
    b = serve.footprint(_req((64, 64, 32), 1, torch.uint16, (8, 8, 8)))
    assert a > b


def test_trace_shape():
    tr = synth.request_trace(200.0, 400, scale=1.0)
    t = np.array([a for a, _ in tr])
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 200.0) < 40.0  # Poisson rate
    kinds = [sp.kind for _, sp in tr]
    assert 0.6 < kinds.count("rgb2d") / len(kinds) < 0.8
    assert all(sp.S[0] in (8, 16) and sp.iterations == 10 for _, sp in tr)


@pytest.mark.gpu
@pytest.mark.parametrize("closed", [False, True])
def test_served_results_equal_alone(closed):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08741_amd import sslic
    trace = synth.request_trace(400.0, 40, key=7, scale=0.12)
    reqs = serve.make_requests(trace, synth.request_image, "cuda")
    srv = serve.Server(hbm_budget=1 << 30, lanes=3, max_batch=8)
    srv.warm(reqs)
    st = srv.serve(reqs, closed_loop=closed)
    torch.cuda.synchronize()
    assert len(st.latencies_ms) == len(reqs)
    assert srv.peak_running > 1  # requests overlapped on the GPU
    ctx = sslic.Context(0)
    for r in reqs:
        assert r.arrival <= r.start <= r.done
        ref = ctx.run(r.image, r.S, r.m, r.iterations, connectivity=False)
        lab, lref = r.out["labels"].cpu().numpy(), ref["labels"].cpu().numpy()
        cen, cref = r.out["centres"].cpu().numpy(), ref["centres"].cpu().numpy()
        if r.image.dtype == torch.float32:
            assert np.mean(lab != lref) <= 1e-4, r.index
            np.testing.assert_allclose(cen, cref, rtol=1e-6, atol=1e-9)
        else:
            np.testing.assert_array_equal(lab, lref, err_msg=str(r.index))
            np.testing.assert_array_equal(cen, cref, err_msg=str(r.index))


@pytest.mark.gpu
def test_admission_keeps_to_the_budget():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    trace = synth.request_trace(1000.0, 16, key=8, scale=0.1)
    reqs = serve.make_requests(trace, synth.request_image, "cuda")
    biggest = max(serve.footprint(r) for r in reqs)
    budget = int(biggest * 2.5)
    srv = serve.Server(hbm_budget=budget, lanes=2, max_batch=4)
    srv.warm(reqs)
    st = srv.serve(reqs, closed_loop=True)
    assert len(st.latencies_ms) == len(reqs)
    assert 0 < srv.peak_used <= budget
    with pytest.raises(ValueError):
        serve.Server(hbm_budget=biggest - 1, lanes=1).serve(reqs, closed_loop=True)


@pytest.mark.gpu
def test_served_against_oracle():
    """One served request of each kind (2D RGB uint8, 3D uint16, 3D 4-channel
    float32) against the FP64 oracle: at least 99% of labels agree with the
    oracle's whole run (as for single images), and the served centres are the
    member means of the served labels (the oracle's update of those labels
    returns them: bit-exact for integer images, 1e-6 relative for float)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    trace = synth.request_trace(400.0, 40, key=7, scale=0.12)
    reqs = serve.make_requests(trace, synth.request_image, "cuda")
    srv = serve.Server(hbm_budget=1 << 30, lanes=3, max_batch=8)
    srv.warm(reqs)
    srv.serve(reqs, closed_loop=True)
    torch.cuda.synchronize()
    kinds = {}
    for r, (_, sp) in zip(reqs, trace):
        if sp.kind not in kinds or r.voxels < kinds[sp.kind][0].voxels:
            kinds[sp.kind] = (r, sp)
    assert set(kinds) == {"rgb2d", "u16-3d", "f32x4-3d"}
    for kind, (r, sp) in sorted(kinds.items()):
        img = r.image.cpu().numpy()
        nd = len(sp.dims)
        print(f"[case] served {kind} {sp.dims} S={sp.S}", flush=True)
        ref = oracle.run(img, nd, sp.S, sp.m, sp.iterations, connectivity=False)
        lab = r.out["labels"].cpu().numpy()
        cen = r.out["centres"].cpu().numpy()
        agree = float(np.mean(lab == ref["labels"]))
        assert agree >= 0.99, (kind, agree)
        exp_c, exp_n, _ = oracle.update(img, nd, sp.S, sp.m, lab, cen)
        np.testing.assert_array_equal(r.out["counts"].cpu().numpy(), exp_n)
        if img.dtype == np.float32:
            np.testing.assert_allclose(cen, exp_c, rtol=1e-6, atol=1e-9)
        else:
            np.testing.assert_array_equal(cen, exp_c)
