"""GPU rate-distortion sweep (persistent launches; a plan runs the DCT and
integer kernels side by side on two streams) against the oracle's
per-(image, transform, r) definition."""

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import batch as OB
from oracle import codec as Co
from oracle import matrices as M
from synth import ar1_image, batch_images, batch_specs

pytestmark = pytest.mark.gpu

ALL = ["DCT", "T1", "LO", "T6", "RDCT", "T4", "T2"]


def _pack(images, cuda, pad_pitch=0):
    """Concatenate images into one device buffer; returns (tensor, planes)."""
    import torch
    planes, parts, off = [], [], 0
    for img in images:
        h, w = img.shape
        pitch = w + pad_pitch
        buf = np.zeros((h, pitch), dtype=np.uint8)
        buf[:, :w] = img
        parts.append(buf.ravel())
        planes.append((off, h, w, pitch))
        off += h * pitch
    return torch.from_numpy(np.concatenate(parts)).to(cuda), planes


def _check(gpu, ref, names):
    for t, name in enumerate(names):
        g, r = gpu[:, t, :].astype(np.int64), ref[:, t, :].astype(np.int64)
        if name == "DCT":      # float64 reconstruction: equal unless a pixel sits on a half
            assert np.all(np.abs(g - r) <= 1e-6 * r + 2), name
        else:
            assert np.array_equal(g, r), name


@pytest.fixture(scope="module")
def small_set():
    return [ar1_image(72, 136, 0.9, seed=21), ar1_image(64, 64, 0.97, seed=22),
            ar1_image(40, 48, 0.85, seed=23)]


def test_batch_matches_oracle(cuda, small_set):
    base, planes = _pack(small_set, cuda, pad_pitch=8)
    sse = A.evaluate_batch(base, planes, ALL, 1, 64).cpu().numpy()
    ref = OB.sse_table(small_set, ALL, 1, 64)
    _check(sse, ref, ALL)
    assert np.all(sse[:, 1:, -1] == 0)                     # lossless at r = 64


@pytest.mark.parametrize("wgs,split", [(1, 1), (3, 7), (8, 1)])
def test_batch_schedules_agree(cuda, small_set, wgs, split):
    base, planes = _pack(small_set, cuda)
    ref = A.evaluate_batch(base, planes, ALL, 3, 40).cpu().numpy()
    got = A.evaluate_batch(base, planes, ALL, 3, 40, wgs_per_cu=wgs, split=split).cpu().numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("names,r_lo,r_hi", [
    (["DCT", "T1", "T4"], 5, 20),            # the DCT's first coefficient window only
    (["LO", "DCT", "T6"], 40, 64),           # the output range starts in the second window
    (["DCT", "T2", "DCT"], 30, 34),          # the DCT twice, across the window edge
    (["RDCT", "T1"], 1, 63),                 # integer transforms only (no DCT kernel)
    (["DCT"], 1, 33),                        # the DCT only (no integer kernel)
])
def test_batch_lists_and_ranges(cuda, small_set, names, r_lo, r_hi):
    base, planes = _pack(small_set, cuda)
    sse = A.evaluate_batch(base, planes, names, r_lo, r_hi).cpu().numpy()
    ref = OB.sse_table(small_set, names, r_lo, r_hi)
    _check(sse, ref, names)


def test_batch_plan_replays(cuda, small_set):
    import torch
    base, planes = _pack(small_set, cuda)
    names = ["DCT", "T1", "LO", "T6", "RDCT", "T4"]
    eager = A.evaluate_batch(base, planes, names, 1, 63).cpu().numpy()
    plan = A.BatchPlan(base, planes, names, 1, 63, autotune=True)
    info = plan.info()
    assert 1 <= info["wgs_per_cu"] <= 16 and info["split"] >= 1 and info["tuned_ms"] > 0
    scratch = torch.empty(1 << 20, device=cuda)
    for rep in range(4):
        scratch.normal_()                                  # eager work between replays
        torch.cuda.synchronize()
        got = plan.launch().clone()
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), eager), rep
    # back-to-back launches on a side stream, read after the stream alone is synchronised
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        plan.launch(stream=side)
    side.synchronize()
    assert np.array_equal(plan.sse.cpu().numpy(), eager)
    plan.close()


def test_batch_plan_in_captured_graph(cuda, small_set):
    """A plan launch captured by the caller (the fork and join become two graph
    branches): every replay, with eager work and synchronisation between
    replays, equals the eager sweep."""
    import torch
    base, planes = _pack(small_set, cuda)
    names = ["T1", "DCT", "LO"]
    eager = A.evaluate_batch(base, planes, names, 2, 50).cpu().numpy()
    plan = A.BatchPlan(base, planes, names, 2, 50, autotune=False)
    plan.launch()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    scratch = torch.empty(1 << 20, device=cuda)
    for rep in range(4):
        plan.sse.fill_(-1)
        scratch.normal_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(plan.sse.cpu().numpy(), eager), rep
    del g
    plan.close()


def test_batch_45_images_sampled(cuda):
    """The 45-image workload (uneven sizes up to 2048 x 1536): one plan, then
    sampled (image, transform, r) entries of the small images and every
    transform at r = 1, 10, 40, 63 of the three largest against the oracle."""
    specs = batch_specs()
    images = batch_images(specs)
    base, planes = _pack(images, cuda)
    names = ["DCT", "T1", "LO", "T6", "RDCT", "T4"]
    plan = A.BatchPlan(base, planes, names, 1, 63, autotune=False)
    sse = plan.launch().cpu().numpy()
    rng = np.random.default_rng(5)
    small = sorted(range(len(images)), key=lambda i: images[i].size)[:6]
    for _ in range(8):
        i = int(rng.choice(small))
        t = int(rng.integers(len(names)))
        r = int(rng.integers(1, 64))
        img = images[i]
        ref = (Co.evaluate_dct(img, r) if names[t] == "DCT"
               else Co.evaluate(img, M.TRANSFORMS[names[t]], r))["sse"]
        if names[t] == "DCT":
            assert abs(int(sse[i, t, r - 1]) - ref) <= 1e-6 * ref + 2
        else:
            assert int(sse[i, t, r - 1]) == ref, (i, names[t], r)
    # the three largest images (up to 2048 x 1536), every transform, r across the scan
    large = sorted(range(len(images)), key=lambda i: images[i].size)[-3:]
    for i in large:
        img = images[i]
        for t, name in enumerate(names):
            for r in (1, 10, 40, 63):
                ref = (Co.evaluate_dct(img, r) if name == "DCT"
                       else Co.evaluate(img, M.TRANSFORMS[name], r))["sse"]
                if name == "DCT":
                    assert abs(int(sse[i, t, r - 1]) - ref) <= 1e-6 * ref + 2, (i, name, r)
                else:
                    assert int(sse[i, t, r - 1]) == ref, (i, name, r)
    plan.close()


def test_batch_argument_errors(cuda, small_set):
    base, planes = _pack(small_set, cuda)
    with pytest.raises(A.AdctError):
        A.evaluate_batch(base, planes, ["T1"], 0, 10)
    with pytest.raises(A.AdctError):
        A.evaluate_batch(base, planes, ["CUSTOM"], 1, 10)
    with pytest.raises(A.AdctError):
        A.evaluate_batch(base, [(1, 8, 8, 8)], ["T1"], 1, 10)
