"""GPU SSIM (adct_ssim, float64) against the float64 oracle.

Tolerance: each of the five window sums is a float64 sum of 121 products of
magnitude at most 128^2 (pixels centred at 128), so its error is below
2^-53 * 121 * 2 * 16384 < 5e-10 in absolute terms; the variances and the
covariance inherit that, and they enter SSIM beside C2 = 58.5, so a map entry
moves by less than 1e-10; the per-plane fixed-point sum rounds each lane's
partial sum to 2^-37.  The tests allow 1e-9 on every plane's mean."""

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import ssim as S
from synth import ar1_image, video_base_planes, video_frame, video_spec

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _dev(x, cuda):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(cuda)


def _pair(h, w, seed, noise=12):
    x = ar1_image(h, w, 0.93, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    y = np.clip(x.astype(np.int64) + rng.integers(-noise, noise + 1, x.shape), 0, 255).astype(np.uint8)
    return x, y


@pytest.mark.parametrize("h,w", [(11, 11), (11, 75), (75, 11), (99, 74), (98, 75), (37, 45),
                                 (64, 200), (200, 150), (181, 267), (186, 75), (187, 74),
                                 (363, 65)])
def test_ssim_matches_oracle(cuda, h, w):
    x, y = _pair(h, w, seed=h * 1000 + w)
    got = float(A.ssim(_dev(x, cuda), _dev(y, cuda), None).cpu().numpy()[0, 0])
    assert abs(got - S.ssim(x, y)) <= TOL, (got, S.ssim(x, y))


def test_ssim_identity_and_determinism(cuda):
    x, y = _pair(130, 170, seed=7, noise=40)
    dx, dy = _dev(x, cuda), _dev(y, cuda)
    assert abs(float(A.ssim(dx, dx, None).cpu()[0, 0]) - 1.0) <= 1e-12
    a = A.ssim(dx, dy, None).cpu().numpy()
    b = A.ssim(dx, dy, None).cpu().numpy()
    assert np.array_equal(a, b)
    assert abs(float(a[0, 0]) - S.ssim(x, y)) <= TOL


def test_ssim_pitched_stream(cuda):
    """Three 4:2:0 frames with padded rows on both sides (different frame strides)."""
    import torch
    spec = video_spec(n_frames=3, width=176, height=96, seed=8)
    bases = video_base_planes(spec)
    frames = np.stack([video_frame(spec, bases, f) for f in range(3)])
    rng = np.random.default_rng(9)
    noisy = np.clip(frames.astype(np.int64) + rng.integers(-15, 16, frames.shape), 0, 255).astype(np.uint8)
    pad = 16
    planes, ref_parts, tst_parts, off = [], [], [], 0
    for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets):
        planes.append((off, h, w, w + pad))
        off += h * (w + pad)
    ref = np.zeros((3, off + 32), dtype=np.uint8)
    tst = np.zeros((3, off + 64), dtype=np.uint8)
    for f in range(3):
        for (o2, h, w, p), ((hh, ww), o) in zip(planes, zip(spec.plane_shapes, spec.plane_offsets)):
            ref[f, o2:o2 + h * p].reshape(h, p)[:, :w] = frames[f, o:o + h * w].reshape(h, w)
            tst[f, o2:o2 + h * p].reshape(h, p)[:, :w] = noisy[f, o:o + h * w].reshape(h, w)
    got = A.ssim(_dev(ref, cuda), _dev(tst, cuda), planes).cpu().numpy()
    for f in range(3):
        for k, ((h, w), o) in enumerate(zip(spec.plane_shapes, spec.plane_offsets)):
            want = S.ssim(frames[f, o:o + h * w].reshape(h, w), noisy[f, o:o + h * w].reshape(h, w))
            assert abs(got[f, k] - want) <= TOL, (f, k)


def test_ssim_full_4k_frame(cuda):
    """The benchmark's frame shape: a 3840 x 2160 4:2:0 frame against its T1
    reconstruction (r = 10, step 16), every plane against the oracle."""
    import torch
    spec = video_spec(n_frames=1, seed=4)
    bases = video_base_planes(spec)
    frame = video_frame(spec, bases, 0)
    planes = [(o, h, w, w) for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets)]
    d = _dev(frame[None], cuda)
    recon = torch.empty_like(d)
    A.evaluate_stream(d, planes, "T1", 10, 16, recon=recon)
    got = A.ssim(d, recon, planes).cpu().numpy()[0]
    rec = recon.cpu().numpy()[0]
    for k, ((h, w), o) in enumerate(zip(spec.plane_shapes, spec.plane_offsets)):
        want = S.ssim(frame[o:o + h * w].reshape(h, w), rec[o:o + h * w].reshape(h, w))
        assert abs(got[k] - want) <= TOL, (k, got[k], want)
