"""GPU N x N transform coding with the 16- and 32-point JAM matrices
(adct_jam_evaluate_stream) against the oracle.

Bar: reconstructions, squared errors and coefficients bit-exact.  Without a
quantiser both sides reconstruct in exact rational arithmetic.  With one, the
levels are exact (where the quotient is rational, a float32 form whose error is
bounded below the distance to the nearest integer; float64 where it is
irrational, which never sits within float64 error of a half for these
magnitudes), and the float64 reconstruction can only differ from the oracle's
exactly settled one within float64 error of a half, which the allowed steps
(multiples of N) keep away from exact halves."""

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import jam
from oracle import matrices as M
from synth import ar1_image, video_base_planes, video_frame, video_spec

pytestmark = pytest.mark.gpu

TN = {16: jam.jam_n(M.T1, 16), 32: jam.jam_n(M.T1, 32)}


def _dev(x, cuda):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(cuda)


def _run_image(img, n, r, step, cuda, pitch=None):
    import torch
    h, w = img.shape
    pitch = pitch or w
    buf = np.full((h, pitch), 77, dtype=np.uint8)
    buf[:, :w] = img
    frames = _dev(buf.reshape(1, -1), cuda)
    recon = torch.full_like(frames, 3)
    nb = A.jam_blocks_per_frame([(0, h, w, pitch)], n)
    coef = torch.empty(nb * r, dtype=torch.int32, device=cuda)
    sse = A.jam_evaluate_stream(frames, [(0, h, w, pitch)], n, r, step, coef=coef, recon=recon)
    rec = recon.cpu().numpy().reshape(h, pitch)
    assert np.all(rec[:, w:] == 3), "bytes outside the plane were written"
    return rec[:, :w], int(sse.cpu().numpy()[0, 0]), coef.cpu().numpy().reshape(nb, r)


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("shape", [(64, 128), (70, 45), (5, 3), (33, 129), (96, 200)])
@pytest.mark.parametrize("r,step", [(1, 0), (10, 0), (40, 0), (3, 16), (40, 16), (130, 32)])
def test_jam_matches_oracle(cuda, n, shape, r, step):
    if step % n:
        step = 2 * n
    img = ar1_image(*shape, rho=0.93, seed=shape[0] * 7 + shape[1] + r)
    rec, sse, coef = _run_image(img, n, r, step, cuda)
    want = jam.evaluate(img, TN[n], r, step)
    assert np.array_equal(coef, want["coef_int"])
    assert np.array_equal(rec, want["rec"])
    assert sse == want["sse"]


@pytest.mark.parametrize("n", [16, 32])
def test_jam_full_retention_and_wide_band(cuda, n):
    img = ar1_image(2 * n + 5, 3 * n + 7, rho=0.9, seed=n)
    for r in (n * n, n * n - 1, n * n // 2 + 1, 2 * n + 3):
        rec, sse, coef = _run_image(img, n, r, 0, cuda)
        want = jam.evaluate(img, TN[n], r, 0)
        assert np.array_equal(rec, want["rec"]) and sse == want["sse"], r
        assert np.array_equal(coef, want["coef_int"]), r
    rec, sse, _ = _run_image(img, n, n * n, 0, cuda)
    assert sse == 0 and np.array_equal(rec, img)
    for r, step in ((n * n, n), (n * n // 3, 3 * n)):
        rec, sse, coef = _run_image(img, n, r, step, cuda)
        want = jam.evaluate(img, TN[n], r, step)
        assert np.array_equal(coef, want["coef_int"]) and np.array_equal(rec, want["rec"]), (r, step)


def test_jam_pitched_multiplane_stream(cuda):
    """Three 4:2:0 frames (sides not multiples of 16 or 32) with padded rows."""
    import torch
    spec = video_spec(n_frames=3, width=200, height=120, seed=5)
    bases = video_base_planes(spec)
    frames = [video_frame(spec, bases, f) for f in range(3)]
    planes, off = [], 0
    pad = 24
    for h, w in spec.plane_shapes:
        planes.append((off, h, w, w + pad))
        off += h * (w + pad)
    buf = np.zeros((3, off + 40), dtype=np.uint8)
    for f in range(3):
        src = 0
        for (o, h, w, p) in planes:
            buf[f, o:o + h * p].reshape(h, p)[:, :w] = frames[f][src:src + h * w].reshape(h, w)
            src += h * w
    dev = _dev(buf, cuda)
    for n, r, step in ((16, 36, 16), (32, 150, 32), (16, 20, 0)):
        recon = torch.zeros_like(dev)
        sse = A.jam_evaluate_stream(dev, planes, n, r, step, recon=recon).cpu().numpy()
        rec = recon.cpu().numpy()
        for f in range(3):
            src = 0
            for p, (o, h, w, pitch) in enumerate(planes):
                img = frames[f][src:src + h * w].reshape(h, w)
                src += h * w
                want = jam.evaluate(img, TN[n], r, step)
                got = rec[f, o:o + h * pitch].reshape(h, pitch)[:, :w]
                assert np.array_equal(got, want["rec"]), (n, f, p)
                assert int(sse[f, p]) == want["sse"], (n, f, p)


@pytest.mark.parametrize("n,r,step", [(16, 40, 16), (32, 160, 32)])
def test_jam_full_4k_frame(cuda, n, r, step):
    """One 3840 x 2160 4:2:0 frame in the benchmark's launch configuration:
    per-plane squared errors and the luma reconstruction against the oracle."""
    import torch
    spec = video_spec(n_frames=1)
    bases = video_base_planes(spec)
    frame = video_frame(spec, bases, 0)
    dev = _dev(frame.reshape(1, -1), cuda)
    planes, off = [], 0
    for h, w in spec.plane_shapes:
        planes.append((off, h, w, w))
        off += h * w
    recon = torch.zeros_like(dev)
    sse = A.jam_evaluate_stream(dev, planes, n, r, step, recon=recon).cpu().numpy()
    rec = recon.cpu().numpy()[0]
    for p, (o, h, w, _) in enumerate(planes):
        img = frame[o:o + h * w].reshape(h, w)
        want = jam.evaluate(img, TN[n], r, step)
        assert int(sse[0, p]) == want["sse"], p
        if p == 0:
            assert np.array_equal(rec[o:o + h * w].reshape(h, w), want["rec"])


def test_jam_repeat_is_bit_identical(cuda):
    img = ar1_image(300, 260, rho=0.95, seed=3)
    a = _run_image(img, 32, 200, 64, cuda)
    b = _run_image(img, 32, 200, 64, cuda)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("n", [16, 32])
def test_jam_exact_quantiser_ties(cuda, n):
    """Two-level blocks put B(0, 0) / step and B(0, 1) / step exactly on halves
    of both signs."""
    rng = np.random.default_rng(n)
    nb = 8
    img = np.zeros((2 * n, nb * n), dtype=np.uint8)
    for by in range(2):
        for i in range(nb):
            a, b = int(rng.integers(0, 128)) * 2 + 1, int(rng.integers(0, 128)) * 2
            if (by + i) % 2:
                a, b = b, a
            img[by * n:(by + 1) * n, i * n:i * n + n // 2] = a
            img[by * n:(by + 1) * n, i * n + n // 2:(i + 1) * n] = b
    for r, step in ((2, n), (3, n), (10, 3 * n)):
        rec, sse, coef = _run_image(img, n, r, step, cuda)
        want = jam.evaluate(img, TN[n], r, step)
        assert np.array_equal(coef, want["coef_int"]), (r, step)
        assert np.array_equal(rec, want["rec"]) and sse == want["sse"], (r, step)


@pytest.mark.parametrize("n", [16, 32])
def test_jam_degenerate_shapes_and_largest_step(cuda, n):
    """One-pixel, one-row and one-column planes (every block is edge-extended)
    and the largest quantiser step the library takes (4096: nearly every level 0)."""
    for shape in ((1, 1), (1, 700), (700, 1), (n + 1, n - 1)):
        img = ar1_image(*shape, rho=0.9, seed=shape[0] + 3 * shape[1])
        for r, step in ((1, 0), (7, n), (n * n, 4096)):
            rec, sse, coef = _run_image(img, n, r, step, cuda)
            want = jam.evaluate(img, TN[n], r, step)
            assert np.array_equal(coef, want["coef_int"]), (shape, r, step)
            assert np.array_equal(rec, want["rec"]) and sse == want["sse"], (shape, r, step)


def _dc_blocks(n, sums, per_row=256):
    """A plane of n x n blocks in raster order whose pixel sums are `sums`
    (255s first, then the remainder, then zeros), padded with zero blocks."""
    nb = len(sums)
    rows = (nb + per_row - 1) // per_row
    s = np.zeros(rows * per_row, dtype=np.int64)
    s[:nb] = sums
    p = np.arange(n * n, dtype=np.int32)[None, :]
    full = (s // 255).astype(np.int32)[:, None]
    rem = (s % 255).astype(np.int32)[:, None]
    vals = np.where(p < full, 255, np.where(p == full, rem, 0)).astype(np.uint8)
    img = vals.reshape(rows, per_row, n, n).transpose(0, 2, 1, 3).reshape(rows * n, per_row * n)
    return np.ascontiguousarray(img)


@pytest.mark.parametrize("n,lo,hi", [(16, 0, 255 * 256 + 1), (32, 0, 65536), (32, 255 * 1024 - 65535, 255 * 1024 + 1)])
def test_jam_dc_levels_every_sum(cuda, n, lo, hi):
    """The DC level for every pixel sum S in [lo, hi) (for N = 16 every sum a
    block can have), at steps N, 3N and 7N: round-half-away(S / (n_0 step)) with
    n_0 = N, so every sum that is an odd multiple of n_0 step / 2 is an exact
    half.  The closed form, in integers, is checked against the oracle on a row
    of exact halves and their neighbours."""
    import torch
    sums = np.arange(lo, hi, dtype=np.int64)
    img = _dc_blocks(n, sums)
    h, w = img.shape
    frames = _dev(img.reshape(1, -1), cuda)
    nb = A.jam_blocks_per_frame([(0, h, w, w)], n)
    coef = torch.empty(nb, dtype=torch.int32, device=cuda)
    for step in (n, 3 * n, 7 * n):
        A.jam_evaluate_stream(frames, [(0, h, w, w)], n, 1, step, coef=coef)
        got = coef.cpu().numpy()[:len(sums)].astype(np.int64)
        d = n * step
        want = (2 * sums + d) // (2 * d)
        assert np.array_equal(got, want), (n, step, int(np.nonzero(got != want)[0][0]))
        halves = d * (2 * np.arange(1, 9, dtype=np.int64) + 1) // 2
        probe = np.concatenate([halves - 1, halves, halves + 1])
        probe = probe[(probe >= 0) & (probe <= 255 * n * n)]
        ref = jam.evaluate(_dc_blocks(n, probe, per_row=len(probe)), TN[n], 1, step)["coef_int"][:, 0]
        assert np.array_equal(ref.astype(np.int64), (2 * probe + d) // (2 * d))
