"""GPU parity of quantised coding at steps that admit exact reconstruction
halves (Sec. 6.1.1 dequantisation and inverse; the rounding of reading 5 with
the quantiser of reading 6).  With such a step (5, 12, 3, 20 for the
built-in matrices) the library decides every pixel within its tolerance of a
half exactly in the field the row norms generate; levels, pixels and squared
errors must equal the oracle's bit for bit, and the constructed exact halves
must round to even."""

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import codec as Co
from oracle import matrices as M
from synth import ar1_image

pytestmark = pytest.mark.gpu

INT_T = ["T1", "T2", "LO", "T6", "RDCT", "T4"]


def _dev(x, cuda):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(cuda)


@pytest.mark.parametrize("name", INT_T)
@pytest.mark.parametrize("step", [5, 12, 3])
@pytest.mark.parametrize("r", [10, 21, 64])
def test_general_steps_match_oracle(cuda, name, step, r):
    import torch
    img = ar1_image(64, 136, 0.93, seed=7 * r + step)        # 8 x 17 blocks: three waves
    t = M.TRANSFORMS[name]
    ref = Co.evaluate(img, t, r, step)
    d = _dev(img, cuda)
    h, w = img.shape
    recon = torch.empty_like(d)
    coef = torch.empty((A.n_blocks(h, w), r), dtype=torch.int16, device=cuda)
    ev = A.evaluate_coding(d, name, r, step, coef_int=coef, recon=recon)
    assert np.array_equal(coef.cpu().numpy(), ref["coef_int"]), (name, step, r)
    assert np.array_equal(recon.cpu().numpy(), ref["rec"]), (name, step, r)
    assert ev.sse == ref["sse"]
    rec2 = A.decode_blocks(coef, h, w, name, r, step)
    assert np.array_equal(rec2.cpu().numpy(), ref["rec"])


def test_exact_halves_round_to_even(cuda):
    """T1, step 5: a DC level q gives every pixel 5 q / 8; q = 4, 12, -4, 20 sit
    exactly on 2.5, 7.5, -2.5, 12.5 and round to 2, 8, 0, 12.  Random DC and
    (0, 1) levels over many blocks put many pixels on exact halves."""
    import torch
    levels = np.array([4, 12, -4, 20, 36, 100, 204], dtype=np.int16)
    coef = torch.from_numpy(levels.reshape(-1, 1)).to(cuda)
    h, w = 8, 8 * len(levels)
    rec = A.decode_blocks(coef, h, w, "T1", 1, 5).cpu().numpy()
    want = Co.decode(levels.reshape(-1, 1).astype(np.int64), M.T1, 1, h, w, 5)["rec"]
    assert np.array_equal(rec, want)
    assert np.all(rec[:, :8] == 2) and np.all(rec[:, 8:16] == 8) and np.all(rec[:, 24:32] == 12)
    rng = np.random.default_rng(3)
    nb = 64 * 5 + 13
    q = np.zeros((nb, 3), dtype=np.int16)
    q[:, 0] = rng.integers(-8, 420, nb) * 4               # 5 q / 8 on a half for q = 4 mod 8
    q[:, 1] = rng.integers(-20, 20, nb) * 8               # (0, 1): rational class 144
    h, w = 8, 8 * nb
    rec = A.decode_blocks(torch.from_numpy(q).to(cuda), h, w, "T1", 3, 5).cpu().numpy()
    want = Co.decode(q.astype(np.int64), M.T1, 3, h, w, 5)
    assert np.array_equal(rec, want["rec"])
    real = want["real"]
    assert np.sum(np.abs(real - np.floor(real) - 0.5) < 1e-12) > 1000   # many exact halves


def test_near_halves_with_square_roots(cuda):
    """T1 at step 20 with levels q_00 and q_02 (class 160 = 16 x 10): at pixels
    with T[0, x] T[2, y] = 1 the value is 2.5 q_00 + q_02 sqrt(10) / 2; with
    q_02 = b from a convergent p / b of sqrt(10) (p odd) it lies within
    1 / (4 b sqrt 10) of a half, on either side depending on the convergent."""
    import torch
    cases = []
    for p, b in ((721, 228), (4443, 1405), (27379, 8658)):
        for target2 in (497, 499, 501, 503, 505):
            num = target2 - p
            if num % 10 == 0:
                q = np.zeros(6, dtype=np.int16)
                q[0] = num // 5
                q[5] = b
                cases.append(q)
    assert len(cases) >= 3
    q = np.stack(cases)
    h, w = 8, 8 * len(cases)
    rec = A.decode_blocks(torch.from_numpy(q).to(cuda), h, w, "T1", 6, 20).cpu().numpy()
    want = Co.decode(q.astype(np.int64), M.T1, 6, h, w, 20)["rec"]
    assert np.array_equal(rec, want)


def test_general_step_stream(cuda):
    """The stream entry point at step 5 (T6, three planes of a 4:2:0 frame pair)
    equals the oracle plane by plane."""
    import torch
    y = ar1_image(48, 64, 0.9, seed=1)
    u = ar1_image(24, 32, 0.9, seed=2)
    v = ar1_image(24, 32, 0.9, seed=3)
    frame = np.concatenate([y.ravel(), u.ravel(), v.ravel()])
    frames = np.stack([frame, frame[::-1].copy()])
    planes = [(0, 48, 64, 64), (48 * 64, 24, 32, 32), (48 * 64 + 24 * 32, 24, 32, 32)]
    d = torch.from_numpy(frames).to(cuda)
    recon = torch.empty_like(d)
    sse = A.evaluate_stream(d, planes, "T6", 10, 5, recon=recon).cpu().numpy()
    for f in range(2):
        for p, (o, h, w, _) in enumerate(planes):
            img = frames[f, o:o + h * w].reshape(h, w)
            ref = Co.evaluate(img, M.T6, 10, 5)
            assert int(sse[f, p]) == ref["sse"], (f, p)
            assert np.array_equal(recon[f, o:o + h * w].cpu().numpy().reshape(h, w), ref["rec"])


def test_general_step_4k_stream_sampled(cuda):
    """A step that admits exact halves (T1, step 12) on the benchmark's frame
    shape (3840 x 2160 4:2:0, r = 10), through the run-time kernels: every
    plane's squared error of one frame against the oracle, and 300 sampled
    blocks of a second frame (levels and pixels)."""
    import torch
    from synth import video_base_planes, video_frame, video_spec
    spec = video_spec(n_frames=2)
    bases = video_base_planes(spec)
    frames = np.stack([video_frame(spec, bases, f) for f in range(2)])
    planes = [(o, h, w, w) for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets)]
    d = _dev(frames, cuda)
    bpf = A.stream_blocks_per_frame(planes)
    coef = torch.empty((2, bpf, 10), dtype=torch.int16, device=cuda)
    recon = torch.empty_like(d)
    sse = A.evaluate_stream(d, planes, "T1", 10, 12, coef=coef, recon=recon).cpu().numpy()
    for p, ((h, w), off) in enumerate(zip(spec.plane_shapes, spec.plane_offsets)):
        ref = Co.evaluate(frames[0, off:off + h * w].reshape(h, w), M.T1, 10, 12)
        assert int(sse[0, p]) == ref["sse"], p
    rng = np.random.default_rng(12)
    coef_h = coef.cpu().numpy()
    recon_h = recon.cpu().numpy()
    for _ in range(300):
        p = int(rng.integers(3))
        h, w = spec.plane_shapes[p]
        off = spec.plane_offsets[p]
        by, bx = int(rng.integers(h // 8)), int(rng.integers(w // 8))
        blk = frames[1, off:off + h * w].reshape(h, w)[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
        ref_b = Co.evaluate(blk, M.T1, 10, 12)
        b = sum((hh // 8) * (ww // 8) for hh, ww in spec.plane_shapes[:p]) + by * (w // 8) + bx
        assert np.array_equal(coef_h[1, b], ref_b["coef_int"][0])
        rb = recon_h[1, off:off + h * w].reshape(h, w)[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
        assert np.array_equal(rb, ref_b["rec"])
