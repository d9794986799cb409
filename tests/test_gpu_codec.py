"""GPU parity of the fused codec against the CPU oracle (through the C ABI).

Integer stage, quantised levels, reconstructed pixels and squared errors are
compared bit for bit; float coefficients within 1e-5 relative."""

import math

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import codec as Co
from oracle import matrices as M
from synth import ar1_image, video_base_planes, video_frame, video_spec

pytestmark = pytest.mark.gpu

INT_T = ["T1", "T2", "LO", "T6", "RDCT", "T4"]


def _dev(x, cuda):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(cuda)


def _oracle(img, name, r, step=0):
    return Co.evaluate(img, M.TRANSFORMS[name], r, step)


def test_config1_512_t1_r10(cuda):
    import torch
    img = ar1_image(512, 512, 0.95, seed=0)
    ref = _oracle(img, "T1", 10)
    d = _dev(img, cuda)
    ci, cf = A.encode_blocks(d, "T1", 10, want_scaled=True)
    assert np.array_equal(ci.cpu().numpy(), ref["coef_int"])
    b = cf.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(b - ref["coef_scaled"]) <= 1e-5 * np.maximum(np.abs(ref["coef_scaled"]), 1.0))
    rec = A.decode_blocks(ci, 512, 512, "T1", 10)
    assert np.array_equal(rec.cpu().numpy(), ref["rec"])
    recon = torch.empty_like(d)
    coef = torch.empty_like(ci)
    ev = A.evaluate_coding(d, "T1", 10, coef_int=coef, recon=recon)
    assert ev.sse == ref["sse"]
    assert ev.psnr == pytest.approx(ref["psnr"], rel=1e-12)
    assert np.array_equal(recon.cpu().numpy(), ref["rec"])
    assert np.array_equal(coef.cpu().numpy(), ref["coef_int"])


@pytest.mark.parametrize("name", INT_T)
@pytest.mark.parametrize("r", [1, 3, 10, 11, 36, 64])
def test_zonal_all_transforms_ragged(cuda, name, r):
    # 9 x 17 = 153 blocks: three waves, the last one partly empty
    img = ar1_image(72, 136, 0.9, seed=11 + r)
    ref = _oracle(img, name, r)
    d = _dev(img, cuda)
    import torch
    recon = torch.empty_like(d)
    coef = None if name == "LO" else torch.empty((153, r), dtype=torch.int16, device=cuda)
    ev = A.evaluate_coding(d, name, r, coef_int=coef, recon=recon)
    assert ev.sse == ref["sse"]
    assert np.array_equal(recon.cpu().numpy(), ref["rec"])
    if coef is not None:
        assert np.array_equal(coef.cpu().numpy(), ref["coef_int"])
        rec2 = A.decode_blocks(coef, 72, 136, name, r)
        assert np.array_equal(rec2.cpu().numpy(), ref["rec"])


QSTEP = {"T1": 8, "T2": 8, "T6": 8, "RDCT": 8, "T4": 8, "LO": 32}


@pytest.mark.parametrize("name", INT_T)
@pytest.mark.parametrize("r,mult", [(10, 2), (64, 2), (6, 1), (21, 5)])
def test_quantised_all_transforms(cuda, name, r, mult):
    step = QSTEP[name] * mult
    img = ar1_image(64, 200, 0.95, seed=r + step)
    ref = _oracle(img, name, r, step)
    d = _dev(img, cuda)
    import torch
    recon = torch.empty_like(d)
    coef = torch.empty((Co.to_blocks(img).shape[0], r), dtype=torch.int16, device=cuda)
    ev = A.evaluate_coding(d, name, r, step, coef_int=coef, recon=recon)
    assert np.array_equal(coef.cpu().numpy(), ref["coef_int"])
    assert np.array_equal(recon.cpu().numpy(), ref["rec"])
    assert ev.sse == ref["sse"]
    rec2 = A.decode_blocks(coef, 64, 200, name, r, step)
    assert np.array_equal(rec2.cpu().numpy(), ref["rec"])


def test_single_block_and_extremes(cuda):
    import torch
    for img in (np.zeros((8, 8), np.uint8), np.full((8, 8), 255, np.uint8),
                np.tile(np.array([0, 255], np.uint8), (8, 4)),
                (np.indices((8, 8)).sum(0) % 2 * 255).astype(np.uint8)):
        for name in INT_T:
            for r in (1, 10, 64):
                ref = _oracle(img, name, r)
                ev = A.evaluate_coding(_dev(img, cuda), name, r)
                assert ev.sse == ref["sse"], (name, r)


def test_pitched_input(cuda):
    import torch
    img = ar1_image(48, 64, 0.95, seed=4)
    big = torch.zeros((48, 96), dtype=torch.uint8, device=cuda)
    big[:, :64] = _dev(img, cuda)
    view = big[:, :64]
    ref = _oracle(img, "T1", 10)
    recon = torch.zeros((48, 80), dtype=torch.uint8, device=cuda)
    ev = A.evaluate_coding(view, "T1", 10, recon=recon[:, :64])
    assert ev.sse == ref["sse"]
    assert np.array_equal(recon[:, :64].cpu().numpy(), ref["rec"])
    assert int(recon[:, 64:].sum()) == 0          # pitch padding untouched


def _stream_oracle(spec, bases, frames, r, step):
    out = []
    for f in frames:
        buf = video_frame(spec, bases, f)
        per = []
        for (h, w), off in zip(spec.plane_shapes, spec.plane_offsets):
            plane = buf[off:off + h * w].reshape(h, w)
            per.append(Co.evaluate(plane, M.T1, r, step))
        out.append(per)
    return out


def test_stream_small_yuv(cuda):
    import torch
    spec = video_spec(n_frames=3, width=144, height=80, seed=5)
    bases = video_base_planes(spec)
    frames = np.stack([video_frame(spec, bases, f) for f in range(3)])
    planes = [(o, h, w, w) for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets)]
    d = _dev(frames, cuda)
    bpf = A.stream_blocks_per_frame(planes)
    coef = torch.empty((3, bpf, 10), dtype=torch.int16, device=cuda)
    recon = torch.empty_like(d)
    sse = A.evaluate_stream(d, planes, "T1", 10, 16, coef=coef, recon=recon)
    torch.cuda.synchronize()
    ref = _stream_oracle(spec, bases, range(3), 10, 16)
    sse = sse.cpu().numpy()
    coef = coef.cpu().numpy()
    recon = recon.cpu().numpy()
    for f in range(3):
        boff = 0
        for p, ((h, w), off) in enumerate(zip(spec.plane_shapes, spec.plane_offsets)):
            nb = (h // 8) * (w // 8)
            assert sse[f, p] == ref[f][p]["sse"]
            assert np.array_equal(coef[f, boff:boff + nb], ref[f][p]["coef_int"])
            assert np.array_equal(recon[f, off:off + h * w].reshape(h, w), ref[f][p]["rec"])
            boff += nb


def test_stream_4k_sampled(cuda):
    """The benchmark's launch shape (T1, r = 10, step 16, 4K 4:2:0) on a
    shortened stream: two frames checked whole, the others on sampled blocks."""
    import torch
    nf = 12
    spec = video_spec(n_frames=nf)
    bases = video_base_planes(spec)
    frames = np.stack([video_frame(spec, bases, f) for f in range(nf)])
    planes = [(o, h, w, w) for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets)]
    d = _dev(frames, cuda)
    bpf = A.stream_blocks_per_frame(planes)
    coef = torch.empty((nf, bpf, 10), dtype=torch.int16, device=cuda)
    recon = torch.empty_like(d)
    sse = A.evaluate_stream(d, planes, "T1", 10, 16, coef=coef, recon=recon).cpu().numpy()
    ref = _stream_oracle(spec, bases, [0, nf - 1], 10, 16)
    for i, f in enumerate([0, nf - 1]):
        for p in range(3):
            assert sse[f, p] == ref[i][p]["sse"]
    rng = np.random.default_rng(0)
    coef_h = coef.cpu().numpy()
    recon_h = recon.cpu().numpy()
    for _ in range(300):
        f = int(rng.integers(nf))
        p = int(rng.integers(3))
        h, w = spec.plane_shapes[p]
        off = spec.plane_offsets[p]
        by, bx = int(rng.integers(h // 8)), int(rng.integers(w // 8))
        blk = frames[f, off:off + h * w].reshape(h, w)[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
        ref_b = Co.evaluate(blk, M.T1, 10, 16)
        boff = sum((hh // 8) * (ww // 8) for hh, ww in spec.plane_shapes[:p])
        b = boff + by * (w // 8) + bx
        assert np.array_equal(coef_h[f, b], ref_b["coef_int"][0])
        rb = recon_h[f, off:off + h * w].reshape(h, w)[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
        assert np.array_equal(rb, ref_b["rec"])


def test_device_argument_errors(cuda):
    import torch
    img = torch.zeros((16, 16), dtype=torch.uint8, device=cuda)
    with pytest.raises(A.AdctError) as e:
        A.evaluate_coding(img[:, 1:9], "T1", 10)       # misaligned base
    assert e.value.status == -2
    with pytest.raises(A.AdctError) as e:
        A.encode_blocks(img, "LO", 10)                 # LO does not fit int16
    assert e.value.status == -4


def test_bandwidth_probe_moves_the_stream_bytes(cuda):
    """The bandwidth probe (the codec's loads and stores without its arithmetic)
    copies every plane's pixels into recon and fills the coefficient run of every
    block, leaving bytes outside the planes untouched."""
    import torch
    planes = [(0, 48, 64, 72), (48 * 72, 24, 32, 40)]
    fbytes = 48 * 72 + 24 * 40
    rng = np.random.Generator(np.random.PCG64(9))
    frames = rng.integers(0, 255, size=(3, fbytes), dtype=np.uint8)     # no 0xffff byte pair
    d = torch.from_numpy(frames).to(cuda)
    recon = torch.full_like(d, 7)
    nb = A.stream_blocks_per_frame(planes)
    coef = torch.full((3 * nb * 10,), -1, dtype=torch.int16, device=cuda)
    A.stream_bandwidth_probe(d, planes, 10, coef=coef, recon=recon)
    rc = recon.cpu().numpy()
    inside = np.zeros(fbytes, dtype=bool)
    for off, h, w, pitch in planes:
        for y in range(h):
            inside[off + y * pitch: off + y * pitch + w] = True
    assert np.array_equal(rc[:, inside], frames[:, inside])
    assert np.all(rc[:, ~inside] == 7)
    # every coefficient entry was written (with two pixel bytes, never 0xffff)
    assert not np.any(coef.cpu().numpy() == -1)
