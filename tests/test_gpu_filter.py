"""GPU parity of the learned post-filter (through the C ABI) against the
float64 oracle evaluated on the same bfloat16-rounded weights and activations.

Tolerances.  The GPU sums K <= 289 exact bfloat16 products (and the bias) in
float32, so each pre-activation carries an error of at most K u sum|terms|
(u = 2^-24).  The activation is then rounded to bfloat16 on both sides: the two
roundings agree unless the exact pre-activation lies within that error of a
bfloat16 rounding midpoint, where they may differ by one bfloat16 unit.
`_y_bound` propagates exactly this through the three layers, from oracle
quantities only, into a per-pixel bound on |y_gpu - y_oracle|; every pixel
must be within it, and pixels may differ only where 128 + 64 y is within
64 times it of a half-integer.  Besides, the bulk must be tight: at least 90 %
of y within 1e-4 of max(1, |y|), counted separately on the two-pixel border
ring and on the interior (measured: about 96 %; the rest are pixels whose
receptive field holds an activation that rounds to the other side of a
bfloat16 midpoint).  Gradients, per parameter group: the error norm within
1e-3 of the group's norm (measured: below 5e-5), every entry within 1e-3 of
the group's largest (measured: below 1e-4), and every entry of at least a tenth
of the group's largest within 1e-3 of itself (measured: below 5e-4; a
relative bound means nothing for entries near zero, which cancel)."""

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import codec as Co
from oracle import matrices as M
from oracle import postfilter as F
from synth import ar1_image, filter_params, video_base_planes, video_frame, video_spec

pytestmark = pytest.mark.gpu

GROUPS = [(name, int(np.prod(shape))) for name, shape in F.LAYOUT]


def _dev(x, cuda):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(cuda)


def _batch(n, h, w, seed, r=10):
    """Originals from the AR(1) generator, decoded by the oracle codec (T1, r)."""
    orig = np.stack([ar1_image(h, w, 0.9, seed=seed + k) for k in range(n)])
    recon = np.stack([Co.evaluate(o, M.T1, r)["rec"] for o in orig]).astype(np.uint8)
    return recon, orig


U = 2.0 ** -24


def _flip(z, err):
    """Bound on |bf16(relu(z')) - bf16(relu(z))| over |z' - z| <= err."""
    az = np.abs(z)
    ulp = np.exp2(np.floor(np.log2(np.maximum(az, 1e-300))) - 7)
    q = az / ulp
    near = np.abs(q - np.floor(q) - 0.5) * ulp <= err
    may_cross = near | (az <= err)
    return np.where(may_cross, err + np.exp2(np.floor(np.log2(np.maximum(az + err, 1e-300))) - 7), 0.0)


def _y_bound(p, x):
    """Per-pixel bound on |y_gpu - y_oracle| (float32 sums, bfloat16 re-rounding)."""
    P = F.unflatten(p)
    fw = F.forward(p, x, rounding=True)
    w1, w2, w3 = (np.abs(fw[k]) for k in ("w1", "w2", "w3"))
    z1 = F.conv3x3(fw["xn"], fw["w1"], P["b1"])
    e1 = 10 * U * (F.conv3x3(np.abs(fw["xn"]), w1) + np.abs(P["b1"])[None, :, None, None])
    d1 = _flip(z1, e1)
    z2 = F.conv3x3(fw["a1"], fw["w2"], P["b2"])
    e2 = 289 * U * (F.conv3x3(fw["a1"], w2) + np.abs(P["b2"])[None, :, None, None]) + F.conv3x3(d1, w2)
    d2 = _flip(z2, e2)
    e3 = 289 * U * (F.conv3x3(fw["a2"], w3)[:, 0] + abs(P["b3"][0])) + F.conv3x3(d2, w3)[:, 0]
    return e3 + 4 * U * (np.abs(fw["xn"][:, 0]) + np.abs(fw["f"])) + 1e-7, fw


def _groups(v):
    out, o = {}, 0
    for name, n in GROUPS:
        out[name] = v[o:o + n]
        o += n
    return out


@pytest.mark.parametrize("shape,seed", [((2, 32, 64), 1), ((3, 16, 32), 2)])
def test_grad_matches_oracle(cuda, shape, seed):
    import torch
    n, h, w = shape
    recon, orig = _batch(n, h, w, 100 * seed)
    p = filter_params(seed, last_scale=1.0, bias_scale=0.1)
    grad, loss, y = A.filter_grad(_dev(p, cuda), _dev(recon, cuda), _dev(orig, cuda), want_y=True)
    torch.cuda.synchronize()
    rl, rg, fw = F.loss_and_grad(p, recon, orig, rounding=True)
    bound, _ = _y_bound(p, recon)
    yg = y.cpu().numpy().astype(np.float64)
    dy = np.abs(yg - fw["y"])
    ok = dy <= 1e-4 * np.maximum(1.0, np.abs(fw["y"]))
    ring = np.zeros(ok.shape[1:], dtype=bool)
    ring[:2], ring[-2:], ring[:, :2], ring[:, -2:] = True, True, True, True
    tight = min(ok[:, ring].mean(), ok[:, ~ring].mean())
    print(f"y: max |dy| {dy.max():.3g}, mean {dy.mean():.3g}, max dy/bound {np.max(dy / bound):.3g}, "
          f"tight {tight:.5f}; loss {float(loss.item()):.9g} vs {rl:.9g}")
    g = _groups(grad.cpu().numpy().astype(np.float64))
    r = _groups(rg)
    errs, norms, rels = {}, {}, {}
    for name, _ in GROUPS:
        d, a = np.abs(g[name] - r[name]), np.abs(r[name])
        err, scale = d.max(), a.max()
        errs[name] = err / scale
        norms[name] = np.linalg.norm(g[name] - r[name]) / np.linalg.norm(r[name])
        big = a >= 0.1 * scale
        rels[name] = (d[big] / a[big]).max()
        print(f"{name}: max err {err:.3g} of scale {scale:.3g}; rel norm {norms[name]:.3g}; "
              f"rel of entries >= scale / 10: {rels[name]:.3g}")
    assert np.all(dy <= bound)
    assert tight >= 0.90
    assert abs(float(loss.item()) - rl) <= 1e-4 * rl
    for name, e in errs.items():
        assert e <= 1e-3, name
        assert norms[name] <= 1e-3, name
        assert rels[name] <= 1e-3, name


def test_grad_is_deterministic(cuda):
    import torch
    recon, orig = _batch(2, 32, 64, 7)
    p = _dev(filter_params(3, last_scale=1.0, bias_scale=0.1), cuda)
    ws = A.filter_workspace(2, 32, 64, cuda)
    g1, l1, _ = A.filter_grad(p, _dev(recon, cuda), _dev(orig, cuda), workspace=ws)
    g2, l2, _ = A.filter_grad(p, _dev(recon, cuda), _dev(orig, cuda), workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_adam_matches_oracle(cuda):
    """The kernel works in float32 on float32 hyper-parameters: the oracle gets
    the same (float32-valued) hyper-parameters, and each result may differ by a
    few float32 roundings of the terms it sums (m and v can cancel)."""
    import torch
    rng = np.random.default_rng(5)
    p = rng.standard_normal(A.FILTER_PARAMS).astype(np.float32)
    m = (0.01 * rng.standard_normal(A.FILTER_PARAMS)).astype(np.float32)
    v = (0.01 * rng.random(A.FILTER_PARAMS)).astype(np.float32)
    g = rng.standard_normal(A.FILTER_PARAMS).astype(np.float32)
    lr, b1, b2, eps = (float(np.float32(x)) for x in (1e-3, 0.9, 0.999, 1e-8))
    tp, tm, tv = _dev(p, cuda), _dev(m, cuda), _dev(v, cuda)
    A.filter_adam(tp, tm, tv, _dev(g, cuda), 3, lr, b1, b2, eps)
    torch.cuda.synchronize()
    rp, rm, rv = F.adam(p, g, m, v, 3, lr, b1, b2, eps)
    p64, m64, v64, g64 = (x.astype(np.float64) for x in (p, m, v, g))
    em = 4 * U * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64))
    ev = 5 * U * (b2 * v64 + (1 - b2) * g64 * g64)
    assert np.all(np.abs(tm.cpu().numpy() - rm) <= em)
    assert np.all(np.abs(tv.cpu().numpy() - rv) <= ev)
    upd = np.abs(rp - p64)
    ep = U * np.abs(p64) + upd * (10 * U + em / np.abs(rm) + ev / rv) + U * upd
    assert np.all(np.abs(tp.cpu().numpy() - rp) <= ep)


def _check_pixels(out, ref, bound):
    diff = out.astype(np.int64) - ref["out"].astype(np.int64)
    frac = ref["real"] - np.floor(ref["real"])
    near = np.abs(frac - 0.5) <= 64 * bound + 2e-5
    assert np.all(np.abs(diff) <= 1)
    bad = (diff != 0) & ~near
    assert not np.any(bad), f"{int(bad.sum())} pixels differ away from a half"
    return int((diff != 0).sum())


@pytest.mark.parametrize("h,w", [(64, 64), (37, 45), (8, 5), (40, 30), (33, 200), (1, 1), (1, 17), (19, 1)])
def test_apply_matches_oracle(cuda, h, w):
    import torch
    orig = ar1_image(h, w, 0.9, seed=h * 1000 + w)
    recon = np.clip(orig.astype(np.int64) + np.random.default_rng(w).integers(-9, 10, orig.shape), 0, 255)
    recon = recon.astype(np.uint8)
    p = filter_params(11, last_scale=1.0, bias_scale=0.1)
    packed = A.filter_pack(_dev(p, cuda))
    frames = _dev(recon.reshape(1, -1), cuda)
    out, sse = A.filter_apply(packed, frames, [(0, h, w, w)], orig=_dev(orig.reshape(1, -1), cuda))
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(h, w)
    ref = F.apply(p, recon[None])
    ref = {k: v[0] for k, v in ref.items()}
    nd = _check_pixels(got, ref, _y_bound(p, recon[None])[0][0])
    print(f"{h}x{w}: {nd} pixels at a half differ")
    assert int(sse[0, 0]) == int(np.sum((got.astype(np.int64) - orig) ** 2))


def test_apply_pitched_frames_and_planes(cuda):
    """Several frames, three planes with pitch > W inside each frame."""
    import torch
    rng = np.random.default_rng(4)
    planes = [(0, 48, 70, 80), (48 * 80, 24, 35, 40), (48 * 80 + 24 * 40, 24, 35, 40)]
    fb = 48 * 80 + 2 * 24 * 40
    frames = rng.integers(0, 256, size=(3, fb), dtype=np.uint8)
    orig = rng.integers(0, 256, size=(3, fb), dtype=np.uint8)
    p = filter_params(13, last_scale=1.0, bias_scale=0.05)
    packed = A.filter_pack(_dev(p, cuda))
    out, sse = A.filter_apply(packed, _dev(frames, cuda), planes, orig=_dev(orig, cuda))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    s = sse.cpu().numpy()
    for f in range(3):
        for k, (off, h, w, pitch) in enumerate(planes):
            view = lambda buf: buf[f, off:off + h * pitch].reshape(h, pitch)[:, :w]
            ref = F.apply(p, view(frames)[None])
            _check_pixels(view(got), {kk: v[0] for kk, v in ref.items()}, _y_bound(p, view(frames)[None])[0][0])
            assert int(s[f, k]) == int(np.sum((view(got).astype(np.int64) - view(orig)) ** 2))
    # bytes between rows (pitch padding) are never written
    for off, h, w, pitch in planes:
        pad = got[:, off:off + h * pitch].reshape(3, h, pitch)[:, :, w:]
        assert not pad.any()


def test_zero_last_layer_is_identity(cuda):
    import torch
    spec = video_spec(n_frames=2, width=144, height=80, seed=3)
    bases = video_base_planes(spec)
    frames = np.stack([video_frame(spec, bases, f) for f in range(2)])
    planes = [(o, h, w, w) for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets)]
    pd = F.unflatten(filter_params(5, bias_scale=0.1))
    pd["W3"][:] = 0.0
    pd["b3"][:] = 0.0
    packed = A.filter_pack(_dev(F.flatten(pd).astype(np.float32), cuda))
    d = _dev(frames, cuda)
    out, sse = A.filter_apply(packed, d, planes, orig=d)
    torch.cuda.synchronize()
    assert torch.equal(out, d)
    assert not sse.any()


def test_select_keep_rule(cuda):
    import torch
    rng = np.random.default_rng(9)
    planes = [(0, 16, 24, 24), (384, 8, 16, 16)]
    fb = 384 + 128
    plain = rng.integers(0, 256, (4, fb), dtype=np.uint8)
    filt = rng.integers(0, 256, (4, fb), dtype=np.uint8)
    sf = np.array([[10, 5], [30, 0], [0, 0], [7, 9]], dtype=np.int64)
    sr = np.array([[9, 6], [29, 0], [0, 0], [1, 1]], dtype=np.int64)
    out = _dev(filt, cuda)
    keep = A.filter_select(_dev(sf, cuda), _dev(sr, cuda), _dev(plain, cuda), planes, out)
    torch.cuda.synchronize()
    ref = F.keep_filtered(sf, sr)
    assert keep.cpu().numpy().astype(bool).tolist() == ref.tolist()
    got = out.cpu().numpy()
    for f in range(4):
        assert np.array_equal(got[f], filt[f] if ref[f] else plain[f])


def test_filter_argument_errors(cuda):
    import torch
    p = torch.zeros(A.FILTER_PARAMS, dtype=torch.float32, device=cuda)
    x = torch.zeros((2, 48, 48), dtype=torch.uint8, device=cuda)
    with pytest.raises(A.AdctError):
        A.filter_grad(p, x, x)                           # W = 48 unsupported
    with pytest.raises(A.AdctError):
        A.filter_adam(p, p.clone(), p.clone(), p.clone(), 0, 1e-3)   # step 0
    packed = A.filter_pack(p)
    f = torch.zeros((1, 64), dtype=torch.uint8, device=cuda)
    with pytest.raises(A.AdctError):
        A.filter_apply(packed, f, [(0, 8, 8, 7)])        # pitch < W
    with pytest.raises(A.AdctError):
        A.filter_apply(packed, f, [(0, 8, 8, 8)], out=f)  # in place


def _held_out_psnr(packed, vrec, vorg, vtab, cuda):
    n = len(vrec)
    _, s = A.filter_apply(packed, _dev(vrec.reshape(n, -1), cuda), [(0, 64, 64, 64)],
                          orig=_dev(vorg.reshape(n, -1), cuda))
    sf = s.cpu().numpy()[:, 0].astype(np.float64)
    sp = ((vrec.astype(np.int64) - vorg) ** 2).sum(axis=(1, 2)).astype(np.float64)
    out = {}
    for r in (6, 10, 16):
        m = vtab[:, 3] == r
        out[r] = 10 * np.log10(sp[m].sum() / sf[m].sum())      # filtered minus plain, dB
    return out


def test_training_gains_over_plain_decoding(cuda):
    """Train on the GPU (T1-decoded patches at r in {6, 10, 16}) and measure the
    PSNR gain over the plain reconstruction on held-out patches from other
    images; the fresh network is near the identity and loses a little."""
    from synth import patch_specs
    imgs, tab = patch_specs(8192, seed=11)
    vimgs, vtab = patch_specs(1024, seed=12)
    rec, org = A.patch_pairs(imgs, tab)
    vrec, vorg = A.patch_pairs(vimgs, vtab)
    p0 = filter_params(0)
    before = _held_out_psnr(A.filter_pack(_dev(p0, cuda)), vrec, vorg, vtab, cuda)
    params, losses = A.train_filter(p0, rec, org, 1500, batch=64, lr=1e-3, lr_final=1e-4)
    after = _held_out_psnr(A.filter_pack(params), vrec, vorg, vtab, cuda)
    print("gain dB before", {r: round(v, 3) for r, v in before.items()},
          "after", {r: round(v, 3) for r, v in after.items()},
          f"loss {losses[:20].mean():.5f} -> {losses[-100:].mean():.5f}")
    assert losses[-100:].mean() < 0.95 * losses[:20].mean()
    assert all(v > 0.05 for v in after.values())
    assert after[10] > 0.2 and after[6] > 0.2


def test_stream_keep_rule_end_to_end(cuda):
    """Decoded stream (T1, r = 10, step 16), filter, keep rule against the
    exact DCT: each output frame is the filtered one exactly when its squared
    error is not above the DCT's, else the plain reconstruction."""
    import torch
    spec = video_spec(n_frames=4, width=288, height=160, seed=5)
    bases = video_base_planes(spec)
    frames = _dev(np.stack([video_frame(spec, bases, f) for f in range(4)]), cuda)
    planes = [(o, h, w, w) for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets)]
    recon = torch.empty_like(frames)
    sse_plain = A.evaluate_stream(frames, planes, "T1", 10, 16, recon=recon)
    sse_dct = A.evaluate_stream(frames, planes, "DCT", 10, 16)
    # two weight sets: identity (never better than the DCT here) and a random one
    pd = F.unflatten(filter_params(2, bias_scale=0.02))
    pd["W3"][:] = 0.0
    pd["b3"][:] = 0.0
    for p in (F.flatten(pd).astype(np.float32), filter_params(4)):
        packed = A.filter_pack(_dev(p, cuda))
        out, sse_f = A.filter_apply(packed, recon, planes, orig=frames)
        filt = out.clone()
        keep = A.filter_select(sse_f, sse_dct, recon, planes, out)
        torch.cuda.synchronize()
        want = sse_f.cpu().numpy().sum(axis=1) <= sse_dct.cpu().numpy().sum(axis=1)
        assert keep.cpu().numpy().astype(bool).tolist() == want.tolist()
        for f in range(4):
            assert torch.equal(out[f], filt[f] if want[f] else recon[f])



def test_grad_full_training_batch(cuda):
    """The training launch shape (64 patches of 64 x 64, as the benchmark's
    steps): loss and every gradient group against the oracle on the full batch."""
    import torch
    from synth import patch_specs
    imgs, tab = patch_specs(64, seed=21)
    rec, org = A.patch_pairs(imgs, tab)          # decoded by the library, compared as inputs only
    orig = org
    recon = np.stack([Co.evaluate(o, M.T1, int(r))["rec"] for o, r in zip(orig, tab[:, 3])]).astype(np.uint8)
    assert np.array_equal(recon, rec)            # the library's decode of the patches is the oracle's
    p = filter_params(6, last_scale=1.0, bias_scale=0.05)
    grad, loss, _ = A.filter_grad(_dev(p, cuda), _dev(recon, cuda), _dev(orig, cuda))
    torch.cuda.synchronize()
    rl, rg, _ = F.loss_and_grad(p, recon, orig)
    assert abs(float(loss.item()) - rl) <= 1e-4 * rl
    g, r = _groups(grad.cpu().numpy().astype(np.float64)), _groups(rg)
    for name, _ in GROUPS:
        assert np.abs(g[name] - r[name]).max() <= 1e-3 * np.abs(r[name]).max(), name


def test_apply_full_4k_frame_sampled(cuda):
    """One 3840 x 2160 4:2:0 frame in the benchmark's launch configuration;
    about 300 output pixels (borders, corners, tile seams and random ones)
    checked against the oracle on their exact receptive field: the output at
    (y, x) depends on the input within 3 pixels, and clipping that window at
    the image edge reproduces the per-layer zero padding there."""
    import torch
    spec = video_spec(n_frames=2, seed=9)
    bases = video_base_planes(spec)
    frames = np.stack([video_frame(spec, bases, f) for f in range(2)])
    planes = [(o, h, w, w) for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets)]
    p = filter_params(8, last_scale=1.0, bias_scale=0.05)
    packed = A.filter_pack(_dev(p, cuda))
    out, sse = A.filter_apply(packed, _dev(frames[:1], cuda), planes, orig=_dev(frames[1:], cuda))
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    rng = np.random.default_rng(3)
    for k, ((h, w), o) in enumerate(zip(spec.plane_shapes, spec.plane_offsets)):
        img = frames[0, o:o + h * w].reshape(h, w)
        res = got[o:o + h * w].reshape(h, w)
        ys = [0, 1, 2, 31, 32, 33, h // 2, h - 3, h - 2, h - 1]
        xs = [0, 1, 13, 14, 15, 27, 28, w // 2, w - 2, w - 1]
        pts = [(y, x) for y in ys for x in xs] + [tuple(v) for v in
                                                  zip(rng.integers(0, h, 30), rng.integers(0, w, 30))]
        for y, x in pts:
            y0, y1, x0, x1 = max(0, y - 3), min(h, y + 4), max(0, x - 3), min(w, x + 4)
            win = img[y0:y1, x0:x1][None]
            ref = F.apply(p, win)
            bound = _y_bound(p, win)[0][0]
            cy, cx = y - y0, x - x0
            one = {"out": ref["out"][0][cy:cy + 1, cx:cx + 1], "real": ref["real"][0][cy:cy + 1, cx:cx + 1]}
            _check_pixels(res[y:y + 1, x:x + 1], one, bound[cy:cy + 1, cx:cx + 1])
        # the squared error the kernel reports is that of its own output
        org = frames[1, o:o + h * w].reshape(h, w)
        assert int(sse[0, k]) == int(np.sum((res.astype(np.int64) - org) ** 2))


def test_checkpoint_resume_is_exact(cuda, tmp_path):
    """Train 10 steps, checkpoint, resume in a new trainer for 10 more: the
    weights and moments equal those of 20 uninterrupted steps bit for bit."""
    import torch
    from synth import patch_specs
    imgs, tab = patch_specs(256, seed=31)
    rec, org = A.patch_pairs(imgs, tab)
    rd, od = _dev(rec, cuda), _dev(org, cuda)
    p0 = filter_params(3)

    def run(tr, s0, s1):
        for s in range(s0, s1):
            b = (s * 32) % 224
            tr.step(rd[b:b + 32], od[b:b + 32])

    full = A.FilterTrainer(p0, 32, 64, 64, lr=2e-3)
    run(full, 0, 20)
    half = A.FilterTrainer(p0, 32, 64, 64, lr=2e-3)
    run(half, 0, 10)
    path = str(tmp_path / "filter.npz")
    half.save(path)
    resumed = A.FilterTrainer.load(path, device=cuda)
    run(resumed, 10, 20)
    torch.cuda.synchronize()
    assert resumed.step_count == 20
    for a, b in ((full.params, resumed.params), (full.m, resumed.m), (full.v, resumed.v)):
        assert torch.equal(a, b)
    assert not torch.equal(full.params, torch.from_numpy(p0).to(cuda))


def test_checkpoint_blob_roundtrip(cuda):
    """adct_filter_save / adct_filter_load: parameters, moments and step come
    back bit for bit; a corrupted blob is refused before anything is copied."""
    import torch
    p = torch.from_numpy(filter_params(5)).to(cuda)
    m = torch.randn(A.FILTER_PARAMS, device=cuda)
    v = torch.rand(A.FILTER_PARAMS, device=cuda)
    blob = A.filter_save(p, m, v, step=123)
    p2, m2, v2 = torch.zeros_like(p), torch.zeros_like(m), torch.zeros_like(v)
    assert A.filter_load(blob, p2, m2, v2) == 123
    assert torch.equal(p, p2) and torch.equal(m, m2) and torch.equal(v, v2)
    only = A.filter_save(p)
    p3 = torch.zeros_like(p)
    assert A.filter_load(only, p3) == 0 and torch.equal(p, p3)
    bad = bytearray(blob)
    bad[-1] ^= 0x40
    p4 = torch.full_like(p, 7.0)
    with pytest.raises(A.AdctError):
        A.filter_load(bytes(bad), p4)
    assert bool((p4 == 7.0).all())
