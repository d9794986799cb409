"""Benchmark: fused 8x8 approximate-DCT encode + decode + PSNR on one MI355X.

Workload: a video-like stream of 300 frames 3840x2160 YUV 4:2:0 (8-bit, seeded
AR(1) textures translated 0-4 px per frame), all frames resident in HBM.  One
step = one launch over the whole stream: T1 forward by the fast algorithm,
step-16 quantiser on the scaled coefficients of the first r = 10 zig-zag
positions, int16 coefficient write-out, inverse, rounded/clipped uint8
reconstruction write-out, per-frame per-plane squared error.

Prints ONE JSON line on stdout (logs go to stderr).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_stream(spec, dev):
    import numpy as np
    import torch

    from synth import video_base_planes

    bases = [torch.from_numpy(b).to(dev) for b in video_base_planes(spec)]
    offs = spec.offsets()
    frames = torch.empty((spec.n_frames, spec.frame_bytes), dtype=torch.uint8, device=dev)
    for f in range(spec.n_frames):
        dy, dx = int(offs[f][0]), int(offs[f][1])
        for p, ((h, w), o) in enumerate(zip(spec.plane_shapes, spec.plane_offsets)):
            oy, ox = (dy, dx) if p == 0 else (dy // 2, dx // 2)
            frames[f, o:o + h * w].view(h, w).copy_(bases[p][oy:oy + h, ox:ox + w])
    torch.cuda.synchronize()
    return frames


def cpu_baseline(spec, n_frames: int, r: int, step: int, gpu_lists=None):
    """The CPU oracle, untuned, on the first n_frames frames (all planes): one
    thread, then one process per available core (up to 16), with the host's
    core count and CPU model; plus bounded samples of the other workloads."""
    from threadpoolctl import threadpool_limits

    from oracle import codec as Co
    from oracle import matrices as M
    from synth import video_base_planes, video_frame

    bases = video_base_planes(spec)
    samples = 0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for f in range(n_frames):
            buf = video_frame(spec, bases, f)
            for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets):
                Co.evaluate(buf[o:o + h * w].reshape(h, w), M.T1, r, step)
                samples += h * w
        dt = time.perf_counter() - t0
    host = host_info()
    workers = max(1, min(16, host["affinity_cpus"] or 1))
    v_all, dt_all, n_all = cpu_all_cores(spec, workers, 4, r, step)
    out = {"value": samples / dt / 1e6, "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
           "sample": f"first {n_frames} of the {spec.n_frames} frames, all 3 planes, "
                     f"T1 r={r} step {step}, encode+decode+SSE, one thread, {dt:.1f} s",
           "blas_threads": 1, **host,
           "all_cores": {"value": round(v_all, 2), "unit": "Mpixel/s", "cores": workers,
                         "sample": f"{n_all} frames over {workers} single-threaded processes, {dt_all:.1f} s"}}
    if gpu_lists is not None:
        out["legs"] = cpu_legs(gpu_lists)
    return out


def host_info():
    """Host cores and CPU model the CPU oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": aff}


_POOL_STATE = {}


def _pool_init(n_frames, r, step):
    from threadpoolctl import threadpool_limits

    from synth import video_base_planes, video_spec
    spec = video_spec(n_frames=n_frames)
    _POOL_STATE.update(spec=spec, bases=video_base_planes(spec), r=r, step=step,
                       limits=threadpool_limits(1))


def _pool_frame(f):
    from oracle import codec as Co
    from oracle import matrices as M
    from synth import video_frame
    st = _POOL_STATE
    buf = video_frame(st["spec"], st["bases"], f)
    n = 0
    for (h, w), o in zip(st["spec"].plane_shapes, st["spec"].plane_offsets):
        Co.evaluate(buf[o:o + h * w].reshape(h, w), M.T1, st["r"], st["step"])
        n += h * w
    return n


def cpu_all_cores(spec, workers: int, frames_per_worker: int, r: int, step: int):
    """The same oracle, one process per core (each single-threaded), over
    frames_per_worker frames per process; returns (Mpixel/s, seconds, frames)."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    n = workers * frames_per_worker
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(workers, mp_context=ctx, initializer=_pool_init,
                             initargs=(spec.n_frames, r, step)) as ex:
        list(ex.map(_pool_frame, range(workers)))          # warm: bases built, imports done
        t0 = time.perf_counter()
        samples = sum(ex.map(_pool_frame, range(n)))
        dt = time.perf_counter() - t0
    return samples / dt / 1e6, dt, n


def cpu_legs(gpu_lists):
    """The CPU oracle on bounded samples of the other workloads (one thread),
    each scaled to its unit and labelled with what was timed."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import batch as Ob
    from oracle import codec as Co
    from oracle import ctuples
    from oracle import matrices as M
    from oracle import postfilter as Of
    from oracle import search as Os
    from synth import ar1_image, batch_images, batch_specs, filter_params

    legs = {}
    with threadpool_limits(1):
        img = ar1_image(512, 512, 0.95, seed=0)
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            Co.evaluate(img, M.T1, 10)
        t_t1 = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            Co.evaluate_dct(img, 10)
        t_dct = (time.perf_counter() - t0) / reps
        legs["single_512x512_r10"] = {"T1_us_per_call": round(t_t1 * 1e6, 1),
                                      "DCT_us_per_call": round(t_dct * 1e6, 1),
                                      "T1_Mpixel_per_s": round(img.size / t_t1 / 1e6, 2),
                                      "sample": f"encode+decode+SSE of the 512x512 image, mean of {reps} calls"}

        specs = sorted(batch_specs(), key=lambda b: b.h * b.w)[:1]
        imgs = batch_images(specs)
        names = ["DCT", "T1", "LO", "T6", "RDCT", "T4"]
        t0 = time.perf_counter()
        Ob.sse_table(imgs, names, 1, 63)
        dt = time.perf_counter() - t0
        px = sum(im.size for im in imgs)
        all_px = sum(b.h * b.w for b in batch_specs())
        legs["batch_45img_6tf_r1_63"] = {
            "evaluations_per_s": round(len(imgs) * len(names) * 63 / dt, 1),
            "Gpixel_evals_per_s": round(px * len(names) * 63 / dt / 1e9, 4),
            "extrapolated_s_for_45_images": round(dt * all_px / px, 1),
            "sample": f"the smallest of the 45 images ({px} pixels) x 6 transforms x r=1..63 in "
                      f"{dt:.1f} s, extrapolated by pixel count"}

        p4 = [0, 1, -1, 2, -2, 3, -3, 4, -4]
        chunk = 1 << 21
        t0 = time.perf_counter()
        Os.topk_scan(p4[:5], 64, chunk=chunk)                    # warm the numpy paths
        dt_small = time.perf_counter() - t0
        # one chunk of the 9^8 space scanned as the oracle does, extrapolated
        digs = np.array(Os.canonical_digits(p4), dtype=np.int64)
        c = M.dct_matrix()
        t0 = time.perf_counter()
        idx = np.arange(1, 1 + chunk, dtype=np.int64)
        cols = [(idx // 9 ** (7 - q)) % 9 for q in range(8)]
        d = digs[np.stack(cols, axis=1)]
        d = d[Os._gcd_rows(d) == 1].astype(np.float64)
        cs = (d @ c.T) / np.sqrt(np.sum(d * d, axis=1))[:, None]
        for row in range(8):
            np.argpartition(-cs[:, row], 255)[:256]
        dt = time.perf_counter() - t0
        total = 9 ** 8 - 1
        t0 = time.perf_counter()
        _, n256 = ctuples.orthogonal_tuples([gpu_lists[r] for r in range(8)])
        dt_tup = time.perf_counter() - t0
        legs["search_topk_9pow8"] = {
            "Gcand_rows_per_s": round(8 * chunk / dt / 1e9, 4),
            "extrapolated_scan_s": round(dt * total / chunk, 1),
            "tuples_k256_s": round(dt_tup, 3), "tuples_k256": int(n256),
            "sample": f"{chunk} of the {total} candidates (digits, gcd, 8 cosines, per-row top 256) in "
                      f"{dt:.2f} s, extrapolated; the C tuple DFS on the 8 top-256 lists; "
                      f"5^8 warm-up scan {dt_small:.1f} s"}

        pr = filter_params(0)
        rng = np.random.Generator(np.random.PCG64(3))
        x = rng.integers(0, 256, size=(2, 64, 64), dtype=np.uint8)
        o = rng.integers(0, 256, size=(2, 64, 64), dtype=np.uint8)
        t0 = time.perf_counter()
        Of.loss_and_grad(pr, x, o)
        dt = time.perf_counter() - t0
        legs["postfilter_train"] = {
            "patches_per_s": round(2 / dt, 2),
            "extrapolated_epoch_s_200k_patches": round(dt / 2 * 200000, 0),
            "sample": f"forward + backward of 2 patches of 64x64 in float64 ({dt:.2f} s), "
                      f"extrapolated to one epoch of 200,000 patches"}
    return legs


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs, or None when the kernel sources changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "codec_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def other_rows():
    """Timings of the other hot-path rows on the same GPU (each synchronised)."""
    import paper_1808_02950_amd as A

    res = {}
    p2 = [0, 1, -1, 2, -2]
    p4 = [0, 1, -1, 2, -2, 3, -3, 4, -4]
    A.derive_transform(p2, A.SEARCH_CLOSURE)                     # warm
    t0 = time.perf_counter()
    mats, _, leaves, dead = A.derive_transform(p2, A.SEARCH_CLOSURE)
    res["search_closure_P2_720_orders"] = {"ms": round((time.perf_counter() - t0) * 1e3, 2),
                                           "matrices": int(len(mats)), "leaves": leaves,
                                           "dead_paths": dead}
    A.search_topk(p4, 64)
    t0 = time.perf_counter()
    vec, idx, cos = A.search_topk(p4, 64)
    t_scan = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, n64 = A.orthogonal_tuples([vec[r] for r in range(8)])
    t_tup = time.perf_counter() - t0
    res["search_topk_9pow8_k64"] = {"ms": round(t_scan * 1e3, 2), "candidates": 9 ** 8 - 1,
                                    "rows": 8, "Gcand_rows_per_s": round(8 * (9 ** 8 - 1) / t_scan / 1e9, 2),
                                    "tuples_ms": round(t_tup * 1e3, 2), "orthogonal_tuples": n64}
    res["search_full_orders_and_extended_P"] = search_wider_row()
    res["coding_gain_vs_rho"] = coding_gain_row()
    res.update(batch_row())
    return res


def search_wider_row():
    """The searches Sec. 3.5 and 4.1 describe beyond the 720-order runs: all 8!
    orders with no fixed rows on D1 and D2, and the five extended entry sets
    (720 orders, rows 1 and 5 fixed).  Matrices are also counted up to positive
    row scaling (each row divided by the gcd of its entries), which S removes."""
    import math as _m

    import numpy as np

    import paper_1808_02950_amd as A

    def primitive_count(mats):
        keys = set()
        for t in mats:
            rows = []
            for r in np.asarray(t, dtype=np.int64):
                g = 0
                for v in r:
                    g = _m.gcd(g, int(v))
                rows.append(tuple(int(v) // max(g, 1) for v in r))
            keys.add(tuple(rows))
        return len(keys)

    out = {}
    runs = [("D1_all_8!_orders", [0, 1, -1], False), ("D2_all_8!_orders", [0, 1, -1, 2, -2], False)]
    runs += [("P_" + "_".join(str(v) for v in p if v > 0) + "_720_orders", p, True)
             for p in ([0, 1, -1, 4, -4], [0, 1, -1, 8, -8], [0, 1, -1, 2, -2, 4, -4],
                       [0, 1, -1, 2, -2, 8, -8], [0, 2, -2, 4, -4, 8, -8])]
    for name, p, fix in runs:
        t0 = time.perf_counter()
        mats, _, leaves, dead = A.derive_transform(p, A.SEARCH_CLOSURE, fix_rows_1_5=fix)
        out[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 1), "space": len(p) ** 8 - 1,
                     "matrices": int(len(mats)), "up_to_row_scaling": primitive_count(mats),
                     "leaves": leaves, "dead_paths": dead}
    return out


def batch_row():
    """The 45-image rate-distortion sweep as one autotuned plan launch."""
    import numpy as np
    import torch

    import paper_1808_02950_amd as A
    from synth import batch_images, batch_specs

    imgs = batch_images(batch_specs())
    parts, planes, off = [], [], 0
    for im in imgs:
        h, w = im.shape
        parts.append(im.ravel())
        planes.append((off, h, w, w))
        off += h * w
    base = torch.from_numpy(np.concatenate(parts)).cuda()
    names = ["DCT", "T1", "LO", "T6", "RDCT", "T4"]
    plan = A.BatchPlan(base, planes, names, 1, 63, autotune=True)
    plan.launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 5
    for _ in range(reps):
        plan.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    sse = plan.sse.cpu().numpy()
    npix = np.array([im.size for im in imgs], dtype=np.float64)
    psnr = (10 * np.log10(255.0 ** 2 * npix[:, None, None] / np.maximum(sse, 1))).mean(axis=0)
    info = plan.info()
    plan.close()
    evals = len(imgs) * len(names) * 63
    # mean SSIM over the 45 images against r (Sec. 6.1.1 compares the transforms'
    # SSIM curves): decode each image with the library, score it with the SSIM kernel
    rs = [4, 8, 12, 16, 24, 32, 48, 60]
    tfs = ["DCT", "T1", "LO", "T6"]
    curve = {t: [] for t in tfs}
    t0 = time.perf_counter()
    for r in rs:
        for t in tfs:
            vals = []
            for (o, h, w, _) in planes:
                img = base[o:o + h * w].view(h, w)
                rec = torch.empty_like(img)
                A.evaluate_coding(img, t, r, recon=rec)
                vals.append(A.ssim(img, rec, None))
            curve[t].append(round(float(torch.cat(vals).mean().item()), 6))
    ssim_s = time.perf_counter() - t0
    # non-orthogonal competitors with the inverse decoder on the same images
    # (per image; T1 through the same decoder for reference)
    comp = {"SDCT": sdct_matrix(), "BAS2008B": BAS2008B, "T1": A.matrix_get("T1")}
    nonortho = {}
    for name, t in comp.items():
        nonortho[name] = []
        for r in (4, 10, 20, 40):
            vals = []
            for (o, h, w, _) in planes:
                s_ = A.evaluate_inverse(base[o:o + h * w].view(1, -1), [(0, h, w, w)], t, r)
                vals.append(s_)
            s_all = torch.cat(vals).cpu().numpy().ravel()
            nonortho[name].append(round(float(np.mean(10 * np.log10(255.0 ** 2 * npix / np.maximum(s_all, 1)))), 4))
    return {"nonortho_competitors_45img_psnr": {"r": [4, 10, 20, 40], **nonortho},
            "batch_45img_6tf_r1_63": {
        "ms": round(ms, 3), "evaluations": evals, "evaluations_per_s": round(evals / (ms / 1e3)),
        "Gpixel_evals_per_s": round(off * len(names) * 63 / (ms / 1e3) / 1e9, 1),
        "pixels": off, "schedule": info,
        "mean_psnr_r10": {n: round(float(psnr[t, 9]), 4) for t, n in enumerate(names)}},
        "ssim_vs_r_45img": {"r": rs, **curve,
                            "T1_above_DCT_at_r": [r for r, a, b in zip(rs, curve["T1"], curve["DCT"]) if a > b],
                            "seconds": round(ssim_s, 2)}}


# BAS-2008b as printed in the paper's table of low-complexity matrices (Sec. 2);
# the signed DCT is sgn(C) entrywise (Sec. 2).  Inputs of the competitor rows.
BAS2008B = [[1, 1, 1, 1, 1, 1, 1, 1], [1, 1, 1, 0, 0, -1, -1, -1], [1, 1, -1, -1, -1, -1, 1, 1],
            [1, 0, -1, 0, 0, 1, 0, -1], [1, -1, -1, 1, 1, -1, -1, 1], [1, -1, 1, 0, 0, -1, 1, -1],
            [1, -1, 1, -1, -1, 1, -1, 1], [1, -1, 1, -1, 1, -1, 1, -1]]


def dct_rows():
    """Orthonormal 8-point DCT-II from its closed form."""
    import numpy as np
    k = np.arange(8)[:, None]
    n = np.arange(8)[None, :]
    c = np.cos((2 * n + 1) * k * np.pi / 16) / 2.0
    c[0] = 1 / np.sqrt(8.0)
    return c


def sdct_matrix():
    import numpy as np
    return np.sign(dct_rows()).astype(np.int8)


def coding_gain_row():
    """Coding-gain loss against the exact DCT over 0 < rho < 1 (Sec. 4.3's figure)
    for T1, LO, T6 and the two non-orthogonal competitors, one GPU launch."""
    import numpy as np

    import paper_1808_02950_amd as A

    def chat(t):
        t = np.asarray(t, dtype=np.float64)
        return t / np.sqrt((t * t).sum(axis=1))[:, None]

    names = ["T1", "LO", "T6"]
    mats = [dct_rows()] + [chat(A.matrix_get(n)) for n in names] + [chat(sdct_matrix()), chat(BAS2008B)]
    names += ["SDCT", "BAS2008B"]
    rhos = np.linspace(0.001, 0.999, 999)
    A.coding_gain_sweep(np.stack(mats), rhos)
    t0 = time.perf_counter()
    cg = A.coding_gain_sweep(np.stack(mats), rhos)
    ms = (time.perf_counter() - t0) * 1e3
    d = cg[1:] - cg[0]
    i95 = int(np.argmin(np.abs(rhos - 0.95)))
    return {"ms": round(ms, 3), "matrices": len(mats), "rho_points": len(rhos),
            "loss_dB_at_rho_0.95": {n: round(float(d[i, i95]), 4) for i, n in enumerate(names)},
            "T1_smallest_loss_every_rho": bool(np.all(np.abs(d[0]) < np.abs(d[1:]).min(axis=0))),
            "T1_over_LO_loss_at_0.95": round(float(d[0, i95] / d[1, i95]), 3)}


# The paper's own hardware figures (Sec. 5.2 results table): the 1-D 8-point
# cores on a Xilinx Virtex-6 XC6VLX240T-1FFG1156 (ML605 board), fixed point,
# checked by hardware co-simulation on 100,000 random input vectors.  Context
# only: a different device, a 1-D core, and no 2-D block coding throughput.
FPGA_CONTEXT = {
    "device": "Xilinx Virtex-6 XC6VLX240T-1FFG1156 (ML605)",
    "what": "1-D 8-point transform core, fixed point; paper Sec. 5.2 results table",
    "T1": {"CLB": 135, "FF": 408, "T_cpd_ns": 1.750, "F_max_MHz": 571, "D_p_mW_per_GHz": 2.74, "Q_p_W": 3.471},
    "T_LO": {"CLB": 114, "FF": 349, "T_cpd_ns": 1.900, "F_max_MHz": 526, "D_p_mW_per_GHz": 2.82,
             "Q_p_W": 3.468},
    "T6": {"CLB": 125, "FF": 389, "T_cpd_ns": 2.100, "F_max_MHz": 476, "D_p_mW_per_GHz": 2.57, "Q_p_W": 3.460},
    "note": "at one 8-point vector per clock the T1 core would do 571 M 1-D transforms/s, i.e. 35.7 M "
            "8x8 blocks/s (2.28 Gpixel/s) for a 2-D transform; a derived figure the paper does not "
            "state (it assumes full pipelining and excludes I/O)",
}


def single_image_row():
    """The single 512x512 image (seeded AR(1), rho 0.95): one call's latency for
    T1 at r = 10 (zonal) and the exact DCT, with PSNR; the image fits in the
    Infinity Cache, so this is a latency figure, not a roofline case."""
    import torch

    import paper_1808_02950_amd as A
    from synth import ar1_image

    img = torch.from_numpy(ar1_image(512, 512, 0.95, seed=0)).cuda()
    rec = torch.empty_like(img)
    coef = torch.empty((4096, 10), dtype=torch.int16, device=img.device)
    res = {}
    for t in ("T1", "DCT"):
        c = coef if t == "T1" else None
        ev = A.evaluate_coding(img, t, 10, coef_int=c, recon=rec)
        v = img.view(1, -1)
        rv = rec.view(1, -1)
        sse_t = torch.empty((1, 1), dtype=torch.int64, device=img.device)
        pl = [(0, 512, 512, 512)]
        A.evaluate_stream(v, pl, t, 10, coef=c, recon=rv, sse=sse_t)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n = 200
        e0.record()
        for _ in range(n):
            A.evaluate_stream(v, pl, t, 10, coef=c, recon=rv, sse=sse_t)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / n * 1e3
        t0 = time.perf_counter()
        for _ in range(50):
            A.evaluate_coding(img, t, 10, coef_int=c, recon=rec)
        us_sync = (time.perf_counter() - t0) / 50 * 1e6
        res[t] = {"us_per_launch": round(us, 2), "us_per_call_with_psnr_sync": round(us_sync, 1),
                  "Mpixel_per_s": round(img.numel() / (us / 1e6) / 1e6, 1), "psnr": round(ev.psnr, 4)}
    return res


FILTER_FLOP_PER_PX = 2 * (9 * 32 + 288 * 32 + 288)   # 19,584: forward MACs x 2, per output pixel
# SSIM per map position: two separable 11-tap passes over 5 maps (x, y, x^2, y^2, xy)
# as multiply-adds, plus the formula (about 20 operations)
SSIM_FLOP_PER_MAP_PX = 2 * 2 * 5 * 11 + 20


def filter_images(n_train: int, n_val: int):
    """Seeded AR(1) images the training / held-out patches are cut from (host)."""
    from synth import patch_specs
    t0 = time.perf_counter()
    tr = patch_specs(n_train, seed=11)
    va = patch_specs(n_val, seed=12)
    log(f"filter patches: {n_train} training + {n_val} held-out in {time.perf_counter() - t0:.1f} s")
    return tr, va


def filter_row(data, steps, batch, frames, recon, planes, sse_plain, sse_dct, npix, codec_ms):
    """Train the post-filter on the GPU, then run it on the decoded stream."""
    import numpy as np
    import torch

    import paper_1808_02950_amd as A
    from synth import filter_params

    (imgs, tab), (vimgs, vtab) = data
    t0 = time.perf_counter()
    rec, org = A.patch_pairs(imgs, tab)
    vrec, vorg = A.patch_pairs(vimgs, vtab)
    torch.cuda.synchronize()
    log(f"patch pairs decoded in {time.perf_counter() - t0:.1f} s; training {steps} steps")
    rd, od = A.shuffled_pairs(rec, org)            # resident in HBM before the timed region
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    params, losses = A.train_filter(filter_params(0), rd, od, steps, batch=batch, lr=1e-3, lr_final=1e-4)
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    train_tflops = steps * batch * 64 * 64 * 3 * FILTER_FLOP_PER_PX / (train_ms / 1e3) / 1e12
    packed = A.filter_pack(params)

    # held-out patches: PSNR with and without the filter, per retention level
    n = len(vrec)
    vr = torch.from_numpy(vrec.reshape(n, -1)).cuda()
    vo = torch.from_numpy(vorg.reshape(n, -1)).cuda()
    _, vs = A.filter_apply(packed, vr, [(0, 64, 64, 64)], orig=vo)
    sf = vs.cpu().numpy()[:, 0].astype(np.float64)
    sp = ((vrec.astype(np.int64) - vorg) ** 2).sum(axis=(1, 2)).astype(np.float64)
    held = {}
    for r in (6, 10, 16):
        m = vtab[:, 3] == r
        pf = 10 * math.log10(255.0 ** 2 * 4096 * m.sum() / sf[m].sum())
        pp = 10 * math.log10(255.0 ** 2 * 4096 * m.sum() / sp[m].sum())
        held[f"r{r}"] = {"plain": round(pp, 4), "filtered": round(pf, 4), "gain": round(pf - pp, 4)}

    # the decoded 4K stream: filter, keep rule against the exact DCT, fallback
    filt = torch.empty_like(recon)
    sse_f = torch.empty_like(sse_plain)

    def apply_once():
        A.filter_apply(packed, recon, planes, out=filt, orig=frames)

    A.filter_apply(packed, recon, planes, out=filt, orig=frames)
    torch.cuda.synchronize()
    reps = 3
    e0.record()
    for _ in range(reps):
        apply_once()
    e1.record()
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1) / reps
    _, sse_f = A.filter_apply(packed, recon, planes, out=filt, orig=frames)
    ssim_f = A.ssim(frames, filt, planes).cpu().numpy()
    e0.record()
    keep = A.filter_select(sse_f, sse_dct, recon, planes, filt)
    e1.record()
    torch.cuda.synchronize()
    select_ms = e0.elapsed_time(e1)
    samples = frames.numel()
    npix_map = [(h - 10) * (w - 10) for _, h, w, _ in planes]
    sf, sp, sd = (x.cpu().numpy().sum(axis=1).astype(np.float64) for x in (sse_f, sse_plain, sse_dct))
    tot = float(sum(npix))
    ps = lambda v: float(np.mean(10 * np.log10(255.0 ** 2 * tot / np.maximum(v, 1))))
    kept = keep.cpu().numpy().astype(bool)
    final = np.where(kept, sf, sp)
    return {
        "network": "3x3 conv 1->32->32->1, ReLU, residual; bf16 operands, fp32 accumulation",
        "train": {"patches": int(len(rec)), "steps": steps, "batch": batch, "ms": round(train_ms, 2),
                  "ms_per_step": round(train_ms / steps, 4), "tflops_fwd_bwd": round(train_tflops, 1),
                  "loss_first": round(float(losses[:20].mean()), 6),
                  "loss_last": round(float(losses[-100:].mean()), 6)},
        "held_out_psnr_db": held,
        "stream": {"apply_ms": round(apply_ms, 3), "select_ms": round(select_ms, 3),
                   "tflops": round(samples * FILTER_FLOP_PER_PX / (apply_ms / 1e3) / 1e12, 1),
                   "peak_bf16_tflops": 2500.0,
                   "psnr_plain": round(ps(sp), 4), "psnr_filtered": round(ps(sf), 4),
                   "psnr_dct": round(ps(sd), 4), "psnr_output": round(ps(final), 4),
                   "gain_vs_plain": round(ps(sf) - ps(sp), 4), "gain_vs_dct": round(ps(sf) - ps(sd), 4),
                   "ssim_filtered_frame_mean": round(float(np.mean(
                       (ssim_f * np.array(npix_map)).sum(axis=1) / sum(npix_map))), 6),
                   "frames_kept": int(kept.sum()), "frames": int(len(kept)),
                   "plain_Mpixel_per_s": round(samples / (codec_ms / 1e3) / 1e6, 1),
                   "learned_Mpixel_per_s": round(samples / ((codec_ms + apply_ms + select_ms) / 1e3) / 1e6,
                                                 1)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--cpu-frames", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--filter-patches", type=int, default=200000,
                    help="training patches of the post-filter (0 skips the filter row)")
    ap.add_argument("--filter-steps", type=int, default=1500)
    ap.add_argument("--filter-batch", type=int, default=256,
                    help="patches of 64x64 per training step")
    ap.add_argument("--codec-only", action="store_true",
                    help="time only the headline codec step and its bandwidth probe (profiling runs)")
    ap.add_argument("--dct-only", action="store_true",
                    help="time only the headline codec step, its probe and the exact-DCT comparator "
                         "(profiling runs)")
    ap.add_argument("--schedule", type=int, default=0,
                    help="resident workgroups per CU of the codec grid (0 = occupancy limit, "
                         "-1 = one tile per wave)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no multi-GPU "
              f"path (the codec would shard by frame, exchanging only per-frame squared errors).",
              file=sys.stderr)
        sys.exit(2)

    # training images are drawn before the GPU is touched
    fdata = (filter_images(args.filter_patches, 4096)
             if args.filter_patches and not (args.codec_only or args.dct_only) else None)

    import numpy as np
    import torch

    import paper_1808_02950_amd as A
    from synth import video_spec

    r, step = 10, 16
    dev = torch.device("cuda:0")
    A.lib()
    A.codec_set_schedule(args.schedule)
    spec = video_spec(n_frames=args.frames)
    log(f"building {spec.n_frames} frames of {spec.width}x{spec.height} 4:2:0 on the GPU")
    frames = build_stream(spec, dev)
    planes = [(o, h, w, w) for (h, w), o in zip(spec.plane_shapes, spec.plane_offsets)]
    bpf = A.stream_blocks_per_frame(planes)
    coef = torch.empty((spec.n_frames, bpf, r), dtype=torch.int16, device=dev)
    recon = torch.empty_like(frames)
    sse = torch.empty((spec.n_frames, 3), dtype=torch.int64, device=dev)

    def step_once():
        A.evaluate_stream(frames, planes, "T1", r, step, coef=coef, recon=recon, sse=sse)

    for _ in range(args.warmup):
        step_once()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step_once()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    kernel_ms = ev0.elapsed_time(ev1) / args.steps
    samples = spec.n_frames * spec.frame_bytes
    value = samples / (ms_per_step / 1e3) / 1e6

    # algorithmic HBM bytes per launch: 64 B read + 2r B coefficients + 64 B
    # reconstruction per 8x8 block
    blocks = spec.n_frames * bpf
    alg_bytes = blocks * (128 + 2 * r)
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    peak = 8000.0

    npix = [h * w for h, w in spec.plane_shapes]

    def psnrs(sse_t):
        s = sse_t.cpu().numpy()
        planes_ = [float(sum(A.psnr_from_sse(int(s[f, p]), npix[p]) for f in range(spec.n_frames))
                         / spec.n_frames) for p in range(3)]
        frame_ = float(sum(A.psnr_from_sse(int(s[f].sum()), sum(npix))
                           for f in range(spec.n_frames)) / spec.n_frames)
        return frame_, planes_

    psnr_frame, psnr_planes = psnrs(sse)

    # the HBM ceiling of this read / write mix: the same loads and stores without
    # the arithmetic (adct_stream_bandwidth_probe), timed the same way
    for _ in range(2):
        A.stream_bandwidth_probe(frames, planes, r, coef=coef, recon=recon)
    torch.cuda.synchronize()
    evp0 = torch.cuda.Event(enable_timing=True)
    evp1 = torch.cuda.Event(enable_timing=True)
    evp0.record()
    for _ in range(args.steps):
        A.stream_bandwidth_probe(frames, planes, r, coef=coef, recon=recon)
    evp1.record()
    torch.cuda.synchronize()
    probe_ms = evp0.elapsed_time(evp1) / args.steps
    ceiling = alg_bytes / (probe_ms / 1e3) / 1e9
    # restore the codec's outputs (the probe overwrote them)
    step_once()

    if args.codec_only:
        print(json.dumps({"metric": "codec-only profiling run", "kernel_ms": round(kernel_ms, 4),
                          "probe_ms": round(probe_ms, 4), "achieved_GBps": round(achieved, 1),
                          "ceiling_GBps": round(ceiling, 1), "ms_per_step": round(ms_per_step, 4)}),
              flush=True)
        return

    # exact-DCT comparator (float32-exact products on the matrix cores) on the
    # same stream, timed apart
    sse_dct = torch.empty_like(sse)
    recon_dct = torch.empty_like(frames)

    def dct_once():
        A.evaluate_stream(frames, planes, "DCT", r, step, recon=recon_dct, sse=sse_dct)

    dct_once()
    torch.cuda.synchronize()
    ev2 = torch.cuda.Event(enable_timing=True)
    ev3 = torch.cuda.Event(enable_timing=True)
    ev2.record()
    dct_steps = max(1, args.steps // 4)
    for _ in range(dct_steps):
        dct_once()
    ev3.record()
    torch.cuda.synchronize()
    dct_ms = ev2.elapsed_time(ev3) / dct_steps
    if args.dct_only:
        print(json.dumps({"metric": "dct-only profiling run", "kernel_ms": round(kernel_ms, 4),
                          "dct_ms": round(dct_ms, 4)}), flush=True)
        return
    dct_frame, dct_planes = psnrs(sse_dct)
    # algorithmic bytes: every pixel read once, every reconstructed pixel written once
    dct_bytes = 2 * samples
    # which arithmetic form the library runs for this (r, step): for r <= 16 and a
    # power-of-two step >= 8 the three-term bfloat16 split, else float32 products
    split_form = r <= 16 and step >= 8 and (step & (step - 1)) == 0

    # SSIM of the T1 and exact-DCT reconstructions (float64 GPU kernel), timed apart
    ssim_t1 = A.ssim(frames, recon, planes)
    ssim_dct = A.ssim(frames, recon_dct, planes)
    torch.cuda.synchronize()
    ev2.record()
    for _ in range(dct_steps):
        A.ssim(frames, recon, planes, out=ssim_t1)
    ev3.record()
    torch.cuda.synchronize()
    ssim_ms = ev2.elapsed_time(ev3) / dct_steps
    map_px = spec.n_frames * sum((h - 10) * (w - 10) for h, w in spec.plane_shapes)
    ssim_flop = map_px * SSIM_FLOP_PER_MAP_PX
    st1, sdct = ssim_t1.cpu().numpy(), ssim_dct.cpu().numpy()
    wts = np.array([(h - 10) * (w - 10) for h, w in spec.plane_shapes], dtype=np.float64)
    frame_ssim = lambda a: float(np.mean((a * wts).sum(axis=1) / wts.sum()))

    # 16- and 32-point JAM matrices (Sec. 6.2) on the same stream, with the
    # coefficient budget per pixel of r = 10 of 64 (40 of 256, 160 of 1024); the
    # 32-point coder needs a step that is a multiple of 32, so the 8-point T1
    # is also scored at step 32 beside it
    jam = {}
    recon_j = torch.empty_like(frames)
    sse_j = torch.empty_like(sse)
    for n_j, r_j, s_j in ((16, 40, 16), (32, 160, 32)):
        A.jam_evaluate_stream(frames, planes, n_j, r_j, s_j, recon=recon_j, sse=sse_j)
        torch.cuda.synchronize()
        ev2.record()
        for _ in range(dct_steps):
            A.jam_evaluate_stream(frames, planes, n_j, r_j, s_j, recon=recon_j, sse=sse_j)
        ev3.record()
        torch.cuda.synchronize()
        ms_j = ev2.elapsed_time(ev3) / dct_steps
        pj, _ = psnrs(sse_j)
        sj = A.ssim(frames, recon_j, planes).cpu().numpy()
        jam[f"T1_{n_j}x{n_j}_r{r_j}_q{s_j}"] = {
            "kernel_ms": round(ms_j, 4),
            "Mpixel_per_s": round(samples / (ms_j / 1e3) / 1e6, 1),
            "GB_per_s": round(2 * samples / (ms_j / 1e3) / 1e9, 1),
            "hbm_frac": round(2 * samples / (ms_j / 1e3) / 1e9 / peak, 4),
            "psnr_frame_mean": round(pj, 4), "ssim_frame_mean": round(frame_ssim(sj), 6)}
    A.evaluate_stream(frames, planes, "T1", r, 32, sse=sse_j)
    jam["T1_8x8_r10_q32_psnr_frame_mean"] = round(psnrs(sse_j)[0], 4)

    # the inverse decoder (non-orthogonal matrices) on the same stream, SDCT, r = 10
    A.evaluate_inverse(frames, planes, sdct_matrix(), r, recon=recon_j, sse=sse_j)
    torch.cuda.synchronize()
    ev2.record()
    for _ in range(dct_steps):
        A.evaluate_inverse(frames, planes, sdct_matrix(), r, recon=recon_j, sse=sse_j)
    ev3.record()
    torch.cuda.synchronize()
    inv_ms = ev2.elapsed_time(ev3) / dct_steps
    inverse_row = {"kernel_ms": round(inv_ms, 4), "GB_per_s": round(2 * samples / (inv_ms / 1e3) / 1e9, 1),
                   "hbm_frac": round(2 * samples / (inv_ms / 1e3) / 1e9 / peak, 4),
                   "psnr_frame_mean_SDCT_r10": round(psnrs(sse_j)[0], 4)}
    jam["T1_8x8_r10_q16_psnr_frame_mean"] = round(psnr_frame, 4)

    out = {
        "metric": "Mpixel/s 8x8 approx-DCT encode+decode at r=10 (% HBM peak); PSNR dB vs exact",
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/f64",
        "data": "synthetic",
        "config": {"workload": f"video stream {spec.n_frames} frames 3840x2160 YUV 4:2:0 uint8",
                   "transform": "T1", "r": r, "quant_step": step, "schedule": args.schedule,
                   "samples_per_frame": spec.frame_bytes, "blocks_per_launch": blocks},
        "frames_per_s": round(spec.n_frames / (ms_per_step / 1e3), 1),
        "luma_Mpixel_per_s": round(spec.n_frames * spec.width * spec.height / (ms_per_step / 1e3) / 1e6, 1),
        "psnr_db": {"T1_frame_mean": round(psnr_frame, 4),
                    "T1_Y": round(psnr_planes[0], 4), "T1_U": round(psnr_planes[1], 4),
                    "T1_V": round(psnr_planes[2], 4),
                    "DCT_frame_mean": round(dct_frame, 4),
                    "DCT_Y": round(dct_planes[0], 4), "DCT_U": round(dct_planes[1], 4),
                    "DCT_V": round(dct_planes[2], 4),
                    "T1_minus_DCT": round(psnr_frame - dct_frame, 4)},
        "exact_dct_comparator": {"kernel_ms": round(dct_ms, 4),
                                 "Mpixel_per_s": round(samples / (dct_ms / 1e3) / 1e6, 1),
                                 "GB_per_s": round(dct_bytes / (dct_ms / 1e3) / 1e9, 1),
                                 "hbm_frac": round(dct_bytes / (dct_ms / 1e3) / 1e9 / peak, 4),
                                 "form": "3-term bf16 split, float32-exact products" if split_form
                                         else "float32 matrix cores"},
        "ssim": {"T1_frame_mean": round(frame_ssim(st1), 6), "DCT_frame_mean": round(frame_ssim(sdct), 6),
                 "T1_minus_DCT": round(frame_ssim(st1) - frame_ssim(sdct), 6),
                 "T1_Y": round(float(st1[:, 0].mean()), 6), "DCT_Y": round(float(sdct[:, 0].mean()), 6),
                 "kernel_ms": round(ssim_ms, 3), "fp64_tflops": round(ssim_flop / (ssim_ms / 1e3) / 1e12, 1),
                 "peak_fp64_tflops": 78.6},
        "jam_16_32_point": jam,
        "inverse_decoder_SDCT": inverse_row,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": peak, "unit": "GB/s",
                     "frac": round(achieved / peak, 4), "traffic": measured_traffic(),
                     "kernel_ms": round(kernel_ms, 4), "alg_bytes_per_launch": alg_bytes,
                     "ceiling_GBps": round(ceiling, 1), "ceiling_kernel_ms": round(probe_ms, 4),
                     "frac_of_ceiling": round(achieved / ceiling, 4),
                     "ceiling_how": "adct_stream_bandwidth_probe: the codec's loads and stores for the "
                                    "same launch without the arithmetic"},
        "single_512x512": single_image_row(),
        "context_fpga_paper": FPGA_CONTEXT,
    }
    out["other_rows"] = other_rows()
    if fdata is not None:
        out["other_rows"]["postfilter"] = filter_row(fdata, args.filter_steps, args.filter_batch, frames, recon,
                                                     planes, sse,
                                                     sse_dct, npix, kernel_ms)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        vec256, _, _ = A.search_topk([0, 1, -1, 2, -2, 3, -3, 4, -4], 256)
        out["cpu_baseline"] = cpu_baseline(spec, min(args.cpu_frames, spec.n_frames), r, step,
                                           gpu_lists=[vec256[q] for q in range(8)])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
