"""Python binding of libadct.so, the MI355X library for blockwise 8x8 transform
coding with angle-similarity DCT approximations.

Argument marshalling only: every step of the coding path runs in the library's
HIP kernels.  torch is used for device memory and streams.  The library must
have been built (`paper_1808_02950_amd._build.build()`); importing the binding
on a machine without it raises immediately -- there is no fallback.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libadct.so")

# transform ids (adct_transform_id)
DCT, T1, T2, LO, T6, RDCT, T4, CUSTOM = range(8)
TRANSFORM_IDS = {"DCT": DCT, "T1": T1, "T2": T2, "LO": LO, "T6": T6,
                 "RDCT": RDCT, "T4": T4, "CUSTOM": CUSTOM}

STATUS = {0: "ADCT_OK", -1: "ADCT_EINVAL", -2: "ADCT_EDIM", -3: "ADCT_ERANGE",
          -4: "ADCT_EOVERFLOW", -5: "ADCT_ECAP", -6: "ADCT_EDEVICE", -7: "ADCT_ENOTSUP"}


class AdctError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class Matrix(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int8 * 64), ("n", ctypes.c_int32 * 8)]


class Plane(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64

_SIGNATURES = {
    "adct_last_error": (ctypes.c_char_p, []),
    "adct_version": (_I, []),
    "adct_matrix_get": (_I, [_I, ctypes.POINTER(Matrix)]),
    "adct_codec_set_schedule": (_I, [_I]),
    "adct_release_caches": (_I, [ctypes.POINTER(_I64)]),
    "adct_check_codec_args": (_I, [_I, ctypes.POINTER(Matrix), _I, _I, _I]),
    "adct_transform_bounds": (_I, [_I, ctypes.POINTER(Matrix), _I, _I,
                                   ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "adct_encode_blocks": (_I, [_P, _I, _I, _I, _I, ctypes.POINTER(Matrix), _I, _I, _P, _P, _P]),
    "adct_decode_blocks": (_I, [_P, _P, _I, _I, _P, _I, _I, ctypes.POINTER(Matrix), _I, _I, _P]),
    "adct_evaluate_coding": (_I, [_P, _I, _I, _I, _I, ctypes.POINTER(Matrix), _I, _I, _P, _P, _I,
                                  _P, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), _P]),
    "adct_evaluate_stream": (_I, [_P, _I64, _I, ctypes.POINTER(Plane), _I, _I,
                                  ctypes.POINTER(Matrix), _I, _I, _P, _P, _I64, _P, _P]),
    "adct_stream_bandwidth_probe": (_I, [_P, _I64, _I, ctypes.POINTER(Plane), _I, _I, _P, _P, _I64, _P]),
    "adct_ssim": (_I, [_P, _I64, _P, _I64, _I, ctypes.POINTER(Plane), _I, _P, _P]),
    "adct_jam_matrix": (_I, [_I, _I, _P, _P]),
    "adct_evaluate_inverse": (_I, [_P, _I64, _I, ctypes.POINTER(Plane), _I, _P, _I, _P, _I64, _P, _P]),
    "adct_coding_gain_sweep": (_I, [_P, _I, _P, _I, _P, _P]),
    "adct_coding_gain_sweep_noalloc": (_I, [_P, _I, _P, _I, _P, _P]),
    "adct_jam_evaluate_stream": (_I, [_P, _I64, _I, ctypes.POINTER(Plane), _I, _I, _I, _I, _I,
                                      _P, _P, _I64, _P, _P]),
    "adct_derive_transform": (_I, [_P, _I, _I, _P, _I, _I, ctypes.POINTER(Matrix), _I,
                                   ctypes.POINTER(_I), _P, ctypes.POINTER(_I64),
                                   ctypes.POINTER(_I64), _P]),
    "adct_search_topk": (_I, [_P, _I, _I, _I, _P, _P, _P, _P]),
    "adct_orthogonal_tuples": (_I, [_P, ctypes.POINTER(_I), _P, _I64, ctypes.POINTER(_I64), _P]),
    "adct_evaluate_batch": (_I, [_P, ctypes.POINTER(Plane), _I, _P, _I, _I, _I, _P, _I, _I, _P]),
    "adct_batch_plan_create": (_I, [_P, ctypes.POINTER(Plane), _I, _P, _I, _I, _I, _P, _I,
                                    ctypes.POINTER(_P), _P]),
    "adct_batch_plan_launch": (_I, [_P, _P]),
    "adct_batch_plan_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                  ctypes.POINTER(ctypes.c_double)]),
    "adct_batch_plan_destroy": (_I, [_P]),
    "adct_filter_packed_bytes": (_I64, []),
    "adct_filter_pack": (_I, [_P, _P, _P]),
    "adct_filter_workspace_bytes": (_I64, [_I, _I, _I]),
    "adct_filter_grad": (_I, [_P, _P, _P, _I, _I, _I, _P, _I64, _P, _P, _P, _P]),
    "adct_filter_adam": (_I, [_P, _P, _P, _P, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, _P]),
    "adct_filter_train_step": (_I, [_P, _P, _P, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _P, _P, _I, _I, _I, _P, _I64, _P, _P]),
    "adct_filter_apply": (_I, [_P, _P, _I64, _I, ctypes.POINTER(Plane), _I, _P, _I64, _P, _I64, _P, _P]),
    "adct_filter_select": (_I, [_P, _P, _I, _I, _P, _I64, ctypes.POINTER(Plane), _P, _I64, _P, _P]),
    "adct_filter_checkpoint_bytes": (_I64, [_I]),
    "adct_filter_save": (_I, [_P, _P, _P, _I, _P, _I64, _P]),
    "adct_filter_load": (_I, [_P, _I64, _P, _P, _P, ctypes.POINTER(_I), _P]),
}


def lib():
    """Load libadct.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1808_02950_amd._build.build()")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def _check(status: int):
    if status != 0:
        raise AdctError(status, lib().adct_last_error().decode())


def _tid(t) -> int:
    return TRANSFORM_IDS[t] if isinstance(t, str) else int(t)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need_cuda(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")


def _need_out(t, dtype, need: int, name: str):
    """A caller-supplied buffer the library writes (or reads) as `need` elements
    of `dtype` from its data pointer: a contiguous CUDA tensor of that dtype
    with at least that many elements (None passes)."""
    if t is None:
        return
    _need_cuda(t, dtype, name)
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < need:
        raise ValueError(f"{name} needs at least {need} elements of {dtype}, has {t.numel()}")


def _need_image(t, h: int, w: int, name: str):
    """A caller-supplied 2-D uint8 image of exactly (h, w) with unit column
    stride: the library addresses it as h rows of w bytes, stride(0) apart."""
    if t is None:
        return
    import torch
    _need_cuda(t, torch.uint8, name)
    if t.dim() != 2 or tuple(t.shape) != (h, w) or t.stride(1) != 1:
        raise ValueError(f"{name} must be a ({h}, {w}) uint8 image with unit column stride")


def _check_buffer(name, buf, planes):
    """Every byte a kernel reaches through `planes` (offset, H, W, pitch) must
    lie inside the contiguous tensor `buf`."""
    if not buf.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    total = buf.numel()
    for off, h, w, pitch in planes:
        if off < 0 or h < 1 or w < 1 or pitch < w or off + (h - 1) * pitch + w > total:
            raise ValueError(f"an image reaches outside {name}")


def _matrix_arg(t):
    """(transform id, Matrix or None): a name / id, or an 8x8 integer matrix,
    which is passed as ADCT_CUSTOM."""
    if isinstance(t, (str, int, np.integer)):
        return _tid(t), None
    m = np.asarray(t)
    if m.shape != (8, 8) or not np.issubdtype(m.dtype, np.integer) or np.abs(m).max() > 127:
        raise ValueError("a custom transform must be an 8x8 integer matrix with int8 entries")
    return CUSTOM, _matrix_struct(m)


def _mref(m):
    return ctypes.byref(m) if m is not None else None


def _check_frames(name, buf, planes, nf):
    """Every byte a kernel reads or writes through `planes` must lie inside the
    (n_frames, frame_bytes) tensor `buf` (None passes)."""
    if buf is None:
        return
    if buf.dim() != 2 or buf.stride(1) != 1 or buf.shape[0] != nf:
        raise ValueError(f"{name} must be (n_frames, frame_bytes) with unit inner stride")
    for off, h, w, pitch in planes:
        if off < 0 or h < 1 or w < 1 or off + (h - 1) * pitch + w > buf.shape[1]:
            raise ValueError(f"a plane reaches outside a frame of {name}")


# ---------------------------------------------------------------- host-only

def version() -> int:
    return lib().adct_version()


def codec_set_schedule(workgroups_per_cu: int) -> None:
    """adct_codec_set_schedule: 0 = occupancy-limited persistent grid,
    -1 = one tile per wave, k > 0 = at most k workgroups per CU."""
    _check(lib().adct_codec_set_schedule(int(workgroups_per_cu)))



def release_caches() -> int:
    """adct_release_caches: free the device buffers the searches and the
    coding-gain sweep keep on the current device; returns the bytes freed."""
    n = _I64()
    _check(lib().adct_release_caches(ctypes.byref(n)))
    return int(n.value)

def matrix_get(t) -> np.ndarray:
    m = Matrix()
    _check(lib().adct_matrix_get(_tid(t), ctypes.byref(m)))
    return np.array(list(m.T), dtype=np.int64).reshape(8, 8)


def transform_bounds(t, r: int, quant_step: int = 0, custom: np.ndarray | None = None):
    m = _matrix_struct(custom) if custom is not None else None
    f, i = _I64(), _I64()
    _check(lib().adct_transform_bounds(_tid(t), ctypes.byref(m) if m else None, r, quant_step,
                                       ctypes.byref(f), ctypes.byref(i)))
    return f.value, i.value


def _matrix_struct(t: np.ndarray) -> Matrix:
    t = np.asarray(t, dtype=np.int64).reshape(8, 8)
    m = Matrix()
    for k in range(64):
        m.T[k] = int(t.ravel()[k])
    for k in range(8):
        m.n[k] = int(np.dot(t[k], t[k]))
    return m


# ---------------------------------------------------------------- codec

def n_blocks(h: int, w: int) -> int:
    return (h // 8) * (w // 8)


def encode_blocks(img, t, r: int, quant_step: int = 0, want_int: bool = True,
                  want_scaled: bool = False, coef_int=None, coef_scaled=None, stream=None):
    """adct_encode_blocks.  img: uint8 CUDA tensor (H, W) (row pitch = stride(0)).
    t: a transform name / id, or an 8x8 integer matrix with orthogonal rows
    (ADCT_CUSTOM).  Returns (coef_int or None, coef_scaled or None), each
    (n_blocks, r)."""
    import torch
    _need_cuda(img, torch.uint8, "img")
    if img.dim() != 2 or img.stride(1) != 1:
        raise ValueError("img must be a 2-D image with unit column stride")
    tid, mat = _matrix_arg(t)
    h, w = img.shape
    nb = n_blocks(h, w)
    _need_out(coef_int, torch.int16, nb * r, "coef_int")
    _need_out(coef_scaled, torch.float32, nb * r, "coef_scaled")
    if want_int and coef_int is None:
        coef_int = torch.empty((nb, r), dtype=torch.int16, device=img.device)
    if want_scaled and coef_scaled is None:
        coef_scaled = torch.empty((nb, r), dtype=torch.float32, device=img.device)
    _check(lib().adct_encode_blocks(_ptr(img), h, w, img.stride(0), tid, _mref(mat), r, quant_step,
                                    _ptr(coef_int), _ptr(coef_scaled), _stream(stream)))
    return coef_int, coef_scaled


def decode_blocks(coef_int, h: int, w: int, t, r: int, quant_step: int = 0, out=None,
                  coef_scaled=None, stream=None):
    """adct_decode_blocks from int16 levels (coef_int) or float32 B
    (coef_scaled; no quantiser step).  t as in encode_blocks.  Returns the
    (H, W) uint8 reconstruction."""
    import torch
    tid, mat = _matrix_arg(t)
    nb = n_blocks(h, w)
    _need_out(coef_int, torch.int16, nb * r, "coef_int")
    _need_out(coef_scaled, torch.float32, nb * r, "coef_scaled")
    src = coef_int if coef_int is not None else coef_scaled
    if src is None:
        raise ValueError("coef_int or coef_scaled is required")
    _need_image(out, h, w, "out")
    if out is None:
        out = torch.empty((h, w), dtype=torch.uint8, device=src.device)
    _check(lib().adct_decode_blocks(_ptr(coef_int), _ptr(coef_scaled), h, w, _ptr(out),
                                    out.stride(0), tid, _mref(mat), r, quant_step, _stream(stream)))
    return out


@dataclass
class Evaluation:
    sse: int
    mse: float
    psnr: float


def evaluate_coding(img, t, r: int, quant_step: int = 0, coef_int=None, recon=None,
                    sse=None, stream=None) -> Evaluation:
    """adct_evaluate_coding (synchronises the stream to return MSE / PSNR).
    t as in encode_blocks."""
    import torch
    _need_cuda(img, torch.uint8, "img")
    if img.dim() != 2 or img.stride(1) != 1:
        raise ValueError("img must be a 2-D image with unit column stride")
    tid, mat = _matrix_arg(t)
    h, w = img.shape
    _need_out(coef_int, torch.int16, n_blocks(h, w) * r, "coef_int")
    _need_image(recon, h, w, "recon")
    _need_out(sse, torch.int64, 1, "sse")
    if sse is None:
        sse = torch.empty(1, dtype=torch.int64, device=img.device)
    mse, psnr = ctypes.c_double(), ctypes.c_double()
    _check(lib().adct_evaluate_coding(_ptr(img), h, w, img.stride(0), tid, _mref(mat), r, quant_step,
                                      _ptr(coef_int), _ptr(recon),
                                      recon.stride(0) if recon is not None else 0,
                                      _ptr(sse), ctypes.byref(mse), ctypes.byref(psnr),
                                      _stream(stream)))
    return Evaluation(int(sse.item()), mse.value, psnr.value)


def planes_struct(planes) -> ctypes.Array:
    arr = (Plane * len(planes))()
    for i, (off, h, w, pitch) in enumerate(planes):
        arr[i].offset, arr[i].H, arr[i].W, arr[i].pitch = int(off), int(h), int(w), int(pitch)
    return arr


def evaluate_stream(frames, planes, t, r: int, quant_step: int = 0, coef=None, recon=None,
                    sse=None, stream=None):
    """adct_evaluate_stream over frames (uint8 CUDA tensor (n_frames, frame_bytes)).
    planes: list of (offset, H, W, pitch).  Returns the device SSE tensor
    (n_frames, n_planes) int64 (uint64 values); does not synchronise."""
    import torch
    _need_cuda(frames, torch.uint8, "frames")
    tid, mat = _matrix_arg(t)
    nf = frames.shape[0]
    _check_frames("frames", frames, planes, nf)
    if recon is not None:
        _need_cuda(recon, torch.uint8, "recon")
        _check_frames("recon", recon, planes, nf)
    _need_out(coef, torch.int16, nf * stream_blocks_per_frame(planes) * r, "coef")
    _need_out(sse, torch.int64, nf * len(planes), "sse")
    if sse is None:
        sse = torch.empty((nf, len(planes)), dtype=torch.int64, device=frames.device)
    arr = planes_struct(planes)
    _check(lib().adct_evaluate_stream(_ptr(frames), frames.stride(0), nf, arr, len(planes), tid,
                                      _mref(mat), r, quant_step, _ptr(coef), _ptr(recon),
                                      recon.stride(0) if recon is not None else 0,
                                      _ptr(sse), _stream(stream)))
    return sse


def stream_bandwidth_probe(frames, planes, r: int, coef=None, recon=None, stream=None):
    """adct_stream_bandwidth_probe: the loads and stores of evaluate_stream for
    these arguments without the arithmetic (the HBM ceiling of that mix)."""
    import torch
    _need_cuda(frames, torch.uint8, "frames")
    nf = frames.shape[0]
    _check_frames("frames", frames, planes, nf)
    if recon is not None:
        _need_cuda(recon, torch.uint8, "recon")
        _check_frames("recon", recon, planes, nf)
    _need_out(coef, torch.int16, nf * stream_blocks_per_frame(planes) * r, "coef")
    _check(lib().adct_stream_bandwidth_probe(_ptr(frames), frames.stride(0), nf, planes_struct(planes), len(planes),
                                             r, _ptr(coef), _ptr(recon), recon.stride(0) if recon is not None else 0,
                                             _stream(stream)))


def ssim(ref, test, planes, out=None, stream=None):
    """adct_ssim: mean SSIM of every plane of every frame of `test` against `ref`.
    With planes (a list of (offset, H, W, pitch)) the inputs are uint8 CUDA
    tensors (n_frames, frame_bytes); with planes=None they are two 2-D images
    (one frame, one plane).  Returns the device float64 tensor
    (n_frames, n_planes); does not synchronise."""
    import torch
    _need_cuda(ref, torch.uint8, "ref")
    _need_cuda(test, torch.uint8, "test")
    if planes is None:
        if ref.dim() != 2 or ref.shape != test.shape or test.stride(0) != ref.stride(0):
            raise ValueError("two 2-D images of one shape and pitch are required")
        planes = [(0, ref.shape[0], ref.shape[1], ref.stride(0))]
        nf, fs_r, fs_t = 1, 0, 0
    else:
        nf, fs_r, fs_t = ref.shape[0], ref.stride(0), test.stride(0)
        _check_frames("ref", ref, planes, nf)
        _check_frames("test", test, planes, nf)
    if test.shape[0] != ref.shape[0]:
        raise ValueError("ref and test need the same number of frames")
    _need_out(out, torch.float64, nf * len(planes), "out")
    if out is None:
        out = torch.empty((nf, len(planes)), dtype=torch.float64, device=ref.device)
    arr = planes_struct(planes)
    _check(lib().adct_ssim(_ptr(ref), fs_r, _ptr(test), fs_t, nf, arr, len(planes), _ptr(out),
                           _stream(stream)))
    return out


def jam_matrix(n: int, base="T1"):
    """adct_jam_matrix: the n-point matrix (n = 16 or 32) as numpy int8 (n, n)
    and its row norms as int32 (n,)."""
    import numpy as np
    t = np.zeros((n, n), dtype=np.int8)
    nr = np.zeros(n, dtype=np.int32)
    _check(lib().adct_jam_matrix(_tid(base), n, t.ctypes.data, nr.ctypes.data))
    return t, nr


def jam_blocks_per_frame(planes, n: int) -> int:
    return sum(((h + n - 1) // n) * ((w + n - 1) // n) for _, h, w, _ in planes)


def jam_evaluate_stream(frames, planes, n: int, r: int, quant_step: int = 0, coef=None, recon=None,
                        sse=None, base="T1", stream=None):
    """adct_jam_evaluate_stream over frames (uint8 CUDA tensor (n_frames, frame_bytes)),
    n x n blocks.  planes: list of (offset, H, W, pitch).  Returns the device SSE
    tensor (n_frames, n_planes) int64 (uint64 values); does not synchronise."""
    import torch
    _need_cuda(frames, torch.uint8, "frames")
    nf = frames.shape[0]
    # every byte the kernel touches must lie inside the tensors
    _check_frames("frames", frames, planes, nf)
    _check_frames("recon", recon, planes, nf)
    _need_out(sse, torch.int64, nf * len(planes), "sse")
    if sse is None:
        sse = torch.empty((nf, len(planes)), dtype=torch.int64, device=frames.device)
    _need_out(coef, torch.int32, nf * jam_blocks_per_frame(planes, n) * r, "coef")
    if recon is not None:
        _need_cuda(recon, torch.uint8, "recon")
    arr = planes_struct(planes)
    _check(lib().adct_jam_evaluate_stream(_ptr(frames), frames.stride(0), nf, arr, len(planes), _tid(base),
                                          n, r, quant_step, _ptr(coef), _ptr(recon),
                                          recon.stride(0) if recon is not None else 0,
                                          _ptr(sse), _stream(stream)))
    return sse


def evaluate_inverse(frames, planes, T, r: int, recon=None, sse=None, stream=None):
    """adct_evaluate_inverse: zonal coding with an invertible (not necessarily
    orthogonal) int8 matrix T (8, 8) and the inverse decoder.  frames: uint8 CUDA
    tensor (n_frames, frame_bytes); planes: list of (offset, H, W, pitch).
    Returns the device SSE tensor (n_frames, n_planes); does not synchronise."""
    import torch
    _need_cuda(frames, torch.uint8, "frames")
    nf = frames.shape[0]
    _check_frames("frames", frames, planes, nf)
    _check_frames("recon", recon, planes, nf)
    if recon is not None:
        _need_cuda(recon, torch.uint8, "recon")
    t = np.ascontiguousarray(np.asarray(T, dtype=np.int8).reshape(64))
    _need_out(sse, torch.int64, nf * len(planes), "sse")
    if sse is None:
        sse = torch.empty((nf, len(planes)), dtype=torch.int64, device=frames.device)
    arr = planes_struct(planes)
    _check(lib().adct_evaluate_inverse(_ptr(frames), frames.stride(0), nf, arr, len(planes), t.ctypes.data,
                                       r, _ptr(recon), recon.stride(0) if recon is not None else 0,
                                       _ptr(sse), _stream(stream)))
    return sse


def coding_gain_sweep(c_hats, rhos, stream=None):
    """adct_coding_gain_sweep: unified coding gain (dB) of each real 8x8 matrix
    at each correlation.  Returns numpy (n_t, n_rho)."""
    c = np.ascontiguousarray(np.asarray(c_hats, dtype=np.float64).reshape(-1, 64))
    r = np.ascontiguousarray(np.asarray(rhos, dtype=np.float64).reshape(-1))
    out = np.zeros((c.shape[0], r.shape[0]), dtype=np.float64)
    _check(lib().adct_coding_gain_sweep(c.ctypes.data, c.shape[0], r.ctypes.data, r.shape[0],
                                        out.ctypes.data, _stream(stream)))
    return out


def coding_gain_sweep_noalloc(c_hats, rhos, stream=None):
    """adct_coding_gain_sweep_noalloc: the same results without any device
    allocation (fixed per-device staging; calls on one GPU must not overlap)."""
    c = np.ascontiguousarray(np.asarray(c_hats, dtype=np.float64).reshape(-1, 64))
    r = np.ascontiguousarray(np.asarray(rhos, dtype=np.float64).reshape(-1))
    out = np.zeros((c.shape[0], r.shape[0]), dtype=np.float64)
    _check(lib().adct_coding_gain_sweep_noalloc(c.ctypes.data, c.shape[0], r.ctypes.data, r.shape[0],
                                                out.ctypes.data, _stream(stream)))
    return out


def stream_blocks_per_frame(planes) -> int:
    return sum(n_blocks(h, w) for _, h, w, _ in planes)


def psnr_from_sse(sse: int, npix: int) -> float:
    if sse == 0:
        return math.inf
    return 10.0 * math.log10(255.0 * 255.0 * npix / sse)


# ---------------------------------------------------------------- search

SEARCH_CLOSURE, SEARCH_CANONICAL = 0, 1


def derive_transform(P, mode: int = SEARCH_CLOSURE, orders=None, fix_rows_1_5: bool = True,
                     cap: int = 4096, stream=None):
    """adct_derive_transform.  Returns (matrices (n, 8, 8) int64, angles (n, 8)
    radians, leaves, dead)."""
    p = np.ascontiguousarray(np.asarray(P, dtype=np.int8))
    if orders is not None:
        o = np.ascontiguousarray(np.asarray(orders, dtype=np.uint8))
        optr, n_orders = o.ctypes.data, o.shape[0]
    else:
        o, optr, n_orders = None, None, 0
    out = (Matrix * cap)()
    ang = np.zeros((cap, 8), dtype=np.float64)
    n, leaves, dead = _I(), _I64(), _I64()
    _check(lib().adct_derive_transform(p.ctypes.data, len(p), mode, optr, n_orders,
                                       1 if fix_rows_1_5 else 0, out, cap, ctypes.byref(n),
                                       ang.ctypes.data, ctypes.byref(leaves), ctypes.byref(dead),
                                       _stream(stream)))
    mats = np.array([np.array(list(out[i].T), dtype=np.int64).reshape(8, 8)
                     for i in range(n.value)]).reshape(-1, 8, 8)
    return mats, ang[:n.value], leaves.value, dead.value


def search_topk(P, k: int, primitive: bool = True, stream=None):
    """adct_search_topk.  Returns (vec (8, k, 8) int8, idx (8, k), cos (8, k))."""
    p = np.ascontiguousarray(np.asarray(P, dtype=np.int8))
    vec = np.zeros((8, k, 8), dtype=np.int8)
    idx = np.zeros((8, k), dtype=np.int64)
    cos = np.zeros((8, k), dtype=np.float64)
    _check(lib().adct_search_topk(p.ctypes.data, len(p), k, 1 if primitive else 0, vec.ctypes.data,
                                  idx.ctypes.data, cos.ctypes.data, _stream(stream)))
    return vec, idx, cos


def orthogonal_tuples(lists, cap: int = 1 << 20, stream=None):
    """adct_orthogonal_tuples.  lists: 8 arrays (len_r, 8).  Returns
    (tuples (min(n, cap), 8) int32, n)."""
    arrs = [np.asarray(l, dtype=np.int8).reshape(-1, 8) for l in lists]
    flat = np.ascontiguousarray(np.concatenate(arrs, axis=0))
    lens = (_I * 8)(*[a.shape[0] for a in arrs])
    out = np.zeros((max(cap, 1), 8), dtype=np.int32)
    n = _I64()
    _check(lib().adct_orthogonal_tuples(flat.ctypes.data, lens, out.ctypes.data, cap,
                                        ctypes.byref(n), _stream(stream)))
    return out[:min(n.value, cap)], n.value


# ---------------------------------------------------------------- batch

def _tid_array(transforms):
    arr = (ctypes.c_int * len(transforms))(*[_tid(t) for t in transforms])
    return arr


def evaluate_batch(base, images, transforms, r_lo: int = 1, r_hi: int = 63, sse=None,
                   wgs_per_cu: int = 4, split: int = 1, stream=None):
    """adct_evaluate_batch.  base: uint8 CUDA tensor holding every image;
    images: list of (offset, H, W, pitch).  Returns the device table
    (n_images, n_transforms, r_hi - r_lo + 1) int64 (uint64 values)."""
    import torch
    _need_cuda(base, torch.uint8, "base")
    _check_buffer("base", base, images)
    n = len(images)
    _need_out(sse, torch.int64, n * len(transforms) * max(r_hi - r_lo + 1, 0), "sse")
    if sse is None:
        sse = torch.empty((n, len(transforms), r_hi - r_lo + 1), dtype=torch.int64, device=base.device)
    tids = _tid_array(transforms)
    _check(lib().adct_evaluate_batch(_ptr(base), planes_struct(images), n, ctypes.cast(tids, _P),
                                     len(transforms), r_lo, r_hi, _ptr(sse), wgs_per_cu, split,
                                     _stream(stream)))
    return sse


class BatchPlan:
    """adct_batch_plan_*: the sweep with a tuned schedule (optionally autotuned);
    a launch runs the DCT and integer kernels side by side on two streams.
    Keeps references to the buffers it was built on."""

    def __init__(self, base, images, transforms, r_lo: int = 1, r_hi: int = 63, sse=None,
                 autotune: bool = True, stream=None):
        import torch
        self._h = _P()
        _need_cuda(base, torch.uint8, "base")
        _check_buffer("base", base, images)
        n = len(images)
        _need_out(sse, torch.int64, n * len(transforms) * max(r_hi - r_lo + 1, 0), "sse")
        self.base = base
        self.sse = sse if sse is not None else torch.empty(
            (n, len(transforms), r_hi - r_lo + 1), dtype=torch.int64, device=base.device)
        self._planes = planes_struct(images)
        self._tids = _tid_array(transforms)
        _check(lib().adct_batch_plan_create(_ptr(base), self._planes, n, ctypes.cast(self._tids, _P),
                                            len(transforms), r_lo, r_hi, _ptr(self.sse),
                                            1 if autotune else 0, ctypes.byref(self._h),
                                            _stream(stream)))

    def launch(self, stream=None):
        _check(lib().adct_batch_plan_launch(self._h, _stream(stream)))
        return self.sse

    def info(self):
        w, s, ms = _I(), _I(), ctypes.c_double()
        _check(lib().adct_batch_plan_info(self._h, ctypes.byref(w), ctypes.byref(s), ctypes.byref(ms)))
        return {"wgs_per_cu": w.value, "split": s.value, "tuned_ms": ms.value}

    def close(self):
        if self._h:
            lib().adct_batch_plan_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned post-filter

FILTER_PARAMS = 9857


def filter_pack(params, packed=None, stream=None):
    """adct_filter_pack: float32 CUDA params (9857,) -> packed uint8 CUDA tensor."""
    import torch
    _need_cuda(params, torch.float32, "params")
    if packed is None:
        packed = torch.empty(lib().adct_filter_packed_bytes(), dtype=torch.uint8, device=params.device)
    _check(lib().adct_filter_pack(_ptr(params), _ptr(packed), _stream(stream)))
    return packed


def filter_workspace(n: int, h: int, w: int, device="cuda"):
    import torch
    nb = lib().adct_filter_workspace_bytes(n, h, w)
    if nb < 0:
        raise AdctError(-2, f"unsupported training shape n={n} H={h} W={w}")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def filter_grad(params, recon, orig, workspace=None, want_y: bool = False, stream=None):
    """adct_filter_grad on uint8 CUDA tensors (n, H, W).  Returns (grad, loss, y)
    as CUDA tensors (y None unless want_y); does not synchronise."""
    import torch
    _need_cuda(params, torch.float32, "params")
    _need_cuda(recon, torch.uint8, "recon")
    _need_cuda(orig, torch.uint8, "orig")
    n, h, w = recon.shape
    if orig.shape != recon.shape or not recon.is_contiguous() or not orig.is_contiguous():
        raise ValueError("recon and orig must be contiguous tensors of one shape")
    if workspace is not None:
        _need_out(workspace, torch.uint8, lib().adct_filter_workspace_bytes(n, h, w), "workspace")
    else:
        workspace = filter_workspace(n, h, w, recon.device)
    grad = torch.empty(FILTER_PARAMS, dtype=torch.float32, device=recon.device)
    loss = torch.empty(1, dtype=torch.float32, device=recon.device)
    y = torch.empty((n, h, w), dtype=torch.float32, device=recon.device) if want_y else None
    _check(lib().adct_filter_grad(_ptr(params), _ptr(recon), _ptr(orig), n, h, w, _ptr(workspace),
                                  workspace.numel(), _ptr(grad), _ptr(loss), _ptr(y), _stream(stream)))
    return grad, loss, y


def filter_adam(params, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                eps: float = 1e-8, stream=None):
    _check(lib().adct_filter_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), step, lr, beta1, beta2, eps,
                                  _stream(stream)))


def filter_save(params, m=None, v=None, step: int = 0, stream=None) -> bytes:
    """adct_filter_save: a checkpoint blob of the float32 CUDA parameters (and the
    Adam moments m, v with the step, when given)."""
    import torch
    _need_cuda(params, torch.float32, "params")
    n = lib().adct_filter_checkpoint_bytes(1 if m is not None else 0)
    buf = ctypes.create_string_buffer(n)
    _check(lib().adct_filter_save(_ptr(params), _ptr(m), _ptr(v), step, ctypes.cast(buf, _P), n, _stream(stream)))
    return buf.raw


def filter_load(blob: bytes, params, m=None, v=None, stream=None) -> int:
    """adct_filter_load into float32 CUDA tensors; returns the saved Adam step."""
    import torch
    _need_cuda(params, torch.float32, "params")
    for name, t in (("params", params), ("m", m), ("v", v)):
        if t is not None and (t.numel() != FILTER_PARAMS or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous tensor of {FILTER_PARAMS} floats")
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    step = _I()
    _check(lib().adct_filter_load(ctypes.cast(buf, _P), len(blob), _ptr(params), _ptr(m), _ptr(v),
                                  ctypes.byref(step), _stream(stream)))
    return step.value


class FilterTrainer:
    """Adam training of the post-filter on device batches through
    adct_filter_train_step.  params: float32 (9857,) numpy or CUDA tensor."""

    def __init__(self, params, n: int, h: int, w: int, lr: float = 1e-3, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, device="cuda"):
        import torch
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32) if not isinstance(params, torch.Tensor)
                                      else params, dtype=torch.float32).to(device).contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.ws = filter_workspace(n, h, w, device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.shape = (n, h, w)
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.step_count = 0

    def step(self, recon, orig, loss_out=None, stream=None):
        """One step on a batch (uint8 CUDA (n, H, W)); the batch loss (before
        the update) goes to loss_out (a one-element float32 CUDA tensor) or to
        self.loss, which is returned; does not synchronise."""
        if tuple(recon.shape) != self.shape or tuple(orig.shape) != self.shape:
            raise ValueError(f"batch shape must be {self.shape}")
        self.step_count += 1
        dst = self.loss if loss_out is None else loss_out
        _check(lib().adct_filter_train_step(_ptr(self.params), _ptr(self.m), _ptr(self.v), self.step_count,
                                            self.lr, self.beta1, self.beta2, self.eps, _ptr(recon), _ptr(orig),
                                            *self.shape, _ptr(self.ws), self.ws.numel(), _ptr(dst),
                                            _stream(stream)))
        return dst

    def packed(self, stream=None):
        return filter_pack(self.params, stream=stream)

    def save(self, path: str):
        """Checkpoint: the library's self-checking blob (float32 master weights,
        Adam moments, step; adct_filter_save) with the batch shape and the
        hyper-parameters, in a numpy .npz file (plain arrays, no pickled objects)."""
        blob = filter_save(self.params, self.m, self.v, self.step_count)
        np.savez(path, blob=np.frombuffer(blob, dtype=np.uint8), shape=np.array(self.shape, dtype=np.int64),
                 hyper=np.array([self.lr, self.beta1, self.beta2, self.eps], dtype=np.float64))

    @classmethod
    def load(cls, path: str, device="cuda"):
        """Resume from a checkpoint written by save(); continuing gives the same
        weights as an uninterrupted run (the gradient is deterministic).  The
        blob is validated (magic, version, size, hash) by adct_filter_load."""
        with np.load(path, allow_pickle=False) as z:
            n, h, w = (int(x) for x in z["shape"])
            lr, b1, b2, eps = (float(x) for x in z["hyper"])
            blob = z["blob"].tobytes()
        tr = cls(np.zeros(FILTER_PARAMS, dtype=np.float32), n, h, w, lr=lr, beta1=b1, beta2=b2, eps=eps,
                 device=device)
        tr.step_count = filter_load(blob, tr.params, tr.m, tr.v)
        return tr


def filter_apply(packed, frames, planes, out=None, orig=None, stream=None):
    """adct_filter_apply over frames (uint8 CUDA (n_frames, frame_bytes)).
    Returns (out, sse) -- sse (n_frames, n_planes) int64 when orig is given."""
    import torch
    _need_cuda(frames, torch.uint8, "frames")
    _need_out(packed, torch.uint8, lib().adct_filter_packed_bytes(), "packed")
    nf = frames.shape[0]
    if out is None:
        out = torch.zeros_like(frames)
    for name, buf in (("frames", frames), ("out", out), ("orig", orig)):
        if buf is not None:
            _need_cuda(buf, torch.uint8, name)
        _check_frames(name, buf, planes, nf)
    sse = torch.empty((nf, len(planes)), dtype=torch.int64, device=frames.device) if orig is not None else None
    arr = planes_struct(planes)
    _check(lib().adct_filter_apply(_ptr(packed), _ptr(frames), frames.stride(0), nf, arr, len(planes), _ptr(out),
                                   out.stride(0), _ptr(orig), orig.stride(0) if orig is not None else 0,
                                   _ptr(sse), _stream(stream)))
    return out, sse


def filter_select(sse_filtered, sse_reference, plain, planes, out, keep=None, stream=None):
    """adct_filter_select: frames whose filtered SSE exceeds the reference's get
    the plain reconstruction copied into out.  Returns the keep flags (uint8)."""
    import torch
    _need_cuda(plain, torch.uint8, "plain")
    _need_cuda(out, torch.uint8, "out")
    nf = plain.shape[0]
    _check_frames("plain", plain, planes, nf)
    _check_frames("out", out, planes, nf)
    _need_out(sse_filtered, torch.int64, nf * len(planes), "sse_filtered")
    _need_out(sse_reference, torch.int64, nf * len(planes), "sse_reference")
    if sse_filtered is None or sse_reference is None:
        raise ValueError("sse_filtered and sse_reference are required")
    _need_out(keep, torch.uint8, nf, "keep")
    if keep is None:
        keep = torch.empty(nf, dtype=torch.uint8, device=plain.device)
    arr = planes_struct(planes)
    _check(lib().adct_filter_select(_ptr(sse_filtered), _ptr(sse_reference), nf, len(planes), _ptr(plain),
                                    plain.stride(0), arr, _ptr(out), out.stride(0), _ptr(keep), _stream(stream)))
    return keep


def patch_pairs(images, table, transform="T1", quant_step: int = 0, size: int = 64, device="cuda"):
    """Training pairs for the post-filter, decoded by this library's codec.

    images: list of 2-D uint8 numpy arrays; table: int rows (image, y0, x0, r)
    with (y0, x0) on the 8x8 grid.  Patch k is the size x size block of
    images[image] at (y0, x0), coded with `transform` keeping r coefficients
    (and `quant_step`).  Blocks are coded independently, so coding the patch
    alone equals cutting it from the coded image.  Returns host uint8 arrays
    (recon, orig) of shape (n, size, size)."""
    import torch
    table = np.asarray(table, dtype=np.int64)
    n = len(table)
    orig = np.empty((n, size, size), dtype=np.uint8)
    for i in np.unique(table[:, 0]):
        rows = np.nonzero(table[:, 0] == i)[0]
        img = images[int(i)]
        for k in rows:
            y0, x0 = int(table[k, 1]), int(table[k, 2])
            orig[k] = img[y0:y0 + size, x0:x0 + size]
    order = np.argsort(table[:, 3], kind="stable")
    od = torch.from_numpy(orig[order].reshape(n, size * size)).to(device)
    rec = torch.empty_like(od)
    start = 0
    for r in np.unique(table[:, 3]):
        cnt = int(np.sum(table[:, 3] == r))
        evaluate_stream(od[start:start + cnt], [(0, size, size, size)], transform, int(r), quant_step,
                        recon=rec[start:start + cnt])
        start += cnt
    out = np.empty_like(orig)
    out[order] = rec.cpu().numpy().reshape(n, size, size)
    return out, orig


def shuffled_pairs(recon, orig, seed: int = 0, device="cuda"):
    """The (recon, orig) host pairs in train_filter's seeded order, on the device."""
    import torch
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(recon))
    return (torch.from_numpy(np.ascontiguousarray(recon[perm])).to(device),
            torch.from_numpy(np.ascontiguousarray(orig[perm])).to(device))


def train_filter(params, recon, orig, steps: int, batch: int = 64, lr: float = 1e-3, lr_final: float = 1e-4,
                 seed: int = 0, device="cuda", log_every: int = 0):
    """Adam training of the post-filter on the GPU.  recon, orig: host uint8
    (n, H, W) pairs (see patch_pairs), shuffled once (seeded) and uploaded, or
    CUDA uint8 tensors used as they are (see shuffled_pairs); step s trains on
    the next contiguous batch (wrapping), with the learning rate decayed
    geometrically from lr to lr_final.  Returns (trained params as a CUDA
    float32 tensor, per-step losses as numpy)."""
    import torch
    n, h, w = recon.shape
    if isinstance(recon, torch.Tensor):
        rd, od = recon, orig
    else:
        rd, od = shuffled_pairs(recon, orig, seed, device)
    tr = FilterTrainer(params, batch, h, w, lr=lr, device=device)
    losses = torch.empty(steps, dtype=torch.float32, device=device)
    decay = (lr_final / lr) ** (1.0 / max(1, steps - 1))
    for s in range(steps):
        b0 = (s * batch) % (n - batch + 1)
        tr.lr = lr * decay ** s
        loss = tr.step(rd[b0:b0 + batch], od[b0:b0 + batch], loss_out=losses[s:s + 1])
        if log_every and (s + 1) % log_every == 0:
            print(f"step {s + 1}: loss {float(loss.item()):.6f}", flush=True)
    return tr.params, losses.cpu().numpy()
