"""The binding validates every caller-supplied buffer (device, dtype,
contiguity, size, and that planes and images lie inside their tensors) BEFORE
the library is called: a wrong buffer raises TypeError / ValueError and no
kernel ever sees it.  Runs on the CPU: the library handle is replaced by one
that fails the test if anything reaches it, and the CUDA-device test accepts
CPU tensors so that the checks after it run."""

import numpy as np
import pytest
import torch

import paper_1808_02950_amd as A
from oracle import matrices as M


@pytest.fixture
def no_library(monkeypatch):
    def reached(*a, **k):
        raise AssertionError("the library was reached before the arguments were validated")

    def dtype_only(t, dtype, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}")

    monkeypatch.setattr(A, "lib", reached)
    monkeypatch.setattr(A, "_need_cuda", dtype_only)


def u8(*shape):
    return torch.zeros(shape, dtype=torch.uint8)


def test_cpu_tensor_is_refused_by_the_real_device_check():
    with pytest.raises(TypeError):
        A._need_cuda(u8(8, 8), torch.uint8, "img")


def test_codec_outputs(no_library):
    img = u8(16, 16)                                     # 4 blocks
    with pytest.raises(ValueError):
        A.encode_blocks(img, "T1", 10, coef_int=torch.zeros(39, dtype=torch.int16))
    with pytest.raises(TypeError):
        A.encode_blocks(img, "T1", 10, coef_int=torch.zeros(40, dtype=torch.int32))
    with pytest.raises(ValueError):
        A.encode_blocks(img, "T1", 10, coef_scaled=torch.zeros((40, 2), dtype=torch.float32)[:, 0])
    with pytest.raises(ValueError):
        A.decode_blocks(torch.zeros(40, dtype=torch.int16), 16, 16, "T1", 10, out=u8(16, 8))
    with pytest.raises(ValueError):
        A.decode_blocks(torch.zeros(30, dtype=torch.int16), 16, 16, "T1", 10)
    with pytest.raises(ValueError):
        A.evaluate_coding(img, "T1", 10, recon=u8(8, 16))
    with pytest.raises(ValueError):
        A.evaluate_coding(img, "T1", 10, recon=u8(16, 32)[:, ::2])
    with pytest.raises(ValueError):
        A.evaluate_coding(img, "T1", 10, coef_int=torch.zeros(10, dtype=torch.int16))
    with pytest.raises(TypeError):
        A.evaluate_coding(img, "T1", 10, sse=torch.zeros(1, dtype=torch.float64))
    with pytest.raises(ValueError):
        A.evaluate_coding(img, np.ones((4, 4), dtype=np.int64), 10)     # not 8 x 8


def test_stream_outputs(no_library):
    planes = [(0, 16, 16, 16)]
    frames = u8(2, 256)
    with pytest.raises(ValueError):
        A.evaluate_stream(frames, planes, "T1", 10, coef=torch.zeros(79, dtype=torch.int16))
    with pytest.raises(TypeError):
        A.evaluate_stream(frames, planes, "T1", 10, coef=torch.zeros(80, dtype=torch.int8))
    with pytest.raises(ValueError):
        A.evaluate_stream(frames, planes, "T1", 10, sse=torch.zeros(1, dtype=torch.int64))
    with pytest.raises(TypeError):
        A.evaluate_stream(frames, planes, "T1", 10, sse=torch.zeros(2, dtype=torch.int32))
    with pytest.raises(ValueError):
        A.evaluate_stream(frames, [(8, 16, 16, 16)], "T1", 10)          # plane past the frame
    with pytest.raises(ValueError):
        A.evaluate_stream(frames, planes, "T1", 10, recon=u8(2, 255))
    with pytest.raises(ValueError):
        A.jam_evaluate_stream(frames, planes, 16, 10, sse=torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ValueError):
        A.evaluate_inverse(frames, planes, M.t_sdct(), 10, sse=torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ValueError):
        A.ssim(frames, frames, planes, out=torch.zeros(1, dtype=torch.float64))


def test_batch_images_inside_base(no_library):
    base = u8(1024)
    with pytest.raises(ValueError):
        A.evaluate_batch(base, [(0, 32, 40, 40)], ["T1"])              # 1,280 bytes > 1,024
    with pytest.raises(ValueError):
        A.evaluate_batch(base, [(0, 16, 16, 16)], ["T1"], sse=torch.zeros(62, dtype=torch.int64))
    with pytest.raises(ValueError):
        A.BatchPlan(base, [(1000, 8, 8, 8)], ["T1"])
    with pytest.raises(ValueError):
        A.evaluate_batch(torch.zeros((64, 32), dtype=torch.uint8)[:, :16], [(0, 8, 8, 8)], ["T1"])


def test_filter_buffers(no_library):
    planes = [(0, 16, 16, 16)]
    frames = u8(2, 256)
    sse = torch.zeros((2, 1), dtype=torch.int64)
    with pytest.raises(ValueError):
        A.filter_select(sse[:1], sse, frames, planes, u8(2, 256))
    with pytest.raises(ValueError):
        A.filter_select(sse, None, frames, planes, u8(2, 256))
    with pytest.raises(ValueError):
        A.filter_select(sse, sse, frames, planes, u8(2, 256), keep=u8(1))
    with pytest.raises(TypeError):
        A.filter_select(sse, sse, frames, planes, torch.zeros((2, 256), dtype=torch.int16))
