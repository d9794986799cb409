"""Learned post-filter on decoded frames: float64 forward and backward.

TEST INFRASTRUCTURE: see the package docstring.

The filter is not part of the paper's method; it is a small network put behind
the decoder of Sec. 6 (encode, keep r zig-zag coefficients, invert) to remove
part of the error the approximate transform leaves.  Parity of this module is
therefore unpinned by the paper: it is pinned here by mathematics instead
(finite differences of the unrounded network, the adjoint identities of the
three convolution forms, scipy's 2-D correlation, torch's bfloat16 conversion,
the identity map when the last layer is zero, Adam's first step in closed form).

Network, on a decoded 8-bit image x (one channel):
    xn = (x - 128) / 64
    a1 = relu(conv3x3(xn; W1, b1))      1 -> 32 channels
    a2 = relu(conv3x3(a1; W2, b2))      32 -> 32
    f  = conv3x3(a2; W3, b3)            32 -> 1
    y  = xn + f,   output pixel = clip(round_half_even(128 + 64 y), 0, 255)
Every convolution is a 3x3 cross-correlation with zero padding of its own input
("same" size).  Loss: mean over all pixels of (y - (orig - 128) / 64)^2.

Rounding points (rounding=True), the places where the GPU kernels feed bfloat16
operands to the matrix cores: the weights W1, W2, W3; the activations a1, a2;
the loss gradient g3 = dL/dy; the masked input gradients dz2 and dz1.  Biases,
accumulations, f and y stay wide.  Weight gradients are taken with respect to
the rounded weights (the usual mixed-precision convention).  With
rounding=False the same code is the exact float64 network.

Parameters are one flat float32 vector in PyTorch Conv2d order:
W1 (32,1,3,3), b1 (32), W2 (32,32,3,3), b2 (32), W3 (1,32,3,3), b3 (1): 9857.
"""

from __future__ import annotations

import numpy as np

CH = 32
LAYOUT = (("W1", (CH, 1, 3, 3)), ("b1", (CH,)),
          ("W2", (CH, CH, 3, 3)), ("b2", (CH,)),
          ("W3", (1, CH, 3, 3)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in LAYOUT)          # 9857


def unflatten(p) -> dict:
    p = np.asarray(p, dtype=np.float64).ravel()
    assert p.size == N_PARAMS
    out, o = {}, 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def flatten(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in LAYOUT])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (8 significant bits), ties to even, kept in float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


def _ident(x):
    return np.asarray(x, dtype=np.float64)


def conv3x3(a: np.ndarray, w: np.ndarray, b=None) -> np.ndarray:
    """out[n,o,y,x] = b[o] + sum_{i,dy,dx} w[o,i,dy,dx] a[n,i,y+dy-1,x+dx-1]."""
    n, ci, h, wd = a.shape
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((n, w.shape[0], h, wd))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oi,nihw->nohw", w[:, :, dy, dx], ap[:, :, dy:dy + h, dx:dx + wd])
    if b is not None:
        out += np.asarray(b)[None, :, None, None]
    return out


def conv3x3_input_grad(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 in its input: da[n,i,y,x] = sum_{o,dy,dx}
    w[o,i,dy,dx] g[n,o,y-dy+1,x-dx+1] (zero outside)."""
    n, co, h, wd = g.shape
    gp = np.pad(g, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((n, w.shape[1], h, wd))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oi,nohw->nihw", w[:, :, dy, dx],
                             gp[:, :, 2 - dy:2 - dy + h, 2 - dx:2 - dx + wd])
    return out


def conv3x3_weight_grad(g: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 in its weights: dw[o,i,dy,dx] = sum_{n,y,x}
    g[n,o,y,x] a[n,i,y+dy-1,x+dx-1]."""
    n, ci, h, wd = a.shape
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((g.shape[1], ci, 3, 3))
    for dy in range(3):
        for dx in range(3):
            out[:, :, dy, dx] = np.einsum("nohw,nihw->oi", g, ap[:, :, dy:dy + h, dx:dx + wd])
    return out


def normalise(x_u8) -> np.ndarray:
    return (np.asarray(x_u8, dtype=np.float64) - 128.0) / 64.0


def forward(params, x_u8, rounding: bool = True) -> dict:
    """x_u8: [n][H][W] uint8 decoded images.  Returns the activations and y."""
    r = bf16 if rounding else _ident
    P = unflatten(params)
    x = np.asarray(x_u8)
    xn = normalise(x)[:, None]
    w1, w2, w3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    z1 = conv3x3(xn, w1, P["b1"])
    a1 = r(np.maximum(z1, 0.0))
    z2 = conv3x3(a1, w2, P["b2"])
    a2 = r(np.maximum(z2, 0.0))
    f = conv3x3(a2, w3, P["b3"])[:, 0]
    return {"xn": xn, "w1": w1, "w2": w2, "w3": w3, "a1": a1, "a2": a2,
            "f": f, "y": xn[:, 0] + f}


def loss_and_grad(params, x_u8, orig_u8, rounding: bool = True):
    """Mean squared error of y against the original and its gradient with
    respect to the 9857 parameters (flat, the order of LAYOUT)."""
    r = bf16 if rounding else _ident
    fw = forward(params, x_u8, rounding)
    tn = normalise(orig_u8)
    d = fw["y"] - tn
    count = d.size
    loss = float(np.sum(d * d) / count)
    g3 = r(2.0 * d / count)[:, None]
    grads = {"W3": conv3x3_weight_grad(g3, fw["a2"]), "b3": g3.sum(axis=(0, 2, 3))}
    dz2 = r(conv3x3_input_grad(g3, fw["w3"]) * (fw["a2"] > 0))
    grads["W2"] = conv3x3_weight_grad(dz2, fw["a1"])
    grads["b2"] = dz2.sum(axis=(0, 2, 3))
    dz1 = r(conv3x3_input_grad(dz2, fw["w2"]) * (fw["a1"] > 0))
    grads["W1"] = conv3x3_weight_grad(dz1, fw["xn"])
    grads["b1"] = dz1.sum(axis=(0, 2, 3))
    return loss, flatten(grads), fw


def loss_only(params, x_u8, orig_u8, rounding: bool = False) -> float:
    d = forward(params, x_u8, rounding)["y"] - normalise(orig_u8)
    return float(np.mean(d * d))


def apply(params, x_u8, rounding: bool = True) -> dict:
    """Filtered 8-bit image: round half to even of 128 + 64 y, clipped."""
    fw = forward(params, x_u8, rounding)
    real = 128.0 + 64.0 * fw["y"]
    out = np.clip(np.rint(real), 0, 255).astype(np.uint8)
    return {"out": out, "real": real, "y": fw["y"]}


def adam(params, grad, m, v, step: int, lr: float, beta1: float = 0.9,
         beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba), bias-corrected, step counted from 1."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def keep_filtered(sse_filtered, sse_reference) -> np.ndarray:
    """Keep rule per frame: the filtered frame is kept when its PSNR is at least
    that of the reference coding (same samples, so: when its squared error is
    not larger); otherwise the plain reconstruction is the output."""
    return (np.asarray(sse_filtered, dtype=np.uint64).reshape(len(sse_filtered), -1).sum(axis=1)
            <= np.asarray(sse_reference, dtype=np.uint64).reshape(len(sse_reference), -1).sum(axis=1))
