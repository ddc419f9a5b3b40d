"""FP64 reference of the convolutional surrogate (TEST INFRASTRUCTURE ONLY:
used by the tests to check the GPU kernels; the product never imports it).

Network: x -> tanh(conv1(s_in x)) -> tanh(conv2) -> tanh(conv3) -> s_out conv4,
each conv a periodic 3x3 correlation z[b,o,y,x] = sum_{c,dy,dx} w[o,c,dy+1,dx+1]
x[b,c,y+dy,x+dx] + bias[o].  Loss: mean squared error over the interior.
Gradients by the chain rule written out layer by layer.

Precision model (bf16=True), the storage precision of the device kernels:
the three hidden activations are rounded to bfloat16 after the tanh, and
the gradients with respect to the hidden pre-activations (after the
factor 1 - a^2) are rounded to bfloat16; the input, the output, dL/dy and
all sums stay in full precision here.  Weights are passed in already
rounded.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(x, dy, dx):
    """out[..., y, x] = x[..., y + dy, x + dx] with periodic wrap."""
    return np.roll(x, shift=(-dy, -dx), axis=(-2, -1))


def conv(x, w, b, iscale=1.0, oscale=1.0):
    B, C, H, W = x.shape
    O = w.shape[0]
    z = np.zeros((B, O, H, W))
    for dy, dx in TAPS:
        xs = shift(x, dy, dx) * iscale
        z += np.einsum("oc,bchw->bohw", w[:, :, dy + 1, dx + 1], xs)
    return oscale * (z + b[None, :, None, None])


def conv_backward(dz, x, w, iscale=1.0, oscale=1.0):
    """Gradients of L through z = oscale (w * (iscale x) + b) given dL/dz."""
    g = oscale * dz
    dw = np.zeros_like(w)
    dx = np.zeros_like(x)
    for dy, dx_ in TAPS:
        xs = shift(x, dy, dx_) * iscale
        dw[:, :, dy + 1, dx_ + 1] = np.einsum("bohw,bchw->oc", g, xs)
        # z[q] uses x[q + off]: dx[p] gets w * g[p - off]
        dx += iscale * np.einsum("oc,bohw->bchw", w[:, :, dy + 1, dx_ + 1], shift(g, -dy, -dx_))
    db = g.sum(axis=(0, 2, 3))
    return dx, dw, db


def forward(params, x, s_in, s_out, bf16=False):
    """params: list of 4 (w, b).  Returns output and the activations."""
    r = bf16_round if bf16 else (lambda a: a)
    a0 = x[:, None]
    a1 = r(np.tanh(conv(a0, *params[0], iscale=s_in)))
    a2 = r(np.tanh(conv(a1, *params[1])))
    a3 = r(np.tanh(conv(a2, *params[2])))
    y = conv(a3, *params[3], oscale=s_out)
    return y[:, 0], (a0, a1, a2, a3)


def mse(pred, target, border):
    H, W = pred.shape[-2:]
    m = np.zeros(pred.shape, dtype=bool)
    m[..., border:H - border, border:W - border] = True
    n = m.sum()
    d = np.where(m, pred - target, 0.0)
    return (d * d).sum() / n, 2.0 * d / n


def backward(params, acts, dy, s_in, s_out, bf16=False):
    """dL/dx and [(dL/dw, dL/db)] for the layers given dL/dy."""
    r = bf16_round if bf16 else (lambda a: a)
    a0, a1, a2, a3 = acts
    grads = [None] * 4
    g = dy[:, None]
    dx3, dw, db = conv_backward(g, a3, params[3][0], oscale=s_out)
    grads[3] = (dw, db)
    g = r(dx3 * (1 - a3 * a3))
    dx2, dw, db = conv_backward(g, a2, params[2][0])
    grads[2] = (dw, db)
    g = r(dx2 * (1 - a2 * a2))
    dx1, dw, db = conv_backward(g, a1, params[1][0])
    grads[1] = (dw, db)
    g = r(dx1 * (1 - a1 * a1))
    dx0, dw, db = conv_backward(g, a0, params[0][0], iscale=s_in)
    grads[0] = (dw, db)
    return dx0[:, 0], grads


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    wn = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return wn, m, v


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
