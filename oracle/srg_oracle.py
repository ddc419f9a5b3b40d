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
rounded.  bf16=False is the unrounded network: every value in FP64.

Error budget of BF16 storage (`storage_noise_budget`): the standard
probabilistic model of rounding, each stored value a carrying an
independent error uniform in [-ulp(a)/2, ulp(a)/2] (ulp = the bfloat16
spacing at a: 8 significant bits, so 2^-8 relative at most).  The budget of
an output is the RMS, over seeded draws of those errors at the storage
points, of its deviation from the unrounded network; the tests allow three
times that (plus the FP32 accumulation term of `fp32_sum_slack`) between
the device and the unrounded network.  The model itself is pinned against
the deterministic round-to-nearest network (bf16=True) on the CPU.
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
        z += np.einsum("oc,bchw->bohw", w[:, :, dy + 1, dx + 1], xs, optimize=True)
    return oscale * (z + b[None, :, None, None])


def conv_backward(dz, x, w, iscale=1.0, oscale=1.0):
    """Gradients of L through z = oscale (w * (iscale x) + b) given dL/dz."""
    g = oscale * dz
    dw = np.zeros_like(w)
    dx = np.zeros_like(x)
    for dy, dx_ in TAPS:
        xs = shift(x, dy, dx_) * iscale
        dw[:, :, dy + 1, dx_ + 1] = np.einsum("bohw,bchw->oc", g, xs, optimize=True)
        # z[q] uses x[q + off]: dx[p] gets w * g[p - off]
        dx += iscale * np.einsum("oc,bohw->bchw", w[:, :, dy + 1, dx_ + 1], shift(g, -dy, -dx_),
                                optimize=True)
    db = g.sum(axis=(0, 2, 3))
    return dx, dw, db


def _store(bf16, store):
    if store is not None:
        return store
    return bf16_round if bf16 else (lambda a: a)


def forward(params, x, s_in, s_out, bf16=False, store=None):
    """params: list of 4 (w, b).  Returns output and the activations.
    `store`, if given, is applied to each stored hidden activation in place
    of the bf16 flag's rounding."""
    r = _store(bf16, store)
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


def backward(params, acts, dy, s_in, s_out, bf16=False, store=None):
    """dL/dx and [(dL/dw, dL/db)] for the layers given dL/dy; `store` as in
    forward, applied to each stored hidden gradient."""
    r = _store(bf16, store)
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


def bf16_ulp(a):
    """Spacing of bfloat16 numbers at |a| (8 significant bits): 2^(e - 7)
    for 2^e <= |a| < 2^(e+1); 0 at 0."""
    a = np.abs(np.asarray(a, dtype=np.float64))
    out = np.zeros_like(a)
    nz = a > 0
    out[nz] = np.exp2(np.floor(np.log2(a[nz])) - 7.0)
    return out


def storage_noise(rng):
    """A store function for forward/backward: adds to each value an
    independent error uniform within half a bfloat16 spacing."""
    def noisy(a):
        return a + rng.uniform(-0.5, 0.5, a.shape) * bf16_ulp(a)
    return noisy


def _outputs(params, x, s_in, s_out, dy, target, border, store):
    y, acts = forward(params, x, s_in, s_out, store=store)
    out = {"y": y}
    if target is not None:
        out["loss"], dy = mse(y, target, border)
    if dy is not None:
        dx, grads = backward(params, acts, dy, s_in, s_out, store=store)
        out["dx"] = dx
        for k, (dw, db) in enumerate(grads):
            out[f"dW{k}"], out[f"db{k}"] = dw, db
    return out


def storage_noise_budget(params, x, s_in, s_out, dy=None, target=None, border=0,
                         samples=8, seed=0):
    """Unrounded outputs and the RMS deviation of each from them under the
    storage-noise model: y always; with dy (or target and border, the MSE
    loss) also dx and every dW_k, db_k, and the loss.  Returns
    (exact, sigma), two dicts of arrays / floats keyed alike."""
    exact = _outputs(params, x, s_in, s_out, dy, target, border, None)
    noisy = storage_noise(np.random.default_rng(seed))
    acc = {k: 0.0 for k in exact}
    for _ in range(samples):
        o = _outputs(params, x, s_in, s_out, dy, target, border, noisy)
        for k in exact:
            acc[k] += float(np.sum((np.asarray(o[k]) - np.asarray(exact[k])) ** 2))
    sigma = {k: np.sqrt(v / samples) for k, v in acc.items()}
    return exact, sigma


def fp32_sum_slack(norm, n_terms, k=3.0):
    """k standard deviations of the error of FP32 sums of n_terms values
    (random-walk model, unit roundoff 2^-24 per addition) relative to the
    norm of the result."""
    return k * 2.0 ** -24 * np.sqrt(n_terms) * norm
