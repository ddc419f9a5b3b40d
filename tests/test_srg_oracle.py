"""Pins of the FP64 surrogate reference: the periodic 3x3 correlation against
scipy's wrap-mode correlation, and every gradient against central
differences."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import srg_oracle as S


def _params(rng, C=4):
    shapes = [(C, 1), (C, C), (C, C), (1, C)]
    return [(rng.normal(0, 0.4, (o, c, 3, 3)), rng.normal(0, 0.1, o)) for o, c in shapes]


def test_conv_matches_scipy_wrap_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 7, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    z = S.conv(x, w, b, iscale=0.7, oscale=1.3)
    for bi in range(2):
        for o in range(4):
            ref = sum(ndimage.correlate(0.7 * x[bi, c], w[o, c], mode="wrap") for c in range(3))
            np.testing.assert_allclose(z[bi, o], 1.3 * (ref + b[o]), atol=1e-12)


def test_bf16_rounding():
    vals = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 1e-3])
    r = S.bf16_round(vals)
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125
    assert abs(r[3] + 3.140625) < 1e-12
    assert abs(r[4] / 1e-3 - 1) < 2 ** -8


@pytest.mark.parametrize("which", ["x", "w0", "b1", "w3", "b3"])
def test_network_gradients_central_differences(which):
    rng = np.random.default_rng(1)
    params = _params(rng)
    x = rng.standard_normal((2, 8, 8))
    t = rng.standard_normal((2, 8, 8)) * 0.1
    s_in, s_out, border = 0.5, 0.3, 1

    def loss(params, x):
        y, _ = S.forward(params, x, s_in, s_out)
        return S.mse(y, t, border)[0]

    y, acts = S.forward(params, x, s_in, s_out)
    _, dy = S.mse(y, t, border)
    dx, grads = S.backward(params, acts, dy, s_in, s_out)
    eps = 1e-6
    for trial in range(4):
        d = {"x": rng.standard_normal(x.shape)}
        if which == "x":
            an = (dx * d["x"]).sum()
            fd = (loss(params, x + eps * d["x"]) - loss(params, x - eps * d["x"])) / (2 * eps)
        else:
            layer, kind = int(which[1]), 0 if which[0] == "w" else 1
            h = rng.standard_normal(params[layer][kind].shape)

            def moved(s):
                p = [list(q) for q in params]
                p[layer][kind] = p[layer][kind] + s * h
                return [tuple(q) for q in p]

            an = (grads[layer][kind] * h).sum()
            fd = (loss(moved(eps), x) - loss(moved(-eps), x)) / (2 * eps)
        assert abs(an - fd) <= 1e-7 * max(abs(fd), 1e-12)


def test_adam_first_step_moves_by_lr():
    """Adam's bias-corrected first step moves each weight by lr * sign(g)."""
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    wn, m, v = S.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(wn, w - 0.01 * np.sign(g), rtol=0, atol=1e-7)
