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


def test_adam_second_moment_decay_closed_form():
    """Two steps with gradients g then 2g: the bias-corrected moments are the
    normalised exponentially weighted sums m^ = (b1 g + 2g)(1 - b1)/(1 - b1^2)
    = (b1 + 2) g/(1 + b1) and v^ = (b2 + 4) g^2/(1 + b2), so the second move
    is lr (b1 + 2)/(1 + b1) sqrt((1 + b2)/(b2 + 4)) sign(g); it depends on b2
    (with b1 in its place the move differs by 1.5%)."""
    b1, b2, lr, eps = 0.9, 0.999, 0.01, 1e-8
    g = np.array([0.3, -4.0, 2.5e-3, 7.0])
    w0 = np.array([1.0, -2.0, 0.5, 0.0])
    w1, m, v = S.adam(w0, g, np.zeros(4), np.zeros(4), 1, lr)
    w2, m, v = S.adam(w1, 2.0 * g, m, v, 2, lr)
    move = lr * (b1 + 2.0) / (1.0 + b1) * np.sqrt((1.0 + b2) / (b2 + 4.0))
    np.testing.assert_allclose(w1 - w2, move * np.sign(g), rtol=1e-5, atol=0)
    # the raw moments are the weighted sums themselves
    np.testing.assert_allclose(m, (1 - b1) * (b1 * g + 2.0 * g), rtol=1e-14)
    np.testing.assert_allclose(v, (1 - b2) * (b2 * g * g + 4.0 * g * g), rtol=1e-14)
    # a third step back to g: v^ = (b2^2 + 4 b2 + 1) g^2 (1 - b2)/(1 - b2^3)
    w3, m, v = S.adam(w2, g, m, v, 3, lr)
    mh = (b1 * b1 + 2.0 * b1 + 1.0) * (1 - b1) / (1 - b1 ** 3)
    vh = (b2 * b2 + 4.0 * b2 + 1.0) * (1 - b2) / (1 - b2 ** 3)
    np.testing.assert_allclose(w2 - w3, lr * mh / np.sqrt(vh) * np.sign(g), rtol=1e-5, atol=0)


def test_mse_counts_interior_pixels_only():
    """Hand case: B = 2 fields of 6 x 7 with a border of 2 leave 2 x 3
    interior pixels each, n = 12.  A unit error on every interior pixel of
    the first field and errors of 5 on border pixels give loss 6/12 and
    gradient 2/12 inside, 0 on the border and in the second field."""
    pred = np.zeros((2, 6, 7))
    pred[0, 2:4, 2:5] = 1.0
    pred[0, 0, :] = 5.0
    pred[1, :, 6] = -5.0
    pred[1, 5, 3] = 5.0
    loss, g = S.mse(pred, np.zeros_like(pred), border=2)
    assert loss == 0.5
    want = np.zeros_like(pred)
    want[0, 2:4, 2:5] = 2.0 / 12.0
    np.testing.assert_array_equal(g, want)


@pytest.mark.parametrize("B,H,W", [(3, 24, 20), (2, 37, 45)])
def test_storage_noise_model_matches_round_to_nearest(B, H, W):
    """The BF16 storage budget's noise model (independent uniform errors of
    half a bfloat16 spacing at each stored hidden activation and gradient)
    predicts the deviation of the deterministic round-to-nearest network
    from the unrounded one: their ratio is close to 1 for the output, the
    input gradient and every weight gradient (each a sum of many errors),
    and within a factor 2 for the bias gradients (sums over few channels)."""
    rng = np.random.default_rng(B * 7 + H)
    shapes = [(32, 1), (32, 32), (32, 32), (1, 32)]
    params = [(S.bf16_round(rng.normal(0, 1 / np.sqrt(9 * c), (o, c, 3, 3))),
               rng.normal(0, 0.1, o)) for o, c in shapes]
    x = rng.normal(0, 3.0, (B, H, W))
    dy = rng.standard_normal((B, H, W))
    exact, sigma = S.storage_noise_budget(params, x, 0.2, 0.1, dy=dy, samples=8, seed=3)
    y, acts = S.forward(params, x, 0.2, 0.1, bf16=True)
    dx, grads = S.backward(params, acts, dy, 0.2, 0.1, bf16=True)
    det = {"y": y, "dx": dx}
    for k, (dw, db) in enumerate(grads):
        det[f"dW{k}"], det[f"db{k}"] = dw, db
    for k, v in det.items():
        d = np.linalg.norm(v - exact[k])
        if k == "db3":  # s_out * sum(dy): nothing stored on its path
            assert d == 0.0 and sigma[k] == 0.0
            continue
        lo, hi = (0.5, 2.0) if k.startswith("db") else (0.7, 1.4)
        assert lo * sigma[k] <= d <= hi * sigma[k], (k, d / sigma[k])
    # BF16 storage costs about 2^-8 relative on every output
    rel = np.linalg.norm(y - exact["y"]) / np.linalg.norm(exact["y"])
    assert 5e-4 < rel < 1e-2


def test_bf16_ulp():
    a = np.array([1.0, 1.5, 0.75, -3.0, 0.0, 2.0 ** -20])
    np.testing.assert_array_equal(S.bf16_ulp(a), [2.0 ** -7, 2.0 ** -7, 2.0 ** -8, 2.0 ** -6,
                                                  0.0, 2.0 ** -27])
    # every bfloat16 rounding error is within half a spacing
    x = np.random.default_rng(0).normal(0, 10, 10000)
    assert np.all(np.abs(S.bf16_round(x) - x) <= 0.5 * S.bf16_ulp(x))
