"""Pins of the learned-warm-start oracle (oracle/surrogate.py) against what
the definitions fix, independent of the library used inside it:
  * the 3x3x3 zero-padded cross-correlation against explicit loops;
  * reverse-mode gradients of the network and of one layer against central
    finite differences;
  * Adam's first two steps against the update written out by hand;
  * the local row order against the rule stated in include/mrcm.h.
"""
import numpy as np
import pytest

pytest.importorskip("torch")

from oracle.surrogate import adam_step, conv3d, layer_grads, local_order, loss_and_grads, net_forward  # noqa: E402


def _brute_conv(x, w, b, dil=1):
    B, Ci, D, H, W = x.shape
    Co = w.shape[0]
    y = np.zeros((B, Co, D, H, W))
    for n in range(B):
        for o in range(Co):
            for z in range(D):
                for yy in range(H):
                    for xx in range(W):
                        s = b[o]
                        for i in range(Ci):
                            for kd in range(3):
                                for kh in range(3):
                                    for kw in range(3):
                                        zi, yi, xi = z + dil * (kd - 1), yy + dil * (kh - 1), xx + dil * (kw - 1)
                                        if 0 <= zi < D and 0 <= yi < H and 0 <= xi < W:
                                            s += w[o, i, kd, kh, kw] * x[n, i, zi, yi, xi]
                        y[n, o, z, yy, xx] = s
    return y


def test_conv3d_is_the_zero_padded_cross_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 2, 3, 4, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    assert np.allclose(conv3d(x, w, b).numpy(), _brute_conv(x, w, b), rtol=1e-13, atol=1e-13)
    x = rng.standard_normal((1, 2, 5, 4, 6))
    assert np.allclose(conv3d(x, w, b, 2).numpy(), _brute_conv(x, w, b, 2), rtol=1e-13, atol=1e-13)


def _params(rng, ch):
    ps = []
    for ci, co in zip(ch[:-1], ch[1:]):
        ps.append(rng.standard_normal((co, ci, 3, 3, 3)) * 0.3)
        ps.append(rng.standard_normal(co) * 0.1)
    return ps


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    ps = _params(rng, (2, 3, 3, 1))
    x = rng.standard_normal((2, 2, 3, 3, 4))
    t = rng.standard_normal((2, 1, 3, 3, 4))
    dils = [1, 2, 1]
    loss, grads, _ = loss_and_grads(ps, x, t, dils)

    def L(qs):
        y = net_forward(qs, x, dils).numpy()
        return np.mean((y - t) ** 2)

    assert abs(loss - L(ps)) < 1e-14
    h = 1e-6
    for k, p in enumerate(ps):
        flat = p.reshape(-1)
        for j in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            qp = [q.copy() for q in ps]
            qm = [q.copy() for q in ps]
            qp[k].reshape(-1)[j] += h
            qm[k].reshape(-1)[j] -= h
            fd = (L(qp) - L(qm)) / (2 * h)
            assert abs(fd - grads[k].reshape(-1)[j]) <= 1e-6 * max(1.0, abs(fd)), (k, j)


def test_layer_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 2, 2, 3, 3))
    w = rng.standard_normal((2, 2, 3, 3, 3))
    b = rng.standard_normal(2)
    dy = rng.standard_normal((1, 2, 2, 3, 3))
    dx, dw, db = layer_grads(x, w, b, dy)

    def f(xx, ww, bb):
        return float(np.sum(conv3d(xx, ww, bb).numpy() * dy))

    h = 1e-6
    for j in range(0, x.size, 5):
        xp, xm = x.copy(), x.copy()
        xp.reshape(-1)[j] += h
        xm.reshape(-1)[j] -= h
        assert abs((f(xp, w, b) - f(xm, w, b)) / (2 * h) - dx.reshape(-1)[j]) < 1e-6
    for j in range(0, w.size, 7):
        wp, wm = w.copy(), w.copy()
        wp.reshape(-1)[j] += h
        wm.reshape(-1)[j] -= h
        assert abs((f(x, wp, b) - f(x, wm, b)) / (2 * h) - dw.reshape(-1)[j]) < 1e-6
    assert np.allclose(db, dy.sum(axis=(0, 2, 3, 4)), rtol=1e-14)


def test_adam_first_two_steps_by_hand():
    p = np.array([1.0, -2.0, 0.5])
    g1 = np.array([0.3, -0.1, 0.0])
    g2 = np.array([-0.2, 0.4, 1.0])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    p1, m1, v1 = adam_step(p, g1, np.zeros(3), np.zeros(3), 1, lr, b1, b2, eps)
    # step 1: the bias-corrected moments are g and g^2
    assert np.allclose(p1, p - lr * g1 / (np.abs(g1) + eps), rtol=1e-15, atol=1e-15)
    p2, _, _ = adam_step(p1, g2, m1, v1, 2, lr, b1, b2, eps)
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    mh, vh = m / (1 - 0.81), v / (1 - 0.999 ** 2)
    assert np.allclose(p2, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=1e-14, atol=1e-15)


def test_local_order_follows_the_stated_rule():
    # extents (4, 4, 2): z shortest, then x before y (tie broken by lower axis id)
    coords, dhw = local_order((10, 20, 30), (4, 4, 2))
    assert dhw == (4, 4, 2)
    assert tuple(coords[0]) == (10, 20, 30)
    assert tuple(coords[1]) == (10, 20, 31)   # t0 runs along z
    assert tuple(coords[2]) == (11, 20, 30)   # then x
    assert tuple(coords[8]) == (10, 21, 30)   # then y
    assert len({tuple(c) for c in coords}) == 32


# ------------------------------------------------- the encoder-decoder -----
from oracle.surrogate import bf16, pool2, unet_forward, unet_loss_and_grads, unet_params, up2  # noqa: E402

SMALL = [("conv", 2, 3, True), ("pool",), ("conv", 3, 4, True), ("conv", 4, 4, True), ("up",),
         ("conv", 4, 3, True), ("conv", 3, 1, False)]


def test_bf16_rounding_is_round_to_nearest_even():
    """Against the float32 -> bfloat16 conversion of torch (round to nearest,
    ties to even), on random values and on exact ties."""
    import torch
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000)).astype(np.float32)
    assert np.array_equal(bf16(x), torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy())
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even significand (1)
    assert bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def test_pool_and_upsampling_by_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 4, 6, 5))
    p = pool2(x).numpy()
    for d in range(2):
        for h in range(3):
            want = 0.25 * (x[:, :, 2 * d, 2 * h] + x[:, :, 2 * d + 1, 2 * h] + x[:, :, 2 * d, 2 * h + 1]
                           + x[:, :, 2 * d + 1, 2 * h + 1])
            assert np.allclose(p[:, :, d, h], want, rtol=1e-14, atol=1e-14)
    u = up2(p).numpy()
    for d in range(4):
        for h in range(6):
            assert np.array_equal(u[:, :, d, h], p[:, :, d // 2, h // 2])


def test_encoder_decoder_gradients_match_finite_differences():
    """The backward pass of the encoder-decoder (convolutions, ReLUs, pooling,
    upsampling) without the bfloat16 roundings, against central differences
    of the loss."""
    rng = np.random.default_rng(2)
    ps = unet_params(SMALL, 3)
    ps = [p + 0.05 * rng.standard_normal(p.shape) for p in ps]  # nonzero biases
    x = rng.standard_normal((2, 2, 4, 4, 3))
    t = rng.standard_normal((2, 1, 4, 4, 3))
    _, g, _ = unet_loss_and_grads(SMALL, ps, x, t, rounding=False)
    eps = 1e-6
    for k in range(len(ps)):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in ps[k].shape)
            pp = [p.copy() for p in ps]
            pp[k][idx] += eps
            lp = unet_loss_and_grads(SMALL, pp, x, t, rounding=False)[0]
            pp[k][idx] -= 2 * eps
            lm = unet_loss_and_grads(SMALL, pp, x, t, rounding=False)[0]
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_roundings_change_nothing_on_bf16_values_of_one_layer():
    """With inputs and weights already bfloat16 numbers, one convolution's
    rounded forward pass and parameter gradients equal the exact ones (the
    roundings pass straight through)."""
    rng = np.random.default_rng(4)
    layers = [("conv", 2, 3, False)]
    w = bf16(0.3 * rng.standard_normal((3, 2, 3, 3, 3)))
    b = rng.standard_normal(3)
    x = bf16(rng.standard_normal((2, 2, 3, 4, 5)))
    t = rng.standard_normal((2, 3, 3, 4, 5))
    l0, g0, y0 = unet_loss_and_grads(layers, [w, b], x, t, rounding=False)
    l1, g1, y1 = unet_loss_and_grads(layers, [w, b], x, t, rounding=True)
    assert np.array_equal(y0, y1) and l0 == l1
    assert all(np.array_equal(a, c) for a, c in zip(g0, g1))
    y, _ = unet_forward(layers, [w, b], x)
    assert np.allclose(y, conv3d(x, w, b).numpy(), rtol=1e-14, atol=1e-14)
