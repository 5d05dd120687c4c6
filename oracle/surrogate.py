"""Oracle of the learned warm start for the conjugate-gradient local solves.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU baseline, never by the library.

The network maps, per right-hand-side column of a subdomain, two channels on
the subdomain's cell grid to one: the centred log-permeability and the column's
right-hand side scaled to a largest magnitude of one, to the column's solution
(an MBF of (2.25) or the particular solution of (2.26)) scaled to unit root
mean square.  Everything here is the plain definition, in float64 on the CPU:

* conv3d: zero-padded 3x3x3 cross-correlation with bias and dilation d (taps
  at offsets -d, 0, +d), the convolution of deep-learning libraries
  (torch.nn.functional.conv3d is the step);
* the network: convolutions with a ReLU after every one but the last;
* the loss: mean squared error over all outputs;
* gradients: reverse-mode differentiation of that composition (torch
  autograd as the step);
* Adam (Kingma and Ba, 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

The grid layout is the library's local row order: the box's axes sorted by
extent, shortest first, ties by lower axis id; row r = t0 + n0 (t1 + n1 t2);
a column is viewed as an array [n2][n1][n0] (D, H, W).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def conv3d(x, w, b, dil=1):
    """x [B, Cin, D, H, W], w [Cout, Cin, 3, 3, 3], b [Cout] -> [B, Cout, D, H, W]."""
    x = torch.as_tensor(x, dtype=torch.float64)
    w = torch.as_tensor(w, dtype=torch.float64)
    b = torch.as_tensor(b, dtype=torch.float64)
    return F.conv3d(x, w, b, padding=dil, dilation=dil)


def net_forward(params, x, dils=None):
    """params: [w0, b0, w1, b1, ...]; dils: dilation per layer (default 1);
    ReLU after every layer but the last."""
    h = torch.as_tensor(x, dtype=torch.float64)
    n = len(params) // 2
    dils = dils or [1] * n
    for i in range(n):
        h = conv3d(h, params[2 * i], params[2 * i + 1], dils[i])
        if i < n - 1:
            h = torch.relu(h)
    return h


def loss_and_grads(params, x, t, dils=None):
    """Mean squared error of the network on (x, t) and its gradients."""
    ps = [torch.tensor(np.asarray(p), dtype=torch.float64, requires_grad=True) for p in params]
    y = net_forward(ps, x, dils)
    tt = torch.as_tensor(t, dtype=torch.float64)
    loss = torch.mean((y - tt) ** 2)
    loss.backward()
    return float(loss.detach()), [p.grad.numpy().copy() for p in ps], y.detach().numpy()


def layer_grads(x, w, b, dy, dil=1):
    """Gradients of one convolution: dL/dx, dL/dw, dL/db given dL/dy."""
    xt = torch.tensor(np.asarray(x), dtype=torch.float64, requires_grad=True)
    wt = torch.tensor(np.asarray(w), dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(np.asarray(b), dtype=torch.float64, requires_grad=True)
    y = conv3d(xt, wt, bt, dil)
    y.backward(torch.as_tensor(dy, dtype=torch.float64))
    return xt.grad.numpy(), wt.grad.numpy(), bt.grad.numpy()


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def local_order(lo, ext):
    """Global (x, y, z) of every local row of a box, in the library's order."""
    ax = sorted(range(3), key=lambda d: (ext[d], d))
    n0, n1, n2 = ext[ax[0]], ext[ax[1]], ext[ax[2]]
    out = np.zeros((n0 * n1 * n2, 3), dtype=np.int64)
    r = 0
    for t2 in range(n2):
        for t1 in range(n1):
            for t0 in range(n0):
                c = [0, 0, 0]
                c[ax[0]] = lo[ax[0]] + t0
                c[ax[1]] = lo[ax[1]] + t1
                c[ax[2]] = lo[ax[2]] + t2
                out[r] = c
                r += 1
    return out, (n2, n1, n0)


def features_and_targets(pb, ls, lo, ext, X=None):
    """Network input [m, 2, D, H, W] for every column of one subdomain, and
    (when the columns' solutions X [N_l, m] in the oracle's row order, x
    fastest, are given) the unit-RMS targets [m, 1, D, H, W]."""
    coords, dhw = local_order(lo, ext)
    nx, ny = pb.nx, pb.ny
    gidx = coords[:, 0] + nx * (coords[:, 1] + ny * coords[:, 2])
    # the oracle's local rows run x fastest within the box
    lx = coords[:, 0] - lo[0] + ext[0] * ((coords[:, 1] - lo[1]) + ext[1] * (coords[:, 2] - lo[2]))
    logk = np.log(pb.kx[gidx])
    logk = logk - logk.mean()
    R = ls.R[lx]
    m = R.shape[1]
    inp = np.zeros((m, 2) + dhw)
    tgt = None if X is None else np.zeros((m, 1) + dhw)
    for c in range(m):
        inp[c, 0] = logk.reshape(dhw)
        s = np.max(np.abs(R[:, c]))
        inp[c, 1] = (R[:, c] / s if s > 0 else 0.0 * R[:, c]).reshape(dhw)
        if X is not None:
            x = X[lx, c]
            rms = np.sqrt(np.mean(x * x))
            tgt[c, 0] = (x / rms if rms > 0 else 0.0 * x).reshape(dhw)
    return inp, tgt


# ---------------------------------------------------------------------------
# The encoder-decoder of the learned warm start, with BF16 operands.
#
# Layers (a list of tuples): ("conv", cin, cout, relu) -- a zero-padded
# 3x3x3 convolution with bias; ("pool",) -- the average of 2x2 cells over the
# two leading grid axes (D, H); ("up",) -- nearest-neighbour upsampling by two
# over the same axes.  Every convolution rounds its input and its weights to
# bfloat16 (round to nearest, ties to even, from the float32 value) and sums
# the products exactly here (float64); the result, the bias, the ReLU and
# every other tensor stay unrounded.  The backward pass is the exact gradient
# of that computation with the roundings passed straight through: for a
# convolution y = conv(r(x), r(w)) + b with upstream gradient g (after the
# ReLU mask),
#   dL/dw = correlation of g with r(x),  dL/db = sum of g,
#   dL/dx = transposed convolution of r(g) with r(w),
# where r rounds to bfloat16.
# ---------------------------------------------------------------------------

def bf16(a):
    """Round to bfloat16 (nearest, ties to even) via the float32 value,
    returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(a):
    """The float32 value of a (what the GPU stores between layers)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def pool2(x):
    """Average over 2x2 cells of the (D, H) axes of [B, C, D, H, W]."""
    return F.avg_pool3d(torch.as_tensor(x, dtype=torch.float64), kernel_size=(2, 2, 1))


def up2(x):
    """Nearest-neighbour upsampling by two over (D, H) of [B, C, D, H, W]."""
    return F.interpolate(torch.as_tensor(x, dtype=torch.float64), scale_factor=(2, 2, 1), mode="nearest")


def unet_params(layers, seed):
    """Seeded initial parameters (He-uniform weights, zero biases): one
    (w [cout, cin, 3, 3, 3], b [cout]) per convolution, float32 values."""
    rng = np.random.default_rng(seed)
    ps = []
    for L in layers:
        if L[0] != "conv":
            continue
        _, ci, co, _ = L
        bound = np.sqrt(6.0 / (27 * ci))
        ps.append(f32(rng.uniform(-bound, bound, size=(co, ci, 3, 3, 3))))
        ps.append(np.zeros(co))
    return ps


def unet_forward(layers, params, x, rounding=True):
    """Network output and every layer's input (for the backward pass).
    rounding=False drops the bfloat16 roundings (the exact float64 network)."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    h = np.asarray(x, dtype=np.float64)
    acts = []
    k = 0
    for L in layers:
        acts.append(h)
        if L[0] == "conv":
            w, b = params[2 * k], params[2 * k + 1]
            k += 1
            h = conv3d(r(h), r(w), b).numpy()
            if L[3]:
                h = np.maximum(h, 0.0)
        elif L[0] == "pool":
            h = pool2(h).numpy()
        else:
            h = up2(h).numpy()
    return h, acts


def unet_loss_and_grads(layers, params, x, t, rounding=True):
    """Mean squared error of the network on (x, t) and the gradients of
    every parameter, by the backward pass stated above."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    y, acts = unet_forward(layers, params, x, rounding)
    t = np.asarray(t, dtype=np.float64)
    loss = float(np.mean((y - t) ** 2))
    g = 2.0 * (y - t) / y.size
    grads = [None] * len(params)
    k = sum(1 for L in layers if L[0] == "conv")
    out = y
    for i in reversed(range(len(layers))):
        L, a = layers[i], acts[i]
        if L[0] == "conv":
            k -= 1
            w = params[2 * k]
            if L[3]:
                g = g * (out > 0.0)
            xr = torch.tensor(r(a), dtype=torch.float64, requires_grad=True)
            wr = torch.tensor(r(w), dtype=torch.float64, requires_grad=True)
            y_ = F.conv3d(xr, wr, None, padding=1)
            y_.backward(torch.as_tensor(g, dtype=torch.float64))
            grads[2 * k] = wr.grad.numpy()
            grads[2 * k + 1] = g.sum(axis=(0, 2, 3, 4))
            # dL/dx from the rounded upstream gradient and rounded weights
            xs = torch.zeros(a.shape, dtype=torch.float64, requires_grad=True)
            y2 = F.conv3d(xs, torch.as_tensor(r(w), dtype=torch.float64), None, padding=1)
            y2.backward(torch.as_tensor(r(g), dtype=torch.float64))
            g = xs.grad.numpy()
        elif L[0] == "pool":
            xs = torch.zeros(a.shape, dtype=torch.float64, requires_grad=True)
            pool2(xs).backward(torch.as_tensor(g, dtype=torch.float64))
            g = xs.grad.numpy()
        else:
            xs = torch.zeros(a.shape, dtype=torch.float64, requires_grad=True)
            up2(xs).backward(torch.as_tensor(g, dtype=torch.float64))
            g = xs.grad.numpy()
        out = a
    return loss, grads, y
