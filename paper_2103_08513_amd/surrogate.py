"""Learned warm start for the conjugate-gradient local solves (include/mrcm_nn.h).

A small 3D convolutional network (3x3x3 convolutions with growing dilation,
zero padding, a ReLU after all but the last, so that the receptive field
spans a 20x20x5 block) maps each right-hand-side column of a subdomain -- its centred
log-permeability and its right-hand side scaled to a largest magnitude of
one -- to the column's solution up to scale.  It is trained on the MBFs the
library itself builds, and its output starts the conjugate gradients of
``MRCM(precision=PCG)`` (with the Galerkin scaling ``pcg_x0_scale``).

Every operation runs in the library's kernels: this module allocates the
parameters, activations and optimiser state as torch device tensors and
passes them to the C ABI.  The initial weights are drawn from a seeded
generator (He-uniform) and are inputs to the kernels.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_float, c_int32, c_void_p

import numpy as np

from . import _lib
from ._lib import CInfo


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _f32(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32 \
            or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor on the HIP device")
    return t


class WarmStartNet:
    """Network, Adam state and the calls that train and apply it."""

    def __init__(self, channels=(2, 12, 12, 12, 1), dilations=(1, 2, 4, 1), seed=0, device="cuda"):
        import torch
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.channels = tuple(int(c) for c in channels)
        cmax = self.lib.mrcm_conv3d_max_channels()
        if self.channels[0] != 2 or self.channels[-1] != 1 or max(self.channels) > cmax:
            raise ValueError(f"channels must run from 2 to 1 with at most {cmax} per layer")
        self.dilations = tuple(int(d) for d in dilations)
        if len(self.dilations) != len(self.channels) - 1 or min(self.dilations) < 1:
            raise ValueError("one dilation (>= 1) per layer")
        rng = np.random.default_rng(seed)
        self.params = []
        for ci, co in zip(self.channels[:-1], self.channels[1:]):
            bound = np.sqrt(6.0 / (27 * ci))
            w = rng.uniform(-bound, bound, size=(co, ci, 3, 3, 3)).astype(np.float32)
            self.params.append(torch.as_tensor(w, device=self.device))
            self.params.append(torch.zeros(co, dtype=torch.float32, device=self.device))
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0
        self.loss_buf = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.work = torch.zeros(1024, dtype=torch.float64, device=self.device)
        self.wt = torch.zeros(max(self.channels) ** 2 * 27, dtype=torch.float32, device=self.device)

    @property
    def n_layers(self):
        return len(self.channels) - 1

    def n_params(self):
        return int(sum(p.numel() for p in self.params))

    # -- forward and backward ---------------------------------------------
    def forward(self, x, dims, keep=False):
        """x [B, 2, D, H, W] float32 -> output [B, 1, D, H, W]; keep: also
        return every layer's input (for backward)."""
        import torch
        _f32(x, "x")
        B = x.shape[0]
        d, h, w = dims
        acts = [x]
        for i in range(self.n_layers):
            ci, co = self.channels[i], self.channels[i + 1]
            y = torch.empty((B, co, d, h, w), dtype=torch.float32, device=self.device)
            code = self.lib.mrcm_conv3d_forward(_ptr(acts[-1]), _ptr(self.params[2 * i]),
                                                _ptr(self.params[2 * i + 1]), _ptr(y), None, B, ci, co, d, h, w,
                                                self.dilations[i], 1 if i < self.n_layers - 1 else 0, _stream())
            _lib.check(code, "mrcm_conv3d_forward")
            acts.append(y)
        return (acts[-1], acts) if keep else acts[-1]

    def loss_and_grads(self, x, t, dims):
        """Mean squared error on (x, t) and the gradients of every parameter
        (loss as a device scalar: no synchronisation)."""
        import torch
        _f32(t, "t")
        out, acts = self.forward(x, dims, keep=True)
        B = x.shape[0]
        d, h, w = dims
        dy = torch.empty_like(out)
        _lib.check(self.lib.mrcm_mse(_ptr(out), _ptr(t), _ptr(dy), _ptr(self.loss_buf), _ptr(self.work),
                                     out.numel(), _stream()), "mrcm_mse")
        grads = [torch.empty_like(p) for p in self.params]
        for i in reversed(range(self.n_layers)):
            ci, co = self.channels[i], self.channels[i + 1]
            dx = torch.empty_like(acts[i]) if i > 0 else None
            mask = acts[i] if i > 0 else None
            code = self.lib.mrcm_conv3d_backward(_ptr(acts[i]), _ptr(self.params[2 * i]), _ptr(dy), _ptr(dx),
                                                 _ptr(grads[2 * i]), _ptr(grads[2 * i + 1]), _ptr(self.wt),
                                                 _ptr(mask), B, ci, co, d, h, w, self.dilations[i], _stream())
            _lib.check(code, "mrcm_conv3d_backward")
            dy = dx
        return self.loss_buf, grads

    def adam(self, grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        for p, g, m, v in zip(self.params, grads, self.m, self.v):
            code = self.lib.mrcm_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), self.t, c_float(lr),
                                           c_float(b1), c_float(b2), c_float(eps), _stream())
            _lib.check(code, "mrcm_adam_step")

    def train(self, inp, tgt, dims, epochs=4, batch=256, lr=2e-3, seed=0):
        """Mini-batch Adam over the samples (shuffled each epoch with a seeded
        generator); returns the mean loss of each epoch."""
        import torch
        n = inp.shape[0]
        rng = np.random.default_rng(seed)
        history = []
        for _ in range(epochs):
            order = torch.as_tensor(rng.permutation(n), device=self.device)
            total = torch.zeros(1, dtype=torch.float64, device=self.device)
            nb = 0
            for s in range(0, n, batch):
                idx = order[s:s + batch]
                xb = inp.index_select(0, idx).contiguous()
                tb = tgt.index_select(0, idx).contiguous()
                loss, grads = self.loss_and_grads(xb, tb, dims)
                total += loss
                nb += 1
                self.adam(grads, lr)
            history.append(float(total.item()) / nb)
        return history

    def predict(self, inp, dims, batch=1024):
        import torch
        outs = [self.forward(inp[s:s + batch], dims) for s in range(0, inp.shape[0], batch)]
        return torch.cat(outs, 0)


# -- data exchange with an MBF handle ------------------------------------------
def net_subdomains(model):
    """The subdomains of the handle's most common grid (n2, n1, n0), and that grid."""
    from collections import Counter
    info = model.info()
    shapes = []
    for l in range(info.n_sub):
        si = model.subdomain(l)
        shapes.append((si.ext[si.ax[2]], si.ext[si.ax[1]], si.ext[si.ax[0]]))
    grid = Counter(shapes).most_common(1)[0][0]
    return [l for l in range(info.n_sub) if shapes[l] == grid], grid


def features(model, subs, dims, targets=True):
    """Inputs [S, 2, D, H, W] (and unit-RMS targets [S, 1, D, H, W]) of every
    column of the listed subdomains, from the handle's current build."""
    import torch
    lib = _lib.load()
    n = sum(model.subdomain(l).n_rhs for l in subs)
    inp = torch.empty((n, 2) + tuple(dims), dtype=torch.float32, device=model.device)
    tgt = torch.empty((n, 1) + tuple(dims), dtype=torch.float32, device=model.device) if targets else None
    arr = (c_int32 * len(subs))(*subs)
    code = lib.mrcm_nn_features(model._mbfs, arr, len(subs), _ptr(inp), _ptr(tgt), _stream())
    _lib.check(code, "mrcm_nn_features")
    return inp, tgt


def warm_start(model, net, subs, dims, x0=None, chunk=4096):
    """Starting guess in the MBF layout from the network (zero for
    subdomains not listed), `chunk` subdomains at a time so that the
    network's inputs and outputs stay a few GB at any workload size."""
    import torch
    lib = _lib.load()
    if x0 is None:
        x0 = torch.zeros(model.mbf_layout()[-1], dtype=torch.float64, device=model.device)
    for c0 in range(0, len(subs), chunk):
        part = subs[c0:c0 + chunk]
        inp, _ = features(model, part, dims, targets=False)
        out = net.predict(inp, dims)
        arr = (c_int32 * len(part))(*part)
        code = lib.mrcm_nn_scatter(model._mbfs, arr, len(part), _ptr(out), _ptr(x0), _stream())
        _lib.check(code, "mrcm_nn_scatter")
        del inp, out
    return x0
