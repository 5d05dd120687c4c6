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


# -- the encoder-decoder (BF16 MFMA convolutions) ----------------------------
# Layers: ("conv", cin, cout, relu), ("pool",) -- average over 2x2 cells of
# the two long grid axes, ("up",) -- nearest upsampling by two over them.  On
# a 20x20x5 block the three resolutions are 20x20x5, 10x10x5 and 5x5x5.
UNET_LAYERS = (("conv", 2, 24, True), ("conv", 24, 24, True), ("pool",),
               ("conv", 24, 48, True), ("conv", 48, 48, True), ("pool",),
               ("conv", 48, 80, True), ("conv", 80, 80, True), ("up",),
               ("conv", 80, 48, True), ("conv", 48, 48, True), ("up",),
               ("conv", 48, 24, True), ("conv", 24, 1, False))


def _u16(t):
    return t  # packed bfloat16 weights live in int16 tensors


class EncoderDecoder:
    """The learned warm start as an encoder-decoder of 3x3x3 convolutions on
    BF16 matrix cores (FP32 accumulation, FP32 master weights and Adam).
    Inputs [S, D, H, W, 2] (channels last), outputs [S, D, H, W, 1]."""

    def __init__(self, layers=UNET_LAYERS, seed=0, device="cuda", init=None):
        import torch
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.layers = tuple(tuple(L) for L in layers)
        cmax = self.lib.mrcm_unet_max_channels()
        convs = [L for L in self.layers if L[0] == "conv"]
        if any(L[1] > cmax or L[2] > cmax for L in convs):
            raise ValueError(f"at most {cmax} channels per convolution")
        rng = np.random.default_rng(seed)
        self.params = []
        for k, (_, ci, co, _) in enumerate(convs):
            if init is not None:
                w = np.asarray(init[2 * k], dtype=np.float32).reshape(co, ci * 27)
                b = np.asarray(init[2 * k + 1], dtype=np.float32)
            else:
                bound = np.sqrt(6.0 / (27 * ci))
                w = rng.uniform(-bound, bound, size=(co, ci * 27)).astype(np.float32)
                b = np.zeros(co, dtype=np.float32)
            self.params.append(torch.as_tensor(w.reshape(-1), device=self.device).contiguous())
            self.params.append(torch.as_tensor(b, device=self.device).contiguous())
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0
        self.packed = []
        for (_, ci, co, _) in convs:
            pi, po = self.lib.mrcm_unet_padded(ci), self.lib.mrcm_unet_padded(co)
            wf = torch.zeros(po * 27 * pi, dtype=torch.int16, device=self.device)
            wt = torch.zeros(pi * 27 * po, dtype=torch.int16, device=self.device)
            self.packed.append((wf, wt))
        self.loss_buf = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.work = torch.zeros(1024, dtype=torch.float64, device=self.device)
        self._wg = {}
        self.pack()

    def n_params(self):
        return int(sum(p.numel() for p in self.params))

    def pack(self):
        k = 0
        for L in self.layers:
            if L[0] != "conv":
                continue
            wf, wt = self.packed[k]
            _lib.check(self.lib.mrcm_unet_pack(_ptr(self.params[2 * k]), _ptr(wf), _ptr(wt), L[1], L[2], _stream()),
                       "mrcm_unet_pack")
            k += 1

    def forward(self, x, keep=False):
        """x [B, D, H, W, C] float32 -> output [B, D, H, W, 1]; keep: also the
        input of every layer."""
        import torch
        _f32(x, "x")
        B, D, H, W, _ = x.shape
        h = x
        acts = []
        k = 0
        for L in self.layers:
            acts.append(h)
            if L[0] == "conv":
                _, ci, co, relu = L
                y = torch.empty((B, D, H, W, co), dtype=torch.float32, device=self.device)
                _lib.check(self.lib.mrcm_unet_conv(_ptr(h), _ptr(self.packed[k][0]), _ptr(self.params[2 * k + 1]),
                                                   _ptr(y), None, B, D, H, W, ci, co, 1 if relu else 0, _stream()),
                           "mrcm_unet_conv")
                k += 1
            elif L[0] == "pool":
                C = h.shape[-1]
                y = torch.empty((B, D // 2, H // 2, W, C), dtype=torch.float32, device=self.device)
                _lib.check(self.lib.mrcm_unet_pool(_ptr(h), _ptr(y), B, D, H, W, C, 0, _stream()), "mrcm_unet_pool")
                D, H = D // 2, H // 2
            else:
                C = h.shape[-1]
                y = torch.empty((B, 2 * D, 2 * H, W, C), dtype=torch.float32, device=self.device)
                _lib.check(self.lib.mrcm_unet_upsample(_ptr(h), _ptr(y), B, D, H, W, C, 0, _stream()),
                           "mrcm_unet_upsample")
                D, H = 2 * D, 2 * H
            h = y
        return (h, acts) if keep else h

    def _wgrad_work(self, B, D, H, W, ci, co):
        import torch
        n = int(self.lib.mrcm_unet_wgrad_workspace(B, D, H, W, ci, co))
        if n < 0:
            raise ValueError("invalid convolution shape")
        key = "w"
        if key not in self._wg or self._wg[key].numel() < n:
            self._wg[key] = torch.empty(n, dtype=torch.float32, device=self.device)
        return self._wg[key]

    def loss_and_grads(self, x, t):
        """Mean squared error on (x, t) and every parameter's gradient (loss as
        a device scalar: no synchronisation)."""
        import torch
        _f32(t, "t")
        out, acts = self.forward(x, keep=True)
        g = torch.empty_like(out)
        _lib.check(self.lib.mrcm_mse(_ptr(out), _ptr(t), _ptr(g), _ptr(self.loss_buf), _ptr(self.work),
                                     out.numel(), _stream()), "mrcm_mse")
        grads = [None] * len(self.params)
        k = sum(1 for L in self.layers if L[0] == "conv")
        y = out
        for i in reversed(range(len(self.layers))):
            L, a = self.layers[i], acts[i]
            B, D, H, W, C = a.shape
            if L[0] == "conv":
                k -= 1
                _, ci, co, relu = L
                if relu:
                    _lib.check(self.lib.mrcm_unet_relu_mask(_ptr(g), _ptr(y), g.numel(), _stream()),
                               "mrcm_unet_relu_mask")
                dw = torch.empty_like(self.params[2 * k])
                db = torch.empty_like(self.params[2 * k + 1])
                work = self._wgrad_work(B, D, H, W, ci, co)
                _lib.check(self.lib.mrcm_unet_wgrad(_ptr(a), _ptr(g), _ptr(dw), _ptr(db), _ptr(work), B, D, H, W, ci,
                                                    co, _stream()), "mrcm_unet_wgrad")
                grads[2 * k], grads[2 * k + 1] = dw, db
                if i > 0:
                    dx = torch.empty_like(a)
                    _lib.check(self.lib.mrcm_unet_conv(_ptr(g), _ptr(self.packed[k][1]), None, _ptr(dx), None, B, D,
                                                       H, W, co, ci, 0, _stream()), "mrcm_unet_conv")
                    g = dx
            elif L[0] == "pool":
                dx = torch.empty_like(a)
                _lib.check(self.lib.mrcm_unet_pool(_ptr(g), _ptr(dx), B, D, H, W, C, 1, _stream()), "mrcm_unet_pool")
                g = dx
            else:
                dx = torch.empty_like(a)
                _lib.check(self.lib.mrcm_unet_upsample(_ptr(g), _ptr(dx), B, D, H, W, C, 1, _stream()),
                           "mrcm_unet_upsample")
                g = dx
            y = a
        return self.loss_buf, grads

    def adam(self, grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        for p, g, m, v in zip(self.params, grads, self.m, self.v):
            code = self.lib.mrcm_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), self.t, c_float(lr),
                                           c_float(b1), c_float(b2), c_float(eps), _stream())
            _lib.check(code, "mrcm_adam_step")
        self.pack()

    def train(self, inp, tgt, epochs=4, batch=128, lr=1e-3, seed=0, lr_decay=0.7):
        """Mini-batch Adam over the samples (shuffled each epoch with a seeded
        generator, the step size scaled by lr_decay after each epoch);
        returns the mean loss of each epoch."""
        import torch
        n = inp.shape[0]
        rng = np.random.default_rng(seed)
        history = []
        for ep in range(epochs):
            order = torch.as_tensor(rng.permutation(n), device=self.device)
            total = torch.zeros(1, dtype=torch.float64, device=self.device)
            nb = 0
            for s in range(0, n - batch + 1, batch):
                idx = order[s:s + batch]
                xb = inp.index_select(0, idx).contiguous()
                tb = tgt.index_select(0, idx).contiguous()
                loss, grads = self.loss_and_grads(xb, tb)
                total += loss
                nb += 1
                self.adam(grads, lr * lr_decay ** ep)
            history.append(float(total.item()) / max(1, nb))
        return history

    def predict(self, inp, batch=2048):
        import torch
        outs = [self.forward(inp[s:s + batch]) for s in range(0, inp.shape[0], batch)]
        return torch.cat(outs, 0)


def channels_last(x):
    """[S, C, D, H, W] -> [S, D, H, W, C] by the library's permute kernel."""
    import torch
    S, C = x.shape[0], x.shape[1]
    V = int(np.prod(x.shape[2:]))
    y = torch.empty((S,) + tuple(x.shape[2:]) + (C,), dtype=torch.float32, device=x.device)
    _lib.check(_lib.load().mrcm_nn_channels_last(_ptr(x), _ptr(y), S, C, V, _stream()), "mrcm_nn_channels_last")
    return y


def warm_start_unet(model, net, subs, dims, x0=None, chunk=2048):
    """Starting guess in the MBF layout from the encoder-decoder, `chunk`
    subdomains at a time."""
    import torch
    lib = _lib.load()
    if x0 is None:
        x0 = torch.zeros(model.mbf_layout()[-1], dtype=torch.float64, device=model.device)
    for c0 in range(0, len(subs), chunk):
        part = subs[c0:c0 + chunk]
        inp, _ = features(model, part, dims, targets=False)
        out = net.predict(channels_last(inp))
        del inp
        arr = (c_int32 * len(part))(*part)
        code = lib.mrcm_nn_scatter(model._mbfs, arr, len(part), _ptr(out), _ptr(x0), _stream())
        _lib.check(code, "mrcm_nn_scatter")
        del out
    return x0


def mbf_dataset(seeds, per_field=50, make_case=None):
    """Training or test samples: for each seed, the channelised field of
    `make_case(seed)` built by the FP64 direct path, and `per_field` of its
    MBF columns (particular columns excluded) drawn with default_rng(seed);
    returns channels-last inputs [S, D, H, W, 2], unit-RMS targets
    [S, D, H, W, 1] and the grid."""
    import torch
    from . import MRCM, FP64
    if make_case is None:
        from mrcm_inputs import config4_field
        make_case = config4_field
    inps, tgts = [], []
    dims = None
    for seed in seeds:
        c = make_case(seed)
        pb = c.problem
        m = MRCM(pb, c.partition, c.iface, alpha=c.alpha, precision=FP64)
        m.build_mbfs(*(torch.as_tensor(a, dtype=torch.float64, device="cuda") for a in (pb.kx, pb.ky, pb.kz, pb.q)))
        subs, dims = net_subdomains(m)
        inp, tgt = features(m, subs, dims)
        # MBF columns only: column 0 of each subdomain is the particular problem
        cols, s0 = [], 0
        for l in subs:
            mr = m.subdomain(l).n_rhs
            cols += list(range(s0 + 1, s0 + mr))
            s0 += mr
        pick = np.random.default_rng(seed).choice(cols, size=min(per_field, len(cols)), replace=False)
        idx = torch.as_tensor(np.sort(pick), device=inp.device)
        inps.append(channels_last(inp.index_select(0, idx).contiguous()))
        tgts.append(tgt.index_select(0, idx).contiguous())
        m.close()
    return torch.cat(inps), torch.cat(tgts), dims
