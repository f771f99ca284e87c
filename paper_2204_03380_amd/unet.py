"""Learned crosstalk filter: a 3-D U-Net on the library's kernels.

A single-realisation random-boundary RTM image carries crosstalk from waves
scattered by the random boundary; it is uncorrelated between realisations of
the boundary (different seeds), so the average over many realisations keeps
the image and loses the crosstalk.  The network learns the map from one
realisation to that average.  It is a project extension of the method; the
images come from the library's own RTM (Eq. (3) with wavefield
reconstruction).

Every layer runs in librtm's kernels (include/unet.h): bfloat16 MFMA
convolutions with float32 accumulation, pooling, upsampling, ReLU gradient,
loss and Adam.  This module only allocates torch buffers and sequences the
calls.  Architecture (16/32/64/128 channels, one 3x3x3 convolution per level,
additive skips, residual output):

    e1 = relu(c1(x))          e2 = relu(c2(pool e1))     e3 = relu(c3(pool e2))
    e4 = relu(c4(pool e3))    d3 = relu(c5(up e4)) + e3  d2 = relu(c6(up d3)) + e2
    d1 = relu(c7(up d2)) + e1 out = x + c8(d1)

The one-channel input and output layers (c1: 1 -> 16, c8: 16 -> 1) run in
the library's vector-unit kernels for those channel pairs.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import UnetConvDesc, check, load

LAYERS = (("c1", 1, 16), ("c2", 16, 32), ("c3", 32, 64), ("c4", 64, 128),
          ("c5", 128, 64), ("c6", 64, 32), ("c7", 32, 16), ("c8", 16, 1))
_BF = torch.bfloat16


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _st():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _desc(shape, cin, cout):
    n, d, h, w = shape
    return UnetConvDesc(n, d, h, w, cin, cout)


# ---------------------------------------------------------------------------
# Thin wrappers, one per entry point of include/unet.h
# ---------------------------------------------------------------------------
def weight_pack(w, cin, cout, w_fwd, w_bwd):
    check(load().unet_weight_pack(ctypes.byref(_desc((1, 1, 1, 1), cin, cout)), _ptr(w), _ptr(w_fwd), _ptr(w_bwd),
                                  _st()))


def weight_pack_many(layers):
    """weight_pack for [(w, cin, cout, w_fwd, w_bwd), ...] in one launch."""
    from ._lib import UnetPackItem
    items = (UnetPackItem * len(layers))()
    for it, (w, cin, cout, wf, wb) in zip(items, layers):
        it.w, it.cin, it.cout, it.w_fwd, it.w_bwd = _ptr(w), cin, cout, _ptr(wf), _ptr(wb)
    check(load().unet_weight_pack_many(len(layers), items, _st()))


def conv3d_fwd(shape, cin, cout, x, w_fwd, bias=None, relu=False, skip=None, y=None, y_channels=None, r=None,
               out=None):
    ych = (y_channels or cout) if y is not None else 0
    check(load().unet_conv3d_fwd(ctypes.byref(_desc(shape, cin, cout)), _ptr(x), _ptr(w_fwd), _ptr(bias), int(relu),
                                 _ptr(skip), _ptr(y), ych, _ptr(r), _ptr(out), _st()))


def conv3d_dgrad(shape, cin, cout, dy, w_bwd, dx, mask=None, g_out=None):
    """Input gradient dx; with mask (the layer below's stored ReLU output)
    also g_out, the gradient through that ReLU, in the same pass."""
    if mask is None and g_out is None:
        check(load().unet_conv3d_dgrad(ctypes.byref(_desc(shape, cin, cout)), _ptr(dy), _ptr(w_bwd), _ptr(dx), _st()))
    else:
        check(load().unet_conv3d_dgrad_relu(ctypes.byref(_desc(shape, cin, cout)), _ptr(dy), _ptr(w_bwd), _ptr(dx),
                                            _ptr(mask), _ptr(g_out), _st()))


def wgrad_ws_bytes(shape, cin, cout):
    b = ctypes.c_size_t()
    check(load().unet_wgrad_ws_bytes(ctypes.byref(_desc(shape, cin, cout)), ctypes.byref(b)))
    return b.value


def conv3d_wgrad(shape, cin, cout, x, dy, dw, db, ws):
    check(load().unet_conv3d_wgrad(ctypes.byref(_desc(shape, cin, cout)), _ptr(x), _ptr(dy), _ptr(dw), _ptr(db),
                                   _ptr(ws), ws.numel(), _st()))


def conv3d_wgrad_partial(shape, cin, cout, x, dy, ws):
    """The split-K pass of conv3d_wgrad: partial sums into ws, reduced later
    by wgrad_reduce_many."""
    check(load().unet_conv3d_wgrad_partial(ctypes.byref(_desc(shape, cin, cout)), _ptr(x), _ptr(dy), _ptr(ws),
                                           ws.numel(), _st()))


def wgrad_reduce_many(layers):
    """Reduces [(shape, cin, cout, ws, dw, db), ...] (partials written by
    conv3d_wgrad_partial) in two launches; dw and db get conv3d_wgrad's bits."""
    from ._lib import UnetWgradItem
    items = (UnetWgradItem * len(layers))()
    for it, (shape, cin, cout, ws, dw, db) in zip(items, layers):
        it.desc = _desc(shape, cin, cout)
        it.ws, it.ws_bytes, it.dw, it.db = _ptr(ws), ws.numel(), _ptr(dw), _ptr(db)
    check(load().unet_wgrad_reduce_many(len(layers), items, _st()))


def embed(img, channels, scale, x):
    check(load().unet_embed(img.numel(), channels, _ptr(img), float(scale), _ptr(x), _st()))


def pool2(shape, c, x, y):
    check(load().unet_pool2(*shape, c, _ptr(x), _ptr(y), _st()))


def up2(shape, c, x, y):
    check(load().unet_up2(*shape, c, _ptr(x), _ptr(y), _st()))


def up2_bwd(shape, c, g_fine, g_coarse, mask=None, g_out=None):
    """Adjoint of up2; with mask (the coarse level's stored ReLU output) also
    g_out, the gradient through that ReLU, in the same pass."""
    if mask is None and g_out is None:
        check(load().unet_up2_bwd(*shape, c, _ptr(g_fine), _ptr(g_coarse), _st()))
    else:
        check(load().unet_up2_bwd_relu(*shape, c, _ptr(g_fine), _ptr(g_coarse), _ptr(mask), _ptr(g_out), _st()))


def relu_grad(shape, c, g1, g2, g_pool, mask, out):
    check(load().unet_relu_grad(*shape, c, _ptr(g1), _ptr(g2), _ptr(g_pool), _ptr(mask), _ptr(out), _st()))


def mse_ws_bytes(nvox):
    b = ctypes.c_size_t()
    check(load().unet_mse_ws_bytes(nvox, ctypes.byref(b)))
    return b.value


def mse(img, y, target, out, gy, channels, ws, want_loss=True):
    loss = ctypes.c_double(0.0)
    check(load().unet_mse(img.numel(), channels, _ptr(img), _ptr(y), _ptr(target), _ptr(out), _ptr(gy),
                          ctypes.byref(loss) if want_loss else None, _ptr(ws), 0 if ws is None else ws.numel(),
                          _st()))
    return loss.value if want_loss else None


def set_conv_lds(on: bool) -> None:
    """Forward and input-gradient convolutions of <= 32 input and output
    channels, and 64 -> 32, on grids >= 64 voxels wide stage their input in
    LDS (default) or not."""
    check(load().unet_set_conv_lds(1 if on else 0))


def get_conv_lds() -> bool:
    v = ctypes.c_int32(0)
    check(load().unet_get_conv_lds(ctypes.byref(v)))
    return bool(v.value)


def adam(p, g, m, v, lr, b1, b2, eps, step):
    check(load().unet_adam(p.numel(), _ptr(p), _ptr(g), _ptr(m), _ptr(v), float(lr), float(b1), float(b2),
                           float(eps), int(step), _st()))


# ---------------------------------------------------------------------------
# The network
# ---------------------------------------------------------------------------
def he_init(seed=0):
    """He-normal weights, zero biases and a zero output layer (so that the
    untrained network is the identity), in the (Cout, Cin, 3, 3, 3) layout."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, ci, co in LAYERS:
        if name == "c8":
            P[name + ".w"] = np.zeros((co, ci, 3, 3, 3))
        else:
            P[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (ci * 27))
        P[name + ".b"] = np.zeros(co)
    return P


@dataclass
class _Acts:
    shape: tuple
    t: dict


class UNet:
    """Parameters (float32 masters, Adam moments, bfloat16 packs) and the
    forward / backward / update sequence."""

    def __init__(self, params=None, device="cuda:0", seed=0):
        self.dev = torch.device(device)
        self.slots = {}
        off = 0
        for name, ci, co in LAYERS:
            self.slots[name + ".w"] = (off, (co, 27, ci))
            off += co * 27 * ci
            self.slots[name + ".b"] = (off, (co,))
            off += co
        self.nparam = off
        z = lambda: torch.zeros(off, dtype=torch.float32, device=self.dev)  # noqa: E731
        self.p, self.g, self.m, self.v = z(), z(), z(), z()
        self.wf, self.wb = {}, {}
        for name, ci, co in LAYERS:
            self.wf[name] = torch.zeros((co, 27 * ci), dtype=_BF, device=self.dev)
            self.wb[name] = torch.zeros((ci, 27 * co), dtype=_BF, device=self.dev)
        self.step_count = 0
        self._acts = None
        self._ws = None
        self.set_params(params if params is not None else he_init(seed))

    # -- parameters -------------------------------------------------------
    def view(self, buf, key):
        off, shape = self.slots[key]
        n = int(np.prod(shape))
        return buf[off:off + n].view(shape)

    def set_params(self, P):
        host = np.zeros(self.nparam, np.float32)
        for name, ci, co in LAYERS:
            off, _ = self.slots[name + ".w"]
            w = np.transpose(np.asarray(P[name + ".w"], np.float32).reshape(co, ci, 27), (0, 2, 1))
            host[off:off + w.size] = w.ravel()
            off, _ = self.slots[name + ".b"]
            host[off:off + co] = np.asarray(P[name + ".b"])
        self.p.copy_(torch.from_numpy(host).to(self.dev))
        self.m.zero_()
        self.v.zero_()
        self.step_count = 0
        self._pack()

    def get_params(self, buf=None):
        host = (self.p if buf is None else buf).detach().cpu().numpy().astype(np.float64)
        P = {}
        for name, ci, co in LAYERS:
            off, _ = self.slots[name + ".w"]
            w = host[off:off + co * 27 * ci].reshape(co, 27, ci)
            P[name + ".w"] = np.transpose(w, (0, 2, 1)).reshape(co, ci, 3, 3, 3)
            off, _ = self.slots[name + ".b"]
            P[name + ".b"] = host[off:off + co].copy()
        return P

    def grads(self):
        return self.get_params(self.g)

    def _pack(self):
        weight_pack_many([(self.view(self.p, name + ".w"), ci, co, self.wf[name], self.wb[name])
                          for name, ci, co in LAYERS])

    # -- buffers ------------------------------------------------------------
    def _buffers(self, shape):
        if self._acts is not None and self._acts.shape == shape:
            return self._acts.t
        n, d, h, w = shape
        if d % 8 or h % 8 or w % 8:
            raise ValueError("image extents must be multiples of 8 (three 2x pooling levels)")
        s = [(n, d >> k, h >> k, w >> k) for k in range(4)]
        vox = [int(np.prod(x)) for x in s]

        def bf(k, c):
            return torch.empty((vox[k], c), dtype=_BF, device=self.dev)

        def f32(k, c):
            return torch.empty((vox[k], c), dtype=torch.float32, device=self.dev)

        t = dict(x0=bf(0, 1), e1=bf(0, 16), p1=bf(1, 16), e2=bf(1, 32), p2=bf(2, 32), e3=bf(2, 64), p3=bf(3, 64),
                 e4=bf(3, 128), u4=bf(2, 128), r5=bf(2, 64), d3=bf(2, 64), u3=bf(1, 64), r6=bf(1, 32), d2=bf(1, 32),
                 u2=bf(0, 32), r7=bf(0, 16), d1=bf(0, 16), y8=f32(0, 1), out=f32(0, 1), gy8=bf(0, 1),
                 g_d1=f32(0, 16), gp7=bf(0, 16), g_u2=f32(0, 32), g_d2=f32(1, 32), gp6=bf(1, 32), g_u3=f32(1, 64),
                 g_d3=f32(2, 64), gp5=bf(2, 64), g_u4=f32(2, 128), g_e4=f32(3, 128), gp4=bf(3, 128),
                 g_p3=f32(3, 64), gp3=bf(2, 64), g_p2=f32(2, 32), gp2=bf(1, 32), g_p1=f32(1, 16), gp1=bf(0, 16))
        t["s"] = s
        # one weight-gradient workspace per layer (256-byte aligned slices of
        # one buffer): the partials of all layers wait for one reduction at
        # the end of backward()
        sizes = [(wgrad_ws_bytes(s[k], ci, co) + 255) // 256 * 256 for k, ci, co in self._conv_levels()]
        self._ws = torch.empty(sum(sizes), dtype=torch.uint8, device=self.dev)
        offs = np.concatenate([[0], np.cumsum(sizes)])
        self._wg_ws = {name: self._ws[int(offs[i]):int(offs[i + 1])] for i, (name, _, _) in enumerate(LAYERS)}
        self._mse_ws = torch.empty(mse_ws_bytes(vox[0]), dtype=torch.uint8, device=self.dev)
        self._acts = _Acts(shape, t)
        return t

    @staticmethod
    def _conv_levels():
        return ((0, 1, 16), (1, 16, 32), (2, 32, 64), (3, 64, 128), (2, 128, 64), (1, 64, 32), (0, 32, 16),
                (0, 16, 1))

    # -- forward / backward ---------------------------------------------------
    def forward(self, img, target=None, want_loss=True):
        """img: float32 (N, D, H, W) on the device (already normalised).
        Returns the network output (N, D, H, W) and, with a target, the loss."""
        img = img.contiguous()
        shape = tuple(img.shape)
        t = self._buffers(shape)
        s = t["s"]
        b = lambda k: self.view(self.p, k)  # noqa: E731
        embed(img, 1, 1.0, t["x0"])
        conv3d_fwd(s[0], 1, 16, t["x0"], self.wf["c1"], b("c1.b"), True, out=t["e1"])
        pool2(s[0], 16, t["e1"], t["p1"])
        conv3d_fwd(s[1], 16, 32, t["p1"], self.wf["c2"], b("c2.b"), True, out=t["e2"])
        pool2(s[1], 32, t["e2"], t["p2"])
        conv3d_fwd(s[2], 32, 64, t["p2"], self.wf["c3"], b("c3.b"), True, out=t["e3"])
        pool2(s[2], 64, t["e3"], t["p3"])
        conv3d_fwd(s[3], 64, 128, t["p3"], self.wf["c4"], b("c4.b"), True, out=t["e4"])
        up2(s[3], 128, t["e4"], t["u4"])
        conv3d_fwd(s[2], 128, 64, t["u4"], self.wf["c5"], b("c5.b"), True, skip=t["e3"], r=t["r5"], out=t["d3"])
        up2(s[2], 64, t["d3"], t["u3"])
        conv3d_fwd(s[1], 64, 32, t["u3"], self.wf["c6"], b("c6.b"), True, skip=t["e2"], r=t["r6"], out=t["d2"])
        up2(s[1], 32, t["d2"], t["u2"])
        conv3d_fwd(s[0], 32, 16, t["u2"], self.wf["c7"], b("c7.b"), True, skip=t["e1"], r=t["r7"], out=t["d1"])
        conv3d_fwd(s[0], 16, 1, t["d1"], self.wf["c8"], b("c8.b"), False, y=t["y8"], y_channels=1)
        loss = mse(img, t["y8"], target, t["out"], t["gy8"] if target is not None else None, 1,
                   self._mse_ws, want_loss=want_loss and target is not None)
        return t["out"].view(shape), loss

    def backward(self):
        """Parameter gradients of the loss of the last forward (with target)."""
        t = self._acts.t
        s = t["s"]
        G = lambda k: self.view(self.g, k)  # noqa: E731
        wsl = self._wg_ws

        def layer(name, k, ci, co, x, gp, gx=None, mask=None, g_out=None):
            conv3d_wgrad_partial(s[k], ci, co, x, gp, wsl[name])
            if gx is not None:
                conv3d_dgrad(s[k], ci, co, gp, self.wb[name], gx, mask, g_out)

        # the ReLU gradients that take one input are fused into the pass
        # that produces it (the input gradient of c8, the upsampling adjoints)
        layer("c8", 0, 16, 1, t["d1"], t["gy8"], t["g_d1"], t["r7"], t["gp7"])
        layer("c7", 0, 32, 16, t["u2"], t["gp7"], t["g_u2"])
        up2_bwd(s[1], 32, t["g_u2"], t["g_d2"], t["r6"], t["gp6"])
        layer("c6", 1, 64, 32, t["u3"], t["gp6"], t["g_u3"])
        up2_bwd(s[2], 64, t["g_u3"], t["g_d3"], t["r5"], t["gp5"])
        layer("c5", 2, 128, 64, t["u4"], t["gp5"], t["g_u4"])
        up2_bwd(s[3], 128, t["g_u4"], t["g_e4"], t["e4"], t["gp4"])
        layer("c4", 3, 64, 128, t["p3"], t["gp4"], t["g_p3"])
        relu_grad(s[2], 64, t["g_d3"], None, t["g_p3"], t["e3"], t["gp3"])
        layer("c3", 2, 32, 64, t["p2"], t["gp3"], t["g_p2"])
        relu_grad(s[1], 32, t["g_d2"], None, t["g_p2"], t["e2"], t["gp2"])
        layer("c2", 1, 16, 32, t["p1"], t["gp2"], t["g_p1"])
        relu_grad(s[0], 16, t["g_d1"], None, t["g_p1"], t["e1"], t["gp1"])
        layer("c1", 0, 1, 16, t["x0"], t["gp1"])
        wgrad_reduce_many([(s[k], ci, co, wsl[name], G(name + ".w"), G(name + ".b"))
                           for (name, ci, co), (k, _, _) in zip(LAYERS, self._conv_levels())])

    def step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        adam(self.p, self.g, self.m, self.v, lr, b1, b2, eps, self.step_count)
        self._pack()

    def capture_pass(self, img, target):
        """A HIP graph of one forward (without the loss read-back) and
        backward pass on these fixed input and target tensors: replaying it
        does what forward(img, target, want_loss=False) and backward() do,
        with one launch from the host instead of one per kernel.  step()
        stays outside the graph (its bias correction depends on the step
        count); replay, then step(), is one training step.  Buffers are
        made by a first eager pass; the graph keeps reading the network's
        parameter, packed-weight and activation tensors, which stay in place."""
        self.forward(img, target, want_loss=False)
        self.backward()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.forward(img, target, want_loss=False)
            self.backward()
        torch.cuda.synchronize()
        return graph

    def train_step(self, img, target, lr=1e-3):
        _, loss = self.forward(img, target)
        self.backward()
        self.step(lr)
        return loss

    def __call__(self, img):
        with torch.no_grad():
            out, _ = self.forward(img)
            return out.clone()


def layer_timings(net: UNet, img, target, reps=5):
    """Device time of every convolution of one training step (forward,
    input gradient, weight gradient) with torch events on the current stream
    (the library launches on it), after a warm-up step.  Flops are the
    algorithmic 2 x voxels x 27 x Cin x Cout of the real channel counts."""
    net.forward(img, target)
    net.backward()
    t = net._acts.t
    s = t["s"]
    n_img = img.shape[0]
    wsb = net._ws
    plan = (("c1", 0, 1, 16, "x0", "e1", None, "gp1", None), ("c2", 1, 16, 32, "p1", "e2", None, "gp2", "g_p1"),
            ("c3", 2, 32, 64, "p2", "e3", None, "gp3", "g_p2"), ("c4", 3, 64, 128, "p3", "e4", None, "gp4", "g_p3"),
            ("c5", 2, 128, 64, "u4", "d3", "e3", "gp5", "g_u4"), ("c6", 1, 64, 32, "u3", "d2", "e2", "gp6", "g_u3"),
            ("c7", 0, 32, 16, "u2", "d1", "e1", "gp7", "g_u2"), ("c8", 0, 16, 1, "d1", None, None, "gy8", "g_d1"))
    real = {n: (ci, co) for n, ci, co in LAYERS}
    b = lambda k: net.view(net.p, k)  # noqa: E731
    G = lambda k: net.view(net.g, k)  # noqa: E731
    out = []
    for name, k, ci, co, xin, yout, skip, gp, gx in plan:
        vox = int(np.prod(s[k]))
        flops = 2.0 * vox * 27 * real[name][0] * real[name][1]
        calls = {
            "fwd": lambda: conv3d_fwd(s[k], ci, co, t[xin], net.wf[name], b(name + ".b"), name != "c8",
                                      skip=t[skip] if skip else None, y=t["y8"] if yout is None else None,
                                      y_channels=1 if yout is None else None,
                                      r=t["r" + name[1]] if skip else None, out=t[yout] if yout else None),
            "wgrad": lambda: conv3d_wgrad(s[k], ci, co, t[xin], t[gp], G(name + ".w"), G(name + ".b"), wsb),
        }
        if gx is not None:
            calls["dgrad"] = lambda: conv3d_dgrad(s[k], ci, co, t[gp], net.wb[name], t[gx])
        row = {"layer": name, "voxels": vox // n_img, "cin": real[name][0], "cout": real[name][1],
               "gflop": flops / 1e9}
        for kind, fn in calls.items():
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            row[kind + "_ms"] = ms
            row[kind + "_tflops"] = flops / (ms * 1e-3) / 1e12
        out.append(row)
    return out
