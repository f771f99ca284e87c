"""Training data, training loop and fallback of the learned crosstalk filter.

Data come from the library's own RTM.  For one geometry (3-D velocity model,
source, surface receivers):

 1. the observed traces are modelled on the model extended by edge
    replication, far enough that waves in the slowest layer do not reach its
    random boundary and return within the record (whatever boundary energy
    remains is common to all realisations and so part of the target);
 2. the shot is migrated K times, each with its own random boundary
    (seeds s_1 .. s_K, one batched launch per time step for the K shots);
 3. pair k maps image k to the mean of the other K - 1 images (the
    leave-one-out stack, whose crosstalk is independent of image k's), both
    divided by a scale computed from image k alone: its RMS ("rms", the
    default) or a depth gain, the RMS of each depth slice smoothed over a few
    slices ("depth": every depth counts equally in the loss, whereas under
    "rms" the strong shallow part of the image dominates it).

The network (unet.UNet) is trained with its own kernels; the Denoiser keeps
the plain image as fallback: it is used when the network has not shown a
gain on held-out geometries or when its output is not finite.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import RTM_OP_RTM, BatchPlan, BatchShot, Grid, rtm_model_shot, rtm_rbc_pad
from .unet import UNet


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def observed_data(v_int, h, dt, wavelet, src, rec, ext, nb=16, seed=1, remove_direct=True, device="cuda:0"):
    """Traces of one shot modelled on v_int (nz, ny, nx) extended by `ext`
    replicated cells on every face.  Positions are interior grid units.
    With remove_direct, the same shot modelled on the homogeneous model of
    the source cell's velocity is subtracted (direct wave removed, leaving
    the reflected and transmitted energy)."""
    v_ext = np.pad(np.asarray(v_int, np.float32), ext, mode="edge")
    g = Grid.for_model(v_ext, h, nb)
    shift = np.array([ext, ext, ext], np.float64)
    s = np.asarray(src, np.float64) + shift
    r = np.asarray(rec, np.float32) + shift.astype(np.float32)
    w = _t(wavelet, device)
    d = rtm_model_shot(g, rtm_rbc_pad(g, _t(v_ext, device), seed, float(v_ext.max())), dt, w, s, r)
    if remove_direct:
        v0 = float(v_int[int(round(src[2])), int(round(src[1])), int(round(src[0]))])
        vh = np.full(v_ext.shape, v0, np.float32)
        d -= rtm_model_shot(g, rtm_rbc_pad(g, _t(vh, device), seed, v0), dt, w, s, r)
    return d


def realisation_images(v_int, h, nb, dt, wavelet, src, rec, d_obs, seeds, eps_rel=1e-3, device="cuda:0"):
    """RTM images (K, nz, ny, nx) of one shot, one per random-boundary seed,
    all K shots in one batched launch per time step."""
    g = Grid.for_model(v_int, h, nb)
    vt = _t(v_int, device)
    cap = float(np.max(v_int))
    w = _t(wavelet, device)
    imgs = torch.empty((len(seeds),) + tuple(np.shape(v_int)), dtype=torch.float32, device=device)
    shots = [BatchShot(g, rtm_rbc_pad(g, vt, int(s), cap), w, src, rec, traces_in=d_obs, image=imgs[k])
             for k, s in enumerate(seeds)]
    BatchPlan(RTM_OP_RTM, shots, dt, len(wavelet), eps_rel=eps_rel).run()
    return imgs


def _rms(x):
    return float(torch.sqrt(torch.mean(x.double() * x.double())))


def image_scale(img, norm="rms"):
    """Scale that divides an image (and its target) before the network."""
    if norm == "rms":
        return _rms(img)
    if norm == "depth":
        return depth_gain(img)
    raise ValueError("norm must be 'rms' or 'depth'")


def depth_gain(img, half_window=2, floor=1e-3):
    """(nz, 1, 1) gain of one image (nz, ny, nx): RMS of each depth slice,
    averaged over +-half_window slices, floored at `floor` x its maximum."""
    r = torch.sqrt(torch.mean(img.double() ** 2, dim=(1, 2)))
    k = 2 * half_window + 1
    rp = torch.nn.functional.pad(r[None, None], (half_window, half_window), mode="replicate")
    a = torch.nn.functional.avg_pool1d(rp, k, stride=1)[0, 0]
    a = torch.clamp(a, min=floor * float(a.max()))
    return a.float()[:, None, None]


@dataclass
class PairSet:
    inputs: list = field(default_factory=list)    # normalised single-realisation images (D, H, W)
    targets: list = field(default_factory=list)   # normalised leave-one-out stacks
    geometry: list = field(default_factory=list)

    def add_geometry(self, imgs, gid, norm="rms"):
        K = imgs.shape[0]
        total = imgs.sum(0)
        for k in range(K):
            a = image_scale(imgs[k], norm)
            self.inputs.append((imgs[k] / a).contiguous())
            self.targets.append(((total - imgs[k]) / ((K - 1) * a)).contiguous())
            self.geometry.append(gid)

    def split(self, held_out):
        a, b = PairSet(), PairSet()
        for x, t, gg in zip(self.inputs, self.targets, self.geometry):
            (b if gg in held_out else a).inputs.append(x)
            (b if gg in held_out else a).targets.append(t)
            (b if gg in held_out else a).geometry.append(gg)
        return a, b

    def __len__(self):
        return len(self.inputs)


def train(net: UNet, data: PairSet, epochs: int, lr: float = 1e-3, batch: int = 1, seed: int = 0,
          lr_decay: float = 1.0, flips: bool = True, log=None, warmup: int = 0):
    """Adam on the mean squared error; returns the mean loss of each epoch.
    With flips, each sample is mirrored along x and/or y at random (the
    acquisition and the crosstalk statistics have no preferred lateral
    direction).  The learning rate rises linearly over the first `warmup`
    epochs (per step) to `lr`, then decays by `lr_decay` per epoch."""
    rng = np.random.default_rng(seed)
    hist = []
    steps_per_epoch = (len(data) + batch - 1) // batch
    step = 0

    def aug(a, f):
        dims = [d for d, on in ((-1, f & 1), (-2, f & 2)) if on]
        return torch.flip(a, dims) if dims else a

    for ep in range(epochs):
        order = rng.permutation(len(data))
        tot, cnt = 0.0, 0
        for i in range(0, len(order), batch):
            idx = order[i:i + batch]
            fl = rng.integers(0, 4, len(idx)) if flips else np.zeros(len(idx), int)
            x = torch.stack([aug(data.inputs[j], f) for j, f in zip(idx, fl)])
            t = torch.stack([aug(data.targets[j], f) for j, f in zip(idx, fl)])
            ramp = min(1.0, (step + 1) / (warmup * steps_per_epoch)) if warmup > 0 else 1.0
            tot += net.train_step(x, t, lr * ramp)
            cnt += 1
            step += 1
        hist.append(tot / cnt)
        if ep >= warmup:
            lr *= lr_decay
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.5f}")
    return hist


def evaluate(net, data: PairSet):
    """Mean relative L2 distance to the leave-one-out stack of the plain
    single-realisation images and of the network's outputs, in the scaled
    amplitudes the network sees."""
    ep, en = [], []
    for x, t in zip(data.inputs, data.targets):
        y = net(x[None])[0]
        nt_ = float(torch.linalg.norm(t))
        ep.append(float(torch.linalg.norm(x - t)) / nt_)
        en.append(float(torch.linalg.norm(y - t)) / nt_)
    ep, en = float(np.mean(ep)), float(np.mean(en))
    return {"plain_rel_l2": ep, "net_rel_l2": en, "gain": ep / en if en > 0 else float("inf"), "pairs": len(data)}


class Denoiser:
    """Applies the network to single-realisation images, keeping the plain
    image as fallback."""

    def __init__(self, net: UNet, min_gain: float = 1.0, norm: str = "rms"):
        self.net = net
        self.min_gain = min_gain
        self.norm = norm
        self.enabled = False
        self.validation = None

    def validate(self, held_out: PairSet):
        self.validation = evaluate(self.net, held_out)
        self.enabled = self.validation["gain"] > self.min_gain
        return self.validation

    def __call__(self, img):
        """img (D, H, W) float32 on the device -> (image, network_used)."""
        if not self.enabled:
            return img, False
        if not bool(torch.isfinite(img).all()) or _rms(img) == 0.0:
            return img, False
        a = image_scale(img, self.norm)
        y = self.net((img / a)[None])[0] * a
        if not bool(torch.isfinite(y).all()):
            return img, False
        return y, True


def build_dataset(models, h, nb, dt, wavelet, K, seed0=100, ext=None, norm="rms", device="cuda:0", log=None):
    """Pairs from a list of 3-D interior models (nz, ny, nx): one shot per
    model at a seeded surface position in the central half, receivers on
    every other surface cell."""
    data = PairSet()
    wav = np.asarray(wavelet, np.float32)
    nt = wav.size
    rng = np.random.default_rng(seed0)
    for gid, v in enumerate(models):
        nz, ny, nx = v.shape
        src = np.array([rng.uniform(0.25, 0.75) * (nx - 1), rng.uniform(0.25, 0.75) * (ny - 1), 2.0])
        xs, ys = np.meshgrid(np.arange(0, nx, 2, dtype=np.float32), np.arange(0, ny, 2, dtype=np.float32))
        rec = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, 2.0, np.float32)], 1)
        # far enough that a wave in the slowest (top) layer cannot reach the
        # random boundary and return within nt steps
        e = ext if ext is not None else int(np.ceil(nt * dt * float(np.min(v)) / (2.0 * h))) + 2
        t0 = time.time()
        d_obs = observed_data(v, h, dt, wav, src, rec, e, nb=nb, seed=seed0 + gid, device=device)
        imgs = realisation_images(v, h, nb, dt, wav, src, rec, d_obs, [seed0 * 1000 + gid * K + k for k in range(K)],
                                  device=device)
        data.add_geometry(imgs, gid, norm)
        if log:
            torch.cuda.synchronize()
            log(f"geometry {gid}: {K} realisations in {time.time() - t0:.2f} s (extension {e} cells)")
    return data


def main(argv=None):
    ap = argparse.ArgumentParser(description="Train the crosstalk filter on the library's RTM images")
    ap.add_argument("--n", type=int, default=128, help="cube edge of the interior models (multiple of 8)")
    ap.add_argument("--geometries", type=int, default=32)
    ap.add_argument("--held-out", type=int, default=4)
    ap.add_argument("--realisations", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--lr-decay", type=float, default=0.97, help="learning-rate factor per epoch after the warm-up")
    ap.add_argument("--warmup", type=int, default=0, help="epochs of linear learning-rate warm-up")
    ap.add_argument("--nt", type=int, default=1100)
    ap.add_argument("--infer-shape", default=None,
                    help="after training, migrate one model of this interior shape NZ,NY,NX (multiples of 8) with "
                         "the same acquisition and realisations, and report the filter's gain on it and its time")
    ap.add_argument("--out", default=None, help="write a JSON summary here")
    a = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    log = lambda m: print(m, flush=True)  # noqa: E731
    models = synth.config_c5_models(a.geometries, 5000, a.n)
    t0 = time.time()
    data = build_dataset(models, 10.0, 30, 1e-3, synth.ricker(15.0, 1e-3, a.nt), a.realisations, log=log)
    torch.cuda.synchronize()
    t_data = time.time() - t0
    train_set, test_set = data.split(set(range(a.geometries - a.held_out, a.geometries)))
    net = UNet(seed=0)
    t0 = time.time()
    hist = train(net, train_set, a.epochs, a.lr, a.batch, lr_decay=a.lr_decay, log=log, warmup=a.warmup)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    den = Denoiser(net)
    res = {"train": evaluate(net, train_set), "held_out": den.validate(test_set), "enabled": den.enabled,
           "loss_history": hist, "data_s": t_data, "train_s": t_train,
           "config": {"n": a.n, "geometries": a.geometries, "held_out": a.held_out, "realisations": a.realisations,
                      "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "nt": a.nt, "pairs_train": len(train_set),
                      "pairs_held_out": len(test_set)}}
    if a.infer_shape:
        nz, ny, nx = (int(v) for v in a.infer_shape.split(","))
        big = synth.layered_salt_3d(nx, ny, nz, 7777)
        t0 = time.time()
        bset = build_dataset([big], 10.0, 30, 1e-3, synth.ricker(15.0, 1e-3, a.nt), a.realisations, seed0=900,
                             log=log)
        torch.cuda.synchronize()
        t_big = time.time() - t0
        x = bset.inputs[0][None]
        net(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        net(x)
        e1.record()
        e1.synchronize()
        res["infer"] = {"shape": [nz, ny, nx], "data_s": t_big, "forward_ms": e0.elapsed_time(e1),
                        **evaluate(net, bset)}
        log(f"inference on {nz}x{ny}x{nx}: {res['infer']}")
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main()
