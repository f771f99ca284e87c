"""The learned crosstalk filter end to end on the GPU: training pairs from
the library's own 3-D RTM (single random-boundary realisation -> leave-one-
out stack of the others), training with the library's kernels, the gain on a
held-out geometry over the plain image, and the fallback to the plain image."""
import numpy as np
import pytest
import torch

import synth
from paper_2204_03380_amd import crosstalk as X
from paper_2204_03380_amd.unet import UNet

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_filter_gain_over_plain_image_on_held_out_geometry():
    """Six networks trained from different seeds (initial weights, sample
    order, flips) on 56 geometries.  Each is switched on by four validation
    geometries and does better than the plain image on eight other held-out
    geometries; the one the validation split prefers gains at least 8% on
    them.  Training either leaves its initial loss plateau (loss 0.007 ->
    0.004-0.006, test gains 1.10-1.22) or stays on it through the 30 epochs
    (loss 0.0064, gains 1.05-1.06): a quarter to a third of the runs in
    studies of 20 and 12 runs, which runs depending on float32 summation
    order.  The validation gain tells the two apart, so model selection on
    the validation split over six seeds is what makes the result robust
    (all six stay on the plateau in about one of 700 orderings)."""
    n, K, nt, G = 64, 8, 600, 68
    models = [synth.layered_salt_3d(n, n, n, 900 + i) for i in range(G)]
    data = X.build_dataset(models, 10.0, 16, 1e-3, synth.ricker(15.0, 1e-3, nt), K)
    assert len(data) == G * K
    train_set, held = data.split(set(range(56, G)))
    test_set, val_set = held.split(set(range(56, 60)))
    best = None
    for seed in range(6):
        net = UNet(seed=seed)
        hist = X.train(net, train_set, epochs=30, lr=1e-3, batch=4, seed=seed, lr_decay=0.95, warmup=2)
        den = X.Denoiser(net)
        val = den.validate(val_set)
        res = X.evaluate(net, test_set)
        print(f"seed {seed}: loss {hist[0]:.5f} -> {hist[-1]:.5f}; validation gain {val['gain']:.4f}, "
              f"test gain {res['gain']:.4f} ({res['pairs']} pairs)")
        assert np.isfinite(hist).all() and hist[-1] < hist[0]
        assert den.enabled and res["gain"] > 1.0
        if best is None or val["gain"] > best[0]:
            best = (val["gain"], res["gain"], den)
    print(f"validation-selected network: test gain {best[1]:.4f}")
    assert best[1] > 1.08
    den = best[2]
    img, used = den(test_set.inputs[0])
    assert used and img.shape == test_set.inputs[0].shape and bool(torch.isfinite(img).all())

    # fallback: the untrained network is the identity (zero output layer):
    # no gain, so the plain image is returned
    den0 = X.Denoiser(UNet(seed=0))
    r0 = den0.validate(test_set)
    assert r0["gain"] == pytest.approx(1.0, abs=1e-6) and not den0.enabled
    x = test_set.inputs[0]
    img0, used0 = den0(x)
    assert img0 is x and not used0
    # a non-finite input is passed through unchanged
    bad = x.clone()
    bad[0, 0, 0] = float("inf")
    out, used = den(bad)
    assert not used and out is bad
