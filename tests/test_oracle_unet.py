"""Pins of the U-Net oracle against what the definitions fix independently:
brute-force sums, closed forms, adjoint (dot-product) identities, the
identity network at initialisation and central finite differences of the
float64 network."""
import itertools

import numpy as np
import pytest

from oracle import unet as U


def test_bf16_rounding_cases():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even
    # significand (1); 1 + 3 * 2^-8 ties between 1 + 2^-7 and 1 + 2^-6 and
    # goes to 1 + 2^-6; anything above a tie rounds up.
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, -(1 + 2.0 ** -8 + 2.0 ** -20),
                  0.0, 3.0e38, 1e-40], np.float64)
    got = U.bf16(x)
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -(1 + 2.0 ** -7), 0.0, 2.99980756e38, 9.99e-41])
    assert np.array_equal(got[:6], want[:6])
    assert abs(got[6] - 3.0e38) / 3.0e38 < 2.0 ** -8
    # bfloat16 keeps float32's exponent range: a subnormal stays subnormal
    assert got[7] > 0 and abs(got[7] - 1e-40) / 1e-40 < 2.0 ** -1
    # every rounded value is exactly representable: 16 low bits clear
    r = np.random.default_rng(0).standard_normal(1000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 1000)
    b = U.bf16(r).astype(np.float32).view(np.uint32)
    assert np.all((b & 0xFFFF) == 0)
    assert np.all(np.abs(U.bf16(r) - r) <= np.abs(r) * 2.0 ** -8 * (1 + 1e-6))


def _brute_conv(x, w, b):
    C, D, H, W = x.shape
    O = w.shape[0]
    y = np.zeros((O, D, H, W))
    for o, z, yy, xx in itertools.product(range(O), range(D), range(H), range(W)):
        s = b[o]
        for i, kz, ky, kx in itertools.product(range(C), range(3), range(3), range(3)):
            zz, y2, x2 = z + kz - 1, yy + ky - 1, xx + kx - 1
            if 0 <= zz < D and 0 <= y2 < H and 0 <= x2 < W:
                s += w[o, i, kz, ky, kx] * x[i, zz, y2, x2]
        y[o, z, yy, xx] = s
    return y


def test_conv3d_brute_force():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 4, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    assert np.allclose(U.conv3d(x, w, b), _brute_conv(x, w, b), rtol=0, atol=1e-12)


def test_pointwise_forms_match_the_brute_force_and_adjoint():
    """conv3d_at equals the brute-force sum at every voxel of a small tensor
    (faces and corners included); conv3d_dgrad_at satisfies the dot-product
    identity <conv(x), dy> = <x, dgrad(dy)> voxel by voxel summed."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, 4, 3, 5))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    pts = np.argwhere(np.ones(x.shape[1:], bool))
    y = U.conv3d_at(x, w, b, pts)
    ref = _brute_conv(x, w, b)
    assert np.allclose(y, ref.reshape(2, -1).T, rtol=0, atol=1e-12)
    dy = rng.standard_normal((2,) + x.shape[1:])
    dx = U.conv3d_dgrad_at(dy, w, pts)
    lhs = np.sum(_brute_conv(x, w, np.zeros(2)) * dy)
    assert abs(lhs - np.sum(x.reshape(3, -1).T * dx)) < 1e-10 * abs(lhs)


def test_conv3d_delta_response():
    # a unit impulse at p0 gives y[o, p0 - k + 1] = w[o, 0, k]
    rng = np.random.default_rng(2)
    w = rng.standard_normal((4, 1, 3, 3, 3))
    x = np.zeros((1, 5, 5, 5))
    x[0, 2, 2, 2] = 1.0
    y = U.conv3d(x, w)
    for kz, ky, kx in itertools.product(range(3), repeat=3):
        assert np.array_equal(y[:, 3 - kz, 3 - ky, 3 - kx], w[:, 0, kz, ky, kx])
    assert np.count_nonzero(y) == np.count_nonzero(w)


def test_dgrad_and_wgrad_are_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 4, 6, 5))
    w = rng.standard_normal((5, 3, 3, 3, 3))
    dy = rng.standard_normal((5, 4, 6, 5))
    lhs = np.sum(U.conv3d(x, w) * dy)
    assert abs(lhs - np.sum(x * U.conv3d_dgrad(dy, w))) <= 1e-12 * abs(lhs) * 100
    dw, db = U.conv3d_wgrad(x, dy)
    assert abs(lhs - np.sum(w * dw)) <= 1e-12 * abs(lhs) * 100
    b = rng.standard_normal(5)
    assert abs(np.sum(U.conv3d(x, 0 * w, b) * dy) - np.sum(b * db)) <= 1e-10


def test_pool_up_adjoint_and_inverse():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 4, 6, 8))
    c = rng.standard_normal((2, 2, 3, 4))
    assert abs(np.sum(U.pool2(x) * c) - np.sum(x * U.pool2_bwd(c))) < 1e-12
    assert abs(np.sum(U.up2(c) * x) - np.sum(c * U.up2_bwd(x))) < 1e-12
    assert np.array_equal(U.pool2(U.up2(c)), c)
    assert U.pool2(x)[1, 0, 1, 2] == pytest.approx(x[1, 0:2, 2:4, 4:6].mean(), abs=1e-15)


def test_identity_at_initialisation():
    P = U.init_params(0)
    img = np.random.default_rng(5).standard_normal((8, 8, 16))
    out, _, _ = U.forward(P, img, quant=True)
    assert np.array_equal(out, img)


def test_mse_gradient():
    rng = np.random.default_rng(6)
    o, t = rng.standard_normal(50), rng.standard_normal(50)
    L, g = U.mse(o, t)
    assert L == pytest.approx(np.sum((o - t) ** 2) / 50, rel=1e-14)
    e = np.zeros(50)
    e[7] = 1e-6
    fd = (U.mse(o + e, t)[0] - U.mse(o - e, t)[0]) / 2e-6
    assert fd == pytest.approx(g[7], rel=1e-7)


def test_adam_first_step_closed_form():
    # after one step the bias-corrected moments are g and g^2, so each
    # parameter moves by lr * g / (|g| + eps)
    rng = np.random.default_rng(7)
    p, g = rng.standard_normal(20), rng.standard_normal(20)
    z = np.zeros(20)
    p1, m, v = U.adam(p, g, z, z, 1, lr=1e-2)
    assert np.allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a constant gradient keeps the bias-corrected moments at g and g^2
    p2, m, v = U.adam(p1, g, m, v, 2, lr=1e-2)
    assert np.allclose(p2 - p1, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_network_gradient_finite_differences():
    """Float64 network: backward against central differences of the loss on
    sampled weights and biases of every layer."""
    rng = np.random.default_rng(8)
    P = U.init_params(3)
    P["c8.w"] = rng.standard_normal(P["c8.w"].shape) * 0.1
    for n, _, co in U.LAYERS:
        P[n + ".b"] = rng.standard_normal(co) * 0.05
    img = rng.standard_normal((8, 8, 8))
    tgt = img + 0.3 * rng.standard_normal((8, 8, 8))
    L, G, _ = U.backward(P, img, tgt, quant=False)
    checked = 0
    for name, _, _ in U.LAYERS:
        for kind in ("w", "b"):
            key = f"{name}.{kind}"
            flat = G[key].ravel()
            for j in (int(np.argmax(np.abs(flat))), int(rng.integers(flat.size))):
                if abs(flat[j]) < 1e-9 * max(abs(L), 1.0):
                    continue
                h = 1e-6
                Pp = {k: v.copy() for k, v in P.items()}
                Pm = {k: v.copy() for k, v in P.items()}
                Pp[key].ravel()[j] += h
                Pm[key].ravel()[j] -= h
                Lp = U.mse(U.forward(Pp, img, quant=False)[0], tgt)[0]
                Lm = U.mse(U.forward(Pm, img, quant=False)[0], tgt)[0]
                fd = (Lp - Lm) / (2 * h)
                assert fd == pytest.approx(flat[j], rel=1e-5, abs=1e-10), (key, j, fd, flat[j])
                checked += 1
    assert checked >= 24
