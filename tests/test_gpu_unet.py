"""GPU parity of the U-Net kernels against the FP64 oracle on the same
bfloat16-quantised operands (only float32 accumulation order differs), on
ragged extents that leave partial 64-voxel tiles and partial 32-voxel
weight-gradient segments, and of the whole network's output and parameter
gradients."""
import numpy as np
import pytest
import torch

from oracle import unet as U
from paper_2204_03380_amd import unet as N

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# the MFMA pairs and the one-channel input / output pairs (vector units)
PAIRS = ((16, 16), (16, 32), (32, 64), (64, 128), (128, 64), (64, 32), (32, 16), (1, 16), (16, 1))


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def bf_tensor(a):
    """bfloat16 device tensor holding a (which must be bf16-representable)."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV).to(torch.bfloat16)


def f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def to_cf(a, shape, c):
    """channels-last (N*D*H*W, C) -> list of (C, D, H, W) per sample."""
    n, d, h, w = shape
    a = np.asarray(a).reshape(n, d, h, w, c)
    return [np.transpose(a[i], (3, 0, 1, 2)) for i in range(n)]


def from_cf(lst):
    return np.stack([np.transpose(x, (1, 2, 3, 0)) for x in lst]).reshape(-1, lst[0].shape[0])


def pack(w_oracle):
    co, ci = w_oracle.shape[:2]
    wm = f32(np.transpose(w_oracle.reshape(co, ci, 27), (0, 2, 1)))
    wf = torch.empty((co, 27 * ci), dtype=torch.bfloat16, device=DEV)
    wb = torch.empty((ci, 27 * co), dtype=torch.bfloat16, device=DEV)
    N.weight_pack(wm, ci, co, wf, wb)
    return wf, wb


def _operands(shape, ci, co, seed):
    rng = np.random.default_rng(seed)
    n, d, h, w = shape
    x = U.bf16(rng.standard_normal((n * d * h * w, ci)))
    wo = rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci))
    b = rng.standard_normal(co) * 0.1
    return rng, x, wo, b


@pytest.mark.parametrize("ci,co", PAIRS)
def test_conv_forward_parity(ci, co):
    shape = (2, 5, 6, 37) if ci <= 32 else (1, 5, 6, 37)
    rng, x, wo, b = _operands(shape, ci, co, ci * 1000 + co)
    wf, _ = pack(wo)
    y = torch.empty((x.shape[0], co), dtype=torch.float32, device=DEV)
    N.conv3d_fwd(shape, ci, co, bf_tensor(x), wf, f32(b), False, y=y)
    ref = from_cf([U.conv3d(xc, U.bf16(wo), b) for xc in to_cf(x, shape, ci)])
    e = rel_l2(host(y), ref)
    print(f"conv fwd {ci}->{co} {shape}: rel-L2 {e:.2e}")
    assert e < 1e-5
    # fused epilogue: relu, stored relu value, skip-add, all rounded once
    skip = U.bf16(rng.standard_normal(y.shape))
    y2 = torch.empty_like(y)
    r = torch.empty(y.shape, dtype=torch.bfloat16, device=DEV)
    out = torch.empty_like(r)
    N.conv3d_fwd(shape, ci, co, bf_tensor(x), wf, f32(b), True, skip=bf_tensor(skip), y=y2, r=r, out=out)
    yg = host(y2).astype(np.float32)
    assert np.array_equal(yg, np.maximum(host(y).astype(np.float32), 0))
    assert np.array_equal(host(r), U.bf16(yg))
    assert np.array_equal(host(out), U.bf16(yg + skip.astype(np.float32)))


@pytest.mark.parametrize("ci,co,shape", [(128, 64, (1, 8, 8, 300)), (64, 128, (1, 2, 4, 300))])
def test_conv_forward_channel_split_grids(ci, co, shape):
    """Grids of 300 and 38 wavefronts, which split the output channels two
    and four ways over the grid (the smaller one also splits the reduction
    over four wavefronts of a workgroup, with a partly empty last
    workgroup): same bar as the other forward tests."""
    _, x, wo, b = _operands(shape, ci, co, 5 + ci + co)
    wf, _ = pack(wo)
    y = torch.empty((x.shape[0], co), dtype=torch.float32, device=DEV)
    N.conv3d_fwd(shape, ci, co, bf_tensor(x), wf, f32(b), False, y=y)
    ref = from_cf([U.conv3d(xc, U.bf16(wo), b) for xc in to_cf(x, shape, ci)])
    e = rel_l2(host(y), ref)
    print(f"conv fwd {ci}->{co} {shape}: rel-L2 {e:.2e}")
    assert e < 1e-5


@pytest.mark.parametrize("ci,co", PAIRS)
def test_conv_dgrad_parity(ci, co):
    shape = (1, 6, 5, 41)
    rng, _, wo, _ = _operands(shape, ci, co, 7 + ci + co)
    dy = U.bf16(rng.standard_normal((int(np.prod(shape)), co)))
    _, wb = pack(wo)
    dx = torch.empty((dy.shape[0], ci), dtype=torch.float32, device=DEV)
    N.conv3d_dgrad(shape, ci, co, bf_tensor(dy), wb, dx)
    ref = from_cf([U.conv3d_dgrad(g, U.bf16(wo)) for g in to_cf(dy, shape, co)])
    e = rel_l2(host(dx), ref)
    print(f"conv dgrad {ci}->{co}: rel-L2 {e:.2e}")
    assert e < 1e-5


@pytest.mark.parametrize("ci,co", PAIRS)
def test_conv_wgrad_parity_and_determinism(ci, co):
    _wgrad_check((2, 4, 7, 45), ci, co)


@pytest.mark.parametrize("ci,co", [(16, 32), (32, 16), (64, 32), (1, 16), (16, 1)])
def test_ring_wgrad_parity_ragged(ci, co):
    """The ring-staged weight gradients (MFMA pairs of at most 64 input
    channels on grids of 2^17 voxels or more, and the one-channel pairs on
    the matrix cores at any size) on a ragged two-sample grid: 19 planes
    (not a multiple of the 4- or 2-plane block), 150 columns (a partial
    32-voxel segment), 23 rows split into unequal y ranges."""
    _wgrad_check((2, 19, 23, 150), ci, co)


def _wgrad_check(shape, ci, co):
    """Weight and bias gradients against the oracle, and equal bit for bit
    on a second call."""
    rng, x, _, _ = _operands(shape, ci, co, 11 + ci * co)
    dy = U.bf16(rng.standard_normal((x.shape[0], co)))
    ws = torch.empty(N.wgrad_ws_bytes(shape, ci, co), dtype=torch.uint8, device=DEV)
    outs = []
    for _ in range(2):
        dw = torch.empty((co, 27, ci), dtype=torch.float32, device=DEV)
        db = torch.empty(co, dtype=torch.float32, device=DEV)
        N.conv3d_wgrad(shape, ci, co, bf_tensor(x), bf_tensor(dy), dw, db, ws)
        outs.append((host(dw), host(db)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    ref_w, ref_b = 0.0, 0.0
    for xc, gc in zip(to_cf(x, shape, ci), to_cf(dy, shape, co)):
        a, bb = U.conv3d_wgrad(xc, gc)
        ref_w, ref_b = ref_w + a, ref_b + bb
    ref_w = np.transpose(ref_w.reshape(co, ci, 27), (0, 2, 1))
    e, eb = rel_l2(outs[0][0], ref_w), rel_l2(outs[0][1], ref_b)
    print(f"conv wgrad {ci}->{co}: dw rel-L2 {e:.2e} db {eb:.2e}")
    assert e < 1e-5 and eb < 1e-5


@pytest.mark.parametrize("c,with_g2", [(32, True), (32, False), (6, True)])
def test_relu_grad_float32_exact(c, with_g2):
    """relu_grad in float32 arithmetic, order g1 (+ g2) + g_pool/8, then one
    bfloat16 rounding, masked: equal bit for bit to the same float32 steps
    in numpy (4 channels per thread when 4 divides c, else one)."""
    rng = np.random.default_rng(c + 2 * with_g2)
    shape = (2, 6, 4, 10)
    n, d, h, w = shape
    cs = (n, d // 2, h // 2, w // 2)
    nf = n * d * h * w
    g1 = rng.standard_normal((nf, c)).astype(np.float32)
    g2 = rng.standard_normal((nf, c)).astype(np.float32) if with_g2 else None
    gp = rng.standard_normal((int(np.prod(cs)), c)).astype(np.float32)
    mask = U.bf16(np.maximum(rng.standard_normal((nf, c)), 0))
    out = torch.empty((nf, c), dtype=torch.bfloat16, device=DEV)
    N.relu_grad(shape, c, f32(g1), f32(g2) if with_g2 else None, f32(gp), bf_tensor(mask), out)
    up = gp.reshape(n, d // 2, h // 2, w // 2, c).repeat(2, 1).repeat(2, 2).repeat(2, 3).reshape(nf, c)
    g = g1 + g2 if with_g2 else g1.copy()
    g = g + up * np.float32(0.125)
    ref = np.where(mask > 0, U.bf16(g.astype(np.float64)), 0.0)
    assert np.array_equal(host(out), ref)


def test_resampling_and_elementwise_kernels():
    rng = np.random.default_rng(3)
    shape, c = (2, 6, 4, 10), 32
    n, d, h, w = shape
    cs = (n, d // 2, h // 2, w // 2)
    x = U.bf16(rng.standard_normal((n * d * h * w, c)))
    y = torch.empty((n * d * h * w // 8, c), dtype=torch.bfloat16, device=DEV)
    N.pool2(shape, c, bf_tensor(x), y)
    ref = from_cf([U.bf16(U.pool2(a)) for a in to_cf(x, shape, c)])
    assert np.array_equal(host(y), ref)
    xc = U.bf16(rng.standard_normal((int(np.prod(cs)), c)))
    up = torch.empty((n * d * h * w, c), dtype=torch.bfloat16, device=DEV)
    N.up2(cs, c, bf_tensor(xc), up)
    assert np.array_equal(host(up), from_cf([U.up2(a) for a in to_cf(xc, cs, c)]))
    gf = rng.standard_normal((n * d * h * w, c)).astype(np.float32)
    gc = torch.empty((int(np.prod(cs)), c), dtype=torch.float32, device=DEV)
    N.up2_bwd(cs, c, f32(gf), gc)
    assert rel_l2(host(gc), from_cf([U.up2_bwd(a) for a in to_cf(gf, shape, c)])) < 1e-6
    # relu gradient with skip gradient and fused pooling adjoint
    g1 = rng.standard_normal(gf.shape).astype(np.float32)
    gp = rng.standard_normal((int(np.prod(cs)), c)).astype(np.float32)
    mask = U.bf16(np.maximum(rng.standard_normal(gf.shape), 0))
    out = torch.empty(gf.shape, dtype=torch.bfloat16, device=DEV)
    N.relu_grad(shape, c, f32(g1), None, f32(gp), bf_tensor(mask), out)
    ref = from_cf([U.bf16((a + U.pool2_bwd(b)) * (m > 0)) for a, b, m in
                   zip(to_cf(g1, shape, c), to_cf(gp, cs, c), to_cf(mask, shape, c))])
    got = host(out)
    # float32 sum vs float64 sum may straddle a bf16 rounding boundary
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)) <= 2.0 ** -7
    assert np.mean(got == ref) > 0.999
    # embed, residual output, loss and gradient
    img = rng.standard_normal(n * d * h * w).astype(np.float32)
    x0 = torch.empty((img.size, 16), dtype=torch.bfloat16, device=DEV)
    N.embed(f32(img), 16, 1.0, x0)
    xh = host(x0)
    assert np.array_equal(xh[:, 0], U.bf16(img)) and not xh[:, 1:].any()
    yv, tg = rng.standard_normal(img.size).astype(np.float32), rng.standard_normal(img.size).astype(np.float32)
    o = torch.empty(img.size, dtype=torch.float32, device=DEV)
    gy = torch.empty((img.size, 16), dtype=torch.bfloat16, device=DEV)
    ws = torch.empty(N.mse_ws_bytes(img.size), dtype=torch.uint8, device=DEV)
    loss = N.mse(f32(img), f32(yv), f32(tg), o, gy, 16, ws)
    L, g = U.mse(img.astype(np.float64) + yv, tg)
    assert np.array_equal(host(o), (img + yv).astype(np.float64))
    assert loss == pytest.approx(L, rel=1e-6)
    gyh = host(gy)
    assert np.max(np.abs(gyh[:, 0] - U.bf16(g)) / np.abs(U.bf16(g))) <= 2.0 ** -7 and not gyh[:, 1:].any()
    # Adam: three steps against the oracle's update
    p, m, v = (rng.standard_normal(1000) for _ in range(3))
    m, v = m * 0.1, np.abs(v) * 0.01
    pt, mt, vt = f32(p), f32(m), f32(v)
    for step in (1, 2, 3):
        gg = rng.standard_normal(1000)
        N.adam(pt, f32(gg), mt, vt, 1e-3, 0.9, 0.999, 1e-8, step)
        p, m, v = U.adam(p.astype(np.float32).astype(np.float64), gg.astype(np.float32).astype(np.float64),
                         m.astype(np.float32).astype(np.float64), v.astype(np.float32).astype(np.float64), step,
                         lr=1e-3)
        for a, b_ in ((pt, p), (mt, m), (vt, v)):
            assert rel_l2(host(a), b_) < 1e-6
        p, m, v = host(pt), host(mt), host(vt)


def _random_params(seed):
    rng = np.random.default_rng(seed)
    P = U.init_params(seed)
    P["c8.w"] = rng.standard_normal(P["c8.w"].shape) * 0.05
    for n, _, co in U.LAYERS:
        P[n + ".b"] = rng.standard_normal(co) * 0.05
    return P


def test_network_forward_and_gradients_vs_oracle():
    rng = np.random.default_rng(21)
    P = _random_params(4)
    img = rng.standard_normal((16, 16, 24)).astype(np.float32)
    tgt = (img + 0.3 * rng.standard_normal(img.shape)).astype(np.float32)
    net = N.UNet(P)
    out, loss = net.forward(f32(img)[None], f32(tgt)[None])
    net.backward()
    L, G, out_o = U.backward(P, img.astype(np.float64), tgt.astype(np.float64), quant=True)
    e_out = rel_l2(host(out)[0], out_o)
    print(f"network: loss {loss:.6e} vs {L:.6e}; output rel-L2 {e_out:.2e}")
    assert abs(loss - L) <= 1e-4 * L and e_out < 1e-4
    Gg = net.grads()
    errs = {k: rel_l2(Gg[k], G[k]) for k in G}
    print("gradient rel-L2:", {k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-3, errs
    # the one-channel layers hold only their real weights
    assert net.slots["c1.w"][1] == (16, 27, 1) and net.slots["c8.w"][1] == (1, 27, 16)


# The eight convolutions of the crosstalk network on a 128^3 image, each at
# the size it runs at (name, cin, cout, cube edge).
NET128 = (("c1", 1, 16, 128), ("c2", 16, 32, 64), ("c3", 32, 64, 32), ("c4", 64, 128, 16),
          ("c5", 128, 64, 32), ("c6", 64, 32, 64), ("c7", 32, 16, 128), ("c8", 16, 1, 128))


def _sample_points(n, rng, count=3000):
    """Random voxels of an n^3 cube plus its corners and face centres."""
    pts = rng.integers(0, n, (count, 3))
    e = (0, n - 1)
    corners = np.array([(a, b, c) for a in e for b in e for c in e])
    m = n // 2
    faces = np.array([(0, m, m), (n - 1, m, m), (m, 0, m), (m, n - 1, m), (m, m, 0), (m, m, n - 1)])
    return np.concatenate([pts, corners, faces])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,ci,co,n", NET128, ids=[r[0] for r in NET128])
def test_layer_parity_at_training_size(name, ci, co, n):
    """Each convolution of the 128^3 network at its real size (the one-
    channel weight gradients at their block cap, the coarse levels on their
    split grids): forward and input gradient on sampled voxels (faces and
    corners included) and the weight and bias gradients in full, against the
    oracle on the same bfloat16 operands."""
    rng = np.random.default_rng(1000 + ci * 7 + co)
    shape = (1, n, n, n)
    nvox = n ** 3
    x = U.bf16(rng.standard_normal((nvox, ci)).astype(np.float32))
    dy = U.bf16(rng.standard_normal((nvox, co)).astype(np.float32))
    wo = U.bf16(rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci)))
    b = rng.standard_normal(co) * 0.1
    wf, wb = pack(wo)
    xt, dyt = bf_tensor(x), bf_tensor(dy)
    y = torch.empty((nvox, co), dtype=torch.float32, device=DEV)
    N.conv3d_fwd(shape, ci, co, xt, wf, f32(b), False, y=y)
    dx = torch.empty((nvox, ci), dtype=torch.float32, device=DEV)
    N.conv3d_dgrad(shape, ci, co, dyt, wb, dx)
    ws = torch.empty(N.wgrad_ws_bytes(shape, ci, co), dtype=torch.uint8, device=DEV)
    dw = torch.empty((co, 27, ci), dtype=torch.float32, device=DEV)
    db = torch.empty(co, dtype=torch.float32, device=DEV)
    N.conv3d_wgrad(shape, ci, co, xt, dyt, dw, db, ws)
    pts = _sample_points(n, rng)
    flat = (pts[:, 0] * n + pts[:, 1]) * n + pts[:, 2]
    x_cf = x.reshape(n, n, n, ci).transpose(3, 0, 1, 2)
    dy_cf = dy.reshape(n, n, n, co).transpose(3, 0, 1, 2)
    e_f = rel_l2(host(y)[flat], U.conv3d_at(x_cf, wo, b, pts))
    e_d = rel_l2(host(dx)[flat], U.conv3d_dgrad_at(dy_cf, wo, pts))
    del y, dx
    ref_w, ref_b = U.conv3d_wgrad(x_cf, dy_cf)
    ref_w = np.transpose(ref_w.reshape(co, ci, 27), (0, 2, 1))
    e_w, e_b = rel_l2(host(dw), ref_w), rel_l2(host(db), ref_b)
    print(f"{name} {ci}->{co} at {n}^3: fwd {e_f:.2e} dgrad {e_d:.2e} wgrad {e_w:.2e} bias {e_b:.2e}")
    assert max(e_f, e_d, e_w, e_b) < 1e-5


# Channel pairs the LDS-staged kernel takes (<= 32 input and output
# channels, and 64 -> 32), as forward layers or as the flipped input-gradient
# convolutions.
LDS_PAIRS = ((16, 16), (16, 32), (32, 16), (32, 32), (64, 32))


@pytest.mark.parametrize("ci,co", LDS_PAIRS)
def test_lds_staged_convolution_equals_direct(ci, co):
    """On a ragged grid wide and large enough for the LDS-staged kernel
    (partial x-segment, y-rows and z-chunk, two samples) its forward
    convolution with the fused epilogue and its input gradient equal the
    direct kernel bit for bit, and the forward matches the oracle."""
    shape = (2, 67, 31, 131)
    rng, x, wo, b = _operands(shape, ci, co, 77 + ci + co)
    wf, wb = pack(wo)
    skip = U.bf16(rng.standard_normal((x.shape[0], co)))
    dy = U.bf16(rng.standard_normal((x.shape[0], co)))
    outs = []
    try:
        for lds in (True, False):
            N.set_conv_lds(lds)
            y = torch.empty((x.shape[0], co), dtype=torch.float32, device=DEV)
            r = torch.empty((x.shape[0], co), dtype=torch.bfloat16, device=DEV)
            out = torch.empty_like(r)
            N.conv3d_fwd(shape, ci, co, bf_tensor(x), wf, f32(b), True, skip=bf_tensor(skip), y=y, r=r, out=out)
            dx = torch.empty((x.shape[0], ci), dtype=torch.float32, device=DEV)
            N.conv3d_dgrad(shape, ci, co, bf_tensor(dy), wb, dx)
            outs.append((y, r, out, dx))
    finally:
        N.set_conv_lds(True)
    for a, c in zip(*outs):
        assert torch.equal(a, c)
    y0 = outs[0][0]
    ref = np.maximum(from_cf([U.conv3d(xc, U.bf16(wo), b) for xc in to_cf(x, shape, ci)]), 0.0)
    e = rel_l2(host(y0), ref)
    print(f"LDS conv {ci}->{co} {shape}: equal to the direct kernel; forward vs oracle {e:.2e}")
    assert e < 1e-5


@pytest.mark.parametrize("ci,co,shape", [(16, 1, (2, 9, 7, 70)), (16, 32, (2, 67, 31, 131)), (64, 128, (1, 6, 5, 9)),
                                         (32, 64, (2, 7, 6, 11))])
def test_dgrad_with_fused_relu_gradient(ci, co, shape):
    """The input gradient with the layer below's ReLU gradient fused in
    (one-channel, LDS-staged and direct kernels): dx equals the plain input
    gradient and g_out equals unet_relu_grad of that dx, bit for bit."""
    rng, x, wo, b = _operands(shape, ci, co, 5 + ci + co)
    _, wb = pack(wo)
    nv = x.shape[0]
    dy = bf_tensor(U.bf16(rng.standard_normal((nv, co))))
    mask = bf_tensor(U.bf16(np.maximum(rng.standard_normal((nv, ci)), 0)))
    dx0 = torch.empty((nv, ci), dtype=torch.float32, device=DEV)
    N.conv3d_dgrad(shape, ci, co, dy, wb, dx0)
    g0 = torch.empty((nv, ci), dtype=torch.bfloat16, device=DEV)
    N.relu_grad(shape, ci, dx0, None, None, mask, g0)
    dx1 = torch.empty_like(dx0)
    g1 = torch.empty_like(g0)
    N.conv3d_dgrad(shape, ci, co, dy, wb, dx1, mask, g1)
    assert torch.equal(dx1, dx0) and torch.equal(g1, g0)
    assert bool((host(g1) != 0).any())


@pytest.mark.parametrize("c", [32, 6])
def test_up2_bwd_with_fused_relu_gradient(c):
    """The upsampling adjoint with the coarse level's ReLU gradient fused in
    equals up2_bwd followed by relu_grad, bit for bit (4 channels per thread
    and 1)."""
    rng = np.random.default_rng(c)
    shape = (2, 3, 4, 5)
    nc = int(np.prod(shape))
    gf = f32(rng.standard_normal((nc * 8, c)).astype(np.float32))
    mask = bf_tensor(U.bf16(np.maximum(rng.standard_normal((nc, c)), 0)))
    gc0 = torch.empty((nc, c), dtype=torch.float32, device=DEV)
    N.up2_bwd(shape, c, gf, gc0)
    o0 = torch.empty((nc, c), dtype=torch.bfloat16, device=DEV)
    N.relu_grad(shape, c, gc0, None, None, mask, o0)
    gc1 = torch.empty_like(gc0)
    o1 = torch.empty_like(o0)
    N.up2_bwd(shape, c, gf, gc1, mask, o1)
    assert torch.equal(gc1, gc0) and torch.equal(o1, o0)


def test_weight_pack_many_equals_per_layer_packing():
    """One launch for several layers packs the same bits as one call each."""
    rng = np.random.default_rng(9)
    layers = [(1, 16), (16, 32), (64, 128), (16, 1)]
    singles, many = [], []
    for ci, co in layers:
        w = f32(rng.standard_normal((co, 27 * ci)).astype(np.float32))
        a = (torch.empty((co, 27 * ci), dtype=torch.bfloat16, device=DEV),
             torch.empty((ci, 27 * co), dtype=torch.bfloat16, device=DEV))
        b = (torch.zeros_like(a[0]), torch.zeros_like(a[1]))
        N.weight_pack(w, ci, co, *a)
        singles.append(a)
        many.append((w, ci, co) + b)
    N.weight_pack_many(many)
    for a, (_, _, _, bf, bb) in zip(singles, many):
        assert torch.equal(a[0], bf) and torch.equal(a[1], bb)


def test_wgrad_partial_and_reduce_many_equal_per_layer_wgrad():
    """The partial pass per layer plus one batched reduction gives the bits of
    one conv3d_wgrad call per layer, for every partial layout: the
    one-channel pairs on the matrix cores, the ring-staged pairs (64^3), the
    plain split-K kernel on the coarse grids; one item without a bias."""
    rng = np.random.default_rng(21)
    cases = [((1, 64, 64, 64), 1, 16), ((1, 64, 64, 64), 16, 1), ((1, 64, 64, 64), 16, 32),
             ((1, 64, 64, 64), 32, 16), ((1, 32, 32, 32), 64, 32), ((1, 16, 16, 16), 64, 128),
             ((1, 16, 16, 16), 128, 64), ((2, 8, 12, 20), 32, 64)]
    singles, items = [], []
    for i, (shape, ci, co) in enumerate(cases):
        nvox = int(np.prod(shape))
        xt = bf_tensor(U.bf16(rng.standard_normal((nvox, ci)).astype(np.float32)))
        dyt = bf_tensor(U.bf16(rng.standard_normal((nvox, co)).astype(np.float32)))
        nb = N.wgrad_ws_bytes(shape, ci, co)
        ws1 = torch.empty(nb, dtype=torch.uint8, device=DEV)
        ws2 = torch.empty(nb, dtype=torch.uint8, device=DEV)
        dw1 = torch.empty((co, 27, ci), dtype=torch.float32, device=DEV)
        db1 = torch.empty(co, dtype=torch.float32, device=DEV)
        N.conv3d_wgrad(shape, ci, co, xt, dyt, dw1, db1, ws1)
        dw2 = torch.full_like(dw1, float("nan"))
        db2 = None if i == 2 else torch.full_like(db1, float("nan"))
        N.conv3d_wgrad_partial(shape, ci, co, xt, dyt, ws2)
        singles.append((dw1, db1))
        items.append((shape, ci, co, ws2, dw2, db2))
    N.wgrad_reduce_many(items)
    torch.cuda.synchronize()
    for (dw1, db1), (shape, ci, co, _, dw2, db2) in zip(singles, items):
        assert torch.equal(dw1, dw2), (shape, ci, co)
        assert db2 is None or torch.equal(db1, db2), (shape, ci, co)
        assert float(dw1.abs().max()) > 0


def test_captured_pass_matches_eager_training():
    """Three training steps as graph replay + step() give the same
    parameters, bit for bit, as three eager steps from the same start, with
    eager work and synchronisation between the replays."""
    g = torch.Generator(device=DEV).manual_seed(3)
    img = torch.randn((1, 16, 16, 16), device=DEV, generator=g)
    tgt = img + 0.1 * torch.randn((1, 16, 16, 16), device=DEV, generator=g)
    eager = N.UNet(seed=1)
    graphed = N.UNet(seed=1)
    # the identity start (zero output layer) gives zero gradients below it at
    # step one; two eager steps first make every layer's gradient nonzero
    for net in (eager, graphed):
        for _ in range(2):
            net.train_step(img, tgt, 1e-3)
    graph = graphed.capture_pass(img, tgt)
    for k in range(3):
        eager.forward(img, tgt, want_loss=False)
        eager.backward()
        eager.step(1e-3)
        junk = torch.randn(1 << 18, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        graphed.step(1e-3)
        torch.cuda.synchronize()
        assert torch.equal(graphed.p, eager.p), f"step {k}"
        assert torch.equal(graphed.g, eager.g), f"step {k}"
        del junk
    assert bool((eager.g != 0).any())
