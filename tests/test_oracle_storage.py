"""Pins of the storage-RTM oracle (Algorithm 2 with the snapshot
decimation of Eq. (7)) against values fixed outside the oracle: the paper's
printed Nyquist steps and storage sizes, the derivative identity of the image
numerator, brute force over separately computed wavefields, and the
partition of the time levels over decimation phases."""
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nyquist_storage.txt")


def _golden():
    out = {}
    with open(GOLD) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[line[0]] = [float(x) for x in line[1:]]
    return out


def kept_levels(nt, stride, phase):
    """Time levels k in [0, nt) with k = phase (mod stride), by enumeration."""
    return [k for k in range(nt) if k % stride == phase]


def test_nyquist_stride_paper_examples():
    g = _golden()
    f_max, f_min, dt, dtn, stride = g["nyquist"]
    assert 1.0 / (2.0 * (f_max - f_min)) == pytest.approx(dtn, rel=1e-12)
    assert oracle.nyquist_stride(dt, f_max, f_min) == int(stride)
    dtn3, dt3, stride3 = g["nyquist_dt"]
    # 3-D: dt_nyq = 10 ms means a 50 Hz band (Eq. (7) solved for f_max)
    assert oracle.nyquist_stride(dt3, 1.0 / (2.0 * dtn3)) == int(stride3)
    # a band narrower than the Nyquist rate of dt never gives stride 0
    assert oracle.nyquist_stride(1e-3, 1000.0) == 1


def test_storage_size_matches_table4():
    """Levels 0 .. T/dt (inclusive) every stride-th step, full padded grid,
    4-byte samples: the printed 132.062 GB is that count in GiB."""
    nx, ny, nz, T, dt, stride, gb_store, gb_rec, ratio = _golden()["storage3d"]
    cells = int(nx) * int(ny) * int(nz)
    nlev = int(round(T / dt)) + 1
    count = len(kept_levels(nlev, int(stride), 0))
    assert count == 601
    gib = 2.0 ** 30
    assert round(count * cells * 4 / gib, 3) == gb_store
    assert round(2 * cells * 4 / gib, 3) == gb_rec
    assert round(gb_store / gb_rec, 2) == ratio  # the printed ratio is that of the rounded sizes


def _setup(nt=120, seed=23):
    s = synth.config_small2d(nt=nt)
    vp = oracle.rbc_pad(s.v_int, s.nb, seed, 0.0)
    return s, vp


def test_storage_stride1_numerator_is_derivative():
    """Stride 1: num equals the derivative of <g, d> with respect to a model
    perturbation (the pairing of p^k with mu^(k+1) in Eq. (3))."""
    s, vp = _setup()
    rng = np.random.default_rng(11)
    g = rng.standard_normal((s.rec.shape[0], s.nt + 1))
    out = oracle.rtm_storage_shot(vp, s.h, s.nb, s.dt, s.wavelet, s.src[0], s.rec, g, stride=1)
    num = out["num"]
    big = np.argwhere(np.abs(num) >= 1e-2 * np.abs(num).max())
    cells = big[np.random.default_rng(12).choice(len(big), size=4, replace=False)]
    eps = 1e-5
    for (iz, ix) in cells:
        m = np.zeros(vp.shape)
        m[iz + s.nb, ix + s.nb] = eps
        dp = oracle.model_shot(vp, s.h, s.nb, s.dt, s.wavelet, s.src[0], s.rec, m=m)
        dm = oracle.model_shot(vp, s.h, s.nb, s.dt, s.wavelet, s.src[0], s.rec, m=-m)
        fd = (np.sum(g * dp) - np.sum(g * dm)) / (2 * eps)
        assert abs(fd - num[iz, ix]) <= 1e-6 * abs(num[iz, ix]) + 1e-9 * np.abs(num).max(), (iz, ix)


def _mu_level(vp, s, w, g, j):
    """mu^j of the reverse pass for trace g, from the reconstruction oracle's
    snapshot.  Two zero samples appended to the trace (and the wavelet) leave
    every level j <= nt unchanged and bring j = nt - 1 and nt in range."""
    g2 = np.concatenate([g, np.zeros((g.shape[0], 2))], axis=1)
    w2 = np.concatenate([w, [0.0, 0.0]])
    return oracle.rtm_shot(vp, s.h, s.nb, s.dt, w2, s.src[0], s.rec, g2, snap_k=j)["snap_mu"]


@pytest.mark.parametrize("stride,phase", [(7, 0), (7, 3), (4, 3)])
def test_storage_sums_bruteforce(stride, phase):
    """num and den over the kept levels, each level's source wavefield from
    its own modeling run and each receiver wavefield from the reconstruction
    oracle's snapshot (pinned separately by the adjoint and time-reversal
    tests)."""
    nt = 60
    s, vp = _setup(nt=nt)
    rng = np.random.default_rng(13)
    g = rng.standard_normal((s.rec.shape[0], nt + 1))
    w = s.wavelet[:nt]
    out = oracle.rtm_storage_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec, g, stride=stride, phase=phase)
    num = np.zeros(vp.shape)
    den = np.zeros(vp.shape)
    kept = kept_levels(nt, stride, phase)
    assert kept[-1] >= nt - stride  # the top levels are covered
    for k in kept:
        if k == 0:
            continue  # p^0 = 0
        _, pk, _ = oracle.model_shot(vp, s.h, s.nb, s.dt, w[:k], s.src[0], s.rec, want_last=True)
        mu = _mu_level(vp, s, w, g, k + 1)
        num += pk * mu
        den += pk * pk
    crop = (slice(s.nb, s.nb + s.v_int.shape[0]), slice(s.nb, s.nb + s.v_int.shape[1]))
    assert np.abs(out["num"] - num[crop]).max() <= 1e-12 * np.abs(num[crop]).max()
    assert np.abs(out["den"] - den[crop]).max() <= 1e-12 * np.abs(den[crop]).max()


def test_storage_phases_partition_stride1():
    """Summing the decimated sums over every phase gives the stride-1 sums,
    which equal the reconstruction oracle's sums."""
    s, vp = _setup(nt=90)
    rng = np.random.default_rng(14)
    g = rng.standard_normal((s.rec.shape[0], s.nt + 1))
    full = oracle.rtm_storage_shot(vp, s.h, s.nb, s.dt, s.wavelet, s.src[0], s.rec, g, stride=1)
    rec = oracle.rtm_shot(vp, s.h, s.nb, s.dt, s.wavelet, s.src[0], s.rec, g, eps_rel=1e-3)
    for key in ("num", "den"):
        assert np.abs(full[key] - rec[key]).max() <= 1e-12 * np.abs(rec[key]).max()
    acc = {"num": 0.0, "den": 0.0}
    for ph in range(5):
        o = oracle.rtm_storage_shot(vp, s.h, s.nb, s.dt, s.wavelet, s.src[0], s.rec, g, stride=5, phase=ph)
        for key in acc:
            acc[key] = acc[key] + o[key]
    for key in acc:
        assert np.abs(acc[key] - full[key]).max() <= 1e-12 * np.abs(full[key]).max()
    img = full["num"] / (full["den"] + 1e-3 * full["den"].max())
    assert np.allclose(full["image"], img, rtol=1e-14, atol=0)


def test_storage_rejects_bad_decimation():
    s, vp = _setup(nt=20)
    g = np.zeros((s.rec.shape[0], s.nt + 1))
    for stride, phase in ((0, 0), (3, 3), (3, -1)):
        with pytest.raises(RuntimeError):
            oracle.rtm_storage_shot(vp, s.h, s.nb, s.dt, s.wavelet, s.src[0], s.rec, g, stride=stride, phase=phase)
