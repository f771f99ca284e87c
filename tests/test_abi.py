"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and rejects bad arguments on the host before any GPU work is queued."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2204_03380_amd as rtm
from paper_2204_03380_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b((?:rtm|unet)_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == names
    assert lib.rtm_abi_version() == 1


def test_workspace_bytes_and_grid_validation():
    g = rtm.Grid(2, 201, 1, 201, 10.0, 40)
    sizes = [rtm.rtm_workspace_bytes(g, op, 201, 1000) for op in range(4)]
    assert sizes[0] > 0 and sizes[1] < sizes[3] <= sizes[2] * 2
    assert rtm.rtm_workspace_bytes(g, rtm.RTM_OP_RTM, 201, 2000) > sizes[2]
    for bad in (rtm.Grid(4, 10, 1, 10, 10.0, 2), rtm.Grid(2, 0, 1, 10, 10.0, 2), rtm.Grid(2, 10, 1, 10, 0.0, 2),
                rtm.Grid(2, 10, 1, 10, 10.0, -1), rtm.Grid(3, 10, 0, 10, 10.0, 2)):
        with pytest.raises(rtm.RtmError) as e:
            rtm.rtm_workspace_bytes(bad, rtm.RTM_OP_MODEL, 1, 1)
        assert e.value.status == _lib.RTM_EINVAL
    with pytest.raises(rtm.RtmError):
        rtm.rtm_workspace_bytes(g, 7, 1, 1)
    # every extent is allowed on its own, but a field of 2^31 floats or more
    # is refused (cell offsets are 32-bit), in 3-D and in 2-D
    assert rtm.rtm_workspace_bytes(rtm.Grid(3, 1250, 1250, 1250, 10.0, 0), rtm.RTM_OP_MODEL, 1, 1) > 0
    for big in (rtm.Grid(3, 1300, 1300, 1300, 10.0, 0), rtm.Grid(3, 200000, 10, 1000, 10.0, 0),
                rtm.Grid(2, 60000, 1, 40000, 10.0, 0)):
        with pytest.raises(rtm.RtmError) as e:
            rtm.rtm_workspace_bytes(big, rtm.RTM_OP_MODEL, 1, 1)
        assert e.value.status == _lib.RTM_EINVAL and "2^31" in str(e.value)


def test_set_tuning_validation():
    with pytest.raises(rtm.RtmError):
        rtm.rtm_set_tuning(rtm.RTM_OP_MODEL, 3, 16)
    with pytest.raises(rtm.RtmError):
        rtm.rtm_set_tuning(rtm.RTM_OP_MODEL, 1, 2)
    with pytest.raises(rtm.RtmError):
        rtm.rtm_set_tuning(rtm.RTM_OP_MODEL, 1, 16)   # not a multiple of 9
    old = rtm.rtm_get_tuning2d(rtm.RTM_OP_RTM)
    with pytest.raises(rtm.RtmError):
        rtm.rtm_set_tuning2d(rtm.RTM_OP_RTM, 1, 3, 9)    # tx must be 1, 2 or 4
    rtm.rtm_set_tuning2d(rtm.RTM_OP_RTM, 2, 4, 27)
    assert rtm.rtm_get_tuning2d(rtm.RTM_OP_RTM) == (2, 4, 27)
    rtm.rtm_set_tuning(rtm.RTM_OP_RTM, 1, 9)              # keeps tx
    assert rtm.rtm_get_tuning2d(rtm.RTM_OP_RTM) == (1, 4, 9)
    rtm.rtm_set_tuning2d(rtm.RTM_OP_RTM, *old)
    rtm.rtm_set_tuning(rtm.RTM_OP_MODEL, 1, 18)


def test_set_tuning3d_validation():
    old_f, old_r = rtm.rtm_get_tuning3d(rtm.RTM_OP_MODEL), rtm.rtm_get_tuning3d(rtm.RTM_OP_RTM)
    try:
        for op, vec, ty, zseg in ((rtm.RTM_OP_MODEL, 1, 2, 18),     # ty must be 4, 8 or 16
                                  (rtm.RTM_OP_MODEL, 4, 16, 18),    # 16 rows: vec <= 2
                                  (rtm.RTM_OP_RTM, 2, 16, 18),      # 16 rows, reverse: vec 1
                                  (rtm.RTM_OP_VJP, 2, 16, 18),
                                  (rtm.RTM_OP_RTM, 1, 16, 10)):     # zseg not a multiple of 9
            with pytest.raises(rtm.RtmError):
                rtm.rtm_set_tuning3d(op, vec, ty, zseg)
        rtm.rtm_set_tuning3d(rtm.RTM_OP_MODEL, 2, 16, 27)
        rtm.rtm_set_tuning3d(rtm.RTM_OP_RTM, 1, 16, 18)
        assert rtm.rtm_get_tuning3d(rtm.RTM_OP_MODEL) == (2, 16, 27)
        assert rtm.rtm_get_tuning3d(rtm.RTM_OP_RTM) == (1, 16, 18)
        # tile order: 0 or 1, per operation, kept by rtm_set_tuning3d
        for bad_order in (-1, 2):
            with pytest.raises(rtm.RtmError):
                rtm.rtm_set_tile_order3d(rtm.RTM_OP_RTM, bad_order)
        with pytest.raises(rtm.RtmError):
            rtm.rtm_set_tile_order3d(99, 1)
        assert rtm.rtm_get_tile_order3d(rtm.RTM_OP_RTM) == 0
        rtm.rtm_set_tile_order3d(rtm.RTM_OP_RTM, 1)
        rtm.rtm_set_tuning3d(rtm.RTM_OP_RTM, 1, 8, 36)
        assert rtm.rtm_get_tile_order3d(rtm.RTM_OP_RTM) == 1 and rtm.rtm_get_tile_order3d(rtm.RTM_OP_MODEL) == 0
        assert rtm.rtm_get_tile_order3d(rtm.RTM_OP_VJP) == 1  # the reverse kernels' setting
    finally:
        rtm.rtm_set_tuning3d(rtm.RTM_OP_MODEL, *old_f)
        rtm.rtm_set_tuning3d(rtm.RTM_OP_RTM, *old_r)
        rtm.rtm_set_tile_order3d(rtm.RTM_OP_MODEL, 0)
        rtm.rtm_set_tile_order3d(rtm.RTM_OP_RTM, 0)


def _call_model(grid, nt=10, src=(5.0, 0.0, 3.0), rec=((1.0, 0.0, 2.0),), ws_bytes=None, ws=0x100000,
                nrec=None, traces=0x3000):
    """Call rtm_model_shot with fake (never dereferenced) device addresses:
    every case below fails host validation before any device work."""
    lib = _lib.load()
    g = grid.c()
    s = np.ascontiguousarray(np.array(src, np.float32))
    r = np.ascontiguousarray(np.array(rec, np.float32).reshape(-1, 3))
    n = r.shape[0] if nrec is None else nrec
    if ws_bytes is None:
        ws_bytes = rtm.rtm_workspace_bytes(grid, rtm.RTM_OP_MODEL, max(n, 1), max(nt, 1))
    return lib.rtm_model_shot(ctypes.byref(g), 0x1000, 1e-3, nt, 0x2000, s.ctypes.data_as(ctypes.c_void_p), n,
                              r.ctypes.data_as(ctypes.c_void_p), traces, None, None, 0, ws, ws_bytes, None)


def test_host_validation_errors():
    g = rtm.Grid(2, 20, 1, 12, 10.0, 4)
    assert _call_model(g, nt=0) == _lib.RTM_EINVAL
    assert _call_model(g, nrec=0) == _lib.RTM_EINVAL
    assert _call_model(g, traces=None) == _lib.RTM_EINVAL
    assert _call_model(g, src=(20.0, 0.0, 3.0)) == _lib.RTM_ERANGE      # x == nx: outside
    assert _call_model(g, src=(-0.01, 0.0, 3.0)) == _lib.RTM_ERANGE
    assert _call_model(g, rec=((1.0, 0.0, 11.5),)) == _lib.RTM_ERANGE   # z > nz - 1
    assert _call_model(g, ws=None) == _lib.RTM_EWORKSPACE
    assert _call_model(g, ws=0x100010) == _lib.RTM_EWORKSPACE           # misaligned
    assert _call_model(g, ws_bytes=1024) == _lib.RTM_EWORKSPACE
    msg = _lib.load().rtm_last_error().decode()
    assert "workspace" in msg


def test_storage_host_helpers():
    """Eq. (7) step and stored-level count (host-only entry points), against
    the paper's printed examples and enumeration."""
    assert rtm.rtm_nyquist_stride(0.5e-3, 100.0, 0.0) == 10     # 5 ms / 0.5 ms
    assert rtm.rtm_nyquist_stride(1e-3, 50.0) == 10             # 10 ms / 1 ms (3-D)
    assert rtm.rtm_nyquist_stride(1e-3, 1000.0) == 1
    assert rtm.rtm_nyquist_stride(1e-3, 60.0, 10.0) == 10       # band of 50 Hz
    for bad in ((0.0, 100.0, 0.0), (1e-3, 10.0, 10.0), (1e-3, 10.0, -1.0), (1e-3, float("inf"), 0.0)):
        with pytest.raises(rtm.RtmError):
            rtm.rtm_nyquist_stride(*bad)
    assert rtm.rtm_storage_count(6001, 10, 0) == 601            # 0 .. 6 s every 10 ms
    for nt, stride, phase in ((1, 1, 0), (10, 3, 2), (9, 3, 2), (5, 7, 6), (100, 10, 9)):
        assert rtm.rtm_storage_count(nt, stride, phase) == len([k for k in range(nt) if k % stride == phase])
    for bad in ((0, 1, 0), (10, 0, 0), (10, 3, 3), (10, 3, -1)):
        with pytest.raises(rtm.RtmError):
            rtm.rtm_storage_count(*bad)


def test_storage_shot_validation():
    """rtm_storage_shot rejects a short snapshot buffer and a bad
    decimation before any device work (fake device addresses)."""
    lib = _lib.load()
    grid = rtm.Grid(2, 20, 1, 12, 10.0, 4)
    g = grid.c()
    nt = 10
    s = np.ascontiguousarray(np.array((5.0, 0.0, 3.0), np.float32))
    r = np.ascontiguousarray(np.array(((1.0, 0.0, 2.0),), np.float32))
    ws_bytes = rtm.rtm_workspace_bytes(grid, rtm.RTM_OP_STORAGE, 1, nt)
    assert ws_bytes > 0

    def call(stride, phase, snap_bytes, snaps=0x4000):
        return lib.rtm_storage_shot(ctypes.byref(g), 0x1000, 1e-3, nt, 0x2000, s.ctypes.data_as(ctypes.c_void_p), 1,
                                    r.ctypes.data_as(ctypes.c_void_p), 0x3000, stride, phase, 1e-3, 0x5000, None,
                                    None, snaps, snap_bytes, 0, 0x100000, ws_bytes, None)

    need = 4 * 20 * 12 * 4      # stride 3: levels 0, 3, 6, 9
    assert call(3, 0, need - 1) == _lib.RTM_EINVAL
    assert call(3, 0, need, snaps=None) == _lib.RTM_EINVAL
    assert call(0, 0, need) == _lib.RTM_EINVAL
    assert call(3, 3, need) == _lib.RTM_EINVAL


def test_band_options_validation():
    """rtm_rbc_pad_ex / rtm_pad_adjoint_ex reject bad options on the host
    (fake device addresses, never dereferenced)."""
    lib = _lib.load()
    for nb, flags, alpha in ((4, 0x1, 1.5), (4, 0x1, -0.1), (4, 0x4, 0.0), (300, 0x1, 0.5)):
        g = rtm.Grid(2, 20, 1, 12, 10.0, nb).c()
        o = _lib.RtmRbcOpts(1, 3000.0, flags, alpha)
        assert lib.rtm_rbc_pad_ex(ctypes.byref(g), 0x1000, ctypes.byref(o), 0x2000, None, 0, None) == _lib.RTM_EINVAL
        assert lib.rtm_pad_adjoint_ex(ctypes.byref(g), 0x1000, ctypes.byref(o), 0x3000, 0x2000, None, 0,
                                      None) == _lib.RTM_EINVAL
    g = rtm.Grid(2, 20, 1, 12, 10.0, 4).c()
    assert lib.rtm_rbc_pad_ex(ctypes.byref(g), 0x1000, None, 0x2000, None, 0, None) == _lib.RTM_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more, it exits with status 2 and
    says why, before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and not r.stdout.strip()


def test_unet_channel_pairs_on_the_host():
    """The convolution entry points take two of 16/32/64/128 channels or the
    one-channel pairs (1, 16) and (16, 1); anything else is rejected before
    any launch.  The one-channel weight gradient's workspace holds one
    partial of 27*16 weights and 16 (or 1) biases per wavefront, four per
    job (n, 4 planes, a 32-voxel x segment, a y range of at least 8 rows,
    about 2048 jobs), plus the two-pass chunk sums."""
    lib = _lib.load()
    sz = ctypes.c_size_t(0)

    def ws(shape, ci, co):
        d = _lib.UnetConvDesc(*shape, ci, co)
        return lib.unet_wgrad_ws_bytes(ctypes.byref(d), ctypes.byref(sz)), sz.value

    def rnd(b):
        return (b + 255) // 256 * 256

    def thin_bytes(parts, nb):
        chunk = 128 if parts >= 2048 else 32  # partials per first-pass chunk
        q = (parts + chunk - 1) // chunk
        return rnd(parts * 432 * 4) + rnd(parts * nb * 4) + rnd(q * 432 * 4) + rnd(q * nb * 4)

    for ci, co in ((16, 16), (32, 64), (128, 64), (1, 16), (16, 1)):
        rc, b = ws((1, 8, 8, 8), ci, co)
        assert rc == _lib.RTM_OK and b > 0, (ci, co)
    for ci, co in ((1, 32), (32, 1), (1, 1), (8, 16), (16, 8), (2, 16), (0, 16)):
        rc, _ = ws((1, 8, 8, 8), ci, co)
        assert rc == _lib.RTM_EINVAL, (ci, co)
    # (1, 16) at 64^3: 16 plane blocks x 2 segments, y ranges capped at 64 / 8:
    # 256 jobs, 1024 partials
    rc, b = ws((1, 64, 64, 64), 1, 16)
    assert rc == _lib.RTM_OK and b == thin_bytes(1024, 16)
    # (16, 1) at 128^3: 32 x 4 columns x 16 y ranges = 2048 jobs
    rc, b = ws((1, 128, 128, 128), 16, 1)
    assert rc == _lib.RTM_OK and b == thin_bytes(8192, 1)
    # ragged two-sample grid: 2 x ceil(19 / 4) x ceil(70 / 32) = 30 columns, 23 // 8 = 2 y ranges
    rc, b = ws((2, 19, 23, 70), 1, 16)
    assert rc == _lib.RTM_OK and b == thin_bytes(4 * 60, 16)
    # tiny images still get one job
    rc, b = ws((1, 2, 2, 2), 1, 16)
    assert rc == _lib.RTM_OK and b == thin_bytes(4, 16)


def test_wgrad_reduce_many_validation_on_the_host():
    """The batched reduction rejects a count outside [1, UNET_WGRAD_MAX], a
    missing item array or dw, an unsupported channel pair and a workspace
    that is missing, short or misaligned, all before any launch (the
    pointers below are never dereferenced)."""
    lib = _lib.load()
    sz = ctypes.c_size_t(0)
    d = _lib.UnetConvDesc(1, 8, 8, 8, 16, 32)
    assert lib.unet_wgrad_ws_bytes(ctypes.byref(d), ctypes.byref(sz)) == _lib.RTM_OK
    need = sz.value

    def call(count, **kw):
        items = (_lib.UnetWgradItem * max(count, 1))()
        for it in items:
            it.desc = kw.get("desc", d)
            it.ws, it.ws_bytes, it.dw, it.db = kw.get("ws", 4096), kw.get("ws_bytes", need), kw.get("dw", 8192), None
        return lib.unet_wgrad_reduce_many(count, items, None)

    assert call(0) == _lib.RTM_EINVAL
    assert call(_lib.UNET_WGRAD_MAX + 1) == _lib.RTM_EINVAL
    assert lib.unet_wgrad_reduce_many(1, None, None) == _lib.RTM_EINVAL
    assert call(2, dw=None) == _lib.RTM_EINVAL
    assert call(1, desc=_lib.UnetConvDesc(1, 8, 8, 8, 8, 16)) == _lib.RTM_EINVAL
    for kw in ({"ws": None}, {"ws_bytes": need - 1}, {"ws": 4096 + 128}):
        assert call(1, **kw) == _lib.RTM_EWORKSPACE, kw
    assert "workspace" in lib.rtm_last_error().decode()
    # the partial pass takes the same workspace rules
    assert lib.unet_conv3d_wgrad_partial(ctypes.byref(d), 4096, 4096, 4096, need - 1, None) == _lib.RTM_EWORKSPACE
    assert lib.unet_conv3d_wgrad_partial(ctypes.byref(d), None, 4096, 4096, need, None) == _lib.RTM_EINVAL


def test_persistent_plan_validation_on_the_host():
    """RTM_F_PERSISTENT: refused with RTM_F_GRAPH and for 3-D shots at plan
    time (no device work; fake device addresses are never dereferenced);
    the wait limit is range-checked and read back."""
    lib = _lib.load()

    def plan(grid, flags):
        d = _lib.RtmShotDesc()
        d.grid = grid.c()
        d.v_pad, d.wavelet, d.traces_out = 0x10000, 0x20000, 0x30000
        d.src[0], d.src[1], d.src[2] = 2.0, 1.0 if grid.ndim == 3 else 0.0, 2.0
        rec = np.ascontiguousarray(np.array([[1.0, 1.0 if grid.ndim == 3 else 0.0, 2.0]], np.float32))
        d.nrec, d.rec = 1, rec.ctypes.data
        out, ws = ctypes.c_void_p(), ctypes.c_size_t()
        rc = lib.rtm_batch_plan(rtm.RTM_OP_MODEL, 1, ctypes.byref(d), 1e-3, 20, 1e-3, flags, ctypes.byref(out),
                                ctypes.byref(ws))
        if rc == 0:
            lib.rtm_batch_free(out)
        return rc, ws.value

    g2 = rtm.Grid(2, 30, 1, 20, 10.0, 4)
    rc, ws_p = plan(g2, rtm.RTM_F_PERSISTENT)
    assert rc == 0
    rc, ws_n = plan(g2, 0)
    assert rc == 0 and ws_p > ws_n  # work items, counters and status word
    assert plan(g2, rtm.RTM_F_PERSISTENT | rtm.RTM_F_GRAPH)[0] == _lib.RTM_EINVAL
    assert plan(rtm.Grid(3, 10, 10, 10, 10.0, 2), rtm.RTM_F_PERSISTENT)[0] == _lib.RTM_EINVAL
    old = rtm.rtm_get_persist_wait()
    assert old == 4000.0
    for bad in (-1.0, float("nan"), 4e6):
        with pytest.raises(rtm.RtmError):
            rtm.rtm_set_persist_wait(bad)
    rtm.rtm_set_persist_wait(250.0)
    assert rtm.rtm_get_persist_wait() == 250.0
    rtm.rtm_set_persist_wait(old)
