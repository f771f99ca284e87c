"""Host-side checks of the Python binding's stream handling (no GPU).

BatchPlan.run on a stream other than the current one must order the run
after the current stream's work (wait_stream) and mark every tensor the run
touches as in use on the side stream (record_stream), so that torch's
caching allocator reuses none of that memory, in either direction, before
the run is done with it.  The device call itself is replaced by a recorder.
"""
import types

import paper_2204_03380_amd as rtm
from paper_2204_03380_amd import _lib


class _Stream:
    def __init__(self, handle):
        self.cuda_stream = handle
        self.waited = []

    def wait_stream(self, other):
        self.waited.append(other.cuda_stream)


class _Tensor:
    def __init__(self, name, log):
        self.name, self.log = name, log

    def data_ptr(self):
        return 4096

    def numel(self):
        return 1 << 20

    def record_stream(self, stream):
        self.log.append((self.name, stream.cuda_stream))


def _plan(log):
    plan = object.__new__(rtm.BatchPlan)
    plan._plan = None
    plan.device = "cuda:0"
    plan.ws = _Tensor("ws", log)
    shots = []
    for i in range(2):
        t = {k: _Tensor(f"{k}{i}", log) for k in ("v_pad", "wavelet", "traces_in", "image")}
        shots.append(types.SimpleNamespace(traces_out=None, grad_v_pad=None, **t))
    plan._shots = shots
    return plan


def _patch(monkeypatch, cur, calls):
    monkeypatch.setattr(rtm.torch.cuda, "current_stream", lambda device=None: cur)
    fake = types.SimpleNamespace(rtm_batch_run=lambda p, ws, n, st: calls.append(st) or 0,
                                 rtm_batch_free=lambda p: 0)
    monkeypatch.setattr(_lib, "load", lambda: fake)


def test_side_stream_run_waits_and_records_every_tensor(monkeypatch):
    log, calls = [], []
    cur, side = _Stream(111), _Stream(222)
    _patch(monkeypatch, cur, calls)
    plan = _plan(log)
    plan.run(side)
    assert side.waited == [111]
    assert calls == [222]
    names = {n for n, _ in log}
    assert names == {"ws", "v_pad0", "wavelet0", "traces_in0", "image0", "v_pad1", "wavelet1", "traces_in1",
                     "image1"}
    assert all(s == 222 for _, s in log)


def test_current_stream_run_records_nothing(monkeypatch):
    log, calls = [], []
    cur = _Stream(111)
    _patch(monkeypatch, cur, calls)
    plan = _plan(log)
    plan.run()
    plan.run(_Stream(111))  # the current stream passed explicitly
    assert calls == [111, 111]
    assert log == [] and cur.waited == []


def test_run_without_a_bound_workspace_is_refused(monkeypatch):
    """A plan made with defer_workspace=True has no workspace until
    bind_workspace: run() raises before any device call."""
    log, calls = [], []
    _patch(monkeypatch, _Stream(111), calls)
    plan = _plan(log)
    plan.ws = None
    try:
        plan.run()
    except RuntimeError as e:
        assert "no workspace" in str(e)
    else:
        raise AssertionError("run() without a workspace was not refused")
    assert calls == []
