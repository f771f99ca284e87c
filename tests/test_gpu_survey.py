"""Survey migration with shot-granular checkpoints: an interrupted run that
resumes from its checkpoint ends with the same stack, bit for bit, as an
uninterrupted one, and that stack matches the oracle's sum of shot images."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2204_03380_amd as rtm
import synth
from paper_2204_03380_amd.survey import migrate_survey

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_checkpoint_resume_bit_identical(tmp_path):
    s = synth.config_small2d(nt=150)
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, torch.from_numpy(s.v_int).to(DEV), s.seed, 0.0)
    vo = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)
    w = torch.from_numpy(s.wavelet).to(DEV)
    srcs = [np.array([6.5 + 9.0 * k, 0.0, 2.0 + 0.5 * (k % 2)]) for k in range(6)]
    d = [oracle.model_shot(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), src, s.rec).astype(np.float32)
         for src in srcs]
    traces = [torch.from_numpy(x).to(DEV) for x in d]
    full, n = migrate_survey(g, vg, w, srcs, s.rec, traces, s.dt, batch=2)
    assert n == 6
    ck = os.path.join(str(tmp_path), "stack.npz")
    part, n1 = migrate_survey(g, vg, w, srcs, s.rec, traces, s.dt, batch=2, checkpoint=ck, max_batches=2)
    assert n1 == 4 and os.path.exists(ck)
    resumed, n2 = migrate_survey(g, vg, w, srcs, s.rec, traces, s.dt, batch=2, checkpoint=ck)
    assert n2 == 6
    assert np.array_equal(resumed.cpu().numpy(), full.cpu().numpy())
    ref = sum(oracle.rtm_shot(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), src, s.rec,
                              x.astype(np.float64), eps_rel=1e-3)["image"] for src, x in zip(srcs, d))
    err = np.linalg.norm(full.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < 1e-4, err
    with pytest.raises(ValueError):
        migrate_survey(g, vg, w, srcs, s.rec, traces, s.dt, batch=3, checkpoint=ck)
