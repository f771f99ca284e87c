#!/usr/bin/env python3
"""Benchmark of the random-boundary RTM hot path on one MI355X.

Workload: the 2-D folded-layer survey (2301 x 751 cells at 4 m, velocities
1500-5500 m/s, 60-cell random boundary, 25 Hz Ricker, dt = 0.4 ms, nt = 5000,
240 shots every 38 m, 2301 receivers), seeded and synthetic.  One step
processes a batch of shots through the whole path: random-boundary padding,
modeling of the observed data (forward propagation with receiver sampling),
then RTM of each shot (forward propagation keeping two panels, fused reverse
reconstruction + receiver back-propagation + imaging, normalisation) and
stacking.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  The metric is Gcell-updates/s: padded cells x nt x
propagations (1 for modeling, 3 for RTM) per second of device time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes of one reverse launch (240 shots, three steps per launch, shape
# vec 2, tx 1, zseg 108) from two rocprofv3 counter runs: L2-to-memory read
# requests by size (TCC_EA0_RDREQ_32B/64B/128B) and write requests
# (TCC_EA0_WRREQ, TCC_EA0_WRREQ_64B; the rest are 32 B).  A 1 GiB device copy
# in the same runs reads exactly 8388608 x 128 B and writes 16777216 x 64 B
# (twice that for the 2 GiB copy of the bandwidth reference), so the request
# counts are bytes without further scaling.  Valid only for the kernel
# sources hashed here and this batch; reported as null otherwise.
PMC_REVERSE = {"sources_sha256_16": "95c4dc57367124d7", "shots": 240, "shape": (2, 1, 108), "steps": 3,
               "read_bytes": 150769382 * 128 + 71343 * 64 + (150840725 - 150769382 - 71343) * 32,
               "write_bytes": 182289122 * 64 + (183488193 - 182289122) * 32}
KERNEL_SOURCES = ("prop2d.hip", "stencil.h", "common.h")


def reverse_traffic(B, shape, steps=1):
    import hashlib
    csrc = os.path.join(ROOT, "paper_2204_03380_amd", "csrc")
    try:
        blob = b"".join(open(os.path.join(csrc, f), "rb").read() for f in KERNEL_SOURCES)
    except OSError:
        return None
    rec = PMC_REVERSE
    if (hashlib.sha256(blob).hexdigest()[:16] != rec["sources_sha256_16"] or B != rec["shots"]
            or tuple(shape) != rec["shape"] or steps != rec.get("steps", 1)):
        return None
    return int(rec["read_bytes"] + rec["write_bytes"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shots-per-step", type=int, default=240,
                    help="shots per step (one launch carries them all); 240 = the whole survey, resident in HBM")
    ap.add_argument("--plain-shots", type=int, default=2, help="shots timed through the plain per-shot calls")
    ap.add_argument("--vec", type=int, default=0, help="floats per lane of both propagation kernels (0: tuned)")
    ap.add_argument("--zseg", type=int, default=0, help="rows per tile of both kernels, a multiple of 9 (0: tuned)")
    ap.add_argument("--nt", type=int, default=5000)
    ap.add_argument("--cpu-sample-nt", type=int, default=2000,
                    help="time steps of the oracle's timed sample (one shot, modeling + RTM)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the benchmark, copy a device buffer of this many MiB once (a plain copy kernel of "
                         "known size, to scale hardware byte counters)")
    ap.add_argument("--autotune", action="store_true", help="pick launch shapes with the autotuner first")
    ap.add_argument("--no-unet", action="store_true", help="skip the learned-filter training-step timing")
    ap.add_argument("--no-c3", action="store_true", help="skip the full-size 3-D shot")
    ap.add_argument("--c3-only", action="store_true",
                    help="instead of the survey benchmark: only the full-size 3-D shot (modeling + RTM)")
    ap.add_argument("--c3-nt", type=int, default=4000, help="time steps of the 3-D shot in --c3-only mode")
    ap.add_argument("--unet-only", action="store_true",
                    help="instead of the survey benchmark: only the crosstalk filter's 128^3 training-step timing")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="instead of the survey benchmark: single-shot modeling and RTM at the grid sizes of the "
                         "paper's Tables 1-4 (modeling timed over a shortened nt and scaled to the paper's nt; "
                         "RTM with reconstruction and with storage at the paper's nt)")
    ap.add_argument("--boundary-study", action="store_true",
                    help="instead of the survey benchmark: RTM crosstalk of one shot for the band setups (uniform "
                         "random factors, Eqs. (4)-(5) tapers, free surface)")
    ap.add_argument("--persistent-study", action="store_true",
                    help="instead of the survey benchmark: batch plans run eagerly, as a hipGraph and as persistent "
                         "passes, on the uneven-aperture windows and single shots of the paper's 2-D grids")
    ap.add_argument("--paper-kinds", default="modeling,rtm,storage",
                    help="with --paper-shapes: comma-separated kinds to run")
    return ap.parse_args()


def _cpu_model():
    """The host CPU's model name and the logical CPUs this process may use."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": name, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(survey, nt_sample, nt_one_thread=200):
    """The FP64 oracle on a bounded sample of the same workload: one shot
    (the first, on-grid source), modeling + RTM, nt_sample steps with the
    oracle's default threads, and nt_one_thread steps on one thread."""
    import numpy as np

    import oracle
    s = survey
    v_pad = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)

    def run(nt):
        w = s.wavelet[:nt].astype(np.float64)
        t0 = time.perf_counter()
        d = oracle.model_shot(v_pad, s.h, s.nb, s.dt, w, s.src[0], s.rec)
        oracle.rtm_shot(v_pad, s.h, s.nb, s.dt, w, s.src[0], s.rec, d, eps_rel=1e-3)
        return time.perf_counter() - t0

    cores = oracle.set_threads(0)
    sec = run(nt_sample)
    oracle.set_threads(1)
    sec1 = run(nt_one_thread)
    oracle.set_threads(cores)
    rate = lambda nt, t: v_pad.size * nt * 4 / t / 1e9  # noqa: E731
    return {"value": rate(nt_sample, sec), "unit": "Gcell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"1 shot, modeling + RTM (4 propagations), {nt_sample} of {s.nt} steps, FP64, "
                      f"{sec:.1f} s on {cores} threads",
            "host_cpu": _cpu_model(), "fp_env": oracle.fp_env(),
            "one_thread": {"value": rate(nt_one_thread, sec1), "unit": "Gcell-updates/s",
                           "sample": f"same shot, {nt_one_thread} steps, {sec1:.1f} s on 1 thread"}}


def unet_report(steps=30):
    """Training step of the learned crosstalk filter on one 128^3 image
    (forward, backward, Adam) and each convolution's MFMA throughput."""
    import torch

    from paper_2204_03380_amd import unet as U
    g = torch.Generator(device="cuda").manual_seed(0)
    img = torch.randn((1, 128, 128, 128), device="cuda", generator=g)
    tgt = img + 0.1 * torch.randn((1, 128, 128, 128), device="cuda", generator=g)
    net = U.UNet(seed=0)
    for _ in range(3):
        net.train_step(img, tgt, 1e-4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        net.forward(img, tgt, want_loss=False)
        net.backward()
        net.step(1e-4)
    e1.record()
    e1.synchronize()
    eager_ms = e0.elapsed_time(e1) / steps
    # the same steps with forward + backward replayed from a HIP graph (one
    # host launch instead of one per kernel) and Adam eager
    graph = net.capture_pass(img, tgt)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        graph.replay()
        net.step(1e-4)
    e1.record()
    e1.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    layers = U.layer_timings(net, img, tgt)
    conv_ms = sum(r["fwd_ms"] + r["wgrad_ms"] + r.get("dgrad_ms", 0.0) for r in layers)
    gflop = sum(r["gflop"] * (3 if "dgrad_ms" in r else 2) for r in layers)
    return {"image": "128^3, batch 1, bf16 MFMA (peak 2500 TFLOP/s)",
            "train_step_ms": round(graph_ms, 3),
            "train_step_ms_eager": round(eager_ms, 3),
            "launch": "forward + backward replayed from a HIP graph, Adam step and weight packing eager",
            "conv_ms": round(conv_ms, 3), "conv_tflops": round(gflop / conv_ms, 2),
            "layers": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()} for r in layers]}


def c3_report(nt=4000):
    """One shot of the 3-D layered-salt workload at full size (512 x 512 x 256
    interior, 612 x 612 x 356 padded, nt 4000, 65 536 receivers): modeling
    of the observed data, then RTM (forward, fused reverse, image), timed
    with events; Gcell-updates/s over the four propagations, and the fused
    reverse kernel's rate on its algorithmic bytes (one step per launch:
    28 B per padded cell + 16 B per interior cell)."""
    import numpy as np
    import torch

    import paper_2204_03380_amd as rtm
    import synth
    dev = torch.device("cuda:0")
    s = synth.config_c3(nt=nt)
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vp = rtm.rtm_rbc_pad(g, torch.from_numpy(s.v_int).to(dev), s.seed, 0.0)
    w = torch.from_numpy(s.wavelet).to(dev)
    cells = int(np.prod(g.padded_shape))
    interior = int(s.v_int.size)
    torch.cuda.synchronize()
    rtm.rtm_timing_read()
    rtm.rtm_timing_enable(True)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    d = rtm.rtm_model_shot(g, vp, s.dt, w, s.src[0], s.rec)
    e1.record()
    im = rtm.rtm_rtm_shot(g, vp, s.dt, w, s.src[0], s.rec, d, eps_rel=1e-3)["image"]
    e2.record()
    e2.synchronize()
    rtm.rtm_timing_enable(False)
    loops = rtm.rtm_timing_read()
    assert torch.isfinite(im).all()
    t_model, t_rtm = e0.elapsed_time(e1) * 1e-3, e1.elapsed_time(e2) * 1e-3
    rev_ms, rev_n = loops["reverse_image"]
    fwd_ms, fwd_n = loops["rtm_forward"]
    rev_us, fwd_us = rev_ms * 1e3 / max(rev_n, 1), fwd_ms * 1e3 / max(fwd_n, 1)
    rev_bytes = 28 * cells + 16 * interior
    fwd_bytes = 16 * cells
    vec_f, ty_f, z_f = rtm.rtm_get_tuning3d(rtm.RTM_OP_MODEL)
    vec_r, ty_r, z_r = rtm.rtm_get_tuning3d(rtm.RTM_OP_RTM)
    del d, im
    torch.cuda.empty_cache()
    return {"workload": f"layered salt 3-D 512x512x256 @ 10 m, nb 50, nt {nt}, 12 Hz, 256x256 receivers: one shot "
                        "modeled then migrated",
            "padded_cells": cells, "model_s": round(t_model, 3), "rtm_s": round(t_rtm, 3),
            "value": round(cells * nt * 4 / (t_model + t_rtm) / 1e9, 2), "unit": "Gcell-updates/s",
            "roofline": {"bound": "hbm", "kernel": f"rev3d_kernel<{vec_r},{ty_r},false> (fused reverse, one step)",
                         "avg_launch_us": round(rev_us, 2), "algorithmic_bytes_per_launch": rev_bytes,
                         "achieved": round(rev_bytes / (rev_us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(rev_bytes / (rev_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
            "forward": {"kernel": f"fwd3d_kernel<{vec_f},{ty_f}>", "avg_launch_us": round(fwd_us, 2),
                        "achieved_GBps": round(fwd_bytes / (fwd_us * 1e-6) / 1e9, 1),
                        "frac": round(fwd_bytes / (fwd_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}}


# The paper's single-shot times (seconds) on its hardware: one V100 (OpenACC)
# and one SX-Aurora TSUBASA 10B vector engine.  Grid sizes are the padded
# grids of Tables 1-4 (2-D: nx x nz, 4 s at 0.5 ms = 8000 steps; 3-D:
# nx x ny x nz, 6 s at 1 ms = 6000 steps).
PAPER_CASES = (
    ("modeling", (837, 1, 294), 8000, {"V100": 1.132, "SX-Aurora": 0.488}, "Table 1"),
    ("modeling", (1574, 1, 534), 8000, {"V100": 1.875, "SX-Aurora": 0.912}, "Table 1"),
    ("modeling", (3048, 1, 1014), 8000, {"V100": 2.615, "SX-Aurora": 2.416}, "Table 1"),
    ("modeling", (5996, 1, 1974), 8000, {"V100": 6.962, "SX-Aurora": 7.885}, "Table 1"),
    ("rtm", (1574, 1, 534), 8000, {"V100": 3.500, "SX-Aurora": 4.489}, "Table 2"),
    ("storage", (1574, 1, 534), 8000, {"V100": 7.969, "SX-Aurora": 9.016}, "Table 2"),
    ("modeling", (501, 501, 235), 6000, {"V100": 42.1505, "SX-Aurora": 43.132}, "Table 3"),
    ("modeling", (901, 901, 416), 6000, {"V100": 330.363, "SX-Aurora": 203.940}, "Table 3"),
    ("rtm", (501, 501, 235), 6000, {"V100": 139.786, "SX-Aurora": 108.582}, "Table 4"),
    ("storage", (501, 501, 235), 6000, {"V100": 256.166, "SX-Aurora": 430.944}, "Table 4"),
)
# Stored-wavefield size the paper prints for its storage runs (GB), Tables 2 and 4.
PAPER_STORAGE_GB = {"Table 2": 2.638, "Table 4": 132.062}
# Snapshot step of the paper's storage runs: dt_nyq / dt = 10 in 2-D and 3-D (Eq. (7)).
PAPER_STRIDE = 10


PAPER_3D_SHAPES = tuple((v, y, z, o) for v, y, z in ((1, 4, 18), (1, 8, 18), (2, 8, 18), (1, 4, 36)) for o in (0, 1))


def paper_shapes(nb=50, kinds=("modeling", "rtm", "storage")):
    """Device time of one shot on each paper grid (synthetic smooth velocity;
    runtime does not depend on the values) against the paper's times, at the
    paper's full nt.  Modeling and RTM with reconstruction run as a one-shot
    plan replayed as a hipGraph (tables built once, no launch gaps); RTM with
    storage through rtm_storage_shot, keeping every 10th level in device
    memory.  3-D grids first run the autotuner over PAPER_3D_SHAPES (36
    steps per candidate) and record its choice."""
    import numpy as np
    import torch

    import paper_2204_03380_amd as rtm
    import synth
    dev = torch.device("cuda:0")
    gst = torch.cuda.Stream(device=dev)  # graph capture needs a stream other than the NULL stream
    out = []
    for kind, (nx, ny, nz), nt_paper, paper, table in PAPER_CASES:
        if kind not in kinds:
            continue
        # every allocation and call of a case on the capture stream, so that
        # torch's reuse of freed memory stays ordered with the work using it
        with torch.cuda.stream(gst):
            out.append(_paper_case(rtm, synth, np, torch, dev, gst, nb, kind, nx, ny, nz, nt_paper, paper, table))
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def _paper_case(rtm, synth, np, torch, dev, gst, nb, kind, nx, ny, nz, nt_paper, paper, table):
    """One row of paper_shapes (run with gst as the current stream)."""
    ndim = 2 if ny == 1 else 3
    shape_int = (nz - 2 * nb, nx - 2 * nb) if ndim == 2 else (nz - 2 * nb, ny - 2 * nb, nx - 2 * nb)
    if ndim == 2:
        v = synth.random_model(shape_int, 7, 1500.0, 4000.0, sigma=4.0)
    else:
        v = synth.layered_salt_3d(shape_int[2], shape_int[1], shape_int[0], 7, vmax=4000.0, salt=False)
    h = 10.0
    dt = 0.45 * h / 4000.0 * (0.8 if ndim == 3 else 1.0)
    g = rtm.Grid.for_model(v, h, nb)
    vp = rtm.rtm_rbc_pad(g, torch.from_numpy(v).to(dev), 11, 0.0)
    steps = nt_paper
    w = torch.from_numpy(synth.ricker(15.0, dt, steps)).to(dev)
    src = np.array([shape_int[-1] / 2.0, (shape_int[1] / 2.0 if ndim == 3 else 0.0), 2.0])
    if ndim == 2:
        rec = synth.line_receivers(np.arange(0, shape_int[-1], 1, dtype=np.float64), 2.0)
    else:
        rec = synth.grid_receivers(np.arange(0, shape_int[-1], 2, dtype=np.float64),
                                   np.arange(0, shape_int[1], 2, dtype=np.float64), 2.0)
    extra = {}
    plan = None
    snap = None
    if ndim == 3:
        # 3-D: the autotuner picks shapes and tile order for this grid (the
        # faster tile order depends on the grid)
        from paper_2204_03380_amd import autotune
        snap = rtm.tuning_snapshot()
        res = autotune.tune_batch(g, vp, w, [src], rec, dt, nt_probe=36, reps=1, shapes=PAPER_3D_SHAPES)
        extra["launch_shape"] = {"forward": list(res["forward"][:-1]), "reverse": list(res["reverse"][:-1]),
                                 "fields": "vec, rows per workgroup, planes per tile, z-innermost tile order"}
    if kind == "modeling":
        tr = torch.empty((rec.shape[0], steps + 1), dtype=torch.float32, device=dev)
        plan = rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, vp, w, src, rec, traces_out=tr)], dt, steps,
                             flags=rtm.RTM_F_GRAPH)
        run = lambda: plan.run(gst)  # noqa: E731
    else:
        d = rtm.rtm_model_shot(g, vp, dt, w, src, rec)
    if kind == "rtm":
        im = torch.empty(g.interior_shape, dtype=torch.float32, device=dev)
        plan = rtm.BatchPlan(rtm.RTM_OP_RTM, [rtm.BatchShot(g, vp, w, src, rec, traces_in=d, image=im)], dt,
                             steps, flags=rtm.RTM_F_GRAPH)
        run = lambda: plan.run(gst)  # noqa: E731
        extra["kept_levels"] = 2
        extra["kept_GiB"] = round(2 * nx * ny * nz * 4 / 2 ** 30, 4)
    if kind == "storage":
        count = rtm.rtm_storage_count(steps, PAPER_STRIDE, 0)
        snaps = torch.empty((count,) + tuple(g.interior_shape), dtype=torch.float32, device=dev)
        run = lambda: rtm.rtm_storage_shot(g, vp, dt, w, src, rec, d, PAPER_STRIDE, 0, snapshots=snaps)  # noqa
        extra["stride"] = PAPER_STRIDE
        extra["kept_levels"] = count
        extra["kept_GiB"] = round(snaps.numel() * 4 / 2 ** 30, 3)
        extra["paper_stored_GB"] = PAPER_STORAGE_GB[table]
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(gst)
    run()
    e1.record(gst)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    props = {"modeling": 1, "rtm": 3, "storage": 2}[kind]
    cells = nx * ny * nz
    t_paper_nt = ms * 1e-3 * nt_paper / steps
    row = {"case": f"{kind} {nx}x{nz}" if ndim == 2 else f"{kind} {nx}x{ny}x{nz}", "source": table,
           "padded_cells": cells, "steps_timed": steps, "ms_per_step": round(ms / steps, 4),
           "gcell_updates_per_s": round(cells * props * steps / (ms * 1e-3) / 1e9, 2),
           "seconds_at_paper_nt": round(t_paper_nt, 4),
           "paper_seconds": paper,
           "speedup": {k: round(v_ / t_paper_nt, 1) for k, v_ in paper.items()}}
    row.update(extra)
    if snap is not None:
        rtm.tuning_restore(snap)
    print(json.dumps(row), file=sys.stderr, flush=True)
    if plan is not None:
        plan.free()
    return row


BAND_MODES = (("uniform factors", None), ("taper Gaussian h (alpha 0)", 0.0), ("taper midway (alpha 0.5)", 0.5),
              ("taper linear g (alpha 1)", 1.0))


def boundary_study(K=8, seed0=500):
    """Boundary crosstalk of one RTM shot against the band setup: the
    uniform random factors, the tapers of Eqs. (4)-(5), each with and
    without the free-surface top.  Crosstalk index = mean over K seeds of
    |I_s - I_mean| / |I_mean| (the boundary noise differs between seeds, the
    reflector image does not), over the whole image and below the near
    surface (z >= 20 cells), where it is also given against the first
    setup's stack norm.  Observed data: the same shot on the model
    extended far enough that no boundary energy returns within nt (top
    extended too, or a free surface), direct wave removed."""
    import numpy as np
    import torch

    import paper_2204_03380_amd as rtm
    import synth
    dev = torch.device("cuda:0")
    # three flat layers within two-way reach of the recording time, one dipping
    nz, nx, h, nb, dt, nt = 201, 301, 10.0, 40, 1e-3, 1200
    zz, xx = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    v = np.full((nz, nx), 1500.0, np.float32)
    v[zz >= 40 + 0.15 * (xx - nx / 2)] = 2000.0
    v[zz >= 80] = 2500.0
    w = torch.from_numpy(synth.ricker(15.0, dt, nt)).to(dev)
    src, rec = np.array([nx / 2.0, 0.0, 2.0]), synth.line_receivers(np.arange(nx), 2.0)
    name = f"three-layer 2-D {nx}x{nz} @ {h:g} m, nb {nb}, dt {dt * 1e3:g} ms, nt {nt}, 15 Hz"
    ext = int(nt * dt * float(v.max()) / (2 * h)) + 2
    g = rtm.Grid.for_model(v, h, nb)
    vt = torch.from_numpy(v).to(dev)
    cap = float(v.max())
    rows = []
    ref_norm = None  # the stack of the first setup (uniform factors, no free surface) below the near surface
    for fs in (False, True):
        top = 0 if fs else ext
        v_ext = np.pad(v, ((top, ext), (ext, ext)), mode="edge")
        ge = rtm.Grid.for_model(v_ext, h, 16)
        shift = np.array([ext, 0.0, top])
        v0 = float(v[int(round(src[2])), int(round(src[0]))])

        def model(vm):
            vp = rtm.rtm_rbc_pad(ge, torch.from_numpy(np.ascontiguousarray(vm)).to(dev), 1, float(vm.max()),
                                 free_surface=fs)
            return rtm.rtm_model_shot(ge, vp, dt, w, src + shift, rec + shift.astype(np.float32))

        d_obs = model(v_ext) - model(np.full(v_ext.shape, v0, np.float32))
        for name, alpha in BAND_MODES:
            seeds = [seed0 + k for k in range(K)]
            imgs = torch.empty((K,) + tuple(v.shape), dtype=torch.float32, device=dev)
            shots = [rtm.BatchShot(g, rtm.rtm_rbc_pad(g, vt, sd, cap, free_surface=fs, taper=alpha), w, src, rec,
                                   traces_in=d_obs, image=imgs[i]) for i, sd in enumerate(seeds)]
            rtm.BatchPlan(rtm.RTM_OP_RTM, shots, dt, nt, eps_rel=1e-3).run()
            mean = imgs.double().mean(0)
            nsr = float(np.mean([float(torch.linalg.norm(imgs[i].double() - mean) / torch.linalg.norm(mean))
                                 for i in range(K)]))
            # below the near surface (z >= 20 cells), where the reflectors are
            win = (slice(20, None), slice(None))
            noise = float(np.mean([float(torch.linalg.norm((imgs[i].double() - mean)[win])) for i in range(K)]))
            if ref_norm is None:
                ref_norm = float(torch.linalg.norm(mean[win]))
            # reconstruction still exact: probe p^k against the forward field
            k = nt // 2
            vp0 = shots[0].v_pad
            _, pk, _ = rtm.rtm_model_shot(g, vp0, dt, w[:k].contiguous(), src, rec, want_last=True)
            probe = rtm.rtm_rtm_shot(g, vp0, dt, w, src, rec, d_obs, snap_k=k)["snap_p"]
            rev = float(torch.linalg.norm((probe - pk).double()) / torch.linalg.norm(pk.double()))
            vmax_band = float(vp0.max())
            row = {"band": name, "free_surface": fs, "crosstalk_index": round(nsr, 4),
                   "crosstalk_index_below_20": round(noise / float(torch.linalg.norm(mean[win])), 4),
                   "noise_below_20_vs_uniform_stack": round(noise / ref_norm, 4),
                   "reconstruction_rel_err": float(f"{rev:.2e}"),
                   "courant_max": round(vmax_band * dt / h, 4), "courant_limit": round((315 / 1024) ** 0.5, 4)}
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    return {"model": name, "seeds": K, "rows": rows}


def persistent_study(reps=2):
    """Device time of batch plans run three ways: the default launch per
    one to three time steps (eager), the same schedule replayed as a
    hipGraph, and the persistent passes (one launch per pass, per-shot
    progress counters, one step per pass over a tile).  Workloads: the 64
    uneven-aperture windows (nt 2000; modeling of the observed data, then
    the gradient pass) and single shots at the paper's 2-D grid sizes
    (modeling, nt 8000)."""
    import numpy as np
    import torch

    import paper_2204_03380_amd as rtm
    import synth
    dev = torch.device("cuda:0")
    gst = torch.cuda.Stream(device=dev)
    rows = []

    def timed(run):
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(gst)
        for _ in range(reps):
            run()
        e1.record(gst)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    def modes(make, name, cell_steps):
        out = {"workload": name}
        for mode, flags in (("launch_per_steps", 0), ("graph", rtm.RTM_F_GRAPH), ("persistent", rtm.RTM_F_PERSISTENT)):
            plans = make(flags)
            ms = timed(lambda: [p.run(gst) for p in plans])
            out[mode] = {"ms": round(ms, 3), "gcell_updates_per_s": round(cell_steps / (ms * 1e-3) / 1e9, 2)}
            for p in plans:
                p.free()
        print(json.dumps(out), file=sys.stderr, flush=True)
        rows.append(out)

    with torch.cuda.stream(gst):
        s = synth.config_c4()
        windows = [(int(a), int(b)) for a, b in s.extra["windows"]]
        vt = torch.from_numpy(s.v_int).to(dev)
        w = torch.from_numpy(s.wavelet).to(dev)
        shots = []
        for i, (x0, wd) in enumerate(windows):
            v = rtm.rtm_window_extract(vt, x0, wd)
            g = rtm.Grid.for_model(v, s.h, s.nb)
            vp = rtm.rtm_rbc_pad(g, v, 1000 + i, 3500.0)
            rec = synth.line_receivers(np.arange(wd, dtype=np.float64), 2.0)
            tr = torch.zeros((wd, s.nt + 1), device=dev)
            gv = torch.empty(g.padded_shape, device=dev)
            shots.append((g, vp, s.src[i], rec, tr, gv))
        cells = sum(g.padded_shape[0] * g.padded_shape[1] for g, *_ in shots)

        def c4(flags):
            m = rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, vp, w, src, rec, traces_out=tr)
                                                 for g, vp, src, rec, tr, gv in shots], s.dt, s.nt, flags=flags)
            v = rtm.BatchPlan(rtm.RTM_OP_VJP, [rtm.BatchShot(g, vp, w, src, rec, traces_in=tr, grad_v_pad=gv)
                                               for g, vp, src, rec, tr, gv in shots], s.dt, s.nt, flags=flags)
            return [m, v]

        modes(c4, "64 uneven-aperture windows (401-1201 x 300, nb 40), nt 2000: modeling + gradient pass",
              cells * s.nt * 4)
        del shots
        for nx, nz, nt in ((837, 294, 8000), (1574, 534, 8000)):
            nb = 50
            v = synth.random_model((nz - 2 * nb, nx - 2 * nb), 7, 1500.0, 4000.0, sigma=4.0)
            g = rtm.Grid.for_model(v, 10.0, nb)
            vp = rtm.rtm_rbc_pad(g, torch.from_numpy(v).to(dev), 11, 0.0)
            dt = 0.45 * 10.0 / 4000.0
            ww = torch.from_numpy(synth.ricker(15.0, dt, nt)).to(dev)
            rec = synth.line_receivers(np.arange(0, nx - 2 * nb, 1, dtype=np.float64), 2.0)
            src = np.array([(nx - 2 * nb) / 2.0, 0.0, 2.0])
            tr = torch.empty((rec.shape[0], nt + 1), device=dev)

            def one(flags):
                return [rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, vp, ww, src, rec, traces_out=tr)], dt, nt,
                                      flags=flags)]

            modes(one, f"single shot {nx}x{nz} (padded), modeling, nt {nt}", nx * nz * nt)
    torch.cuda.synchronize()
    return rows


def device_info():
    """What the run was measured on (torch's view of device 0)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": p.gcnArchName, "compute_units": p.multi_processor_count,
            "hbm_gib": round(p.total_memory / 2**30, 1), "l2_bytes": getattr(p, "L2_cache_size", None)}


def copy_rate(dev, mib=2048, reps=5):
    """Device-to-device copy rates (read + write bytes / time) of a 2 GiB
    buffer: torch's copy, and the library's streaming copy kernel (16-byte
    nontemporal loads and stores) at a few grid sizes, the best of which is
    the measured bandwidth reference for the propagation kernels."""
    import torch

    import paper_2204_03380_amd as rtm
    a = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    out = {"torch_copy_GBps": round(timed(lambda: b.copy_(a)), 1), "stream_copy_GBps": {}}
    for bpc in (2, 4, 8, 16):
        out["stream_copy_GBps"][bpc] = round(timed(lambda: rtm.rtm_stream_copy(a, b, bpc)), 1)
    assert torch.equal(a, b)
    best = max(out["stream_copy_GBps"].items(), key=lambda kv: kv[1])
    out["best_stream_copy"] = {"blocks_per_cu": best[0], "GBps": best[1]}
    del a, b
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}): shots are "
              "independent and a multi-GPU run would be a shot partition plus one image all-reduce, which this "
              "build does not include.", file=sys.stderr)
        sys.exit(2)

    if args.boundary_study:
        out = boundary_study()
        print(json.dumps({"metric": "RTM boundary crosstalk index by band setup", "unit": "ratio", "n_gpus": 1,
                          "higher_is_better": False, "dtype": "f32", "data": "synthetic", **out}), flush=True)
        return

    if args.c3_only:
        print(json.dumps({"metric": "Gcell-updates/s", "unit": "Gcell-updates/s", "n_gpus": 1, "higher_is_better": True,
                          "dtype": "f32", "data": "synthetic", "c3": c3_report(args.c3_nt)}), flush=True)
        return

    if args.unet_only:
        print(json.dumps({"metric": "crosstalk filter training step (128^3, forward + backward + Adam)",
                          "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "bf16 (fp32 accumulation)",
                          "data": "synthetic", "unet_train_step": unet_report()}), flush=True)
        return

    if args.persistent_study:
        rows = persistent_study()
        print(json.dumps({"metric": "batch plan device time: launch per step(s), hipGraph, persistent passes",
                          "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
                          "rows": rows}), flush=True)
        return

    if args.paper_shapes:
        rows = paper_shapes(kinds=tuple(args.paper_kinds.split(",")))
        print(json.dumps({"metric": "single-shot time at the paper's grid sizes", "unit": "s", "n_gpus": 1,
                          "higher_is_better": False, "dtype": "f32", "data": "synthetic", "cases": rows}),
              flush=True)
        return

    import numpy as np
    import torch

    import paper_2204_03380_amd as rtm
    import synth

    dev = torch.device("cuda:0")
    s = synth.config_c2(nt=args.nt)
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    v_int = torch.from_numpy(s.v_int).to(dev)
    wav = torch.from_numpy(s.wavelet).to(dev)
    NZ, NX = g.padded_shape
    cells = NX * NZ
    interior = s.v_int.size
    B = args.shots_per_step
    nshot = s.src.shape[0]
    nrec = s.rec.shape[0]
    nt = args.nt
    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    copy = copy_rate(dev)
    copy_gbps = copy["best_stream_copy"]["GBps"]
    if args.vec and args.zseg:
        rtm.rtm_set_tuning(rtm.RTM_OP_MODEL, args.vec, args.zseg)
        rtm.rtm_set_tuning(rtm.RTM_OP_RTM, args.vec, args.zseg)
    tuned = None
    if args.autotune:
        from paper_2204_03380_amd import autotune
        v_tmp = rtm.rtm_rbc_pad(g, v_int, s.seed, 0.0)
        tuned = autotune.tune_batch(g, v_tmp, wav, [s.src[i] for i in range(B)], s.rec, s.dt, nt_probe=90, reps=2)
        del v_tmp
        # the timed batch runs exactly the configuration the tuner picked for it
        rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    fwd_shape = rtm.rtm_get_tuning2d(rtm.RTM_OP_MODEL)   # (vec, tx, zseg)
    rev_shape = rtm.rtm_get_tuning2d(rtm.RTM_OP_RTM)

    # Buffers resident in HBM before timing: padded model, B traces, stack.
    v_pad = rtm.rtm_rbc_pad(g, v_int, s.seed, 0.0)
    traces = [torch.zeros((nrec, nt + 1), dtype=torch.float32, device=dev) for _ in range(B)]
    stack = torch.zeros(g.interior_shape, dtype=torch.float32, device=dev)
    ngroups = max(1, nshot // B)
    groups = [[(k * B + j) % nshot for j in range(B)] for k in range(ngroups)]
    # one workspace for every plan (they run one after another on one
    # stream), sized for the largest: groups of other source positions can
    # need more than the first
    plans = []
    for grp in groups:
        mp = rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, v_pad, wav, s.src[i], s.rec, traces_out=traces[j])
                                              for j, i in enumerate(grp)], s.dt, nt, defer_workspace=True)
        rp = rtm.BatchPlan(rtm.RTM_OP_RTM, [rtm.BatchShot(g, v_pad, wav, s.src[i], s.rec, traces_in=traces[j],
                                                          image=stack) for j, i in enumerate(grp)],
                           s.dt, nt, eps_rel=1e-3, flags=rtm.RTM_F_ACCUMULATE, defer_workspace=True)
        plans.append((mp, rp))
    ws = torch.empty(max(max(mp.ws_bytes, rp.ws_bytes) for mp, rp in plans), dtype=torch.uint8, device=dev)
    for mp, rp in plans:
        mp.bind_workspace(ws)
        rp.bind_workspace(ws)

    def step(i):
        rtm.rtm_rbc_pad(g, v_int, s.seed, 0.0, out=v_pad)
        mp, rp = plans[i % ngroups]
        mp.run()
        rp.run()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    rtm.rtm_timing_read()
    rtm.rtm_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        step(args.warmup + i)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rtm.rtm_timing_enable(False)
    loops = rtm.rtm_timing_read()
    dev_ms = e0.elapsed_time(e1)
    assert torch.isfinite(stack).all()

    shots = args.steps * B
    updates = cells * nt * 4 * shots
    ms_per_step = dev_ms / args.steps
    value = updates / (dev_ms * 1e-3) / 1e9

    # Plain per-shot calls on the same GPU (modeling + RTM), same shots as
    # the first batch; their images must equal the batched ones bit for bit.
    plain_shots = groups[0][:min(B, args.plain_shots)]
    exact = rtm.rtm_get_tuning(rtm.RTM_TUNE_EXACT)[0]
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 0, 0)  # single shots take the library's shapes for small jobs
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    plain = []
    for i in plain_shots:
        d = rtm.rtm_model_shot(g, v_pad, s.dt, wav, s.src[i], s.rec)
        plain.append((d, rtm.rtm_rtm_shot(g, v_pad, s.dt, wav, s.src[i], s.rec, d, eps_rel=1e-3)["image"]))
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - p0
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, exact, 0)
    # The batched side of the comparison is the timed configuration itself:
    # the first group's modeling plan as timed, then an RTM plan of the same
    # B shots at the same launch shape writing one image per shot.  Its launch
    # count (loop timing) shows which kernel ran.
    mp0, _ = plans[0]
    mp0.run()
    imgs = torch.empty((B,) + tuple(g.interior_shape), dtype=torch.float32, device=dev)
    check = rtm.BatchPlan(rtm.RTM_OP_RTM, [rtm.BatchShot(g, v_pad, wav, s.src[i], s.rec, traces_in=traces[j],
                                                         image=imgs[j]) for j, i in enumerate(groups[0])],
                          s.dt, nt, eps_rel=1e-3, ws=ws)
    torch.cuda.synchronize()
    rtm.rtm_timing_read()
    rtm.rtm_timing_enable(True)
    check.run()
    torch.cuda.synchronize()
    rtm.rtm_timing_enable(False)
    check_launches = rtm.rtm_timing_read()["reverse_image"][1]
    check.free()
    tr_equal = all(torch.equal(d, traces[j]) for j, (d, _) in enumerate(plain))
    batch_vs_plain = max(float(torch.linalg.norm(imgs[j] - im) / torch.linalg.norm(im))
                         for j, (_, im) in enumerate(plain))
    del imgs, plain

    # Dominant kernel: the fused reverse kernel (two stencils, imaging sums),
    # one launch covering the B shots of a batch and one to three time steps.
    # Algorithmic bytes per launch: one step reads p^k, p^{k+1}, mu^{k+1},
    # mu^{k+2}, D' and writes p^{k-1}, mu^k on the padded grid (28 B) and
    # reads and writes num, den on the interior (16 B); two or three steps
    # read the same five arrays once, write the last two levels of each field
    # (36 B) and num, den once (16 B).
    steps_f = rtm.rtm_get_steps_per_launch(rtm.RTM_OP_MODEL)
    steps_r = rtm.rtm_get_steps_per_launch(rtm.RTM_OP_RTM)
    rev_ms, rev_n = loops["reverse_image"]
    rev_us = rev_ms * 1e3 / max(rev_n, 1)
    rev_bytes = B * ((36 if steps_r >= 2 else 28) * cells + 16 * interior)
    achieved = rev_bytes / (rev_us * 1e-6) / 1e9
    one_step_bytes = B * (28 * cells + 16 * interior)
    per_step_us = rev_us / steps_r
    traffic = reverse_traffic(B, rev_shape, steps_r)
    rev_kernel = (f"rev2d_t{steps_r}_kernel<{rev_shape[0]}> ({steps_r} reverse steps per launch: reconstruction + "
                  f"receiver field + imaging, {B} shots per launch)" if steps_r >= 2 else
                  f"rev2d_kernel<{rev_shape[0]},false,{rev_shape[1]}> (fused reconstruction + receiver field + "
                  f"imaging, {B} shots per launch)")
    # the reverse launches of the check plan: nt // steps multi-step launches
    # plus the nt % steps single steps
    check_kernel = (f"rev2d_t{steps_r}_kernel<{rev_shape[0]}> at the timed shape, {B} shots"
                    if check_launches == nt // steps_r + nt % steps_r else f"{check_launches} launches")
    fwd_ms, fwd_n = loops["model_forward"]
    rf_ms, rf_n = loops["rtm_forward"]
    line = {
        "metric": "Gcell-updates/s",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"folded-layer 2-D survey 2301x751 @ 4 m, nb 60, nt {nt}, 25 Hz, 2301 receivers, 240 shots: "
                        f"per step {B} shots modeled then migrated (random boundaries, reconstruction), each launch "
                        f"advancing the {B} shots by up to three time steps, images stacked",
            "padded_cells": cells,
            "shots_per_step": B,
            "propagations_per_shot": 4,
            "workspace_bytes": int(ws.numel()),
            "launch_shape": {"forward": {"vec": fwd_shape[0], "tx": fwd_shape[1], "zseg": fwd_shape[2]},
                             "reverse": {"vec": rev_shape[0], "tx": rev_shape[1], "zseg": rev_shape[2]},
                             "autotuned": tuned is not None,
                             "tuner": ({"forward_us_per_step": round(tuned["forward"][-1], 3),
                                        "reverse_us_per_step": round(tuned["reverse"][-1], 3),
                                        "candidates": len(tuned["table"])} if tuned else None)},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": rev_kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "avg_launch_us": round(rev_us, 3),
            "algorithmic_bytes_per_launch": rev_bytes,
            "fractions": {
                "compulsory": round(achieved / HBM_PEAK_GBS, 4),
                "counter_traffic": (round(traffic / (rev_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                    if traffic else None),
                "one_step_equivalent": round(one_step_bytes / (per_step_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "note": (f"compulsory: this kernel's minimum bytes per launch ({steps_r} steps read p^k, p^(k+1), "
                         "mu^(k+1), mu^(k+2), D' once and write the last two levels of both fields, 36 B per "
                         "padded cell, plus num and den read and written once, 16 B per interior cell) over the "
                         "measured launch time; counter_traffic: the HBM bytes the counters saw per launch over "
                         "the same time; one_step_equivalent: a one-step kernel's minimum bytes per step (28 B "
                         "per padded cell + 16 B per interior cell) over the measured time per step, which "
                         "exceeds 1 because the steps of a launch share one pass over memory"),
            },
            "stream_copy_GBps": copy_gbps,
            "frac_of_stream_copy": round(achieved / copy_gbps, 4) if copy_gbps else None,
            "copy_reference": copy,
            "steps_per_launch": steps_r,
            "per_step": {"us": round(per_step_us, 3),
                         "one_step_algorithmic_bytes": one_step_bytes,
                         "equivalent_GBps": round(one_step_bytes / (per_step_us * 1e-6) / 1e9, 1)},
        },
        "rtm_shots_per_s": {"batched": round(shots / (dev_ms * 1e-3), 4),
                            "plain": round(len(plain_shots) / plain_s, 4),
                            "image_rel_l2_batched_vs_plain": batch_vs_plain,
                            "traces_equal_batched_vs_plain": tr_equal,
                            "checked_kernel": check_kernel,
                            "note": "one shot = modeling + RTM; plain = sequential single-shot calls; the check "
                                    f"compares {len(plain_shots)} shots of a {B}-shot plan at the timed shape"},
        "steps_per_launch": {"forward": steps_f, "reverse": steps_r},
        "loop_us_per_launch": {
            "model_forward": round(fwd_ms * 1e3 / max(fwd_n, 1), 3),
            "rtm_forward": round(rf_ms * 1e3 / max(rf_n, 1), 3),
            "reverse_image": round(rev_us, 3),
        },
        "wall_s": round(wall, 3),
        "device": device_info(),
    }
    if not args.no_c3:
        line["c3"] = c3_report()
    if not args.no_unet:
        line["unet_train_step"] = unet_report()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s, args.cpu_sample_nt)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
