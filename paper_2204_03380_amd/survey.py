"""Survey migration with shot-granular checkpoints.

Algorithm 3's shot loop, run in batches of shots (one launch per time step
for a batch, images stacked on the device with RTM_F_ACCUMULATE).  After
every batch the partial stack and the index of the next shot can be written
to a checkpoint file; a run given that file resumes from there and ends with
the same stack, bit for bit, as an uninterrupted run with the same batches.
The checkpoint holds arrays only (numpy .npz, no pickled objects)."""
from __future__ import annotations

import os

import numpy as np
import torch

from . import RTM_F_ACCUMULATE, RTM_OP_RTM, BatchPlan, BatchShot, Grid


def _save(path, image, next_shot, batch):
    tmp = path + ".tmp.npz"
    np.savez(tmp, image=image.detach().cpu().numpy(), next_shot=np.int64(next_shot), batch=np.int64(batch))
    os.replace(tmp, path)  # atomic: a crash leaves the previous checkpoint


def migrate_survey(grid: Grid, v_pad: torch.Tensor, wavelet: torch.Tensor, srcs, rec, traces, dt: float,
                   batch: int = 16, eps_rel: float = 1e-3, checkpoint: str | None = None,
                   max_batches: int | None = None) -> tuple[torch.Tensor, int]:
    """Stacked image of the shots srcs[i] with recorded traces[i] ([nrec][nt
    + 1] device tensors, or a callable i -> tensor), `batch` shots per plan.
    With `checkpoint`, resumes from the file if it exists (same grid and
    batch size required) and rewrites it after every batch.  `max_batches`
    stops early (the checkpoint then holds the partial stack).  Returns
    (image, number of shots stacked)."""
    nt = int(wavelet.numel())
    n = len(srcs)
    image = torch.zeros(grid.interior_shape, dtype=torch.float32, device=v_pad.device)
    start = 0
    if checkpoint and os.path.exists(checkpoint):
        with np.load(checkpoint, allow_pickle=False) as z:
            if tuple(z["image"].shape) != tuple(grid.interior_shape) or int(z["batch"]) != batch:
                raise ValueError(f"checkpoint {checkpoint} is for another grid or batch size")
            image.copy_(torch.from_numpy(z["image"]))
            start = int(z["next_shot"])
    done = 0
    i = start
    while i < n and (max_batches is None or done < max_batches):
        idx = range(i, min(i + batch, n))
        shots = [BatchShot(grid, v_pad, wavelet, srcs[j], rec, traces_in=(traces(j) if callable(traces) else traces[j]),
                           image=image) for j in idx]
        BatchPlan(RTM_OP_RTM, shots, dt, nt, eps_rel=eps_rel, flags=RTM_F_ACCUMULATE).run()
        i = idx[-1] + 1
        done += 1
        if checkpoint:
            _save(checkpoint, image, i, batch)
    return image, i
