"""Training and evaluation of the learned warm start through the C ABI.

The network and its training run in the library's matrix-core kernels
(``xpbd_mlp_*``); this module only orders the calls: record substeps of the
plain solver (features and the correction the sweeps found), derive the
feature and output scales from a pilot recording, and run Adam steps over
windows of the recorded rows.  torch provides device buffers only.
"""
from __future__ import annotations

import numpy as np

from . import xpbd


def he_init(seed: int) -> np.ndarray:
    """Flat float32 parameters: He-uniform weights, zero biases, a small output layer."""
    rng = np.random.default_rng(seed)
    F, H, O = xpbd.MLP_FEATURES, xpbd.MLP_HIDDEN, xpbd.MLP_OUTPUTS
    parts = [rng.uniform(-1, 1, H * F) * np.sqrt(6.0 / F), np.zeros(H),
             rng.uniform(-1, 1, H * H) * np.sqrt(6.0 / H), np.zeros(H),
             rng.uniform(-1, 1, O * H) * np.sqrt(6.0 / H) * 0.1, np.zeros(O)]
    return np.concatenate(parts).astype(np.float32)


def record(batch: "xpbd.Batch", net: "xpbd.Mlp", tool_pos, substeps, iterations):
    """Advance the batch one step per entry of ``substeps`` with the plain
    sweeps and record that substep's features and targets.  tool_pos:
    [len(substeps)][N][tools][3].  Returns device tensors (bfloat16 [R, 32],
    float32 [R, 4]) with R = len(substeps) * total particles."""
    import torch
    NP = int(batch.env_offsets[-1])
    n = len(substeps)
    feats = torch.zeros((n * NP, xpbd.MLP_FEATURE_STRIDE), dtype=torch.bfloat16, device="cuda")
    targets = torch.zeros((n * NP, 4), dtype=torch.float32, device="cuda")
    for k, sub in enumerate(substeps):
        tp = None if tool_pos is None else tool_pos[k:k + 1]
        batch.step_learned(net, 1, tp, iterations, iterations, np.inf, apply_correction=False,
                           record_substep=int(sub), record_features=feats[k * NP:(k + 1) * NP],
                           record_targets=targets[k * NP:(k + 1) * NP])
    return feats, targets


def normalisation(feats, targets):
    """(in_shift, in_scale, out_shift, out_scale): means and 1 / std of the
    features, means and std of the targets, over the free rows of a recording
    made with the identity normalisation (computed by the library's kernels,
    xpbd_mlp_normalisation)."""
    return xpbd.xpbd_mlp_normalisation(feats, targets)


def train(net: "xpbd.Mlp", feats, targets, steps: int, batch: int = 8192, lr: float = 1e-3,
          seed: int = 0, final_lr: float = 1e-4):
    """Adam steps on minibatches of the free recorded rows (the learning rate
    decays geometrically from lr to final_lr).  Returns the loss of every
    step.

    The free rows are shuffled once (seeded); step s takes the next ``batch``
    rows of that order, wrapping around its end, so successive passes over
    the rows start at shifting offsets.  The host queues all steps with one
    library call and reads the losses back once at the end."""
    import torch
    rng = np.random.default_rng(seed)
    free = np.flatnonzero(feats[:, 31].float().cpu().numpy() > 0).astype(np.int32)
    if free.size == 0:
        raise ValueError("the recording holds no free rows to train on")
    batch = min(batch, free.size)
    order = torch.from_numpy(np.ascontiguousarray(free[rng.permutation(free.size)])).cuda()
    xpbd.check_rows(order, feats.shape[0])
    losses = torch.zeros(max(steps, 1), dtype=torch.float32, device="cuda")
    net.train_steps(feats, targets, order, batch, steps, lr, final_lr, losses=losses,
                    rows_checked=True)
    return [float(v) for v in losses[:steps].cpu().numpy()]
