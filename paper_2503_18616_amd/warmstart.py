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


def scales(feats, targets):
    """Feature scales 1 / std and output scales std over the free rows of a
    recording made with unit scales."""
    f = feats.float().cpu().numpy()
    t = targets.cpu().numpy()
    free = f[:, 31] > 0
    sf = f[free, :xpbd.MLP_FEATURES].std(axis=0)
    st = t[free, :3].std(axis=0)
    in_scale = np.where(sf > 0, 1.0 / np.maximum(sf, 1e-30), 1.0).astype(np.float32)
    out_scale = np.maximum(st, 1e-12).astype(np.float32)
    return in_scale, out_scale


def train(net: "xpbd.Mlp", feats, targets, steps: int, window: int = 8192, lr: float = 1e-3,
          seed: int = 0, final_lr: float = 1e-4):
    """Adam steps over random windows of the recorded rows (learning rate decays
    geometrically from lr to final_lr).  Returns the loss of every step."""
    rng = np.random.default_rng(seed)
    rows = feats.shape[0]
    window = min(window, rows)
    losses = []
    for s in range(steps):
        rate = lr * (final_lr / lr) ** (s / max(steps - 1, 1))
        o = int(rng.integers(0, rows - window + 1))
        losses.append(net.train_step(feats[o:o + window], targets[o:o + window], rate))
    return losses
