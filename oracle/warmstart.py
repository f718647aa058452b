"""FP64 reference of the learned warm start (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the GPU library never calls it.

The warm start is not part of FF-SRL's method: it is the learned extension
built on its substep (Alg. 1).  After the prediction of a substep, a small
per-particle network maps 27 local features of the predicted state to a
correction of the predicted position; the Gauss-Seidel iterations of the
substep then start from the corrected positions.  The plain iterations still
decide convergence: after ``min_iterations`` the constraint residual of the
environment is evaluated (the RMS of (C + alpha~ lambda) / rest over all
constraints, as ``oracle_residual`` defines it) and, if it exceeds the
threshold, the substep continues to ``max_iterations``.

Everything here is the plain definition written out in float64:

* Features of free particle i (raw, before scaling), from the start-of-substep
  positions x_prev, the start-of-substep velocity v, the predicted positions
  x_hat and the rest positions X:
    f[0:3]   x_hat_i - x_prev_i              (predicted displacement)
    f[3:6]   v_i                             (velocity before the prediction)
    f[6:9]   x_hat_i - X_i                   (displacement from rest)
    f[9+3k : 12+3k], k = 0..5, the axis neighbours -x, +x, -y, +y, -z, +z:
             (x_hat_n - x_hat_i) - (X_n - X_i), or 0 without a neighbour.
  The axis neighbour of i in direction +x is the particle with the same rest
  y and z and the smallest rest x above X_i (likewise for the other five).
* Network: a0 = bf16((f - in_shift) * in_scale); z1 = a0 W1^T + b1;
  a1 = bf16(relu(z1)); z2 = a1 W2^T + b2; a2 = bf16(relu(z2)); y = a2 W3^T + b3;
  correction = out_shift + clamp(y, -8, 8) * out_scale.  Weights are stored [out][in]; bf16() rounds to the nearest
  bfloat16 (ties to even) at exactly the points where the GPU keeps bfloat16
  operands of its matrix cores; every sum is exact here (float64).
* Loss over the free particles of a batch: L = (1/2n) sum_i |y_i - t_i|^2 with
  t_i = (x_after_i - x_hat_i - out_shift) / out_scale, n the number of free
  particles;
  its gradient by the chain rule, computed on the unnormalised error
  dy_i = y_i - t_i of the free particles with the same bfloat16 rounding of
  the backward operands (bf16(dz) before each product with a weight matrix
  or an activation), bias gradients from the unrounded dz, and every
  gradient divided by n at the end.
* Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FEATURES = 27
HIDDEN = 128
OUTPUTS = 3
CLIP = 8.0     # bound of the network output used as a correction


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    float64 -> float32 first (the GPU holds float32 before it rounds)."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16 << 16
    return (bits.astype(np.uint32)).view(np.float32).astype(np.float64)


def axis_neighbours(rest):
    """[V, 6] particle ids of the -x, +x, -y, +y, -z, +z axis neighbours, -1 if none."""
    rest = np.asarray(rest, np.float64).reshape(-1, 3)
    V = rest.shape[0]
    out = np.full((V, 6), -1, np.int32)
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        for i in range(V):
            same = np.all(rest[:, others] == rest[i, others], axis=1)
            d = rest[:, axis] - rest[i, axis]
            below = np.where(same & (d < 0))[0]
            above = np.where(same & (d > 0))[0]
            if below.size:
                out[i, 2 * axis] = below[np.argmax(d[below])]
            if above.size:
                out[i, 2 * axis + 1] = above[np.argmin(d[above])]
    return out


def features(x_prev, v, x_hat, rest, nbr):
    """[V, 27] raw features (see the module text)."""
    x_prev, v, x_hat, rest = (np.asarray(a, np.float64).reshape(-1, 3)
                              for a in (x_prev, v, x_hat, rest))
    V = rest.shape[0]
    f = np.zeros((V, FEATURES))
    f[:, 0:3] = x_hat - x_prev
    f[:, 3:6] = v
    f[:, 6:9] = x_hat - rest
    for k in range(6):
        n = nbr[:, k]
        has = n >= 0
        nn = np.where(has, n, 0)
        off = (x_hat[nn] - x_hat) - (rest[nn] - rest)
        f[:, 9 + 3 * k:12 + 3 * k] = np.where(has[:, None], off, 0.0)
    return f


@dataclass
class Net:
    W1: np.ndarray                  # [HIDDEN, FEATURES]
    b1: np.ndarray                  # [HIDDEN]
    W2: np.ndarray                  # [HIDDEN, HIDDEN]
    b2: np.ndarray
    W3: np.ndarray                  # [OUTPUTS, HIDDEN]
    b3: np.ndarray
    in_scale: np.ndarray = field(default_factory=lambda: np.ones(FEATURES))
    out_scale: np.ndarray = field(default_factory=lambda: np.ones(OUTPUTS))
    in_shift: np.ndarray = field(default_factory=lambda: np.zeros(FEATURES))
    out_shift: np.ndarray = field(default_factory=lambda: np.zeros(OUTPUTS))

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]


def forward(net: Net, f, emulate_bf16=True):
    """Network output y [n, 3] (scaled units) and the cache for backward."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, np.float64))
    a0 = r((np.asarray(f, np.float64) - net.in_shift) * net.in_scale)
    z1 = a0 @ r(net.W1).T + net.b1
    a1 = r(np.maximum(z1, 0.0))
    z2 = a1 @ r(net.W2).T + net.b2
    a2 = r(np.maximum(z2, 0.0))
    y = a2 @ r(net.W3).T + net.b3
    return y, (a0, z1, a1, z2, a2)


def correction(net: Net, f, free, emulate_bf16=True):
    """Correction of the predicted positions [n, 3] (m); zero for pinned particles."""
    y, _ = forward(net, f, emulate_bf16)
    c = net.out_shift + np.clip(y, -CLIP, CLIP) * net.out_scale
    return np.where(np.asarray(free)[:, None], c, 0.0)


def loss_and_grads(net: Net, f, target, mask, emulate_bf16=True):
    """Loss and gradients (dW1, db1, dW2, db2, dW3, db3) of the masked MSE."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, np.float64))
    y, (a0, z1, a1, z2, a2) = forward(net, f, emulate_bf16)
    m = np.asarray(mask, np.float64).reshape(-1, 1)
    n = max(float(m.sum()), 1.0)
    dy = (y - np.asarray(target, np.float64)) * m
    loss = 0.5 * float(np.sum(dy * dy)) / n
    gy = r(dy)
    dW3 = gy.T @ a2
    db3 = dy.sum(axis=0)
    dz2 = (gy @ r(net.W3)) * (z2 > 0)
    g2 = r(dz2)
    dW2 = g2.T @ a1
    db2 = dz2.sum(axis=0)
    dz1 = (g2 @ r(net.W2)) * (z1 > 0)
    g1 = r(dz1)
    dW1 = g1.T @ a0
    db1 = dz1.sum(axis=0)
    return loss, [g / n for g in (dW1, db1, dW2, db2, dW3, db3)]


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: list = None
    v: list = None

    def step(self, params, grads):
        if self.m is None:
            self.m = [np.zeros_like(p) for p in params]
            self.v = [np.zeros_like(p) for p in params]
        self.t += 1
        c1 = 1.0 - self.beta1 ** self.t
        c2 = 1.0 - self.beta2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.beta1
            m += (1.0 - self.beta1) * g
            v *= self.beta2
            v += (1.0 - self.beta2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


def init_net(seed=0, in_scale=None, out_scale=None) -> Net:
    """He-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)

    def he(o, i):
        lim = np.sqrt(6.0 / i)
        return rng.uniform(-lim, lim, (o, i))
    return Net(he(HIDDEN, FEATURES), np.zeros(HIDDEN), he(HIDDEN, HIDDEN), np.zeros(HIDDEN),
               he(OUTPUTS, HIDDEN) * 0.1, np.zeros(OUTPUTS),
               np.ones(FEATURES) if in_scale is None else np.asarray(in_scale, np.float64),
               np.ones(OUTPUTS) if out_scale is None else np.asarray(out_scale, np.float64))
