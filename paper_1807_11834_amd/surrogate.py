"""Training driver of the learned velocity surrogate (host-side orchestration).

Every arithmetic step runs in the library's kernels: the coupling steps that
generate the training pairs (fine-grid velocity at the particles), the feature
gather (``couple_mlp_features``), the standardisation fit and the training steps
(``couple_mlp_train_step``: BF16 MFMA forward and backward, FP32 Adam).  This
module only draws the random numbers (initial weights, particle samples, batch
order) on the host and moves them to the device.

Target of the surrogate: the residual u_fine - u_bulk at a particle (fine-grid
lookup minus bulk trilinear interpolation), the sub-bulk part of the fluid
velocity that the dual-grid coupling (Sec. 2.1) otherwise obtains from the fine
grid.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import COUPLE_VEL_FINE, MLP_NFEAT, Config, Coupler, Mlp, couple_mlp_features

LAYERS = [(193, 128), (128, 128), (128, 128), (128, 3)]


def he_uniform(seed):
    """Initial parameters: W_l ~ U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)) drawn
    layer by layer as [fan_in][fan_out] with numpy's PCG64 (seed), biases 0;
    flat FP32 in the library's order (W_1, b_1, ..., W_4, b_4)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fin, fout in LAYERS:
        b = math.sqrt(6.0 / fin)
        parts.append(rng.uniform(-b, b, size=(fin, fout)).astype(np.float32).ravel())
        parts.append(np.zeros(fout, np.float32))
    return np.concatenate(parts)


class PairPool:
    """Device buffers of (features, residual) training pairs."""

    def __init__(self, capacity, device="cuda"):
        self.feat = torch.empty((capacity, MLP_NFEAT), dtype=torch.float32, device=device)
        self.resid = torch.empty((capacity, 3), dtype=torch.float32, device=device)
        self.n = 0
        self.capacity = capacity

    def add_from_step(self, cfg: Config, pos, diam, out, sel):
        """Pairs of the particles ``sel`` (device int32) from the outputs of a
        COUPLE_VEL_FINE step that wrote ``out["uf"]`` at positions ``pos``."""
        m = sel.shape[0]
        assert self.n + m <= self.capacity
        couple_mlp_features(cfg, pos, diam, out["bulk_phi"], out["bulk_U"], out["bulk_G"],
                            self.feat[self.n:self.n + m], u_fine=out["uf"], sel=sel,
                            resid=self.resid[self.n:self.n + m])
        self.n += m

    def view(self):
        return self.feat[:self.n], self.resid[:self.n]


def collect(pool: PairPool, cfg: Config, pos, vel, diam, fine, steps, per_step, seed, dev="cuda"):
    """Run ``steps`` coupling steps (fine-grid velocity; the configuration's own
    advection setting) and add ``per_step`` uniformly drawn particles of each
    step to the pool.  ``pos``/``vel`` are advanced in place when advecting."""
    assert cfg.vel_source == COUPLE_VEL_FINE
    rng = np.random.default_rng(seed)
    n = pos.shape[0]
    c = Coupler(cfg)
    try:
        for k in range(steps):
            at = pos.clone() if cfg.advect else pos      # positions the step's velocities belong to
            out = c.step(pos, vel, diam, fine, uf=True, step=k)
            sel = torch.from_numpy(rng.choice(n, per_step, replace=False).astype(np.int32)).to(dev)
            pool.add_from_step(cfg, at, diam, out, sel)
        torch.cuda.synchronize()
    finally:
        c.close()


def train(mlp: Mlp, feat, resid, steps, batch, seed, log_every=0, log=None):
    """``steps`` Adam steps on batches drawn without replacement from a fresh
    permutation of the pairs each epoch, drawn on the device (torch's generator
    seeded with ``seed``: a permutation of millions of pairs drawn on the host
    would cost more than the epoch's training steps).  Returns the losses read
    back every ``log_every`` steps (none when 0)."""
    n = feat.shape[0]
    assert batch <= n and batch % 32 == 0
    dev = feat.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    perm, at = None, n
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        if at + batch > n:
            perm = torch.randperm(n, generator=gen, device=dev, dtype=torch.int32)
            at = 0
        want = log_every and (it % log_every == 0 or it == steps - 1)
        mlp.train_step(feat, resid, batch, idx=perm[at:at + batch], loss=loss if want else None)
        at += batch
        if want:
            v = float(loss.item())
            hist.append((it, v))
            if log:
                log(f"step {it}: loss {v:.4e} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return hist
