"""Learned warm starts for a parametrised family M(eps) = D + eps R (initial guesses,
Sec. 7).

Orchestration only: every solve, target, training step and prediction is a call into
libipt.so.  The family's training solutions come from FP64 IPT solves; the network
learns the standardised entries of (Z - E) / eps as a function of the features
(eps / eps_max, (eps / eps_max)^2); a predicted Z0 warm-starts a solve whose columns
are still certified by FP64 sweeps, so the prediction changes the number of sweeps
but not the answer."""
from __future__ import annotations

import time

import numpy as np

from . import ipt


def features(eps, eps_max):
    e = np.asarray(eps, dtype=np.float64) / eps_max
    return np.stack([e, e * e], axis=1).astype(np.float32)


def solve_family(theta, base, eps_list, idx, z0=None, handle=None, **opts):
    """Solve M(eps) = diag(theta) + eps * base for each eps; returns (z [B, n, k],
    lam [B, k], status [B, k], sweeps [B], seconds).  z0: optional [B, n, k] warm starts."""
    import torch
    n, k = theta.shape[0], idx.shape[0]
    b = len(eps_list)
    z = torch.empty((b, n, k), dtype=torch.float64, device=theta.device)
    lam = torch.empty((b, k), dtype=torch.float64, device=theta.device)
    status = torch.empty((b, k), dtype=torch.int32, device=theta.device)
    sweeps = np.zeros(b, dtype=np.int64)
    deltas = [float(e) * base for e in eps_list]  # the family members, built before timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in range(b):
        r = ipt.ipt_solve_dense(theta, deltas[p], idx=idx, z0=None if z0 is None else z0[p], handle=handle,
                                colinfo=False, z_out=z[p], **opts)
        lam[p] = r.lam
        status[p] = r.status
        sweeps[p] = r.info["sweeps"]
    torch.cuda.synchronize()
    return z, lam, status, sweeps, time.perf_counter() - t0


class WarmStarter:
    """Trains an ipt.MLP on solutions of the family and predicts warm starts."""

    def __init__(self, n, k, hidden=256, depth=2, seed=0, eps_max=0.08, handle=None):
        self.n, self.k, self.eps_max = n, k, eps_max
        self.handle = handle
        self.net = ipt.MLP(2, hidden, depth, n * k, seed=seed, handle=handle)
        self.mu = self.sigma = None

    def fit(self, z_train, eps_train, idx, steps=2000, lr=1e-3):
        import torch
        dev = z_train.device
        scale = torch.from_numpy(np.asarray(eps_train, dtype=np.float64)).to(dev)
        targets, self.mu, self.sigma = ipt.ipt_mlp_targets(z_train, idx, scale, handle=self.handle)
        x = torch.from_numpy(features(eps_train, self.eps_max)).to(dev)
        t0 = time.perf_counter()
        loss = self.net.train(x, targets, steps, lr)
        return loss, time.perf_counter() - t0

    def predict(self, eps, idx):
        import torch
        dev = self.mu.device
        x = torch.from_numpy(features(eps, self.eps_max)).to(dev)
        scale = torch.from_numpy(np.asarray(eps, dtype=np.float64)).to(dev)
        return self.net.predict_z0(x, self.mu, self.sigma, scale, self.n, self.k, idx)
