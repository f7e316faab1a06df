"""Learned warm starts for a parametrised family M(eps) = D + eps R (initial guesses,
Sec. 7).

Orchestration only: every solve, series term, target, training step and prediction is a
call into libipt.so.  The family's Rayleigh-Schroedinger terms T_1..T_p of R on the
requested columns (App. B; IPT contains the series, App. C) are computed once; the base
start of a member is the partial sum E + sum_l eps^l T_l, whose error is O(eps^(p+1)).
The network learns the standardised remainder (Z - base) / eps^(p+1) of FP64 IPT
solutions as a function of the features (eps / eps_max, (eps / eps_max)^2), so its
BF16 error is scaled by eps^(p+1); a predicted Z0 warm-starts a solve whose columns are
still certified by FP64 sweeps, so the prediction changes the number of sweeps but not
the answer.  order = 0 gives the plain scaled start E + eps (mu + sigma y)."""
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
    """Trains an ipt.MLP on solutions of the family and predicts warm starts on top of
    the family's series partial sum of the given order."""

    def __init__(self, n, k, hidden=256, depth=2, seed=0, eps_max=0.08, handle=None, order=2):
        self.n, self.k, self.eps_max, self.order = n, k, eps_max, order
        self.handle = handle
        self.net = ipt.MLP(2, hidden, depth, n * k, seed=seed, handle=handle)
        self.mu = self.sigma = None
        self.terms = None

    def set_family(self, theta, base, idx):
        """The series terms of the family's perturbation (once per family)."""
        self.terms = ipt.ipt_rs_terms(theta, base, idx, self.order, handle=self.handle) if self.order > 0 else None
        return self.terms

    def fit(self, z_train, eps_train, idx, steps=2000, lr=1e-3):
        """Targets, then `steps` Adam steps.  Each member is weighted by
        (eps / eps_max)^(order + 1), the factor its remainder enters Z0 with, so that the
        loss (and the targets' mean and spread) measure the error of the start itself,
        and members whose remainder is mostly the solutions' own rounding (small eps)
        do not steer the fit."""
        import torch
        dev = z_train.device
        e = torch.from_numpy(np.asarray(eps_train, dtype=np.float64)).to(dev)
        w = (np.asarray(eps_train, dtype=np.float64) / self.eps_max) ** (self.order + 1)
        wd = torch.from_numpy(w).to(dev)
        targets, self.mu, self.sigma = ipt.ipt_mlp_targets(z_train, idx, e, self.terms, weights=wd,
                                                           handle=self.handle)
        x = torch.from_numpy(features(eps_train, self.eps_max)).to(dev)
        wf = torch.from_numpy(w.astype(np.float32)).to(dev)
        t0 = time.perf_counter()
        loss = self.net.train(x, targets, steps, lr, weights=wf)
        return loss, time.perf_counter() - t0

    def inputs(self, eps):
        """Device features and parameters of the members eps (for predict_from)."""
        import torch
        dev = self.mu.device
        return (torch.from_numpy(features(eps, self.eps_max)).to(dev),
                torch.from_numpy(np.asarray(eps, dtype=np.float64)).to(dev))

    def predict_from(self, x, e, idx, z0=None):
        return self.net.predict_z0(x, self.mu, self.sigma, e, self.n, self.k, idx, terms=self.terms, z0=z0)

    def predict(self, eps, idx):
        x, e = self.inputs(eps)
        return self.predict_from(x, e, idx)


def series_start(terms, eps, idx, handle=None):
    """The series partial sums E + sum_l eps^l T_l for each eps (no network)."""
    import torch
    e = torch.from_numpy(np.asarray(eps, dtype=np.float64)).to(terms.device)
    return ipt.ipt_rs_start(terms, e, idx, handle=handle)
