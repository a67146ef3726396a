"""Learned quartet screening: data collection, training and threshold tuning.

The estimator (tdgrad.Estimator, HIP kernels) predicts log10 of a screened shell
quartet's largest gradient contribution (scaled by 1/10).  Training data are the
contributions the library itself computes (Plan.collect); training runs the
library's BF16 forward/backward kernels and Adam update on the GPU.  A quartet is
then vetoed when its prediction is below a threshold unless its density-multiplied
Schwarz bound exceeds tau_hi (the rigorous fallback).  The threshold is tuned so
that the gradient stays within a tolerance of a reference evaluated without the
veto at a tighter Schwarz threshold.
"""
from __future__ import annotations

import time

import numpy as np

from . import tdgrad


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda:0"))


def collect(mols, tau=1e-10, cap=2_000_000, stride=1):
    """Features [n, 16] and targets [n] (float32 device tensors) from the surviving
    quartets of every molecule (every stride-th one, at most cap per molecule)."""
    import torch
    feats, tgts = [], []
    for m in mols:
        p = tdgrad.Plan(m, schwarz_tol=tau)
        f = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
        y = torch.zeros(cap, dtype=torch.float32, device="cuda")
        n = p.collect(_dev(m.P0), _dev(m.PD), _dev(m.R), f, y, stride=stride)
        feats.append(f[:n].clone())
        tgts.append(y[:n].clone())
        p.close()
    return torch.cat(feats), torch.cat(tgts)


def train(est, X, Y, epochs=6, batch=4096, lr=2e-3, seed=0, log=None):
    """Adam on shuffled mini-batches (all on the GPU); returns the full-set losses per epoch."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    hist = [est.grad(X, Y)[0]]
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        Xs, Ys = X[perm].contiguous(), Y[perm].contiguous()
        lr_ep = lr * (0.5 ** max(0, ep - epochs // 2))
        for b in range(0, n - batch + 1, batch):
            est.train_step(Xs[b:b + batch], Ys[b:b + batch], lr_ep)
        hist.append(est.grad(X, Y)[0])
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def gradient(plan, mol, out=None):
    import torch
    dens = (_dev(mol.P0), _dev(mol.PD), _dev(mol.R))
    out = out if out is not None else torch.zeros((mol.n_atoms, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = plan.grad_device(*dens, out, stats=True)
    torch.cuda.synchronize()
    st["seconds"] = time.perf_counter() - t
    return out.cpu().numpy(), st


def tune_threshold(mol, est, ref, tau=1e-10, tol=1e-6, tau_hi=1e-6, thresholds=None, precision=0):
    """Largest veto threshold (log10 of a contribution) whose gradient is within tol of ref;
    returns (threshold, error, stats) — threshold None when even the smallest fails."""
    thresholds = thresholds if thresholds is not None else [-9.0, -9.5, -10.0, -10.5, -11.0, -11.5, -12.0, -13.0]
    p = tdgrad.Plan(mol, schwarz_tol=tau, precision=precision, screening=1)
    p.set_screen_model(est, -1e30, 0.0)  # keeps every quartet while the kernel variants are tuned
    gradient(p, mol)  # tune kernel variants first
    best = (None, None, None)
    for thr in sorted(thresholds, reverse=True):
        p.set_screen_model(est, thr, tau_hi)
        g, st = gradient(p, mol)
        err = float(np.abs(g - ref).max())
        if err <= tol:
            best = (thr, err, st)
            break
    p.set_screen_model(None)
    p.close()
    return best


def schwarz_only(mol, ref, tol=1e-6, taus=(1e-7, 3e-8, 1e-8, 3e-9, 1e-9, 3e-10, 1e-10), precision=0):
    """Largest Schwarz threshold alone whose gradient is within tol of ref."""
    for tau in sorted(taus, reverse=True):
        p = tdgrad.Plan(mol, schwarz_tol=tau, precision=precision)
        gradient(p, mol)
        g, st = gradient(p, mol)
        p.close()
        err = float(np.abs(g - ref).max())
        if err <= tol:
            return tau, err, st
    return None, None, None


def budget_threshold(n_quartets, budget=1e-6, margin=2.0):
    """Veto threshold (log10 of a quartet's largest contribution) from an error budget that
    scales with the system: n vetoed contributions of random sign below t add up to about
    t sqrt(n), so t = budget / sqrt(n), lowered by `margin` decades for the estimator's own
    error (one decade left the 133-water gradient between 6e-7 and 2.8e-6 from the reference
    over repeated trainings; two decades)."""
    return float(np.log10(budget) - 0.5 * np.log10(max(n_quartets, 1)) - margin)
