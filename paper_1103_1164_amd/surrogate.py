"""Training and evaluation driver of the learned surrogate.

The surrogate predicts, for a (voxel, beam) row, the six Section 2.1
parameters (u1x, u1y, u2x, u2y, w1, w2) from a density patch along the
source-voxel ray (see include/fspb.h).  Everything numeric runs in libfspb's
kernels: the training rows (gathered on the GPU from plans built with the
density correction on), the BF16 MFMA forward/backward and Adam steps, the
fused gather + inference and the dose with the predicted parameters.  This
module only draws row indices, shuffles the data set once, keeps the
learning-rate schedule and picks the guard thresholds.

    mlp = Mlp.initial(seed)
    data = build_dataset(train_plans, rows_per_plan=5000, seed=1)
    fit(mlp, data, epochs=20)
    guard = calibrate(mlp, heldout_plans, data)
    rep = evaluate(mlp, plan)         # dose error vs the corrected method
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Callable, Iterable, List, Optional

import numpy as np
import torch

from . import Geometry, Mlp


@dataclass
class Dataset:
    x: torch.Tensor          # BF16 [n, 224] scaled inputs
    t: torch.Tensor          # FP32 [n, 6] targets (unstandardised)
    mean: np.ndarray         # standardisation of the network targets
    std: np.ndarray
    rho_lo: float            # density range the rows were gathered from
    rho_hi: float
    t_lo: np.ndarray         # per-output target range
    t_hi: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _draw_rows(rng: np.random.Generator, n_vox: int, n_beams: int, n: int) -> torch.Tensor:
    rows = np.stack([rng.integers(0, n_vox, size=n), rng.integers(0, n_beams, size=n)], axis=1)
    return torch.as_tensor(rows.astype(np.int32), device="cuda")


def rows_of_plan(plan, rows_per_plan: int, seed: int, geo: Optional[Geometry] = None,
                 max_rounds: int = 8):
    """Up to rows_per_plan valid training rows of one plan (uniform over the
    valid (voxel, beam) rows): (x, t, geometry)."""
    geo = geo or Geometry.from_plan(plan, dc_enabled=1)
    rng = np.random.default_rng(seed)
    xs, ts, have = [], [], 0
    for _ in range(max_rounds):
        rows = _draw_rows(rng, geo.n_vox, geo.n_beams, 2 * rows_per_plan)
        x, t, v = geo.surrogate_samples(rows)
        keep = torch.nonzero(v, as_tuple=True)[0][: rows_per_plan - have]
        xs.append(x[keep])
        ts.append(t[keep])
        have += int(keep.numel())
        if have >= rows_per_plan:
            break
    return torch.cat(xs), torch.cat(ts), geo


def build_dataset(plans: Iterable, rows_per_plan: int, seed: int = 0,
                  log: Optional[Callable[[str], None]] = None) -> Dataset:
    """Training rows from every plan (built one at a time), shuffled once."""
    xs, ts = [], []
    rho_lo, rho_hi = np.inf, -np.inf
    t0 = time.perf_counter()
    for k, plan in enumerate(plans):
        x, t, geo = rows_of_plan(plan, rows_per_plan, seed * 100_003 + k)
        xs.append(x)
        ts.append(t)
        rho_lo = min(rho_lo, float(np.min(plan.density)))
        rho_hi = max(rho_hi, float(np.max(plan.density)))
        geo.close()
        if log and (k + 1) % 20 == 0:
            log(f"dataset: {k + 1} plans, {sum(a.shape[0] for a in xs)} rows, "
                f"{time.perf_counter() - t0:.1f} s")
    x = torch.cat(xs)
    t = torch.cat(ts)
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(x.shape[0], generator=g).to(x.device)
    x, t = x[perm].contiguous(), t[perm].contiguous()
    tt = t.double()
    zz = network_targets(t).double()
    mean = zz.mean(0).cpu().numpy()
    std = np.maximum(zz.std(0).cpu().numpy(), 1e-6)
    return Dataset(x, t, mean.astype(np.float32), std.astype(np.float32), rho_lo, rho_hi,
                   tt.min(0).values.cpu().numpy(), tt.max(0).values.cpu().numpy())


def network_targets(t: torch.Tensor) -> torch.Tensor:
    """What the network predicts: (log u1x, log u1y, log u2x, log u2y, w1, w2)."""
    z = t.clone()
    z[:, :4] = torch.log(t[:, :4])
    return z


def standardised_targets(data: Dataset) -> torch.Tensor:
    m = torch.as_tensor(data.mean, device=data.t.device)
    s = torch.as_tensor(data.std, device=data.t.device)
    return ((network_targets(data.t) - m) / s).contiguous()


def fit(mlp: Mlp, data: Dataset, epochs: int = 20, batch: int = 8192, lr: float = 2e-3,
        lr_end: float = 1e-4, seed: int = 0, log: Optional[Callable[[str], None]] = None):
    """Adam on the mean-square loss of the standardised targets, with a
    cosine learning-rate decay; minibatches are contiguous slices of the
    shuffled data set, visited in a fresh order every epoch.  Returns the
    mean loss of each epoch."""
    mlp.set_scaling(data.mean, data.std)
    tz = standardised_targets(data)
    n = data.n
    starts = np.arange(0, n, batch)
    total = epochs * len(starts)
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=data.x.device)
    acc = torch.zeros(1, dtype=torch.float32, device=data.x.device)
    history = []
    step = 0
    for ep in range(epochs):
        acc.zero_()
        for s0 in rng.permutation(starts):
            s1 = min(int(s0) + batch, n)
            a = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * step / max(total - 1, 1)))
            mlp.train_step(data.x[s0:s1], tz[s0:s1], lr=a, loss=loss)
            acc += loss
            step += 1
        history.append(float(acc.item()) / len(starts))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {history[-1]:.5f}")
    return history


def dose_error(d: torch.Tensor, ref: torch.Tensor) -> float:
    """max |d - ref| / max ref over the grid."""
    return float((d - ref).abs().max().item() / ref.max().item())


def evaluate(mlp: Mlp, plan, geo: Optional[Geometry] = None, fluence=None) -> dict:
    """Surrogate dose against the corrected method on one plan, with the
    conventional method's error beside it."""
    own = geo is None
    geo = geo or Geometry.from_plan(plan, dc_enabled=1)
    f = torch.as_tensor(plan.fluence if fluence is None else fluence, device="cuda")
    d_dc = geo.forward(f)
    prm = geo.surrogate_infer(mlp)
    d_s = geo.forward_surrogate(f, prm)
    geo.set_dc(False)
    d_plain = geo.forward(f)
    geo.set_dc(True)
    fb = prm[:, :, 6]
    out = dict(err_surrogate=dose_error(d_s, d_dc), err_plain=dose_error(d_plain, d_dc),
               fallback_fraction=float(fb.mean().item()),
               served_fraction=float((fb == 0).float().mean().item()),
               max_dose=float(d_dc.max().item()))
    if own:
        geo.close()
    return out


def calibrate(mlp: Mlp, plans: List, data: Dataset, target: float = 0.01,
              band_margin: float = 0.05,
              het_grid=(np.inf, 1.0, 0.6, 0.4, 0.3, 0.2, 0.15, 0.1, 0.07, 0.05, 0.03, 0.02,
                        0.01, 0.0, -1.0),
              log: Optional[Callable[[str], None]] = None) -> dict:
    """Guard thresholds: the training density range, the training target
    range widened by band_margin of its width, and the largest near-voxel
    heterogeneity bound for which every held-out plan's dose error stays
    within target (a negative bound sends every row to the fallback)."""
    w = data.t_hi - data.t_lo
    band_lo = data.t_lo - band_margin * w
    band_hi = data.t_hi + band_margin * w
    geos = [Geometry.from_plan(p, dc_enabled=1) for p in plans]
    fl = [torch.as_tensor(p.fluence, device="cuda") for p in plans]
    ref = [g.forward(f) for g, f in zip(geos, fl)]
    chosen = None
    table = []
    for tau in het_grid:
        mlp.set_guard(data.rho_lo, data.rho_hi, tau, band_lo, band_hi)
        errs, fbs = [], []
        for g, f, r in zip(geos, fl, ref):
            prm = g.surrogate_infer(mlp)
            errs.append(dose_error(g.forward_surrogate(f, prm), r))
            fbs.append(float(prm[:, :, 6].mean().item()))
        table.append(dict(het_max=float(tau), max_err=max(errs), fallback=float(np.mean(fbs))))
        if log:
            log(f"guard het_max={tau}: max err {max(errs):.4f}, fallback {np.mean(fbs):.3f}")
        if max(errs) <= target:
            chosen = table[-1]
            break
    for g in geos:
        g.close()
    tau = chosen["het_max"] if chosen else -1.0
    mlp.set_guard(data.rho_lo, data.rho_hi, tau, band_lo, band_hi)
    return dict(het_max=tau, rho_lo=data.rho_lo, rho_hi=data.rho_hi, band_lo=band_lo.tolist(),
                band_hi=band_hi.tolist(), table=table, met=chosen is not None)
