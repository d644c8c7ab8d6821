"""Commissioning: fit the parameters of the commissioned tables to reference
doses (measurements, or a reference dose engine), with the library's own
dose engine in the loop.

The paper commissions its tables against Monte Carlo (Section 2.1); here the
fit is generic: `tables_fn(c)` maps a parameter vector to a tables object
(fields as `fspb_synth.Tables`), the measurement set is a list of plans
(density, beams, fluences) with one reference dose grid each, and the fit
minimises

    sum over plans p and voxels r of ((D_p(r; c) - M_p(r)) / max M_p)^2

by Levenberg-Marquardt with a central-difference Jacobian.  Every dose is a
full plan on the GPU (the tables change the density factors and the depth
tables, so each evaluation rebuilds the geometry); the small normal
equations are solved on the host.
"""
from __future__ import annotations

import time
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

from . import Geometry


def _residuals(c, tables_fn, setups):
    tabs = tables_fn(c)
    out = []
    for p, dens, flu, ref, scale in setups:
        geo = Geometry(dens, p.spacing, p.origin, p.beams, tabs, p.options)
        d = geo.forward(flu)
        geo.close()
        out.append(((d - ref) / scale).reshape(-1))
    return torch.cat(out).double().cpu().numpy()


def fit_tables(plans: Sequence, refs: Sequence[torch.Tensor], tables_fn: Callable,
               c0, iters: int = 30, h: float = 3e-3, tol: float = 1e-9,
               log: Optional[Callable[[str], None]] = None) -> dict:
    """Levenberg-Marquardt fit of the table parameters c (starting at c0).
    Returns dict(c, cost (per iteration), evaluations, seconds)."""
    setups = []
    for p, ref in zip(plans, refs):
        dens = torch.as_tensor(np.ascontiguousarray(p.density, np.float32), device="cuda")
        flu = torch.as_tensor(np.ascontiguousarray(p.fluence, np.float32), device="cuda")
        ref = torch.as_tensor(ref, dtype=torch.float32, device="cuda").reshape(p.density.shape)
        setups.append((p, dens, flu, ref, float(ref.max())))
    t0 = time.perf_counter()
    c = np.asarray(c0, dtype=np.float64).copy()
    n_eval = 1
    r = _residuals(c, tables_fn, setups)
    cost = [float(r @ r)]
    lam = 1e-3
    for it in range(iters):
        J = np.empty((r.size, c.size))
        for k in range(c.size):
            hk = h * max(abs(c[k]), 1e-3)
            e = np.zeros_like(c)
            e[k] = hk
            J[:, k] = (_residuals(c + e, tables_fn, setups) - _residuals(c - e, tables_fn, setups)) / (2 * hk)
            n_eval += 2
        A = J.T @ J
        g = J.T @ r
        improved = False
        for _ in range(12):
            step = np.linalg.solve(A + lam * np.diag(np.diag(A)), -g)
            r_new = _residuals(c + step, tables_fn, setups)
            n_eval += 1
            if float(r_new @ r_new) < cost[-1]:
                c, r = c + step, r_new
                cost.append(float(r @ r))
                lam = max(lam / 3.0, 1e-9)
                improved = True
                break
            lam *= 4.0
        if log:
            log(f"iteration {it + 1}: cost {cost[-1]:.3e}, lambda {lam:.1e}")
        if not improved or np.linalg.norm(step) <= tol * (1.0 + np.linalg.norm(c)):
            break
    return dict(c=c, cost=cost, evaluations=n_eval, seconds=time.perf_counter() - t0)
