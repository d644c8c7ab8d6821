"""Shared helpers of the GPU parity tests: run one plan through the FP64
oracle and through libfspb, and compare under the stated tolerance

    |D_gpu(r) - D_oracle(r)| <= 1e-4 * max_r D_oracle + amb(r)

where amb(r) is the oracle's allowance for pairs within 1e-4 (relative) of
the ROI boundary or 1e-4 cm of the entrance depth, which FP32 and FP64 may
decide differently.
"""
import sys

import numpy as np
import torch

REL_TOL = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def geometry(plan, dc=None, tile=None):
    from paper_1103_1164_amd import Geometry
    return Geometry.from_plan(plan, device="cuda", dc_enabled=dc, tile=tile)


def gpu_dose(geo, fluence):
    f = torch.as_tensor(np.ascontiguousarray(fluence, np.float32), device="cuda")
    d = geo.forward(f)
    torch.cuda.synchronize()
    return d.cpu().numpy().astype(np.float64)


def assert_dose_parity(d_gpu, d_orc, amb, scale=None, what=""):
    d_gpu = np.asarray(d_gpu, np.float64).reshape(-1)
    d_orc = np.asarray(d_orc, np.float64).reshape(-1)
    amb = np.asarray(amb, np.float64).reshape(-1)
    m = float(np.max(np.abs(d_orc))) if scale is None else float(scale)
    err = np.abs(d_gpu - d_orc)
    bound = REL_TOL * m + amb
    bad = err > bound
    worst = float(np.max(err - REL_TOL * m - amb)) if err.size else 0.0
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {err.size} values outside "
                           f"1e-4*max+amb; max err {err.max():.3e} (max {m:.3e}), worst excess {worst:.3e}")
    return float(err.max() / m) if m > 0 else 0.0
