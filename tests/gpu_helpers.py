"""Shared helpers of the GPU parity tests: run one plan through the FP64
oracle and through libfspb, and compare under the stated tolerance

    |D_gpu(r) - D_oracle(r)| <= 1e-4 * max_r D_oracle

The oracle is given the plan as the library's C interface receives it (every
interface float rounded to float32, ``fspb_synth.abi_rounded``), so both
compute on the same instance.  Which pairs count (inside the ROI cylinder,
below the entrance) is a discrete outcome that both sides decide in single
precision by the same recipe; ``assert_pair_consts_equal`` checks that the
per-beamlet constants of that recipe are bitwise equal, and the oracle's
ambiguity allowance is asserted to be zero everywhere.
"""
import sys

import numpy as np
import torch

REL_TOL = 1e-4
AMB_MAX = 2e-4     # bound on max(amb) / max D (the allowance is expected to be 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def abi_oracle(plan, **kw):
    """The FP64 oracle on the plan as the library receives it."""
    import oracle
    import fspb_synth as S
    return oracle.Oracle(S.abi_rounded(plan), **kw)


def geometry(plan, dc=None, tile=None, schedule=None):
    from paper_1103_1164_amd import Geometry
    return Geometry.from_plan(plan, device="cuda", dc_enabled=dc, tile=tile, schedule=schedule)


def gpu_dose(geo, fluence):
    f = torch.as_tensor(np.ascontiguousarray(fluence, np.float32), device="cuda")
    d = geo.forward(f)
    torch.cuda.synchronize()
    return d.cpu().numpy().astype(np.float64)


def amb_stats(amb, scale, what=""):
    """Prints and bounds the oracle's ambiguity allowance: the number of
    values with amb > 0 and max(amb) / scale."""
    amb = np.asarray(amb, np.float64).reshape(-1)
    n_amb = int((amb > 0).sum())
    frac = float(amb.max() / scale) if amb.size and scale > 0 else 0.0
    say(f"{what}: {n_amb} of {amb.size} values with amb > 0, max amb / max = {frac:.2e}")
    assert n_amb == 0 and frac <= AMB_MAX, (what, n_amb, frac)
    return n_amb, frac


def assert_dose_parity(d_gpu, d_orc, amb, scale=None, what=""):
    d_gpu = np.asarray(d_gpu, np.float64).reshape(-1)
    d_orc = np.asarray(d_orc, np.float64).reshape(-1)
    amb = np.asarray(amb, np.float64).reshape(-1)
    m = float(np.max(np.abs(d_orc))) if scale is None else float(scale)
    amb_stats(amb, m, what)
    err = np.abs(d_gpu - d_orc)
    bound = REL_TOL * m
    bad = err > bound
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {err.size} values outside "
                           f"1e-4*max; max err {err.max():.3e} (max {m:.3e})")
    return float(err.max() / m) if m > 0 else 0.0


def assert_pair_consts_equal(geo, orc, beamlets=None):
    """The single-precision constants of the pair test, as the kernels read
    them, against those of the oracle's recipe for every listed beamlet (all
    by default) that reaches the body.  Both sides round their own double-
    precision frames, which agree to about 1e-14 cm; the single-precision
    values are then bitwise equal except where the double value is itself of
    that size (a direction component that is a rounding residue such as
    3.9e-20 against 0, or an offset of 7.5e-8 when the grid centre lies on
    the axis).  Those differ by at most 1e-12: times a coordinate below
    100 cm, 1e-10 cm, which changes a single-precision t, xp or yp only when
    it lies that close to a rounding boundary.  The pair counts compared per
    voxel elsewhere check the decisions themselves.
    Returns (beamlets compared, components not bitwise equal)."""
    ids = range(orc.n_beamlets) if beamlets is None else beamlets
    n = n_diff = 0
    for i in ids:
        g = geo.beamlet(int(i), tables=False)
        if not g["hit"]:
            continue
        a, b = g["pair_consts"], orc.pair_consts(int(i))
        same = a.view(np.uint32) == b.view(np.uint32)
        close = np.abs(a.astype(np.float64) - b.astype(np.float64)) <= 1e-12
        assert np.all(same | close), (i, a, b)
        n += 1
        n_diff += int((~same).sum())
    return n, n_diff
