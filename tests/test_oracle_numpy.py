"""The second oracle (NumPy, oracle/numpy_oracle.py) against the C oracle:
two implementations of the same definitions, organised differently, must
agree to rounding (1e-12 relative) on config 1 and on small plans with
couch rotation, a body in air, anisotropic voxels and plain FSPB; the pair
sets (Algorithm A1 step 8, single precision) must agree exactly.  The
single-precision fused multiply-add emulation is pinned against exact
rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

import fspb_synth as S
from oracle import numpy_oracle as NO


def _fma_exact(a, b, c):
    """fma(a, b, c) rounded once to float32, from the exact rational value
    (round half to even)."""
    x = Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))
    lo = np.float32(float(x))
    # float(x) rounds to double first; step to the float32 neighbours around x
    cands = {lo, np.nextafter(lo, np.float32(np.inf)), np.nextafter(lo, np.float32(-np.inf))}
    best = min(cands, key=lambda v: (abs(Fraction(float(v)) - x),
                                     int(np.frombuffer(np.float32(v).tobytes(), np.uint32)[0]) & 1))
    return best


def test_fma32_is_rounded_once():
    rng = np.random.default_rng(0)
    a = rng.standard_normal(2000).astype(np.float32)
    b = rng.standard_normal(2000).astype(np.float32)
    c = rng.standard_normal(2000).astype(np.float32)
    # products that nearly cancel c, and sums that sit near float32 midpoints
    c[:500] = -(a[:500].astype(np.float64) * b[:500]).astype(np.float32)
    one = np.float32(1.0)
    eps = np.float32(2.0 ** -24)
    a[500:520], b[500:520] = one + 2 * eps, one + 2 * eps
    c[500:520] = np.float32(2.0 ** -30) * np.arange(20, dtype=np.float32)
    got = NO.fma32(a, b, c)
    want = np.array([_fma_exact(x, y, z) for x, y, z in zip(a, b, c)], dtype=np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # a double-rounding case: a*b + c lands exactly on a float32 midpoint in
    # double but not in exact arithmetic
    x = np.float32(1.0 + 2.0 ** -12)
    y = np.float32(1.0 + 2.0 ** -12)        # x*y = 1 + 2^-11 + 2^-24
    z = np.float32(-(2.0 ** -60))
    assert NO.fma32(x, y, z) == _fma_exact(x, y, z)


@pytest.fixture(scope="module")
def c1(oracle_mod):
    plan = S.abi_rounded(S.plan_c1())
    return plan, oracle_mod.Oracle(plan)


def test_smoothing_and_frames_agree(c1):
    plan, orc = c1
    rh = NO.smoothed_density(plan)
    assert np.abs(rh - orc.smoothed()).max() <= 1e-12 * np.abs(rh).max()
    for i, fr in enumerate(NO.beamlet_frames(plan)):
        o = orc.frame(i)
        for k in ("src", "d", "ex", "ey"):
            assert np.abs(fr[k] - o[k]).max() <= 1e-14 * max(1.0, np.abs(o[k]).max()), (i, k)
        assert abs(fr["theta"] - o["theta"]) <= 1e-15


def test_depth_tables_agree(c1):
    plan, orc = c1
    for i, fr in enumerate(NO.beamlet_frames(plan)):
        tr = NO.trace(plan, fr)
        o = orc.trace(i)
        assert (tr is not None) == o["hit"], i
        if tr is None:
            continue
        assert abs(tr["s_entry"] - o["s_entry"]) <= 1e-12 * abs(o["s_entry"])
        assert len(tr["T"]) == o["K"], i
        for k in ("T", "W1", "W2"):
            scale = max(np.abs(o[k]).max(), 1e-30)
            assert np.abs(tr[k] - o[k]).max() <= 1e-12 * scale, (i, k)


def _check_dose(plan, orc):
    d, pairs = NO.dose(plan)
    d_o, amb, pc = orc.dose()
    assert np.array_equal(pairs, pc)
    scale = np.abs(d_o).max()
    assert scale > 0
    err = np.abs(d - d_o).max() / scale
    assert err <= 1e-12, err
    return err


def test_config1_dose_and_pairs_agree(c1):
    plan, orc = c1
    _check_dose(plan, orc)


def _body_plan(dc):
    n, sp = (21, 17, 13), (0.3, 0.25, 0.4)

    def body(Z, Y, X):
        r = (X / 2.6) ** 2 + (Y / 1.9) ** 2 + (Z / 2.2) ** 2
        return np.where(r <= 1.0, 1.0 + 0.5 * np.sin(2.0 * X) * np.cos(Y), 0.001)
    return S.plan_small(n=n, spacing=sp, density=body, seed=5, name="np_body",
                        options=S.Options(roi_radius=1.2, dc_enabled=dc), beams=[
                            S.Beam(gantry=0.7, couch=0.35, nbx=4, nby=3, wx=0.4, wy=0.3, cx=0.1),
                            S.Beam(gantry=3.9, nbx=3, nby=3, wx=0.5, wy=0.5, cy=-0.2)])


@pytest.mark.parametrize("dc", [1, 0])
def test_small_plans_agree(oracle_mod, dc):
    plan = S.abi_rounded(_body_plan(dc))
    _check_dose(plan, oracle_mod.Oracle(plan))
