"""Pins of the oracle's Siddon mode (exact radiological path through
voxel-constant density, the ray-tracing alternative Section 2.2 sets aside),
against closed forms and against a fine numerical march along the axis."""
import math

import numpy as np
import pytest

import fspb_synth as S
from oracle import Oracle


def _opts(**kw):
    return S.Options(siddon=1, **kw)


def _eval(tab, key, slope, t):
    """Integral at depth t from segment tables (last segment at or before t)."""
    m = np.searchsorted(tab["t"], t, side="right") - 1
    return tab[key][m] + slope[m] * (t - tab["t"][m])


def test_water_is_geometric_depth():
    plan = S.plan_small(n=(20, 24, 16), density=1.0, options=_opts(),
                        beams=[S.Beam(gantry=0.5, couch=0.3, nbx=3, nby=3)])
    o = Oracle(plan)
    for i in range(plan.n_beamlets):
        tab = o.trace_siddon(i)
        tr = o.trace(i)
        assert tab["K"] > 5 and tr["hit"]
        assert tr["s_entry"] == pytest.approx(tr["s_in"], abs=1e-12)
        t = np.linspace(0, tab["t"][-1] + 2.0, 50)
        assert np.allclose(_eval(tab, "T", tab["rho"], t), t, atol=1e-12)
        assert np.allclose(tab["W1"], 0.0) and np.allclose(tab["W2"], 0.0)


def test_slabs_closed_form():
    """Config 1's slabs lie on voxel faces, so the exact path integral along
    the central axis is T(t) = t - 0.75 clip(t - 4, 0, 3) + 0.8 clip(t - 10, 0, 1)
    and W1 = 0.02 (-0.75 clip(t - 4, 0, 3) + 0.8 clip(t - 10, 0, 1)), W2 = -W1."""
    plan = S.plan_c1()
    plan.options = _opts()
    o = Oracle(plan)
    # the beamlet whose axis is closest to the central axis: beamlets (4|5, 4|5);
    # the lateral offset is 0.25 cm, parallel to the slabs, so depth is exact
    i = 4 * 10 + 4
    tab = o.trace_siddon(i)
    f = o.frame(i)
    cos = abs(f["d"][1])                        # the slabs are normal to y
    t = np.linspace(0.0, 14.0, 300)
    depth = t * cos                            # slab depth along y
    want = t - (0.75 * np.clip(depth - 4, 0, 3) - 0.8 * np.clip(depth - 10, 0, 1)) / cos
    assert np.allclose(_eval(tab, "T", tab["rho"], t), want, atol=1e-9)
    b = np.array([0.02 * (min(max(r, 0.1), 2.0) - 1.0) for r in tab["rho"]])
    w = 0.02 * (-0.75 * np.clip(depth - 4, 0, 3) + 0.8 * np.clip(depth - 10, 0, 1)) / cos
    assert np.allclose(_eval(tab, "W1", b, t), w, atol=1e-9)
    assert np.allclose(_eval(tab, "W2", -b, t), -w, atol=1e-9)


def _chord(p0, d, lo, hi):
    """Length of the line p0 + s d inside the box [lo, hi] (slab method)."""
    s0, s1 = -np.inf, np.inf
    for a in range(3):
        if d[a] == 0:
            if not lo[a] <= p0[a] <= hi[a]:
                return 0.0
            continue
        u, v = (lo[a] - p0[a]) / d[a], (hi[a] - p0[a]) / d[a]
        s0, s1 = max(s0, min(u, v)), min(s1, max(u, v))
    return max(0.0, s1 - s0)


def test_single_dense_voxel_adds_its_chord():
    n, sp = (15, 17, 13), (0.25, 0.3, 0.2)
    base = S.plan_small(n=n, spacing=sp, density=1.0, options=_opts(),
                        beams=[S.Beam(gantry=0.37, couch=0.21, nbx=1, nby=1, cx=0.13, cy=-0.07)])
    o0 = Oracle(base)
    f = o0.frame(0)
    # the voxel the axis crosses near the middle of its path through the grid
    tab0 = o0.trace_siddon(0)
    tr = o0.trace(0)
    s_mid = 0.5 * (tr["s_in"] + tr["s_out"])
    p = f["src"] + s_mid * f["d"]
    org = np.array(base.origin)
    idx = np.floor((p - (org - 0.5 * np.array(sp))) / np.array(sp)).astype(int)
    rho = np.ones((n[2], n[1], n[0]), np.float32)
    rho[idx[2], idx[1], idx[0]] = 1.7
    plan = S.plan_small(n=n, spacing=sp, density=rho, options=_opts(), beams=base.beams)
    tab = Oracle(plan).trace_siddon(0)
    lo = org + (idx - 0.5) * np.array(sp)
    chord = _chord(f["src"], f["d"], lo, lo + np.array(sp))
    assert chord > 0.05
    t_end = tab["t"][-1] + 1.0
    dT = _eval(tab, "T", tab["rho"], t_end) - _eval(tab0, "T", tab0["rho"], t_end)
    assert dT == pytest.approx((float(np.float32(1.7)) - 1.0) * chord, abs=1e-12)


def test_entrance_of_a_body_in_air():
    """The entrance is where the axis enters the first voxel of density
    >= 0.5, found here by marching the axis in 1e-4 cm steps."""
    n, sp = (22, 26, 18), (0.25, 0.25, 0.25)

    def body(Z, Y, X):
        return np.where((X / 2.5) ** 2 + (Y / 2.0) ** 2 + (Z / 1.8) ** 2 <= 1.0, 1.0, 0.001)
    plan = S.plan_small(n=n, spacing=sp, density=body, options=_opts(),
                        beams=[S.Beam(gantry=0.8, couch=-0.4, nbx=3, nby=2, wx=0.6, wy=0.6)])
    o = Oracle(plan)
    rho = plan.density
    org = np.array(plan.origin)
    lo = org - 0.5 * np.array(sp)
    for i in range(plan.n_beamlets):
        f, tr = o.frame(i), o.trace(i)
        s = np.arange(tr["s_in"], tr["s_out"], 1e-4)
        pts = f["src"] + s[:, None] * f["d"]
        ijk = np.clip(np.floor((pts - lo) / np.array(sp)).astype(int), 0, np.array(n) - 1)
        inside = rho[ijk[:, 2], ijk[:, 1], ijk[:, 0]] >= 0.5
        if not inside.any():
            assert not tr["hit"]
            continue
        assert tr["hit"]
        assert tr["s_entry"] == pytest.approx(s[np.argmax(inside)], abs=2e-4)


def test_siddon_equals_uniform_dose_in_water():
    """In water both tables give t_eq = t and no drift, and both entrances
    are the grid face: the doses agree."""
    beams = [S.Beam(gantry=0.3, nbx=3, nby=4), S.Beam(gantry=2.2, couch=0.3, nbx=2, nby=2)]
    plan = S.plan_small(n=(24, 20, 16), density=1.0, beams=beams)
    d_u, _, _ = Oracle(plan).dose()
    d_s, _, _ = Oracle(plan, siddon=1).dose()
    assert np.allclose(d_s, d_u, rtol=1e-10, atol=1e-14 * d_u.max())
    assert d_u.max() > 0
