"""Pins of the oracle's learned-surrogate support (inputs, targets and the
dose with given parameters).  CPU only.

The surrogate is an extension beside the method; these functions define
what it reads and predicts.  Each pin checks them against something other
than their own formulas: table values interpolated by NumPy, closed forms in
a uniform medium, brute force over beamlets, and sample points recovered
from linear density fields."""
import numpy as np
import pytest

import fspb_synth as S
from oracle import Oracle


def _uniform_plan(rho0, dc=1, beams=None, n=(28, 28, 28)):
    opts = S.Options(dc_enabled=dc)
    return S.plan_small(n=n, density=rho0, beams=beams or [S.Beam(gantry=0.4, nbx=5, nby=4)],
                        options=opts)


def _lerp(tab, x):
    v = np.asarray(tab.values, dtype=np.float64)
    grid = tab.start + tab.step * np.arange(v.shape[-1])
    return np.interp(x, grid, v)


def _counted_pairs(o, rng, n):
    out = []
    while len(out) < n:
        v = int(rng.integers(o.n_vox))
        i = int(rng.integers(o.n_beamlets))
        if o.pair(v, i)[1] & 1:
            out.append((v, i))
    return out


def _depth(o, v, i, plan):
    f, tr = o.frame(i), o.trace(i)
    nz, ny, nx = plan.shape
    r = np.array(plan.origin) + np.array(plan.spacing) * np.array([v % nx, (v // nx) % ny, v // (nx * ny)])
    return float(np.dot(r - f["src"], f["d"]) - tr["s_entry"])


def test_density_at_centres_and_linear_fields():
    rng = np.random.default_rng(0)
    plan = S.plan_small(n=(9, 7, 6), density=lambda Z, Y, X: 1.0 + 0.3 * X - 0.2 * Y + 0.1 * Z)
    o = Oracle(plan)
    nz, ny, nx = plan.shape
    org, sp = np.array(plan.origin), np.array(plan.spacing)
    for _ in range(20):                     # voxel centres reproduce the grid
        i, j, k = rng.integers(nx), rng.integers(ny), rng.integers(nz)
        assert o.density_at(org + sp * [i, j, k])[0] == pytest.approx(plan.density[k, j, i], abs=1e-12)
    # a linear field is reproduced exactly between centres
    lo, hi = org, org + sp * (np.array([nx, ny, nz]) - 1)
    pts = lo + rng.uniform(0, 1, size=(50, 3)) * (hi - lo)
    got = o.density_at(pts)
    rho32 = plan.density.astype(np.float64)
    # reference: the float32-stored linear field is linear only up to storage
    # rounding; compare to the exact field within that rounding
    want = 1.0 + 0.3 * pts[:, 0] - 0.2 * pts[:, 1] + 0.1 * pts[:, 2]
    assert np.allclose(got, want, atol=4e-7 * np.abs(rho32).max())
    # clamp to edge beyond the outermost centres
    p_out = np.array([lo[0] - 3.0, lo[1] + 0.5 * sp[1], lo[2]])
    p_in = np.array([lo[0], lo[1] + 0.5 * sp[1], lo[2]])
    assert o.density_at(p_out)[0] == pytest.approx(o.density_at(p_in)[0], abs=1e-12)


@pytest.mark.parametrize("dc", [1, 0])
def test_params_in_water_are_the_water_tables(dc):
    plan = _uniform_plan(1.0, dc=dc)
    o = Oracle(plan)
    t = plan.tables
    for v, i in _counted_pairs(o, np.random.default_rng(1), 25):
        prm, fl = o.params(v, i)
        d = _depth(o, v, i, plan)
        want = [_lerp(getattr(t, n), d) for n in ("u1x", "u1y", "u2x", "u2y", "w1", "w2")]
        assert np.allclose(prm, want, rtol=2e-6, atol=1e-9), (v, i)


def test_params_in_uniform_medium_closed_form():
    """rho = 0.7 everywhere: u1 = f_u1(0.7) u1w(t), u2 = f_u2(0.7) u2w(t),
    w_c = max(0, f_wc(0.7) (w_cw(t) + b_c(0.7) t)) -- the passing-history
    integral of a constant is the constant times the depth."""
    rho0 = 0.7
    plan = _uniform_plan(rho0, dc=1)
    o = Oracle(plan)
    t = plan.tables
    fu1, fu2 = _lerp(t.fu1, rho0), _lerp(t.fu2, rho0)
    fw1, fw2 = _lerp(t.fw1, rho0), _lerp(t.fw2, rho0)
    b1, b2 = _lerp(t.b1, rho0), _lerp(t.b2, rho0)
    for v, i in _counted_pairs(o, np.random.default_rng(2), 25):
        prm, _ = o.params(v, i)
        d = _depth(o, v, i, plan)
        want = [fu1 * _lerp(t.u1x, d), fu1 * _lerp(t.u1y, d), fu2 * _lerp(t.u2x, d),
                fu2 * _lerp(t.u2y, d), max(0.0, fw1 * (_lerp(t.w1, d) + b1 * d)),
                max(0.0, fw2 * (_lerp(t.w2, d) + b2 * d))]
        assert np.allclose(prm, want, rtol=2e-5, atol=1e-7), (v, i, prm, want)


def test_pair_given_with_own_params_is_the_pair():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.3, 1.9, size=(16, 20, 24)).astype(np.float32)
    plan = S.plan_small(density=rho, beams=[S.Beam(gantry=1.0, nbx=4, nby=3),
                                           S.Beam(gantry=3.5, couch=0.3, nbx=3, nby=3)])
    o = Oracle(plan)
    for v, i in _counted_pairs(o, rng, 40):
        prm, fl = o.params(v, i)
        d, fl2 = o.pair_given(v, i, prm)
        ref, fl3 = o.pair(v, i)
        assert fl == fl2 == fl3
        assert d == pytest.approx(ref, rel=1e-13, abs=1e-300)


def _iso_point(src, direction, cax, sad):
    return src + direction * (sad / np.dot(direction, cax))


@pytest.mark.parametrize("couch", [0.0, 0.35])
def test_nearest_beamlet_brute_force(couch):
    """The nearest beamlet minimises the isocentre-plane distance between the
    beamlet's axis and the voxel's central projection (brute force over the
    beamlets, using their frames)."""
    beam = S.Beam(gantry=0.7, couch=couch, nbx=6, nby=5, wx=0.6, wy=0.45, cx=0.2, cy=-0.1)
    plan = S.plan_small(n=(30, 30, 30), density=1.0, beams=[beam])
    o = Oracle(plan)
    fr = [o.frame(i) for i in range(o.n_beamlets)]
    src = fr[0]["src"]
    centre = np.array(beam.iso)
    cax = (centre - src) / np.linalg.norm(centre - src)
    iso_pts = np.array([_iso_point(src, f["d"], cax, beam.sad) for f in fr])
    nz, ny, nx = plan.shape
    rng = np.random.default_rng(4)
    checked = 0
    for v in rng.choice(o.n_vox, size=300, replace=False):
        r = np.array(plan.origin) + np.array(plan.spacing) * [v % nx, (v // nx) % ny, v // (nx * ny)]
        p = _iso_point(src, r - src, cax, beam.sad)
        dist = np.linalg.norm(iso_pts - p, axis=1)
        i, tie = o.nearest_beamlet(int(v), 0)
        if tie < 1e-6:
            continue
        assert i == int(np.argmin(dist)), v
        checked += 1
    assert checked > 250


def _row_points(plan_fn, vox, beam_idx):
    """Sample points of a surrogate row recovered from three linear fields
    rho = 10 + x, 10 + y, 10 + z (each field reveals one coordinate; all
    three are above the surface threshold everywhere, so they share the
    entrance).  The fields are stored in float32: coordinates carry about
    1e-6 cm of storage rounding."""
    pts = []
    for ax in range(3):
        plan = plan_fn(lambda Z, Y, X, ax=ax: 10.0 + (X, Y, Z)[ax])
        o = Oracle(plan)
        feat, near, _, _ = o.surrogate_rows([vox], beam_idx)
        assert near[0] >= 0
        pts.append(feat[0, :200] - 10.0)
    return np.stack(pts, axis=1).reshape(8, 5, 5, 3), feat[0], near[0], o


def test_surrogate_row_geometry_from_linear_fields():
    n, sp = (56, 56, 56), (0.25, 0.25, 0.25)
    beam = S.Beam(gantry=0.9, couch=0.25, nbx=5, nby=5)
    mk = lambda f: S.plan_small(n=n, spacing=sp, density=f, beams=[beam])
    nz, ny, nx = n[2], n[1], n[0]
    vox = (nz // 2 + 3) * nx * ny + (ny // 2 - 2) * nx + nx // 2 + 1
    P, feat, i, o = _row_points(mk, vox, 0)
    plan = mk(lambda Z, Y, X: 10.0 + X)
    tol = 2e-5
    org, spa = np.array(plan.origin), np.array(plan.spacing)
    lo, hi = org, org + spa * (np.array(n) - 1)
    inside = np.all((P > lo + tol) & (P < hi - tol), axis=-1)
    r = org + spa * np.array([vox % nx, (vox // nx) % ny, vox // (nx * ny)])
    f = o.frame(i)
    src = f["src"]
    u = (r - src) / np.linalg.norm(r - src)
    # plane 7's centre is the voxel centre
    assert inside[7, 2, 2] and np.allclose(P[7, 2, 2], r, atol=tol)
    t = feat[200]
    assert t == pytest.approx(_depth(o, vox, i, plan), abs=1e-12)
    assert feat[201] == pytest.approx(f["theta"], abs=1e-15)
    used = 0
    for k in range(8):
        c = P[k, 2, 2]
        if inside[k, 2, 2]:
            # plane centres lie on the source-voxel ray, t/7 apart
            assert np.allclose(np.cross(c - src, u), 0, atol=tol * 20)
            assert np.dot(r - c, u) == pytest.approx(t * (7 - k) / 7, abs=tol)
        for b in range(5):
            for a in range(4):
                if inside[k, b, a] and inside[k, b, a + 1]:
                    e1 = (P[k, b, a + 1] - P[k, b, a]) / 0.5
                    assert np.linalg.norm(e1) == pytest.approx(1.0, abs=4 * tol)
                    assert abs(np.dot(e1, u)) < 4 * tol
                    used += 1
            for a in range(5):
                if b < 4 and inside[k, b, a] and inside[k, b + 1, a]:
                    e2 = (P[k, b + 1, a] - P[k, b, a]) / 0.5
                    assert np.linalg.norm(e2) == pytest.approx(1.0, abs=4 * tol)
                    assert abs(np.dot(e2, u)) < 4 * tol
    assert used > 100
    # orientation: e1 lies in the plane of u and the beam's lateral x axis
    # (the x axis of the central beamlet of an odd grid is the beam's),
    # pointing along it; e2 = e1 x u
    ex = o.frame(o.n_beamlets // 2)["ex"]
    e1 = (P[7, 2, 3] - P[7, 2, 2]) / 0.5
    e2 = (P[7, 3, 2] - P[7, 2, 2]) / 0.5
    assert abs(np.dot(e1, np.cross(u, ex))) < 4 * tol and np.dot(e1, ex) > 0
    assert np.allclose(e2, np.cross(e1, u), atol=4 * tol)


def test_surrogate_row_validity():
    """Rows are valid exactly when the nearest beamlet's pair is counted."""
    rng = np.random.default_rng(5)
    # body in y > -1 with scattered air voxels; air in front of it
    plan = S.plan_small(density=lambda Z, Y, X: np.where(
        (Y > -1.0) & (rng.uniform(size=X.shape) > 0.1), 1.0, 0.05),
        beams=[S.Beam(gantry=0.2, nbx=3, nby=3, wx=1.0, wy=1.0)])
    o = Oracle(plan)
    vox = rng.choice(o.n_vox, size=200, replace=False)
    _, near, _, _ = o.surrogate_rows(vox, 0)
    for v, i in zip(vox, near):
        j, _ = o.nearest_beamlet(int(v), 0)
        assert (i >= 0) == bool(o.pair(int(v), j)[1] & 1)
        if i >= 0:
            assert i == j
    assert (near >= 0).sum() > 20 and (near < 0).sum() > 5


def test_dose_given_reduces_to_the_method():
    rng = np.random.default_rng(6)
    rho = rng.uniform(0.3, 1.9, size=(16, 20, 24)).astype(np.float32)
    beams = [S.Beam(gantry=0.3, nbx=3, nby=4), S.Beam(gantry=2.9, nbx=4, nby=3)]
    plan = S.plan_small(density=rho, beams=beams, seed=2)
    o = Oracle(plan)
    vox = rng.choice(o.n_vox, size=60, replace=False)
    d_ref, _, _ = o.dose(vox=vox)
    prm = np.zeros((vox.size, 2, 7))
    prm[..., 6] = 1.0                           # every row falls back
    d, _ = o.dose_given(prm, vox=vox)
    assert np.array_equal(d, d_ref)
    # constant tables in a uniform medium: every beamlet's parameters are the
    # same constants, so rows carrying them reproduce the method
    plan_c = S.plan_small(density=1.3, beams=beams, tables=S.constant_tables(), seed=2)
    oc = Oracle(plan_c)
    d_ref, _, _ = oc.dose(vox=vox)
    prm = np.zeros((vox.size, 2, 7))
    prm[..., :6] = [3.0, 3.0, 1.0, 1.0, 0.8, 0.2]
    d, _ = oc.dose_given(prm, vox=vox)
    assert np.allclose(d, d_ref, rtol=1e-6, atol=1e-12 * np.abs(d_ref).max())
    assert np.abs(d_ref).max() > 0
