"""Pins of the FP64 gamma-index reference (Section 2.3's evaluation): the
vectorised per-offset search against closed forms and against a plain
per-voxel search written independently here."""
import itertools
import math

import numpy as np

from oracle import gamma as G


def _brute(R, E, sp, dist, frac, cap):
    """Per-voxel loop over every grid voxel within the sphere."""
    nz, ny, nx = R.shape
    dD = frac * R.max()
    out = np.zeros_like(R)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        best = cap * cap
        for kk, jj, ii in itertools.product(range(nz), range(ny), range(nx)):
            d2 = ((ii - i) * sp[0]) ** 2 + ((jj - j) * sp[1]) ** 2 + ((kk - k) * sp[2]) ** 2
            if d2 > (cap * dist) ** 2:
                continue
            best = min(best, d2 / dist ** 2 + (E[kk, jj, ii] - R[k, j, i]) ** 2 / dD ** 2)
        out[k, j, i] = math.sqrt(best)
    return out


def test_matches_per_voxel_search():
    rng = np.random.default_rng(0)
    R = rng.uniform(0.0, 1.0, (4, 5, 6))
    E = R + rng.normal(0.0, 0.05, R.shape)
    sp = (0.15, 0.2, 0.1)
    for cap in (2.0, 5.0):
        assert np.allclose(G.gamma(R, E, sp, cap=cap), _brute(R, E, sp, 0.3, 0.03, cap), atol=1e-12)


def test_identical_is_zero_and_uniform_shift_is_closed_form():
    R = np.full((6, 7, 8), 2.0)
    assert np.all(G.gamma(R, R, (0.25, 0.25, 0.25)) == 0.0)
    # a uniform field shifted by delta cannot be matched spatially:
    # gamma = |delta| / dD, capped
    for delta, want in ((0.03, 0.5), (-0.09, 1.5), (0.5, 5.0)):
        g = G.gamma(R, R + delta, (0.25, 0.25, 0.25))
        assert np.allclose(g, min(abs(delta) / (0.03 * 2.0), 5.0), atol=1e-12), delta
        assert math.isclose(min(abs(delta) / 0.06, 5.0), want)


def test_spatial_shift_of_a_ramp():
    """A ramp D = a x shifted by one voxel along x: at interior voxels the
    gamma is the 1-D minimum over offsets k of
    sqrt((k dx)^2 / dd^2 + (a dx (k - 1))^2 / dD^2)."""
    n, dx, a = 40, 0.1, 0.5
    x = dx * np.arange(n)
    R = np.broadcast_to(a * x, (3, 4, n)).copy()
    E = np.broadcast_to(a * (x - dx), (3, 4, n)).copy()
    g = G.gamma(R, E, (dx, 0.25, 0.25))
    dD = 0.03 * R.max()
    want = min(math.sqrt((k * dx) ** 2 / 0.09 + (a * dx * (k - 1)) ** 2 / dD ** 2)
               for k in range(-15, 16) if abs(k * dx) <= 1.5)
    assert np.allclose(g[:, :, 16:-16], min(want, 5.0), atol=1e-12)
    assert want < a * dx / dD          # the spatial match beats the dose difference


def test_offsets_are_the_sphere():
    sp = (0.4, 0.4, 0.25)
    off = G.offsets(sp, 1.5)
    got = {(k, j, i) for k, j, i, _ in off}
    want = {(k, j, i) for k in range(-7, 8) for j in range(-4, 5) for i in range(-4, 5)
            if (i * 0.4) ** 2 + (j * 0.4) ** 2 + (k * 0.25) ** 2 <= 1.5 ** 2}
    assert got == want and (0, 0, 0) in got


def test_stats():
    R = np.zeros((2, 2, 2))
    R[0, 0, 0], R[0, 0, 1], R[1, 1, 1] = 10.0, 6.0, 4.0
    g = np.zeros_like(R)
    g[0, 0, 0], g[0, 0, 1], g[1, 1, 1], g[1, 0, 0] = 0.5, 1.5, 3.0, 0.2
    s = G.stats(g, R)
    assert s["n_iso"] == 2 and s["gamma_max"] == 3.0
    assert math.isclose(s["gamma_avg_iso"], 1.0) and s["pass_rate_iso"] == 0.5
