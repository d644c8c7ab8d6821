"""Second FP64 oracle of the DC-FSPB dose, in NumPy: a cross-check of the C
oracle.

TEST INFRASTRUCTURE ONLY.  Only the test suite imports this module.  It
shares no code with the C oracle (``fspb_oracle.c``) or with the GPU package,
and it is organised differently: it works one beamlet at a time over the
whole grid with array operations, and it smooths the density with three 1-D
passes, where the C oracle loops over voxels and sums the 3D Gaussian
directly.  Both follow the paper's definitions and the same readings of what
the paper leaves open (listed in the repository's design notes), so a
transcription mistake in either one shows up as a disagreement between them.

What it computes, in the paper's order:

* the smoothed density (Section 2.1; Algorithm A1, step 1);
* the beamlet frames (Eq. 2 geometry; Algorithm A1, step 3);
* the uniformly sampled radiological depth and weight drift along each
  beamlet axis (Section 2.2; Algorithm A1, steps 4-6);
* the ROI pair test (Algorithm A1, step 8), decided in single precision by
  the fixed recipe both sides use;
* the pair dose, Eqs. 2-4 with the Section 2.1 corrections (Algorithm A1,
  steps 9-12);
* the dose, Eq. 1, summed in beamlet order.

It takes a ``fspb_synth.Plan`` (pass it through ``fspb_synth.abi_rounded``
to compare with the library or the C oracle on the same instance).
"""
from __future__ import annotations

import math

import numpy as np


# -- single precision with one rounding per fused multiply-add -------------
def fma32(a, b, c):
    """Elementwise fma(a, b, c) of float32 values, rounded once to float32.

    a*b is exact in float64 (two 24-bit significands).  The float64 sum s of
    the product and c, and its rounding error e (Knuth's two-sum), are exact.
    s rounds to the correctly rounded float32 result, except when s lies on
    a midpoint between two float32 values; then the sign of e says on which
    side the exact sum lies."""
    a = np.asarray(a, dtype=np.float32).astype(np.float64)
    b = np.asarray(b, dtype=np.float32).astype(np.float64)
    c = np.asarray(c, dtype=np.float32).astype(np.float64)
    p = a * b
    s = p + c
    bv = s - p
    e = (p - (s - bv)) + (c - bv)
    r = s.astype(np.float32)
    rd = r.astype(np.float64)
    above = s > rd
    other = np.where(above, np.nextafter(r, np.float32(np.inf)), np.nextafter(r, np.float32(-np.inf)))
    mid = 0.5 * (rd + other.astype(np.float64))
    tie = (s == mid) & (e != 0.0) & (rd != s)
    return np.where(tie & ((e > 0.0) == above), other, r).astype(np.float32)


# -- tables (interpolation reading: linear, coordinate clamped to the table) -
def lerp_uniform(start, step, values, x):
    """Linear interpolation in a table sampled at start + k step, k < n;
    outside the table the end value holds."""
    v = np.asarray(values, dtype=np.float64).reshape(-1)
    x = np.asarray(x, dtype=np.float64)
    if v.size == 1:
        return np.full(x.shape, v[0])
    c = np.clip((x - start) / step, 0.0, v.size - 1)
    k = np.minimum(np.floor(c).astype(np.int64), v.size - 2)
    f = c - k
    return v[k] + f * (v[k + 1] - v[k])


def lerp_table(tab, x):
    return lerp_uniform(float(tab.start), float(tab.step), tab.values, x)


def a_bilinear(tables, teq, theta):
    """A(t_eq, theta): rows of the A table are theta samples (theta_step
    apart from 0), columns radiological depth; bilinear, clamped."""
    A = np.asarray(tables.A.values, dtype=np.float64).reshape(int(tables.n_theta), -1)
    nth = A.shape[0]
    if nth == 1:
        return lerp_uniform(float(tables.A.start), float(tables.A.step), A[0], teq)
    cr = min(max(theta / float(tables.theta_step), 0.0), nth - 1.0)
    r = min(int(math.floor(cr)), nth - 2)
    fr = cr - r
    a0 = lerp_uniform(float(tables.A.start), float(tables.A.step), A[r], teq)
    a1 = lerp_uniform(float(tables.A.start), float(tables.A.step), A[r + 1], teq)
    return a0 + fr * (a1 - a0)


# -- Eq. 4 -------------------------------------------------------------------
def penumbra(x, u, x0):
    """Eq. 4: a box of half-width x0 convolved with the normalised Laplace
    density (u/2) exp(-u |x|): sinh(u x0) exp(-u |x|) outside the box,
    1 - cosh(u x) exp(-u x0) inside."""
    ax = np.abs(x)
    outside = np.sinh(u * x0) * np.exp(-u * ax)
    inside = 1.0 - np.cosh(u * x) * np.exp(-u * x0)
    return np.where(ax > x0, outside, inside)


# -- Section 2.1, Algorithm A1 step 1 ----------------------------------------
def smoothed_density(plan):
    """The density convolved with a normalised 3D Gaussian of width
    smooth_sigma, truncated to ceil(3 sigma / delta) voxels per axis, with
    clamp-to-edge beyond the grid.  The 3D Gaussian is the product of 1-D
    ones, so three 1-D passes give the same convolution."""
    rho = np.asarray(plan.density, dtype=np.float64)
    sigma = float(plan.options.smooth_sigma)
    if sigma <= 0.0:
        return rho.copy()
    out = rho
    for axis, delta in ((2, plan.spacing[0]), (1, plan.spacing[1]), (0, plan.spacing[2])):
        r = int(math.ceil(3.0 * sigma / float(delta) - 1e-6))
        offs = np.arange(-r, r + 1)
        w = np.exp(-((offs * float(delta)) ** 2) / (2.0 * sigma * sigma))
        w /= w.sum()
        n = out.shape[axis]
        acc = np.zeros_like(out)
        for o, wk in zip(offs, w):
            idx = np.clip(np.arange(n) + o, 0, n - 1)
            acc += wk * np.take(out, idx, axis=axis)
        out = acc
    return out


# -- Eq. 2 geometry, Algorithm A1 step 3 --------------------------------------
def beamlet_frames(plan):
    """Per beamlet: source, unit direction d, lateral axes ex (the beam's x
    axis made orthogonal to d) and ey = ex x d, off-axis angle theta and
    half widths.  Gantry phi rotates about z (source at iso - SAD (0, 1, 0)
    at phi = 0), the couch rotates the beam about y; beamlet (n, m) is
    centred at ((m - (nbx - 1)/2) wx + cx, (n - (nby - 1)/2) wy + cy) in the
    isocentre plane."""
    frames = []
    for beam in plan.beams:
        phi, psi = float(beam.gantry), float(beam.couch)
        cp, sp_ = math.cos(psi), math.sin(psi)

        def couch(v):
            return np.array([cp * v[0] + sp_ * v[2], v[1], -sp_ * v[0] + cp * v[2]])
        cax = couch((-math.sin(phi), math.cos(phi), 0.0))
        bx = couch((math.cos(phi), math.sin(phi), 0.0))
        by = couch((0.0, 0.0, 1.0))
        sad = float(beam.sad)
        src = np.array([float(beam.iso[k]) - sad * cax[k] for k in range(3)])
        for n in range(beam.nby):
            for m in range(beam.nbx):
                a = (m - 0.5 * (beam.nbx - 1)) * float(beam.wx) + float(beam.cx)
                b = (n - 0.5 * (beam.nby - 1)) * float(beam.wy) + float(beam.cy)
                d = sad * cax + a * bx + b * by
                d = d / math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
                ex = bx - (bx[0] * d[0] + bx[1] * d[1] + bx[2] * d[2]) * d
                ex = ex / math.sqrt(ex[0] * ex[0] + ex[1] * ex[1] + ex[2] * ex[2])
                ey = np.array([ex[1] * d[2] - ex[2] * d[1], ex[2] * d[0] - ex[0] * d[2],
                               ex[0] * d[1] - ex[1] * d[0]])
                frames.append(dict(src=src, d=d, ex=ex, ey=ey, sad=sad,
                                   theta=math.atan(math.sqrt(a * a + b * b) / sad),
                                   x0=0.5 * float(beam.wx), y0=0.5 * float(beam.wy)))
    return frames


def trilinear(plan, pts):
    """Density between voxel centres (trilinear), clamp-to-edge, at points
    [n, 3]."""
    rho = np.asarray(plan.density, dtype=np.float64)
    nz, ny, nx = rho.shape
    g = (pts - np.asarray(plan.origin, dtype=np.float64)) / np.asarray(plan.spacing, dtype=np.float64)
    i0 = np.floor(g).astype(np.int64)
    f = g - i0
    out = np.zeros(len(pts))
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                w = ((f[:, 0] if cx else 1.0 - f[:, 0]) * (f[:, 1] if cy else 1.0 - f[:, 1])
                     * (f[:, 2] if cz else 1.0 - f[:, 2]))
                x = np.clip(i0[:, 0] + cx, 0, nx - 1)
                y = np.clip(i0[:, 1] + cy, 0, ny - 1)
                z = np.clip(i0[:, 2] + cz, 0, nz - 1)
                out += w * rho[z, y, x]
    return out


# -- Section 2.2, Algorithm A1 steps 4-6 ---------------------------------------
def sample_step(plan):
    d = float(plan.options.sample_step)
    return d if d > 0.0 else 0.5 * min(float(v) for v in plan.spacing)


def trace(plan, fr):
    """Uniform samples along the beamlet axis from where it enters the grid
    box, one sample past the deepest box corner along the axis.  The
    entrance is the first sample whose density reaches rho_surface; from it
    the radiological depth T and the drifts W_c are trapezoid sums of rho
    and of b_c(rho) (rho clamped to the commissioned range for b_c).
    Returns None when the axis misses the box or never reaches the body."""
    nx, ny, nz = plan.density.shape[2], plan.density.shape[1], plan.density.shape[0]
    o = np.asarray(plan.origin, dtype=np.float64)
    dl = np.asarray(plan.spacing, dtype=np.float64)
    lo = o - 0.5 * dl
    hi = o + (np.array([nx, ny, nz]) - 0.5) * dl
    src, d = fr["src"], fr["d"]
    s_in, s_out = -math.inf, math.inf
    for a in range(3):
        if d[a] == 0.0:
            if src[a] < lo[a] or src[a] > hi[a]:
                return None
            continue
        t1, t2 = (lo[a] - src[a]) / d[a], (hi[a] - src[a]) / d[a]
        s_in, s_out = max(s_in, min(t1, t2)), min(s_out, max(t1, t2))
    s_in = max(s_in, 0.0)
    if not s_in < s_out:
        return None
    corners = np.array([[hi[0] if k & 1 else lo[0], hi[1] if k & 2 else lo[1],
                         hi[2] if k & 4 else lo[2]] for k in range(8)])
    v = corners - src
    s_cover = max(v[k, 0] * d[0] + v[k, 1] * d[1] + v[k, 2] * d[2] for k in range(8))
    step = sample_step(plan)
    n = int(math.floor((s_cover - s_in) / step)) + 2
    s = s_in + np.arange(n) * step
    rho = trilinear(plan, src[None, :] + s[:, None] * d[None, :])
    inside = np.nonzero(rho >= float(plan.options.rho_surface))[0]
    if inside.size == 0:
        return None
    ke = int(inside[0])
    r = rho[ke:]
    rc = np.clip(r, float(plan.options.rho_min), float(plan.options.rho_max))
    t = plan.tables

    def cumtrap(y):
        out = np.zeros(len(y))
        out[1:] = np.cumsum(step * 0.5 * (y[:-1] + y[1:]))
        return out
    return dict(s_entry=s_in + ke * step, step=step, T=cumtrap(r),
                W1=cumtrap(lerp_table(t.b1, rc)), W2=cumtrap(lerp_table(t.b2, rc)))


# -- Algorithm A1 step 8: the pair test in single precision --------------------
def voxel_indices(plan):
    nz, ny, nx = plan.density.shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.reshape(-1), j.reshape(-1), k.reshape(-1)


def pair_mask(plan, fr, tr, idx):
    """The pair counts iff t >= 0 and xp^2 + yp^2 <= R^2, in single
    precision: voxel positions relative to the grid centre P0 and the
    beamlet's direction, lateral axes and offsets rounded to float32 from
    double, each coordinate one chain of fused multiply-adds."""
    n = plan.density.shape[::-1]
    o = [float(v) for v in plan.origin]
    dl = [float(v) for v in plan.spacing]
    P0 = [o[a] + 0.5 * (n[a] - 1) * dl[a] for a in range(3)]
    q = [fma32(idx[a].astype(np.float32), np.float32(dl[a]), np.float32(o[a] - P0[a]))
         for a in range(3)]
    v0 = [P0[a] - fr["src"][a] for a in range(3)]

    def row(axis, offset):
        return [np.float32(axis[0]), np.float32(axis[1]), np.float32(axis[2]), np.float32(offset)]

    def dotv(u):
        return v0[0] * u[0] + v0[1] * u[1] + v0[2] * u[2]
    rt = row(fr["d"], dotv(fr["d"]) - tr["s_entry"])
    rx = row(fr["ex"], dotv(fr["ex"]))
    ry = row(fr["ey"], dotv(fr["ey"]))

    def chain(r):
        return fma32(q[0], r[0], fma32(q[1], r[1], fma32(q[2], r[2], r[3])))
    t, xp, yp = chain(rt), chain(rx), chain(ry)
    rf = np.float32(float(plan.options.roi_radius))
    return (t >= np.float32(0.0)) & (fma32(xp, xp, yp * yp) <= rf * rf)


# -- Eqs. 1-4, Section 2.1 -------------------------------------------------------
def dose(plan, fluence=None):
    """Returns (dose [nz, ny, nx], evaluated pairs per voxel) of Eq. 1:
    D(r) = sum over beamlets i with f_i != 0 of f_i D_i(r), in beamlet
    order, where D_i(r) (Eq. 2) is F A(t_eq, theta_i) (SAD / |r_a|)^2 with
    F = w_1 p_x(u_1x) p_y(u_1y) + w_2 p_x(u_2x) p_y(u_2y) (Eq. 3, Eq. 4) for
    the pairs of Algorithm A1 step 8, and 0 for the others."""
    f = np.asarray(plan.fluence if fluence is None else fluence, dtype=np.float32)
    opt, tab = plan.options, plan.tables
    dc = bool(opt.dc_enabled)
    idx = voxel_indices(plan)
    o = np.asarray(plan.origin, dtype=np.float64)
    dl = np.asarray(plan.spacing, dtype=np.float64)
    r = np.stack([o[a] + idx[a] * dl[a] for a in range(3)], axis=1)
    rho_c = np.clip(np.asarray(plan.density, dtype=np.float64).reshape(-1), float(opt.rho_min),
                    float(opt.rho_max))
    if dc:
        rhohat_c = np.clip(smoothed_density(plan).reshape(-1), float(opt.rho_min), float(opt.rho_max))
        fu1, fu2 = lerp_table(tab.fu1, rho_c), lerp_table(tab.fu2, rhohat_c)
        fw1, fw2 = lerp_table(tab.fw1, rhohat_c), lerp_table(tab.fw2, rhohat_c)
    out = np.zeros(len(r))
    pairs = np.zeros(len(r), dtype=np.int64)
    for i, fr in enumerate(beamlet_frames(plan)):
        if f[i] == 0.0:
            continue
        tr = trace(plan, fr)
        if tr is None:
            continue
        sel = np.nonzero(pair_mask(plan, fr, tr, idx))[0]
        v = r[sel] - fr["src"]
        s = v @ fr["d"]
        keep = s > 0.0
        sel, v, s = sel[keep], v[keep], s[keep]
        xp, yp = v @ fr["ex"], v @ fr["ey"]
        depth = s - tr["s_entry"]
        mag = fr["sad"] / s
        ci = depth / tr["step"]
        teq = lerp_uniform(0.0, 1.0, tr["T"], ci)
        A = a_bilinear(tab, teq, fr["theta"])
        u1x, u1y = lerp_table(tab.u1x, depth), lerp_table(tab.u1y, depth)
        u2x, u2y = lerp_table(tab.u2x, depth), lerp_table(tab.u2y, depth)
        w1, w2 = lerp_table(tab.w1, depth), lerp_table(tab.w2, depth)
        if dc:
            u1x, u1y = u1x * fu1[sel], u1y * fu1[sel]
            u2x, u2y = u2x * fu2[sel], u2y * fu2[sel]
            W1 = lerp_uniform(0.0, 1.0, tr["W1"], ci)
            W2 = lerp_uniform(0.0, 1.0, tr["W2"], ci)
            w1 = np.maximum(fw1[sel] * (w1 + W1), 0.0)
            w2 = np.maximum(fw2[sel] * (w2 + W2), 0.0)
        x, y = xp * mag, yp * mag
        F = (w1 * penumbra(x, u1x, fr["x0"]) * penumbra(y, u1y, fr["y0"])
             + w2 * penumbra(x, u2x, fr["x0"]) * penumbra(y, u2y, fr["y0"]))
        out[sel] += float(f[i]) * (F * A * mag * mag)
        pairs[sel] += 1
    shape = plan.density.shape
    return out.reshape(shape), pairs.reshape(shape)
