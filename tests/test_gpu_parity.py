"""GPU parity of libfspb against the FP64 oracle (run on an MI355X).

Every comparison calls the C ABI through the thin ctypes binding; the
oracle runs independently on the host from the same seeded inputs.
"""
import math

import numpy as np
import pytest
import torch

import fspb_synth as S
from gpu_helpers import (REL_TOL, abi_oracle, amb_stats, assert_dose_parity, assert_pair_consts_equal,
                         geometry, gpu_dose, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1103_1164_amd as M
    M.load()
    yield


# ---------------------------------------------------------------------------
# Config 1: the whole grid, DC and plain
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dc", [1, 0])
def test_c1_full_grid(oracle_mod, dc):
    plan = S.plan_c1()
    say(f"c1 dc={dc}")
    orc = abi_oracle(plan, dc_enabled=dc)
    d_orc, amb, pc = orc.dose()
    geo = geometry(plan, dc)
    d_gpu = gpu_dose(geo, plan.fluence)
    rel = assert_dose_parity(d_gpu, d_orc, amb, what=f"c1 dc={dc}")
    say(f"c1 dc={dc}: max |err|/max D = {rel:.2e}, pairs {int(pc.sum())}")
    assert assert_pair_consts_equal(geo, orc)[0] == 100
    n_gpu = geo.count_pairs(torch.as_tensor(plan.fluence, device="cuda"))
    assert n_gpu == int(pc.sum())


def test_c1_intermediates(oracle_mod):
    plan = S.plan_c1()
    orc = abi_oracle(plan)
    geo = geometry(plan, 1)
    info = geo.info()
    assert info["n_beamlets"] == 100 and info["n_hit"] == 100
    assert info["n_entry_ambiguous"] == 0
    assert info["smooth_radius"] == orc.smooth_radius()
    rh = geo.smoothed_density().cpu().numpy()
    ro = orc.smoothed()
    assert np.max(np.abs(rh - ro)) < 2e-6
    for i in range(orc.n_beamlets):
        g, o = geo.beamlet(i), orc.trace(i)
        f = orc.frame(i)
        assert g["hit"] == o["hit"] and g["k_entry"] == o["k_entry"] and g["K"] == o["K"]
        assert abs(g["s_entry"] - o["s_entry"]) < 1e-9
        assert np.allclose(g["d"], f["d"], atol=1e-12) and np.allclose(g["ex"], f["ex"], atol=1e-12)
        assert np.allclose(g["ey"], f["ey"], atol=1e-12) and abs(g["theta"] - f["theta"]) < 1e-12
        assert np.max(np.abs(g["T"] - o["T"])) <= 2e-6 * max(1.0, o["T"].max())
        assert np.max(np.abs(g["W1"] - o["W1"])) < 1e-7 and np.max(np.abs(g["W2"] - o["W2"])) < 1e-7


@pytest.mark.parametrize("sigma,spacing", [(0.5, (0.2, 0.25, 0.3)), (2.0, (0.2, 0.2, 0.2))])
def test_smoothed_density_lds_and_wide_passes(oracle_mod, sigma, spacing):
    """The smoothed density against the oracle's direct 3D sum: unequal
    radii per axis (8, 6, 5 voxels: the LDS-staged passes) and a radius of
    30 voxels (beyond the LDS tiles: the single-axis passes)."""
    rng = np.random.default_rng(17)
    n = (26, 21, 17)
    rho = rng.uniform(0.05, 2.0, size=(n[2], n[1], n[0])).astype(np.float32)
    plan = S.plan_small(n=n, spacing=spacing, density=rho, seed=17,
                        options=S.Options(smooth_sigma=sigma), name="smooth")
    geo = geometry(plan, 1)
    orc = abi_oracle(plan)
    assert geo.info()["smooth_radius"] == orc.smooth_radius()
    say(f"smoothing sigma={sigma}: radius {orc.smooth_radius()}")
    rh = geo.smoothed_density().cpu().numpy()
    assert np.max(np.abs(rh - orc.smoothed())) < 2e-6
    geo.close()


def test_c1_pair_counts_per_voxel(oracle_mod):
    plan = S.plan_c1()
    orc = abi_oracle(plan)
    counts_o = orc.pair_counts()
    geo = geometry(plan, 1)
    tot, counts_g = geo.count_pairs(None, per_voxel=True)
    counts_g = counts_g.cpu().numpy()
    assert np.array_equal(counts_g, counts_o)
    assert tot == int(counts_o.sum())
    # per beamlet, from the adjoint's traversal: every beamlet exactly
    bpc = geo.beamlet_pair_counts().cpu().numpy().astype(np.int64)
    assert np.array_equal(bpc, orc.beamlet_pair_counts())


def _tight_plans():
    """Small ROI radii (0.3 to 1.2 cm) on grids with unequal voxel sizes,
    couch rotations and beams along grid axes: the row intervals the
    adjoint scans are then short and their ends decide many pairs."""
    rng = np.random.default_rng(31)
    out = []
    for k in range(6):
        n = tuple(int(v) for v in rng.integers(10, 40, 3))
        sp = tuple(float(v) for v in rng.uniform(0.1, 0.5, 3))
        rho = rng.uniform(0.05, 2.2, size=(n[2], n[1], n[0])).astype(np.float32)
        beams = [S.Beam(gantry=float(rng.uniform(0, 6.3)),
                        couch=float(rng.uniform(-1.5, 1.5)) if k % 2 else 0.0,
                        nbx=int(rng.integers(2, 7)), nby=int(rng.integers(2, 7)),
                        wx=float(rng.uniform(0.1, 0.6)), wy=float(rng.uniform(0.1, 0.6)))
                 for _ in range(2)]
        beams.append(S.Beam(gantry=(math.pi / 2) * (k % 4), nbx=3, nby=2))
        opts = S.Options(roi_radius=float(rng.uniform(0.3, 1.2)))
        out.append(S.plan_small(n=n, spacing=sp, density=rho, beams=beams, options=opts,
                                seed=k, name=f"tight{k}"))
    return out


@pytest.mark.parametrize("k", range(6))
def test_beamlet_pair_counts_tight_roi(oracle_mod, k):
    plan = _tight_plans()[k]
    orc = abi_oracle(plan)
    geo = geometry(plan, 1)
    bpc = geo.beamlet_pair_counts().cpu().numpy().astype(np.int64)
    assert np.array_equal(bpc, orc.beamlet_pair_counts())
    assert int(bpc.sum()) == geo.count_pairs(None)
    # and the adjoint on the same plan, every beamlet
    w = np.random.default_rng(k).uniform(0, 1, plan.n_vox).astype(np.float32)
    g = geo.adjoint(torch.as_tensor(w, device="cuda")).cpu().numpy().astype(np.float64)
    g_o, amb = orc.adjoint(w)
    amb_stats(amb, np.abs(g_o).max(), f"tight{k} adjoint")
    assert np.all(np.abs(g - g_o) <= REL_TOL * np.abs(g_o).max())
    geo.close()


# ---------------------------------------------------------------------------
# Small plans with ragged sizes and every geometry option
# ---------------------------------------------------------------------------
def _ragged_plans():
    rng = np.random.default_rng(21)
    out = []
    # heterogeneous noise phantom, two beams, rectangular beamlets, offsets
    n = (23, 19, 13)
    rho = rng.uniform(0.05, 2.3, size=(n[2], n[1], n[0])).astype(np.float32)
    out.append(S.plan_small(n=n, density=rho, seed=1, name="noise2", beams=[
        S.Beam(gantry=0.3, nbx=5, nby=3, wx=0.4, wy=0.6, cx=0.2, cy=-0.1),
        S.Beam(gantry=3.9, nbx=4, nby=4, wx=0.5, wy=0.5)]))
    # body in air (entrance inside the grid), anisotropic voxels, couch rotation
    n, sp = (30, 26, 17), (0.3, 0.25, 0.4)

    def body(Z, Y, X):
        r = (X / 3.2) ** 2 + (Y / 2.6) ** 2 + (Z / 3.0) ** 2
        return np.where(r <= 1.0, 1.0 + 0.3 * np.sin(2 * X) * np.cos(Y), 0.001)
    out.append(S.plan_small(n=n, spacing=sp, density=body, seed=2, name="body_couch", beams=[
        S.Beam(gantry=1.2, couch=0.35, nbx=6, nby=5, wx=0.5, wy=0.5, iso=(0.2, -0.3, 0.1)),
        S.Beam(gantry=5.0, couch=-0.2, sad=80.0, nbx=3, nby=7, wx=0.7, wy=0.3)]))
    # single beamlet, beam along x, 1-voxel-thick grid
    out.append(S.plan_small(n=(25, 9, 1), density=1.1, seed=3, name="thin",
                            beams=[S.Beam(gantry=math.pi / 2, nbx=1, nby=1, wx=1.0, wy=1.0)]))
    return out


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("dc", [1, 0])
def test_ragged_plans_full_grid(oracle_mod, k, dc):
    plan = _ragged_plans()[k]
    say(f"ragged {plan.name} dc={dc}")
    orc = abi_oracle(plan, dc_enabled=dc)
    d_orc, amb, pc = orc.dose()
    geo = geometry(plan, dc)
    d_gpu = gpu_dose(geo, plan.fluence)
    assert d_orc.max() > 0
    assert_dose_parity(d_gpu, d_orc, amb, what=plan.name)
    assert geo.info()["n_entry_ambiguous"] == 0
    assert_pair_consts_equal(geo, orc)
    assert geo.count_pairs(torch.as_tensor(plan.fluence, device="cuda")) == int(pc.sum())


# ---------------------------------------------------------------------------
# Full-size configs 2 and 3, on sampled voxels and beamlets
# ---------------------------------------------------------------------------
def _sample_voxels(shape, d_gpu, n, seed):
    rng = np.random.default_rng(seed)
    nv = int(np.prod(shape))
    rand = rng.choice(nv, size=n, replace=False)
    hot = np.argsort(d_gpu.reshape(-1))[-n // 4:]          # highest-dose voxels
    hot = rng.choice(hot, size=min(len(hot), n // 4), replace=False)
    return np.unique(np.concatenate([rand, hot]))


_FULL = {"c2": S.plan_c2, "c3": S.plan_c3, "paper_h5": S.plan_paper_h5, "paper_l2": S.plan_paper_l2}


@pytest.mark.parametrize("cfg", list(_FULL))
def test_full_size_forward_sampled(oracle_mod, cfg):
    """Configs 2 and 3, and the paper-shaped plans (Table 1 scales: 0.4 x 0.4
    x 0.25 cm voxels, 0.2 x 0.5 cm beamlets, non-coplanar beams for the
    head-and-neck case).  Config 2 runs with the tile bench.py times it with."""
    from bench import C2_TILE
    plan = _FULL[cfg]()
    tile = C2_TILE if cfg == "c2" else None
    say(f"{cfg}: geometry, tile {tile}")
    geo = geometry(plan, 1, tile=tile)
    if tile is not None:
        assert geo.get_tile() == tuple(tile)
    d_gpu = gpu_dose(geo, plan.fluence)
    info = geo.info()
    assert info["n_entry_ambiguous"] == 0
    vox = _sample_voxels(plan.shape, d_gpu, 3000, seed=7)
    say(f"{cfg}: oracle at {vox.size} voxels")
    orc = abi_oracle(plan)
    # beamlets that reach the body: all of them in configs 2 and 3; the
    # paper-shaped head's outer beamlet rows pass beside it
    hits = sum(orc.trace(i)["hit"] for i in range(plan.n_beamlets))
    assert info["n_hit"] == hits
    if cfg in ("c2", "c3"):
        assert hits == plan.n_beamlets
    d_o, amb, pc = orc.dose(vox=vox)
    # the scale is the oracle maximum over the sample, which includes the
    # hottest GPU voxels
    rel = assert_dose_parity(d_gpu.reshape(-1)[vox], d_o, amb, what=cfg)
    say(f"{cfg}: max |err|/max D = {rel:.2e}")
    assert np.all(np.isfinite(d_gpu)) and d_gpu.min() >= 0.0
    # the pair test's single-precision constants of every beamlet, and the
    # evaluated-pair counts at the sampled voxels
    n_eq, n_tiny = assert_pair_consts_equal(geo, orc)
    say(f"{cfg}: pair-test constants of {n_eq} beamlets agree ({n_tiny} not bitwise, within 1e-12)")
    tot, cnt = geo.count_pairs(torch.as_tensor(plan.fluence, device="cuda"), per_voxel=True)
    cnt = cnt.cpu().numpy().reshape(-1)[vox]
    assert np.array_equal(cnt, pc)
    # the adjoint's beamlet-major traversal visits the same pairs: its
    # per-beamlet counts add up to the forward's total, and sampled beamlets
    # match the oracle's count exactly
    bpc = geo.beamlet_pair_counts().cpu().numpy().astype(np.int64)
    assert int(bpc.sum()) == geo.count_pairs(None)
    pick = np.random.default_rng(8).choice(plan.n_beamlets, 6, replace=False)
    say(f"{cfg}: oracle pair counts of beamlets {pick.tolist()}")
    assert np.array_equal(bpc[pick], orc.beamlet_pair_counts(pick))


def test_c3_adjoint_sampled_and_fd(oracle_mod):
    plan = S.plan_c3()
    geo = geometry(plan, 1)
    nb = plan.n_beamlets
    w, u = S.c3_objective(3, plan.n_vox)
    wt = torch.as_tensor(w, device="cuda")
    g = geo.adjoint(wt).cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(g))
    # sampled beamlets: two 4x2 blocks in beams 0 and 4 plus two field corners
    pick = []
    for beam, (n0, m0) in ((0, (13, 13)), (4, (10, 17))):
        pick += [beam * 900 + (n0 + a) * 30 + (m0 + b) for a in range(2) for b in range(4)]
    pick += [2 * 900 + 0, 7 * 900 + 899]
    pick = np.array(pick)
    say(f"c3 adjoint: oracle for {pick.size} beamlets")
    orc = abi_oracle(plan)
    g_o, amb = orc.adjoint(w, pick)
    scale = np.max(np.abs(g_o))
    amb_stats(amb, scale, "c3 adjoint")
    err = np.abs(g[pick] - g_o)
    assert np.all(err <= REL_TOL * scale), (err / scale).max()
    say(f"c3 adjoint: max |err|/max g = {(err / scale).max():.2e}")

    # quadratic objective: central differences of the GPU forward against the
    # adjoint of w' = 2 w (D - D0).  D is linear in f (Eq. 1), so L is exactly
    # quadratic and the central difference has no truncation error at any
    # step; what remains is the FP32 rounding of the two doses, which grows
    # as 1/h.  Steps 0.05 and 1e-3 (fluences are about 1); the difference of
    # L is summed in FP64 from the FP32 doses.  The bound adds to 2e-3 of the
    # gradient the rounding term: 4 ulp of each voxel's dose in D(f + h) and
    # D(f - h), weighted by |w (D+ + D- - 2 D0)| and summed in absolute value,
    # over 2 h.
    f = torch.as_tensor(plan.fluence, device="cuda")
    D = geo.forward(f).reshape(-1)
    D0 = torch.as_tensor(u, device="cuda") * D.max()
    wq = (2.0 * wt * (D - D0)).contiguous()
    gq = geo.adjoint(wq).double()
    rng = np.random.default_rng(5)
    pick_fd = rng.choice(nb, size=16, replace=False)
    worst = {}
    for h in (0.05, 1e-3):
        for i in pick_fd:
            fp, fm = f.clone(), f.clone()
            fp[i] += h
            fm[i] -= h
            hh = (fp[i].double() - fm[i].double()) / 2
            Dp, Dm = geo.forward(fp).reshape(-1).double(), geo.forward(fm).reshape(-1).double()
            c = wt.double() * (Dp + Dm - 2 * D0.double())
            dL = torch.sum(c * (Dp - Dm))
            fd = float(dL / (2 * hh))
            rounding = float(torch.sum(c.abs() * 4 * 2.0 ** -24 * (Dp.abs() + Dm.abs())) / (2 * hh))
            g_i = float(gq[i])
            tol = 2e-3 * max(abs(g_i), 1e-3 * float(gq.abs().max())) + rounding
            assert abs(fd - g_i) <= tol, (h, int(i), fd, g_i, rounding)
            worst[h] = max(worst.get(h, 0.0), abs(fd - g_i) / max(abs(g_i), 1e-30))
    say(f"c3 finite differences: max relative deviation {worst}")


def test_c2_adjoint_sampled(oracle_mod):
    """The adjoint over every beamlet of config 2 (the launch bench.py
    times), against the oracle at sampled beamlets: random ones and those
    with the largest gradients."""
    from bench import C2_TILE
    plan = S.plan_c2()
    geo = geometry(plan, 1, tile=C2_TILE)
    w = np.random.default_rng(13).uniform(0, 1, plan.n_vox).astype(np.float32)
    g = geo.adjoint(torch.as_tensor(w, device="cuda")).cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(g)) and g.min() >= 0.0
    rng = np.random.default_rng(14)
    pick = np.unique(np.concatenate([rng.choice(plan.n_beamlets, 16, replace=False),
                                     np.argsort(g)[-4:]]))
    say(f"c2 adjoint: oracle for {pick.size} beamlets")
    g_o, amb = abi_oracle(plan).adjoint(w, pick)
    scale = np.max(np.abs(g_o))
    amb_stats(amb, scale, "c2 adjoint")
    err = np.abs(g[pick] - g_o)
    assert np.all(err <= REL_TOL * scale), (err / scale).max()
    say(f"c2 adjoint: max |err|/max g = {(err / scale).max():.2e}")
    geo.close()


# ---------------------------------------------------------------------------
# Adjoint on a small plan: every beamlet against the oracle, dot-product test
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dc", [1, 0])
def test_adjoint_full_small(oracle_mod, dc):
    plan = _ragged_plans()[1]
    rng = np.random.default_rng(3)
    w = rng.uniform(0, 1, plan.n_vox).astype(np.float32)
    orc = abi_oracle(plan, dc_enabled=dc)
    g_o, amb = orc.adjoint(w)
    geo = geometry(plan, dc)
    g = geo.adjoint(torch.as_tensor(w, device="cuda")).cpu().numpy()
    amb_stats(amb, np.abs(g_o).max(), f"adjoint small dc={dc}")
    assert np.all(np.abs(g - g_o) <= REL_TOL * np.abs(g_o).max())
    # <D f, w> = <f, D^T w> on the GPU
    f = rng.uniform(0, 1, plan.n_beamlets).astype(np.float32)
    D = gpu_dose(geo, f).reshape(-1)
    lhs = float(D @ w.astype(np.float64))
    rhs = float(f.astype(np.float64) @ g.astype(np.float64))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_adjoint_long_rows_span_several_windows(oracle_mod):
    """A beam along the x rows of a long grid: the 512 rows of a chunk hold
    about 150,000 voxels, more than one window of the adjoint's block table
    (16,384), so several windows per chunk are walked."""
    n = (300, 40, 13)
    rng = np.random.default_rng(21)
    rho = rng.uniform(0.6, 1.4, size=(n[2], n[1], n[0])).astype(np.float32)
    rho[:, :, :4] = 0.001
    rho[:, :, -4:] = 0.001
    beams = [S.Beam(gantry=math.pi / 2, nbx=4, nby=3, wx=0.5, wy=0.5),
             S.Beam(gantry=-math.pi / 2 + 0.05, nbx=3, nby=3, wx=0.5, wy=0.5)]
    plan = S.plan_small(n=n, density=rho, beams=beams, seed=21, name="long_rows")
    w = rng.uniform(0, 1, plan.n_vox).astype(np.float32)
    orc = abi_oracle(plan)
    g_o, amb = orc.adjoint(w)
    geo = geometry(plan, 1)
    g = geo.adjoint(torch.as_tensor(w, device="cuda")).cpu().numpy().astype(np.float64)
    say(f"long rows adjoint: max |err|/max g = {np.abs(g - g_o).max() / np.abs(g_o).max():.2e}")
    bpc = geo.beamlet_pair_counts().cpu().numpy().astype(np.int64)
    assert np.array_equal(bpc, orc.beamlet_pair_counts())
    amb_stats(amb, np.abs(g_o).max(), "long rows adjoint")
    assert np.all(np.abs(g - g_o) <= REL_TOL * np.abs(g_o).max())
    geo.close()


def test_adjoint_slab_thickness(oracle_mod):
    """The adjoint's unit thickness (grid planes per slab) changes only the
    order of its partial sums: every thickness from one plane to the whole
    grid matches the oracle, counts stay exact, a thickness is
    deterministic, and the autotuner keeps one of those it timed."""
    plan = _ragged_plans()[1]              # nz = 17
    nz = plan.shape[0]
    w = np.random.default_rng(6).uniform(0, 1, plan.n_vox).astype(np.float32)
    orc = abi_oracle(plan)
    g_o, amb = orc.adjoint(w)
    cnt_o = orc.beamlet_pair_counts()
    scale = np.abs(g_o).max()
    geo = geometry(plan, 1)
    wt = torch.as_tensor(w, device="cuda")
    default = geo.get_adjoint_slab()
    assert 1 <= default <= nz
    for planes in (1, 2, 5, nz):
        geo.set_adjoint_slab(planes)
        assert geo.get_adjoint_slab() == planes
        g1 = geo.adjoint(wt).clone()
        assert torch.equal(geo.adjoint(wt), g1)
        assert np.all(np.abs(g1.cpu().numpy() - g_o) <= REL_TOL * scale), planes
        assert np.array_equal(geo.beamlet_pair_counts().cpu().numpy(), cnt_o), planes
    geo.set_adjoint_slab(0)
    assert geo.get_adjoint_slab() == default
    for bad in (-1, nz + 1):
        with pytest.raises(RuntimeError):
            geo.set_adjoint_slab(bad)
    res = geo.autotune_adjoint(wt, reps=2)
    assert len(res) >= 2 and all(r["ms"] > 0 for r in res)
    best = min(res, key=lambda r: r["ms"])
    assert geo.get_adjoint_slab() == best["planes"]
    geo.close()


def test_autograd_function():
    from paper_1103_1164_amd import FspbDose
    plan = _ragged_plans()[0]
    geo = geometry(plan, 1)
    f = torch.as_tensor(plan.fluence, device="cuda").requires_grad_(True)
    D = FspbDose.apply(f, geo)
    w = torch.rand(D.shape, device="cuda")
    loss = (w * D).sum()
    loss.backward()
    g = geo.adjoint(w.reshape(-1))
    assert torch.equal(f.grad, g)


# ---------------------------------------------------------------------------
# Invariants through the GPU path
# ---------------------------------------------------------------------------
def test_gpu_invariants():
    plan = _ragged_plans()[0]
    geo = geometry(plan, 1)
    rng = np.random.default_rng(8)
    f = np.round(rng.uniform(0, 1, plan.n_beamlets) * 1024) / 1024
    g = np.round(rng.uniform(0, 1, plan.n_beamlets) * 1024) / 1024
    Df, Dg, Dfg = gpu_dose(geo, f), gpu_dose(geo, g), gpu_dose(geo, 2 * f + 0.5 * g)
    assert np.max(np.abs(Dfg - (2 * Df + 0.5 * Dg))) < 2e-6 * Dfg.max()
    # DC reduces to plain in water
    water = S.plan_small(n=(27, 21, 15), density=1.0, seed=4,
                         beams=[S.Beam(gantry=0.5, nbx=5, nby=4), S.Beam(gantry=3.0, nbx=3, nby=3)])
    a = gpu_dose(geometry(water, 1), water.fluence)
    b = gpu_dose(geometry(water, 0), water.fluence)
    assert np.max(np.abs(a - b)) < 1e-6 * a.max()
    # a DC handle switched to plain equals a plain handle
    geo_w = geometry(water, 1)
    geo_w.set_dc(False)
    assert np.array_equal(gpu_dose(geo_w, water.fluence), b)
    # inverse square along the central axis
    tabs = S.constant_tables(A=1.0, u1=3.0, u2=1.2, w1=0.75, w2=0.25)
    ax = S.plan_small(n=(9, 41, 9), density=1.0, tables=tabs, fluence=np.ones(1),
                      beams=[S.Beam(gantry=0.0, nbx=1, nby=1)])
    d = gpu_dose(geometry(ax, 1), ax.fluence)
    y = ax.origin[1] + 0.25 * np.arange(41)
    v = d[4, :, 4] * (y + 100.0) ** 2
    assert np.max(np.abs(v / v.mean() - 1)) < 2e-6


def test_determinism():
    plan = S.plan_c2()
    geo = geometry(plan, 1)
    f = torch.as_tensor(plan.fluence, device="cuda")
    a, b = geo.forward(f).clone(), geo.forward(f).clone()
    assert torch.equal(a, b)
    w = torch.rand(plan.n_vox, device="cuda")
    assert torch.equal(geo.adjoint(w).clone(), geo.adjoint(w).clone())


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------
def test_edge_cases(oracle_mod):
    # zero fluence: every voxel written with zero
    plan = _ragged_plans()[0]
    geo = geometry(plan, 1)
    out = torch.full(plan.shape, 7.0, device="cuda")
    geo.forward(torch.zeros(plan.n_beamlets, device="cuda"), out=out)
    assert torch.count_nonzero(out) == 0
    # a beamlet that misses the grid contributes nothing, others are unaffected
    beams = [S.Beam(gantry=0.0, nbx=2, nby=1, wx=0.5, cx=0.0), S.Beam(gantry=0.0, nbx=1, nby=1, cx=60.0)]
    p = S.plan_small(n=(12, 10, 6), density=1.0, beams=beams, fluence=np.ones(3), seed=0)
    g = geometry(p, 1)
    assert g.info()["n_hit"] == 2 and not g.beamlet(2)["hit"]
    d_o, amb, _ = abi_oracle(p).dose()
    assert_dose_parity(gpu_dose(g, p.fluence), d_o, amb, what="miss")
    # body entirely below the surface threshold: nothing enters
    p2 = S.plan_small(n=(8, 8, 8), density=0.2, seed=0)
    g2 = geometry(p2, 1)
    assert g2.info()["n_hit"] == 0
    assert gpu_dose(g2, p2.fluence).max() == 0.0
    # 1x1x1 grid
    p3 = S.plan_small(n=(1, 1, 1), density=1.0, beams=[S.Beam(gantry=0.7, nbx=2, nby=2)], seed=0)
    d_o, amb, _ = abi_oracle(p3).dose()
    g3 = geometry(p3, 1)
    assert_dose_parity(gpu_dose(g3, p3.fluence), d_o, amb, what="1x1x1")
    # the adjoint on the same cases: the missing beamlet gets zero, nothing
    # entering gives a zero gradient, the single voxel matches the oracle
    for plan_, geo_, what in ((p, g, "miss"), (p2, g2, "no entry"), (p3, g3, "1x1x1")):
        w = np.random.default_rng(2).uniform(0.5, 1.0, plan_.n_vox).astype(np.float32)
        grad = geo_.adjoint(torch.as_tensor(w, device="cuda")).cpu().numpy().astype(np.float64)
        g_o, amb_g = abi_oracle(plan_).adjoint(w)
        assert not amb_g.any(), what
        assert np.all(np.abs(grad - g_o) <= REL_TOL * max(np.abs(g_o).max(), 1e-30)), what
    assert geometry(p, 1).adjoint(torch.ones(p.n_vox, device="cuda"))[2].item() == 0.0
    assert torch.count_nonzero(g2.adjoint(torch.ones(p2.n_vox, device="cuda"))) == 0


def test_errors_on_gpu():
    from paper_1103_1164_amd import FspbError
    import os
    plan = _ragged_plans()[2]
    geo = geometry(plan, 0)
    with pytest.raises(FspbError):
        geo.set_dc(True)             # created without density correction
    with pytest.raises(FspbError):
        geo.smoothed_density()
    with pytest.raises(ValueError):
        geo.forward(torch.ones(plan.n_beamlets + 1, device="cuda"))
    # injected device allocation failure: clean error, no handle
    os.environ["FSPB_TEST_FAIL_ALLOC"] = "3"
    try:
        with pytest.raises(FspbError) as e:
            geometry(plan, 1)
        assert e.value.code == -3
    finally:
        del os.environ["FSPB_TEST_FAIL_ALLOC"]
    assert geometry(plan, 1).info()["n_hit"] == 1


def test_paper_h5_adjoint_sampled(oracle_mod):
    """The transpose on the paper-shaped head-and-neck plan, on sampled
    beamlets of every beam."""
    plan = S.plan_paper_h5()
    geo = geometry(plan, 1)
    rng = np.random.default_rng(8)
    w = rng.uniform(0.0, 1.0, size=plan.n_vox).astype(np.float32)
    g = geo.adjoint(torch.as_tensor(w, device="cuda")).cpu().numpy().astype(np.float64)
    per = plan.beams[0].n_beamlets
    pick = np.concatenate([b * per + rng.choice(per, size=2, replace=False)
                           for b in range(len(plan.beams))])
    say(f"paper_h5 adjoint: oracle on {pick.size} beamlets")
    g_o, amb = abi_oracle(plan).adjoint(w, beamlets=pick)
    assert_dose_parity(g[pick], g_o, amb, scale=np.abs(g_o).max(), what="paper_h5 adjoint")
