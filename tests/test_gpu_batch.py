"""Batched persistent launch, HIP-graph replay, density updates and tile
configurations (run on an MI355X).

Every voxel sums its pairs in the same order whatever the schedule, the
launch path or the number of waves per workgroup, and a wave evaluates the
same pairs for a given brick shape, so these tests demand bitwise equality
with the single-plan forward of the same brick shape (test_gpu_parity.py
checks that against the oracle).  Across brick shapes a pair may be
evaluated by a different one of the two exact forms of its Eq. 4 profile
product (the form is chosen per wave), so doses agree to rounding: within
SHAPE_TOL of the maximum dose."""
import json

import numpy as np
import pytest
import torch

import fspb_synth as S
from gpu_helpers import abi_oracle, assert_dose_parity, geometry, gpu_dose, say

pytestmark = pytest.mark.gpu

SHAPE_TOL = 2e-6    # relative to max dose: a few FP32 ulps per pair, summed


def _plans():
    rng = np.random.default_rng(40)
    out = []
    for k, (n, gantries) in enumerate([((23, 19, 13), (0.3, 3.9)), ((30, 17, 22), (1.1,)),
                                      ((9, 41, 7), (0.0, 2.0, 4.0)), ((36, 36, 20), (5.5, 0.8))]):
        rho = rng.uniform(0.05, 2.2, size=(n[2], n[1], n[0])).astype(np.float32)
        beams = [S.Beam(gantry=g, nbx=3 + k, nby=4, wx=0.5, wy=0.4 + 0.1 * k) for g in gantries]
        out.append(S.plan_small(n=n, density=rho, beams=beams, seed=k, name=f"b{k}"))
    return out


@pytest.mark.parametrize("dc", [1, 0])
def test_tile_configurations_agree(dc):
    from paper_1103_1164_amd import Geometry
    plan = _plans()[3]
    geo = geometry(plan, dc)
    ref = gpu_dose(geo, plan.fluence)
    shapes = Geometry.tile_shapes()
    assert len(shapes) >= 2 and all(int(np.prod(s)) == 64 for s in shapes)
    scale = float(np.max(np.abs(ref)))
    for sh in range(len(shapes)):
        first = None
        for wpb in (1, 2, 4, 8):          # 8: water table staged in LDS
            geo.set_tile(sh, wpb)
            assert geo.get_tile() == (sh, wpb)
            d = gpu_dose(geo, plan.fluence)
            if first is None:
                first = d
            assert np.array_equal(d, first), (sh, wpb)       # same shape: bitwise
            assert np.max(np.abs(d - ref)) <= SHAPE_TOL * scale, (sh, wpb)
            n = geo.count_pairs(torch.as_tensor(plan.fluence, device="cuda"))
            if sh == 0 and wpb == 1:
                n0 = n
            assert n == n0


@pytest.mark.parametrize("dc", [1, 0])
def test_batch_equals_single_plan(dc):
    from paper_1103_1164_amd import Batch
    plans = _plans()
    geos = [geometry(p, dc) for p in plans]
    fl = [torch.as_tensor(p.fluence, device="cuda") for p in plans]
    for shape, wpb, wpc, pol in ((0, 4, 32, "throughput"), (1, 2, 8, "latency"),
                                 (0, 1, 1, "throughput"), (2, 4, 16, "latency"),
                                 (0, 8, 32, "latency"), (3, 8, 8, "throughput")):
        refs = []                          # single-plan forwards with the batch's shape
        for g, p in zip(geos, plans):
            g.set_tile(shape, 4)
            refs.append(gpu_dose(g, p.fluence))
        b = Batch(geos, shape=shape, waves_per_block=wpb, waves_per_cu=wpc, policy=pol)
        out = [torch.full(p.shape, -1.0, device="cuda") for p in plans]
        b.forward(fl, out)
        torch.cuda.synchronize()
        for o, r in zip(out, refs):
            assert np.array_equal(o.cpu().numpy().astype(np.float64), r), (shape, wpb, wpc, pol)
        ms, total = b.latencies()
        assert total > 0 and all(0 < m <= total + 1e-9 for m in ms)
        sx, sy, sz = geos[0].tile_shapes()[shape]
        n_bricks = sum(-(-p.shape[2] // sx) * -(-p.shape[1] // sy) * -(-p.shape[0] // sz)
                       for p in plans)
        assert b.info()["n_items"] == n_bricks
        b.close()


def _fine_water_tables():
    """The nominal tables with the water (depth) tables resampled every 0.04
    cm: 2001 samples, 96 KB as the kernels hold them, more than the 64 KB
    the forward stages in LDS."""
    import dataclasses
    tab = S.make_tables(0)
    t_new = 0.04 * np.arange(2001)
    def fine(tb):
        t_old = tb.start + tb.step * np.arange(tb.n)
        return S.Table1D(0.0, 0.04, np.interp(t_new, t_old, tb.values).astype(np.float32))
    return dataclasses.replace(tab, **{k: fine(getattr(tab, k))
                                       for k in ("u1x", "u1y", "u2x", "u2y", "w1", "w2")})


@pytest.mark.parametrize("dc", [1, 0])
def test_water_table_too_large_for_lds(oracle_mod, dc):
    """8 waves per workgroup with a water table over 64 KB reads it from
    global memory (4 waves): same dose as the other configurations, and the
    oracle's.  A batch of plans with different tables has no shared table to
    stage and takes the same path."""
    from paper_1103_1164_amd import Batch
    p0 = _plans()[0]
    plan = S.plan_small(n=p0.shape[::-1], density=p0.density, beams=p0.beams,
                        fluence=p0.fluence, tables=_fine_water_tables(), seed=9)
    geo = geometry(plan, dc)
    geo.set_tile(0, 8)
    d8 = gpu_dose(geo, plan.fluence)
    geo.set_tile(0, 4)
    assert np.array_equal(gpu_dose(geo, plan.fluence), d8)
    orc = abi_oracle(plan, dc_enabled=dc)
    d_o, amb, _ = orc.dose()
    assert_dose_parity(d8, d_o, amb, what="fine water tables")
    # the adjoint's global-memory path (4-wave workgroups) on the same tables
    w = np.random.default_rng(3).uniform(0.0, 1.0, plan.n_vox).astype(np.float32)
    g = geo.adjoint(torch.as_tensor(w, device="cuda")).cpu().numpy().astype(np.float64)
    g_o, g_amb = orc.adjoint(w)
    scale = float(np.max(np.abs(g_o)))
    assert np.all(np.abs(g - g_o) <= 1e-4 * scale + g_amb), float(np.max(np.abs(g - g_o)) / scale)
    other = _plans()[1]
    g1 = geometry(other, dc)
    ref1 = gpu_dose(g1, other.fluence)
    b = Batch([geo, g1], shape=0, waves_per_block=8, policy="latency")
    fl = [torch.as_tensor(p.fluence, device="cuda") for p in (plan, other)]
    out = [torch.full(p.shape, -1.0, device="cuda") for p in (plan, other)]
    b.forward(fl, out)
    torch.cuda.synchronize()
    assert np.array_equal(out[0].cpu().numpy().astype(np.float64), d8)
    assert np.array_equal(out[1].cpu().numpy().astype(np.float64), ref1)
    b.close()


def test_update_density_matches_fresh_geometry():
    plans = _plans()
    p0 = plans[0]
    rng = np.random.default_rng(7)
    rho2 = rng.uniform(0.05, 2.2, size=p0.density.shape).astype(np.float32)
    p1 = S.plan_small(n=p0.shape[::-1], density=rho2, beams=p0.beams, fluence=p0.fluence)
    geo = geometry(p0, 1)
    d2 = torch.as_tensor(rho2, device="cuda")
    geo.update_density(d2)
    fresh = geometry(p1, 1)
    assert np.array_equal(gpu_dose(geo, p0.fluence), gpu_dose(fresh, p0.fluence))
    assert torch.equal(geo.smoothed_density(), fresh.smoothed_density())
    for i in range(0, p0.n_beamlets, 3):
        a, b = geo.beamlet(i), fresh.beamlet(i)
        assert a["k_entry"] == b["k_entry"] and np.array_equal(a["T"], b["T"])


def test_graph_replay_with_density_updates():
    from paper_1103_1164_amd import Batch
    plans = _plans()
    geos = [geometry(p, 1) for p in plans]
    rng = np.random.default_rng(11)
    dens = [torch.as_tensor(rng.uniform(0.05, 2.2, size=p.density.shape).astype(np.float32),
                            device="cuda") for p in plans]
    fl = [torch.as_tensor(p.fluence, device="cuda") for p in plans]
    out = [torch.zeros(p.shape, device="cuda") for p in plans]
    # reference: fresh geometries on the new densities
    refs = []
    for p, d in zip(plans, dens):
        q = S.plan_small(n=p.shape[::-1], density=d.cpu().numpy(), beams=p.beams,
                         fluence=p.fluence)
        refs.append(gpu_dose(geometry(q, 1), p.fluence))
    b = Batch(geos)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.capture(fl, out, densities=dens, stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        for o in out:
            o.fill_(-5.0)                      # eager work between replays
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.replay(stream=s)
        s.synchronize()
        for o, r in zip(out, refs):
            assert np.array_equal(o.cpu().numpy().astype(np.float64), r), rep
        ms, total = b.latencies(stream=s)
        assert total > 0


def test_autotune_and_cache(tmp_path):
    from paper_1103_1164_amd.autotune import tune
    plan = _plans()[3]
    geo = geometry(plan, 1)
    ref = gpu_dose(geo, plan.fluence)
    f = torch.as_tensor(plan.fluence, device="cuda")
    cache = tmp_path / "tune.json"
    r1 = tune(geo, f, cache=cache, reps=2)
    # two schedules x shapes x four workgroup sizes
    assert not r1["cached"] and len(r1["all"]) == 2 * 4 * len(geo.tile_shapes())
    assert {r["per_beam"] for r in r1["all"]} == {0, 1}
    assert geo.get_tile() == (r1["shape"], r1["waves_per_block"])
    assert geo.get_schedule() == r1["per_beam"]
    got = gpu_dose(geo, plan.fluence)
    assert np.max(np.abs(got - ref)) <= SHAPE_TOL * float(np.max(np.abs(ref)))
    geo2 = geometry(plan, 1)
    r2 = tune(geo2, f, cache=cache)
    assert r2["cached"] and geo2.get_tile() == geo.get_tile()
    assert geo2.get_schedule() == geo.get_schedule()
    assert r1["key"] in json.loads(cache.read_text())


def test_c4_batch_full_size(oracle_mod):
    """Four config-4 plans (the smallest and largest grids and two in
    between) in one persistent launch: equal to the single-plan forwards and
    to the oracle on sampled voxels."""
    from paper_1103_1164_amd import Batch
    idx = [0, 1, 2, 31]
    plans = S.plans_c4(idx)
    say("c4: geometries")
    geos = [geometry(p, 1) for p in plans]
    fl = [torch.as_tensor(p.fluence, device="cuda") for p in plans]
    out = [torch.empty(p.shape, device="cuda") for p in plans]
    b = Batch(geos)
    b.forward(fl, out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for k, (p, g, o) in enumerate(zip(plans, geos, out)):
        single = gpu_dose(g, p.fluence)
        got = o.cpu().numpy().astype(np.float64)
        assert np.array_equal(got, single), p.name
        if k in (0, 3):
            vox = rng.choice(p.n_vox, size=1500, replace=False)
            hot = np.argsort(got.reshape(-1))[-300:]
            vox = np.unique(np.concatenate([vox, hot]))
            say(f"c4: oracle {p.name} at {vox.size} voxels")
            d_o, amb, _ = abi_oracle(p).dose(vox=vox)
            assert_dose_parity(got.reshape(-1)[vox], d_o, amb, what=p.name)
