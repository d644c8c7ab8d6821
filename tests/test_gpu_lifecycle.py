"""Plan creation and release do not wait for the device: creation returns
once the handle has its own copy of the CT (the geometry kernels may still
run), and a released handle's buffers rejoin the library's pool only after
its queued work is done.  These tests use handles in the ways that ordering
must survive -- another stream right after creation, host reads right after
creation, the caller overwriting its CT at once, and a pipeline of plans
whose buffers are recycled while earlier work is in flight -- and demand
bitwise equality with references computed with a synchronisation after each
step (test_gpu_parity.py ties those to the oracle)."""
import numpy as np
import pytest
import torch

import fspb_synth as S
from gpu_helpers import geometry, gpu_dose

pytestmark = pytest.mark.gpu


def _plans():
    rng = np.random.default_rng(90)
    out = []
    for k, (n, gantries) in enumerate([((26, 22, 18), (0.4, 2.6)), ((34, 30, 14), (1.3,)),
                                      ((18, 40, 24), (0.1, 3.3, 5.0))]):
        rho = rng.uniform(0.05, 2.0, size=(n[2], n[1], n[0])).astype(np.float32)
        beams = [S.Beam(gantry=g, nbx=4 + k, nby=3 + k, wx=0.5, wy=0.5) for g in gantries]
        out.append(S.plan_small(n=n, density=rho, beams=beams, seed=k, name=f"l{k}"))
    return out


def _make(plan, dens, dc, stream=None):
    from paper_1103_1164_amd import Geometry
    o = S.Options(dc_enabled=dc)
    return Geometry(dens, plan.spacing, plan.origin, plan.beams, plan.tables, o, stream=stream)


@pytest.mark.parametrize("dc", [1, 0])
def test_other_stream_and_overwritten_ct_right_after_create(dc):
    """Creation on stream s1; at once the caller overwrites its CT on stream
    s2 and runs the forward on s2: the handle reads its own copy, and the
    forward waits for the creation kernels."""
    plan = _plans()[0]
    ref = gpu_dose(geometry(plan, dc), plan.fluence)
    dens = torch.as_tensor(plan.density, device="cuda").clone()
    f = torch.as_tensor(plan.fluence, device="cuda")
    out = torch.full(plan.shape, -1.0, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    geo = _make(plan, dens, dc, stream=s1)
    with torch.cuda.stream(s2):
        dens.fill_(7.0)
    if dc:
        geo.wait_ready(s2)                 # explicit wait (the forward also orders itself)
    geo.forward(f, out=out, stream=s2)
    s2.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
    geo.close()
    torch.cuda.synchronize()


def test_host_reads_right_after_create():
    plan = _plans()[2]
    ref_geo = geometry(plan, 1)
    torch.cuda.synchronize()
    want = ref_geo.info()
    want_b = [ref_geo.beamlet(i) for i in range(0, plan.n_beamlets, 5)]
    dens = torch.as_tensor(plan.density, device="cuda")
    torch.cuda.synchronize()
    geo = _make(plan, dens, 1)
    got = geo.info()                       # host copies: must wait for the trace
    assert got["n_hit"] == want["n_hit"] and got["k_max"] == want["k_max"]
    for i, b in zip(range(0, plan.n_beamlets, 5), want_b):
        g = geo.beamlet(i)
        assert g["k_entry"] == b["k_entry"] and np.array_equal(g["T"], b["T"])
    geo.close()
    ref_geo.close()


def test_pipeline_of_plans_recycles_buffers_safely():
    """Create, forward and release plans of three sizes in a loop without
    synchronising: released buffers are handed to later plans only once the
    work that used them is done."""
    plans = _plans()
    refs = [gpu_dose(geometry(p, 1), p.fluence) for p in plans]
    dens = [torch.as_tensor(p.density, device="cuda") for p in plans]
    fl = [torch.as_tensor(p.fluence, device="cuda") for p in plans]
    torch.cuda.synchronize()
    outs = []
    for rep in range(5):
        for k, p in enumerate(plans):
            g = _make(p, dens[k], 1)
            o = torch.empty(p.shape, device="cuda")
            g.forward(fl[k], out=o)
            g.close()
            outs.append((k, o))
    torch.cuda.synchronize()
    for k, o in outs:
        assert np.array_equal(o.cpu().numpy().astype(np.float64), refs[k]), k


@pytest.mark.parametrize("shape,waves", [(3, 8), (1, 4), (2, 1), (0, 8)])
def test_tile_given_at_creation_matches_set_tile(shape, waves):
    """options.tile_shape / tile_waves build the forward schedule at
    creation: the same tile and bitwise the same dose as fspb_set_tile
    after a default creation."""
    from paper_1103_1164_amd import Geometry
    plan = _plans()[1]
    dens = torch.as_tensor(plan.density, device="cuda")
    f = torch.as_tensor(plan.fluence, device="cuda")
    o = S.Options(dc_enabled=1)
    a = Geometry(dens, plan.spacing, plan.origin, plan.beams, plan.tables, o, tile=(shape, waves))
    b = Geometry(dens, plan.spacing, plan.origin, plan.beams, plan.tables, o)
    b.set_tile(shape, waves)
    assert a.get_tile() == b.get_tile()
    assert torch.equal(a.forward(f), b.forward(f))
    a.close()
    b.close()


def test_zero_initialised_options_mean_plain_fspb():
    """A zero-initialised fspb_options (every field 0) takes the bracketed
    defaults for its float fields and dc_enabled = 0 (plain FSPB); NULL
    options take the same defaults with the density correction on.  Both
    match plans built with those defaults spelt out, bit for bit."""
    from paper_1103_1164_amd import Geometry

    class Zero:
        roi_radius = rho_surface = smooth_sigma = rho_min = rho_max = sample_step = 0.0
        dc_enabled = siddon = 0

    plan = S.plan_small(n=(19, 17, 13), density=1.0, seed=2,
                        beams=[S.Beam(gantry=0.7, nbx=3, nby=3, wx=0.5, wy=0.5)])
    dens = torch.as_tensor(plan.density, device="cuda")
    f = torch.as_tensor(plan.fluence, device="cuda")

    def make(options):
        return Geometry(dens, plan.spacing, plan.origin, plan.beams, plan.tables, options)

    g_zero, g_null = make(Zero()), make(None)
    assert g_zero.info()["dc_enabled"] == 0
    assert g_null.info()["dc_enabled"] == 1
    spelt = S.Options()                       # roi 5, surface 0.5, sigma 0.5, rho 0.1-2.0
    assert (spelt.roi_radius, spelt.rho_surface, spelt.smooth_sigma,
            spelt.rho_min, spelt.rho_max, spelt.sample_step) == (5.0, 0.5, 0.5, 0.1, 2.0, 0.0)
    spelt.dc_enabled = 0
    assert torch.equal(g_zero.forward(f), make(spelt).forward(f))
    spelt.dc_enabled = 1
    assert torch.equal(g_null.forward(f), make(spelt).forward(f))
    for g in (g_zero, g_null):
        g.close()
