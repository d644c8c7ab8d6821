"""The per-beam forward schedule (fspb_set_schedule): for a given brick shape
its dose is bitwise that of the brick-major schedule, on small ragged plans
(every shape and workgroup size) and on config 2; against the oracle through
the per-beam path; and the schedule follows set_tile, update_density and a
plan too large for LDS-staged water tables.  With 8-wave workgroups the
per-beam kernel is persistent (per-XCD item counters); idle XCDs and
repeated launches are covered too."""
import numpy as np
import pytest
import torch

import fspb_synth as S
from gpu_helpers import abi_oracle, assert_dose_parity, geometry, say

pytestmark = pytest.mark.gpu


def _small():
    rng = np.random.default_rng(41)
    n = (29, 23, 17)
    rho = rng.uniform(0.05, 2.2, size=(n[2], n[1], n[0])).astype(np.float32)
    return S.plan_small(n=n, density=rho, seed=5, name="sched_small", beams=[
        S.Beam(gantry=0.4, nbx=6, nby=4, wx=0.4, wy=0.6, cx=0.1),
        S.Beam(gantry=2.2, couch=0.3, nbx=5, nby=5),
        S.Beam(gantry=4.4, nbx=3, nby=7, wx=0.6, wy=0.3)])


@pytest.mark.parametrize("dc", [1, 0])
def test_per_beam_bitwise_equal_every_tile(dc):
    plan = _small()
    geo = geometry(plan, dc)
    f = torch.as_tensor(plan.fluence, device="cuda")
    for shape in range(4):
        for wpb in (1, 2, 4, 8):
            geo.set_schedule(0)
            geo.set_tile(shape, wpb)
            ref = geo.forward(f).clone()
            geo.set_schedule(1)
            got = geo.forward(f).clone()
            assert geo.get_schedule() == 1
            assert torch.equal(ref, got), (shape, wpb, float((ref - got).abs().max()))
    geo.close()


def test_per_beam_oracle_parity_and_update():
    plan = _small()
    geo = geometry(plan, 1, schedule=1)
    assert geo.get_schedule() == 1
    d = geo.forward(torch.as_tensor(plan.fluence, device="cuda")).cpu().numpy()
    d_o, amb, _ = abi_oracle(plan).dose()
    rel = assert_dose_parity(d, d_o, amb, what="per-beam schedule")
    say(f"per-beam schedule: max |err|/max D = {rel:.2e}")
    # a new density through update_density: the schedule (geometry only) is kept
    rho2 = np.clip(plan.density * 0.9 + 0.05, 0.0, None).astype(np.float32)
    geo.update_density(torch.as_tensor(rho2, device="cuda"))
    d2 = geo.forward(torch.as_tensor(plan.fluence, device="cuda")).cpu().numpy()
    plan2 = S.plan_small(n=(29, 23, 17), density=rho2, seed=5, beams=plan.beams)
    d2_o, amb2, _ = abi_oracle(plan2).dose()
    assert_dose_parity(d2, d2_o, amb2, what="per-beam schedule after update_density")
    geo.close()


def test_per_beam_persistent_idle_xcds_and_repeats():
    """The 8-wave per-beam kernel takes its items from per-XCD counters:
    with a single brick and beam most XCDs get no item, and the counters are
    cleared before every launch, so repeated forwards agree bitwise."""
    rng = np.random.default_rng(3)
    for n, beams in (((4, 4, 4), [S.Beam(gantry=0.9, nbx=2, nby=2)]),
                     ((9, 7, 5), [S.Beam(gantry=0.3, nbx=3, nby=2), S.Beam(gantry=3.5, nbx=2, nby=2)])):
        rho = rng.uniform(0.5, 1.5, size=(n[2], n[1], n[0])).astype(np.float32)
        plan = S.plan_small(n=n, density=rho, seed=9, beams=beams, name="tiny")
        geo = geometry(plan, 1)
        f = torch.as_tensor(plan.fluence, device="cuda")
        geo.set_tile(0, 8)
        ref = geo.forward(f).clone()
        geo.set_schedule(1)
        for _ in range(3):
            assert torch.equal(geo.forward(f), ref), n
        d_o, amb, _ = abi_oracle(plan).dose()
        assert_dose_parity(ref.cpu().numpy(), d_o, amb, what=f"tiny plan {n}")
        geo.close()


def test_per_beam_config2_bitwise():
    from bench import C2_TILE
    plan = S.plan_c2()
    f = torch.as_tensor(plan.fluence, device="cuda")
    geo = geometry(plan, 1, tile=C2_TILE)
    ref = geo.forward(f).clone()
    geo.set_schedule(1)
    got = geo.forward(f).clone()
    assert torch.equal(ref, got)
    assert torch.equal(geo.forward(f), ref)          # again: the counters start from zero
    # the plain model too
    geo.set_dc(False)
    got_p = geo.forward(f).clone()
    geo.set_schedule(0)
    assert torch.equal(geo.forward(f), got_p)
    geo.close()


def test_per_beam_water_table_in_global_memory():
    """Water tables too long for LDS (1,600 samples): both schedules read
    them from global memory and agree bitwise."""
    plan = _small()
    t = plan.tables
    n = 1600
    for name in ("u1x", "u1y", "u2x", "u2y", "w1", "w2"):
        tb = getattr(t, name)
        x = np.linspace(0, 80, n)
        v = np.interp(x, tb.start + tb.step * np.arange(tb.n), tb.values).astype(np.float32)
        setattr(t, name, S.Table1D(0.0, 80.0 / (n - 1), v))
    geo = geometry(plan, 1)
    f = torch.as_tensor(plan.fluence, device="cuda")
    ref = geo.forward(f).clone()
    geo.set_schedule(1)
    assert torch.equal(geo.forward(f), ref)
    geo.close()
