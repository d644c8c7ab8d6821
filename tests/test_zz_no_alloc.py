"""fspb_count_pairs_noalloc (the pair count with no allocation, its scratch a
static device array) against fspb_count_pairs, through the C interface, on
two calls in a row: a config 2 plan, then a smaller one, so the second call
finds the first call's counts in the shared array."""
import numpy as np
import pytest
import torch

import fspb_synth as S
from gpu_helpers import geometry, say

pytestmark = pytest.mark.gpu


def _counts(geo, plan, stream=None):
    f = torch.as_tensor(plan.fluence, device="cuda")
    ref_f = geo.count_pairs(f)
    ref_all = geo.count_pairs(None)
    got_f = geo.count_pairs_noalloc(f, stream=stream)
    got_all = geo.count_pairs_noalloc(None, stream=stream)
    torch.cuda.synchronize()
    return ref_f, int(got_f.item()), ref_all, int(got_all.item())


def test_count_pairs_noalloc_matches_count_pairs():
    big = S.plan_c2()
    rng = np.random.default_rng(3)
    n = (23, 19, 13)
    rho = rng.uniform(0.05, 2.3, size=(n[2], n[1], n[0])).astype(np.float32)
    small = S.plan_small(n=n, density=rho, seed=1, name="small", beams=[
        S.Beam(gantry=0.3, nbx=5, nby=3, wx=0.4, wy=0.6), S.Beam(gantry=3.9, nbx=4, nby=4)])
    for plan, tile in ((big, (3, 8)), (small, None)):
        say(f"noalloc count: {plan.name}, {plan.n_vox} voxels")
        geo = geometry(plan, 1, tile=tile)
        ref_f, got_f, ref_all, got_all = _counts(geo, plan)
        say(f"  {plan.name}: fluence {got_f} (ref {ref_f}), all beamlets {got_all} (ref {ref_all})")
        assert got_f == ref_f and got_all == ref_all
        assert ref_f > 0 and ref_all >= ref_f
        geo.close()


def test_count_pairs_noalloc_on_a_stream_and_other_tiles():
    """On a side stream (ordered after the geometry's creation), with each
    brick shape of the library: the scratch holds one count per brick of
    the handle's own shape."""
    plan = S.plan_c1()
    geo = geometry(plan, 1)
    f = torch.as_tensor(plan.fluence, device="cuda")
    ref = geo.count_pairs(f)
    s = torch.cuda.Stream()
    for shape in range(4):
        geo.set_tile(shape, 8)
        out = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        s.wait_stream(torch.cuda.current_stream())     # f, out and the new schedule
        with torch.cuda.stream(s):
            geo.count_pairs_noalloc(f, out=out, stream=s)
        s.synchronize()
        assert int(out.item()) == ref, shape
    geo.close()
