"""The forward's pipelined candidate loop against the plain one, on the
head-and-neck plan of config 2.

Workgroups of 8 waves keep the water table in LDS and run the candidate
loop that reads the next candidate's depth record while the current pair is
evaluated; workgroups of 4 waves read the water table from global memory
and run the plain loop.  Both evaluate the same pairs of a brick in the same
order with the same arithmetic, so for one brick shape their doses agree bit
for bit: the density-corrected forward, conventional FSPB, and the
surrogate's forward on rows of which the network serves some and the
corrected pair the rest."""
import pytest
import torch

import fspb_synth as S
from gpu_helpers import geometry, say

pytestmark = pytest.mark.gpu


def test_pipelined_loop_bitwise_on_head_plan():
    from paper_1103_1164_amd import Mlp
    plan = S.plan_c2()
    geo = geometry(plan, 1)
    f = torch.as_tensor(plan.fluence, device="cuda")
    mlp = Mlp.initial(0)
    mlp.set_guard(het_max=0.01)
    prm = geo.surrogate_infer(mlp)
    own = float((prm[..., 6] == 0).float().mean())
    say(f"pipeline: rows served by the network {own:.3f}")
    assert 0.0 < own < 1.0
    for shape in (0, 3):
        out = {}
        for waves in (8, 4):
            geo.set_tile(shape, waves)
            for dc in (True, False):
                geo.set_dc(dc)
                out[waves, dc] = geo.forward(f).clone()
            geo.set_dc(True)
            out[waves, "surrogate"] = geo.forward_surrogate(f, prm).clone()
        for what in (True, False, "surrogate"):
            assert torch.equal(out[8, what], out[4, what]), (shape, what)
            assert float(out[8, what].max()) > 0.0, (shape, what)
        say(f"pipeline: brick shape {shape} bitwise")
    geo.close()
