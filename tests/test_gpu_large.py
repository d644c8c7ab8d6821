"""A plan of 2^28 voxels (512 x 512 x 1024 at 1 mm), the size from which the
learned surrogate's 32-bit offsets into its 16-byte CT records would
overflow: the density-corrected forward matches the oracle at sampled voxels
and the pair counts are exact there, and every surrogate entry point rejects
the plan with FSPB_E_ARG before it touches a buffer."""
import ctypes as C

import numpy as np
import pytest
import torch

import fspb_synth as S
from gpu_helpers import abi_oracle, assert_dose_parity, geometry, say

pytestmark = pytest.mark.gpu


def test_grid_of_2_pow_28_voxels(oracle_mod):
    from paper_1103_1164_amd import Mlp, _lib
    n, sp = (512, 512, 1024), (0.1, 0.1, 0.1)
    rho = np.ones((n[2], n[1], n[0]), dtype=np.float32)       # 1 GiB
    rho[:, 180:230, :] = 0.3                                  # a lung-like slab across the beam
    rho[:, 300:320, 200:330] = 1.7                            # and a bone-like block
    plan = S.plan_small(n=n, spacing=sp, density=rho, seed=3, name="large_2_28",
                        beams=[S.Beam(gantry=0.0, nbx=2, nby=2, wx=0.5, wy=0.5)])
    assert plan.n_vox == 1 << 28
    say("large plan: creating the geometry (2^28 voxels)")
    geo = geometry(plan, 1)
    f = torch.as_tensor(plan.fluence, device="cuda")
    dose = geo.forward(f).reshape(-1)
    total, counts = geo.count_pairs(f, per_voxel=True)
    counts = counts.reshape(-1)
    # sampled voxels: around the beamlet axes (x, z near the isocentre), at
    # every depth, and anywhere in the grid
    rng = np.random.default_rng(7)
    i = rng.integers(230, 282, 400)
    k = rng.integers(486, 538, 400)
    j = rng.integers(0, n[1], 400)
    near = (k * n[1] + j) * n[0] + i
    vox = np.concatenate([near, rng.integers(0, plan.n_vox, 100)]).astype(np.int64)
    vt = torch.as_tensor(vox, device="cuda")
    d_gpu = dose[vt].cpu().numpy().astype(np.float64)
    c_gpu = counts[vt].cpu().numpy()
    say("large plan: oracle at 500 sampled voxels")
    orc = abi_oracle(plan)
    d_o, amb, pc = orc.dose(vox=vox)
    assert d_o.max() > 0 and (d_o > 0).sum() > 100
    rel = assert_dose_parity(d_gpu, d_o, amb, what="2^28 voxels")
    assert np.array_equal(c_gpu, pc)
    say(f"large plan: max |err|/max D = {rel:.2e} over {vox.size} voxels, {int(total)} pairs")
    # the surrogate: rejected from this size on, before any buffer is used
    L = _lib.load()
    mlp = Mlp.initial(0)
    dens = torch.as_tensor(rho.reshape(-1)[:16], device="cuda")
    small = torch.zeros(64, device="cuda")
    rows = torch.zeros(2, dtype=torch.int32, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())
    assert L.fspb_surrogate_infer(geo._handle(), mlp._handle(), p(dens), p(small), None) == -1
    assert "surrogate_infer" in L.fspb_last_error().decode()
    assert L.fspb_forward_surrogate(geo._handle(), p(f), p(small), p(small), None) == -1
    assert L.fspb_surrogate_samples(geo._handle(), p(dens), p(rows), 1, p(small), p(small),
                                    p(rows), None) == -1
    geo.close()
