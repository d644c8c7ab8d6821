"""The 3D gamma index on an MI355X against the FP64 reference (oracle.gamma).

Bar: gamma agrees to 1e-5 (FP32 against FP64 of the same input values, on
values of order 1); the statistics agree exactly except for voxels whose
gamma lies within 1e-5 of 1, which FP32 and FP64 may put on either side."""
import numpy as np
import pytest
import torch

import fspb_synth as S
from gpu_helpers import abi_oracle, say
from oracle import gamma as G

pytestmark = pytest.mark.gpu


def _smooth_pair(shape, seed, shift=(0, 0, 1), noise=0.02):
    """Two dose-like fields: Gaussian blobs, the second shifted by a voxel
    offset and perturbed (seeded)."""
    rng = np.random.default_rng(seed)
    Z, Y, X = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    R = np.zeros(shape)
    E = np.zeros(shape)
    for _ in range(4):
        c = rng.uniform(0, 1, 3) * np.array(shape)
        w = rng.uniform(2.0, 6.0)
        a = rng.uniform(0.5, 2.0)
        R += a * np.exp(-((Z - c[0]) ** 2 + (Y - c[1]) ** 2 + (X - c[2]) ** 2) / (2 * w * w))
        E += a * np.exp(-((Z - c[0] - shift[0]) ** 2 + (Y - c[1] - shift[1]) ** 2
                          + (X - c[2] - shift[2]) ** 2) / (2 * w * w))
    E *= 1.0 + noise * rng.standard_normal(shape)
    return R.astype(np.float32), E.astype(np.float32)


def _check(R, E, sp, **kw):
    from paper_1103_1164_amd import gamma_index
    g_gpu, st = gamma_index(torch.as_tensor(R, device="cuda"), torch.as_tensor(E, device="cuda"),
                            sp, **kw)
    g_gpu = g_gpu.cpu().numpy().astype(np.float64)
    cap = kw.get("cap", 5.0)
    g_o = G.gamma(R.astype(np.float64), E.astype(np.float64), sp, dist=kw.get("dist", 0.3),
                  dose_frac=kw.get("dose_frac", 0.03), cap=cap, dose_max=kw.get("dose_max") or None)
    assert np.max(np.abs(g_gpu - g_o)) < 1e-5
    so = G.stats(g_o, R.astype(np.float64), iso_frac=kw.get("iso_frac", 0.5),
                 dose_max=kw.get("dose_max") or None)
    assert st["n_iso"] == so["n_iso"] and st["dose_max"] == pytest.approx(so["dose_max"], rel=1e-7)
    assert st["gamma_max"] == pytest.approx(so["gamma_max"], abs=1e-5)
    assert st["gamma_avg_iso"] == pytest.approx(so["gamma_avg_iso"], abs=1e-5)
    m = R >= kw.get("iso_frac", 0.5) * so["dose_max"]
    near = int(np.sum(np.abs(g_o[m] - 1.0) < 1e-5))
    assert abs(st["pass_rate_iso"] - so["pass_rate_iso"]) * so["n_iso"] <= near + 1e-9
    return g_gpu, st


@pytest.mark.parametrize("sp", [(0.25, 0.25, 0.25), (0.4, 0.4, 0.25), (0.1, 0.3, 0.2)])
def test_gamma_matches_reference(sp):
    R, E = _smooth_pair((22, 27, 31), seed=int(sp[0] * 100), shift=(1, 0, -1))
    say(f"gamma spacing {sp}")
    _, st = _check(R, E, sp)
    assert 0.0 < st["gamma_max"] <= 5.0 and 0.0 < st["pass_rate_iso"] < 1.0


def test_gamma_options_and_edges():
    R, E = _smooth_pair((9, 11, 13), seed=3, noise=0.1)
    _check(R, E, (0.25, 0.25, 0.25), cap=1.5, dist=0.2, dose_frac=0.05, iso_frac=0.2)
    _check(R, E, (0.25, 0.25, 0.25), dose_max=float(R.max()) * 2.0)
    from paper_1103_1164_amd import gamma_index
    t = torch.as_tensor(R, device="cuda")
    g, st = gamma_index(t, t, (0.25, 0.25, 0.25))
    assert float(g.abs().max()) == 0.0 and st["pass_rate_iso"] == 1.0
    # one-voxel grid, and a grid thinner than the search radius
    _check(R[:1, :1, :1] + 1.0, E[:1, :1, :1] + 1.0, (0.25, 0.25, 0.25))
    _check(R[:2], E[:2], (0.25, 0.25, 0.25))


def test_gamma_of_the_method_on_config1(oracle_mod):
    """The paper's evaluation applied to DC against conventional FSPB on
    config 1 (doses from the oracle): gamma grid and statistics agree."""
    plan = S.plan_c1()
    say("c1: oracle doses")
    d_dc = abi_oracle(plan, dc_enabled=1).dose()[0].astype(np.float32)
    d_pl = abi_oracle(plan, dc_enabled=0).dose()[0].astype(np.float32)
    _, st = _check(d_dc, d_pl, plan.spacing)
    assert st["gamma_max"] > 0.5
