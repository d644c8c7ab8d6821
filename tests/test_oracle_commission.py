"""The commissioning measurement set pins down the eight table parameters:
an independent least-squares fit (SciPy) on the FP64 oracle's doses, at a
few thousand sampled voxels of each plan, recovers the truth parameters
from the nominal start.  (The GPU fitter is checked against the same truth
in tests/test_gpu_commission.py.)"""
import numpy as np
import pytest
from scipy.optimize import least_squares

import fspb_synth as S
from oracle import Oracle


@pytest.mark.slow
def test_oracle_fit_recovers_truth():
    truth = S.table_coeffs(7)
    plans = S.commissioning_plans()
    rng = np.random.default_rng(0)
    vox = [rng.choice(p.n_vox, size=1500, replace=False) for p in plans]

    def doses(c):
        out = []
        for p, v in zip(plans, vox):
            q = S.Plan(p.name, p.density, p.spacing, p.origin, p.beams, p.fluence,
                       S.make_tables_coeffs(c), p.options)
            out.append(Oracle(q).dose(vox=v)[0])
        return out

    ref = doses(truth)
    scale = [m.max() for m in ref]

    def res(c):
        return np.concatenate([(d - m) / s for d, m, s in zip(doses(c), ref, scale)])

    fit = least_squares(res, np.ones(8), diff_step=1e-3, x_scale=np.ones(8), xtol=1e-12,
                        ftol=1e-14, gtol=1e-14, max_nfev=400)
    assert np.max(np.abs(fit.x - truth) / truth) < 1e-3, (fit.x, truth)
    assert np.max(np.abs(res(np.ones(8)))) > 1e-3        # the start really is off
