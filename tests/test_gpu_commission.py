"""Commissioning with the library in the loop: the Levenberg-Marquardt
fitter, whose every dose is a GPU plan, recovers the eight table parameters
of a perturbed machine from FP64 oracle "measurements" made with that
machine's tables (water tank and slab phantom), starting from the nominal
machine."""
import numpy as np
import pytest

import fspb_synth as S
from gpu_helpers import abi_oracle, say

pytestmark = pytest.mark.gpu


def test_fit_recovers_perturbed_machine(oracle_mod):
    from paper_1103_1164_amd.commission import fit_tables
    truth = S.table_coeffs(7)
    plans = S.commissioning_plans()
    say("commission: oracle measurements")
    refs = []
    for p in plans:
        q = S.Plan(p.name, p.density, p.spacing, p.origin, p.beams, p.fluence,
                   S.make_tables_coeffs(truth), p.options)
        refs.append(abi_oracle(q).dose()[0].astype(np.float32))
    say("commission: fit")
    res = fit_tables(plans, refs, S.make_tables_coeffs, np.ones(8), iters=30, log=say)
    err = np.abs(res["c"] - truth) / truth
    say(f"commission: {res['evaluations']} evaluations in {res['seconds']:.2f} s, "
        f"max relative parameter error {err.max():.2e}")
    assert err.max() < 1e-3, (res["c"], truth)
    assert res["cost"][-1] < 1e-6 * res["cost"][0]
