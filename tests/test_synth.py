"""The seeded generators are deterministic and produce the stated structure."""
import hashlib

import numpy as np

import fspb_synth as S


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_generators_deterministic():
    a, b = S.plan_c2(), S.plan_c2()
    assert _h(a.density) == _h(b.density) and _h(a.fluence) == _h(b.fluence)
    assert _h(S.c5_phantom(1000)) != _h(S.c5_phantom(1001))
    p, q = S.plan_c4(5), S.plan_c4(5)
    assert _h(p.density) == _h(q.density) and p.shape == q.shape


def test_config_shapes_and_ranges():
    c1 = S.plan_c1()
    assert c1.shape == (64, 64, 64) and c1.n_beamlets == 100
    assert set(np.unique(c1.density).tolist()) == {np.float32(0.25), np.float32(1.0), np.float32(1.8)}
    c2 = S.plan_c2()
    assert c2.shape == (96, 128, 128) and c2.n_beamlets == 2800
    zero = np.mean(c2.fluence == 0)
    assert 0.25 < zero < 0.35
    assert c2.density.min() >= np.float32(0.001) and c2.density.max() <= 1.9
    assert S.plan_c4(0).shape == (96, 96, 96) and S.plan_c4(31).shape == (160, 256, 256)


def test_tables_unit_at_water():
    t = S.make_tables(0)
    i = round((1.0 - t.fu1.start) / t.fu1.step)
    for tab in (t.fu1, t.fu2, t.fw1, t.fw2):
        assert tab.values[i] == np.float32(1.0)
    assert t.b1.values[i] == 0.0 and t.b2.values[i] == 0.0
    assert t.A.values.shape == (26, 801)


def test_paper_shaped_plans():
    """Table 1 shapes: 128 x 128 x 72 (head) and 128 x 128 x 103 (lung) at
    0.4 x 0.4 x 0.25 cm, 0.2 x 0.5 cm beamlets; the head case non-coplanar."""
    import math
    h, l = S.plan_paper_h5(), S.plan_paper_l2()
    assert h.shape == (72, 128, 128) and l.shape == (103, 128, 128)
    assert h.spacing == l.spacing == (0.4, 0.4, 0.25)
    assert len(h.beams) == 7 and len(l.beams) == 6
    assert abs(h.n_beamlets - 10369) < 20 and abs(l.n_beamlets - 1720) < 10
    assert len({round(b.couch, 6) for b in h.beams}) > 1 and all(b.couch == 0 for b in l.beams)
    assert all((b.wx, b.wy) == (0.2, 0.5) for b in h.beams + l.beams)
    assert np.array_equal(h.density, S.plan_paper_h5().density)
    assert 0.25 < float(np.mean(h.fluence == 0)) < 0.35
    assert math.isclose(h.origin[2], -0.5 * 71 * 0.25)
