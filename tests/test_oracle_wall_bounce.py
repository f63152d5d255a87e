"""Case 1 of Section 4 on the oracle: the effective restitution of a sphere
bouncing on a wall in a liquid against the Stokes number, with and without
lubrication (wall_bounce.py describes the case)."""
import numpy as np
import pytest

import wall_bounce as wb

MUS = (1e-3, 5e-3, 2e-2, 5e-2)


@pytest.fixture(scope="module")
def sweep(orc):
    out = {}
    for mu in MUS:
        for lub in (False, True):
            c = wb.case(mu, lubrication=lub)
            z, v = wb.run_oracle(orc, c)
            out[mu, lub] = wb.restitution(c["params"], z, v)
    return out


def test_wall_bounce_effective_restitution_trend(sweep):
    """Without lubrication the wet collision keeps the dry restitution (the
    drag acts only briefly during contact); with it, e falls as St falls,
    strongly below St ~ 50 and little above St ~ 500, the trend the paper
    reports."""
    for mu in MUS:
        e, St, _ = sweep[mu, False]
        assert 0.98 < e < 1.02, (mu, e)
    e_lub = [sweep[mu, True][0] for mu in MUS]
    St = [sweep[mu, True][1] for mu in MUS]
    print("St", np.round(St, 1), "e", np.round(e_lub, 4))
    assert all(a > b for a, b in zip(St, St[1:]))       # viscosity up, St down
    assert all(a > b for a, b in zip(e_lub, e_lub[1:]))  # and e down with it
    assert e_lub[0] > 0.95 and e_lub[-1] < 0.5
    for mu in MUS:
        assert sweep[mu, True][0] < sweep[mu, False][0]
