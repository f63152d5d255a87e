"""Case 1 of Section 4 on the GPU path: the sphere-wall bounce in a liquid
(wall_bounce.py describes the case), step by step against the oracle, and
the effective restitution's trend with the Stokes number."""
import numpy as np
import pytest

import wall_bounce as wb
from gpu_helpers import gpu_context

pytestmark = pytest.mark.gpu

MUS = (1e-3, 5e-3, 2e-2, 5e-2)


def run_gpu(c):
    g = gpu_context(c)
    g.compute_forces(update_history=False)  # initial acceleration, as the oracle's

    def once():
        g.step(1, 0)
        p = g.get_particles()
        return p["x"][0, 2], p["v"][0, 2]
    return wb.follow(once, c["params"])


def test_wall_bounce_matches_oracle_and_trend(orc):
    e_lub, St_lub = [], []
    for mu in MUS:
        for lub in (False, True):
            c = wb.case(mu, lubrication=lub)
            zg, vg = run_gpu(c)
            zo, vo = wb.run_oracle(orc, c)
            assert len(zg) == len(zo)
            eg, Stg, vin = wb.restitution(c["params"], zg, vg)
            eo, _, _ = wb.restitution(c["params"], zo, vo)
            dz = np.abs(zg - zo).max() / wb.D
            dv = np.abs(vg - vo).max() / vin
            print(f"mu {mu:.0e} lub {lub}: St {Stg:.1f} e {eg:.5f} (oracle {eo:.5f}) "
                  f"steps {len(zg)} max|dz|/d {dz:.2e} max|dv|/v_in {dv:.2e}")
            assert dz < 1e-9 and dv < 1e-7
            assert abs(eg - eo) < 1e-7
            if lub:
                e_lub.append(eg)
                St_lub.append(Stg)
            else:
                assert 0.98 < eg < 1.02
    assert all(a > b for a, b in zip(St_lub, St_lub[1:]))
    assert all(a > b for a, b in zip(e_lub, e_lub[1:]))
