"""The oracle's contact model reproduces the restitution coefficients the
paper lists for its three cases (Table 1), with the stiffness, diameter and
density listed beside them: two equal spheres colliding head on, and a sphere
hitting the wall, separate with the listed fraction of the approach speed.
The fixture holds the table's values (tests/golden/table1_dem_parameters.json).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "table1_dem_parameters.json")) as fh:
    TABLE1 = json.load(fh)["cases"]


def _contact_time(kn, e, meff):
    le = math.log(e)
    zeta = -le / math.sqrt(math.pi ** 2 + le ** 2)
    gam = 2 * zeta * math.sqrt(meff * kn)
    return math.pi / math.sqrt(kn / meff - (gam / (2 * meff)) ** 2)


def _dry(case, **kw):
    d = case["d"]
    p = workloads.base_params(Lx=20 * d, Ly=20 * d, Lz=10 * d, nx=1, ny=1, nz=1,
                              drag_law="none", lubrication=0, fluid_forces=0, bottom_wall=0,
                              top_wall=0, gz=0.0, kn=case["kn"],
                              restitution=case["restitution"], friction=case["friction"])
    p.update(kw)
    return p


@pytest.mark.parametrize("name", sorted(TABLE1))
def test_table1_restitution_head_on(orc, name):
    c = TABLE1[name]
    d, rho = c["d"], c["rho_p"]
    m = rho * math.pi / 6 * d ** 3
    tc = _contact_time(c["kn"], c["restitution"], 0.5 * m)
    prm = _dry(c, dt=tc / 2000)
    v0 = 0.05
    xc = 0.5 * prm["Lx"]
    x = np.array([[xc - 0.5 * d - 1e-7, 2 * d, 2 * d], [xc + 0.5 * d + 1e-7, 2 * d, 2 * d]])
    v = np.array([[v0, 0, 0], [-v0, 0, 0]])
    st = orc.State(prm, x, v, np.zeros((2, 3)), np.full(2, d), np.full(2, rho))
    st.init_accel()
    inside = 0
    for _ in range(20000):
        st.run(1)
        if st.x[1, 0] - st.x[0, 0] < d:
            inside += 1
        elif inside:
            break
    e_sim = (st.v[1, 0] - st.v[0, 0]) / (2 * v0)
    assert abs(e_sim - c["restitution"]) < 2e-3, (name, e_sim)
    assert abs(inside * prm["dt"] - tc) < 2e-3 * tc


@pytest.mark.parametrize("name", sorted(TABLE1))
def test_table1_restitution_wall(orc, name):
    c = TABLE1[name]
    d, rho = c["d"], c["rho_p"]
    m = rho * math.pi / 6 * d ** 3
    tc = _contact_time(c["kn"], c["restitution"], m)
    prm = _dry(c, bottom_wall=1, dt=tc / 2000)
    v0 = 0.03
    st = orc.State(prm, np.array([[2 * d, 2 * d, 0.5 * d + 1e-8]]), np.array([[0, 0, -v0]]),
                   np.zeros((1, 3)), np.full(1, d), np.full(1, rho))
    st.init_accel()
    touched = False
    for _ in range(20000):
        st.run(1)
        if st.x[0, 2] < 0.5 * d:
            touched = True
        elif touched:
            break
    assert touched
    assert abs(st.v[0, 2] / v0 - c["restitution"]) < 2e-3, name
