"""The oracle's OpenMP loops change nothing: the pair list, every force
component, the tangential histories and a short coupled run with averaging
are bit-identical on 1 and on several threads (pairs are evaluated in
parallel and added to their particles in pair order; per-particle loops
touch only their own particle)."""
import numpy as np
import pytest

import workloads


def _bed(seed, **kw):
    n = 3000
    d = workloads.lognormal_diameters(n, seed)
    L = 24 * workloads.D50
    prm = workloads.base_params(Lx=L, Ly=L, Lz=14 * workloads.D50, nx=18, ny=18, nz=11, **kw)
    x = workloads.rsd_bed(n, d, L, L, seed)
    rng = np.random.default_rng(seed)
    x = x + rng.normal(scale=0.002 * workloads.D50, size=x.shape)
    x[:, :2] %= L
    x[:, 2] = np.clip(x[:, 2], 0.3 * d, prm["Lz"] - 0.5 * d)
    v = rng.normal(scale=0.01, size=(n, 3))
    w = rng.normal(scale=20.0, size=(n, 3))
    zb = workloads.bed_top(x, d, L, L)
    U, gradp, dudt = workloads.fluid_fields(prm, z_bed=zb, fluct=0.05, seed=seed + 1)
    return prm, x, v, w, d, np.full(n, workloads.RHO_P), U, gradp, dudt


def _everything(orc, threads, seed, **kw):
    orc.set_threads(threads)
    try:
        prm, x, v, w, d, rho, U, gradp, dudt = _bed(seed, **kw)
        pairs = orc.pairs_cells(prm, x, d)
        comps, hist = orc.forces(prm, x, v, w, d, rho, U=U, gradp=gradp, dudt=dudt)
        st = orc.State(prm, x, v, w, d, rho, U=U, gradp=gradp, dudt=dudt)
        st.average()
        st.init_accel()
        st.run(6, average_every=3)
        return pairs, comps, hist, st.x.copy(), st.v.copy(), st.w.copy(), st.avg.copy()
    finally:
        orc.set_threads(1)


@pytest.mark.parametrize("seed,kw", [(3, {}), (4, dict(c_lift=1.6, z_grading=4.0))])
def test_threads_do_not_change_any_bit(orc, seed, kw):
    one = _everything(orc, 1, seed, **kw)
    many = _everything(orc, 4, seed, **kw)
    assert orc.get_threads() == 1
    pairs1, comps1, hist1 = one[:3]
    pairs4, comps4, hist4 = many[:3]
    assert len(pairs1) > 3000
    assert np.array_equal(pairs1, pairs4)
    for k in comps1:
        assert np.array_equal(comps1[k], comps4[k]), k
    assert np.array_equal(hist1, hist4)
    for a, b in zip(one[3:], many[3:]):
        assert np.array_equal(a, b)
