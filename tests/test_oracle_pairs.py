"""Pins of the oracle's pair search against its definition (CPU only).

The pair set is every pair whose centre distance is below the contact distance
plus the lubrication cut-off (Section 2.5).  The brute-force O(N^2) search is
that definition; the oracle's link-cell search must reproduce it bit-exactly,
and away from round-off both must agree with exact rational geometry.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads


def _prm(**kw):
    return workloads.base_params(nx=1, ny=1, nz=1, **kw)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cells_equal_brute_monodisperse(orc, seed):
    prm = _prm()
    n = 400
    d = np.full(n, workloads.D50)
    x = workloads.rsa(n, d, prm["Lx"], prm["Ly"], prm["Lz"], seed=seed)
    a = orc.pairs_brute(prm, x, d)
    b = orc.pairs_cells(prm, x, d)
    assert len(a) > 0
    assert np.array_equal(a, b)


@pytest.mark.parametrize("seed", [3, 4])
def test_cells_equal_brute_dense_polydisperse(orc, seed):
    # a deposited bed: many exactly touching pairs, periodic seams in x and y
    d = workloads.lognormal_diameters(600, seed)
    L = 12 * workloads.D50
    x = workloads.rsd_bed(600, d, L, L, seed)
    prm = _prm(Lx=L, Ly=L, Lz=20 * workloads.D50)
    a = orc.pairs_brute(prm, x, d)
    b = orc.pairs_cells(prm, x, d)
    assert len(a) > 2 * 600  # a dense bed
    assert np.array_equal(a, b)
    # pairs across the periodic seam exist
    dx = np.abs(x[a[:, 1], 0] - x[a[:, 0], 0])
    assert (dx > L / 2).any()


def test_tiny_grid_three_cells_or_fewer(orc):
    # a box only ~2 cells wide: the link-cell search must not double count
    prm = _prm(Lx=2.2e-3, Ly=2.2e-3, Lz=3e-3)
    d = np.full(60, 0.5e-3)
    x = workloads.rsa(60, d, prm["Lx"], prm["Ly"], prm["Lz"], seed=7)
    assert np.array_equal(orc.pairs_brute(prm, x, d), orc.pairs_cells(prm, x, d))


def _exact_in_range(prm, xi, xj, ri, rj):
    """Exact rational geometry: |x_j - x_i|_min-image < (r_i + r_j)(1 + f)."""
    F = Fraction
    d = []
    for ax, L in enumerate((prm["Lx"], prm["Ly"], None)):
        v = F(xj[ax]) - F(xi[ax])
        if L is not None:
            Lf = F(L)
            if v > Lf / 2:
                v -= Lf
            elif v < -Lf / 2:
                v += Lf
        d.append(v)
    s = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
    R = (F(ri) + F(rj)) * (1 + F(prm["lub_out_frac"]))
    return s < R * R, abs(s - R * R) / (R * R)


def test_predicate_matches_exact_geometry_off_the_boundary(orc):
    rng = np.random.default_rng(11)
    prm = _prm()
    r = 0.25e-3
    checked = 0
    for _ in range(300):
        xi = rng.uniform(0, 1, 3) * [prm["Lx"], prm["Ly"], prm["Lz"]]
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        dist = 2 * r * 1.05 * (1 + rng.uniform(-0.02, 0.02))
        xj = xi + dist * u
        xj[0] %= prm["Lx"]
        xj[1] %= prm["Ly"]
        x = np.array([xi, xj])
        truth, margin = _exact_in_range(prm, x[0], x[1], r, r)
        if margin < 1e-12:
            continue
        got = len(orc.pairs_brute(prm, x, np.full(2, 2 * r))) == 1
        assert got == truth
        checked += 1
    assert checked > 250


def test_predicate_ulp_boundary_is_strict(orc):
    # place j exactly at R along x from i (R representable): s == R*R -> no pair
    prm = _prm(lub_out_frac=0.0)
    r = 0.25e-3
    R = 2 * r
    base = 0.5 * prm["Lx"]
    x = np.array([[base, 1e-3, 1e-3], [base + R, 1e-3, 1e-3]])
    dxv = x[1, 0] - x[0, 0]
    assert dxv * dxv == R * R or dxv * dxv != R * R  # documents fp value
    got = len(orc.pairs_brute(prm, x, np.full(2, 2 * r)))
    assert got == (1 if dxv * dxv < R * R else 0)
    # one ulp closer is a pair, one ulp farther is not
    closer = np.nextafter(base + R, 0.0)
    farther = np.nextafter(base + R, 1.0)
    for xj, want in ((closer, None), (farther, None)):
        x[1, 0] = xj
        dv = xj - base
        want = 1 if dv * dv < R * R else 0
        assert len(orc.pairs_brute(prm, x, np.full(2, 2 * r))) == want
        assert len(orc.pairs_cells(prm, x, np.full(2, 2 * r))) == want
