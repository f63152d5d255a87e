"""The seeded input generators (the recipe the design states): log-normal
diameters truncated to [0.3, 0.8] mm, random sequential insertion and
deposition without overlaps, the log-law frozen flow with its pressure
gradient and convective derivative, and the paper's time-step rule.  CPU
only; the generators hold none of the method's arithmetic."""
import math

import numpy as np

import workloads


def _min_gap(x, d, Lx, Ly):
    """Smallest surface gap between any two spheres (minimum image in x, y)."""
    dx = x[:, None, :] - x[None, :, :]
    dx[..., 0] -= Lx * np.round(dx[..., 0] / Lx)
    dx[..., 1] -= Ly * np.round(dx[..., 1] / Ly)
    dist = np.sqrt((dx ** 2).sum(-1))
    gap = dist - 0.5 * (d[:, None] + d[None, :])
    np.fill_diagonal(gap, np.inf)
    return gap.min()


def test_lognormal_diameters_recipe_and_seeding():
    d = workloads.lognormal_diameters(40000, 3)
    assert d.min() >= 0.3e-3 and d.max() <= 0.8e-3
    assert abs(np.median(d) / workloads.D50 - 1) < 0.01
    s = np.log(d).std()
    assert 0.17 < s < 0.2  # sigma 0.2, narrowed slightly by the truncation
    assert np.array_equal(d, workloads.lognormal_diameters(40000, 3))
    assert not np.array_equal(d[:100], workloads.lognormal_diameters(100, 4))


def test_insertion_and_deposition_place_spheres_without_overlap():
    n = 1500
    d = workloads.lognormal_diameters(n, 5)
    L = 20 * workloads.D50
    x = workloads.rsa(n, d, L, L, 12 * workloads.D50, 5)
    assert np.all((x[:, :2] >= 0) & (x[:, :2] < L))
    assert np.all(x[:, 2] >= 0.5 * d - 1e-15) and np.all(x[:, 2] <= 12 * workloads.D50 - 0.5 * d + 1e-15)
    assert _min_gap(x, d, L, L) > -1e-12 * workloads.D50
    b = workloads.rsd_bed(n, d, L, L, 6)
    assert np.all((b[:, :2] >= 0) & (b[:, :2] < L))
    assert np.all(b[:, 2] >= 0.5 * d - 1e-12 * workloads.D50)  # on or above the floor
    assert _min_gap(b, d, L, L) > -1e-9 * workloads.D50
    # a deposited bed is dense: its mean solid fraction below the bed top is high
    top = workloads.bed_top(b, d, L, L)
    frac = (math.pi / 6 * d ** 3).sum() / (L * L * top)
    assert 0.45 < frac < 0.65
    assert np.array_equal(b, workloads.rsd_bed(n, d, L, L, 6))


def test_fluid_fields_log_law_pressure_gradient_and_convective_derivative():
    prm = workloads.base_params(nx=8, ny=6, nz=20, Lz=10e-3)
    zb = 2e-3
    U, gp, du = workloads.fluid_fields(prm, z_bed=zb)
    _, _, zc = workloads.cell_centres(prm)
    z0 = workloads.D50 / 30
    above = zc - zb > z0
    want = workloads.U_STAR / workloads.KAPPA * np.log((zc[above] - zb) / z0)
    assert np.allclose(U[above, 0], want, rtol=1e-14, atol=0)
    assert np.all(U[~above] == 0) and np.all(U[:, 1:] == 0)
    H = prm["Lz"] - zb
    assert np.allclose(gp[:, 0], -prm["rho_f"] * workloads.U_STAR ** 2 / H, rtol=1e-14)
    assert np.allclose(gp[:, 2], prm["rho_f"] * prm["gz"], rtol=1e-14)
    # a pure streamwise log law has U . grad U = 0
    assert np.abs(du).max() == 0.0
    # on a sheared periodic field the central-difference derivative is exact
    # for the discrete sine: U = (A sin(k x), 0, 0) gives u du/dx
    A = 0.1
    xc, _, _ = workloads.cell_centres(prm)
    hx = prm["Lx"] / prm["nx"]
    kx = 2 * math.pi / prm["Lx"]
    V = np.zeros_like(U)
    V[:, 0] = A * np.sin(kx * xc)
    got = workloads.convective_derivative(prm, V)
    assert np.allclose(got[:, 0], V[:, 0] * A * math.sin(kx * hx) / hx * np.cos(kx * xc),
                       rtol=0, atol=1e-12 * A * A * kx)


def test_time_step_is_one_fiftieth_of_the_shortest_contact():
    prm = workloads.base_params()
    dmin = 0.3e-3
    m = workloads.RHO_P * math.pi / 6 * dmin ** 3
    e = prm["restitution"]
    zeta = -math.log(e) / math.sqrt(math.pi ** 2 + math.log(e) ** 2)
    k, me = prm["kn"], 0.5 * m
    wn = math.sqrt(k / me)
    tc = math.pi / (wn * math.sqrt(1 - zeta ** 2))
    assert abs(workloads.dt_rule(prm, dmin) - tc / 50) < 1e-15 * tc


def test_graded_mesh_geometry_and_fields():
    """z_grading: geometric faces with the requested top/bottom height
    ratio; the log law is sampled at the graded centres, and the convective
    derivative of a field linear in z is exact on them."""
    prm = workloads.base_params(nx=4, ny=3, nz=16, Lz=8e-3, z_grading=5.0)
    zf = workloads.z_faces(prm)
    h = np.diff(zf)
    assert zf[0] == 0 and zf[-1] == prm["Lz"] and np.all(h > 0)
    assert abs(h[-1] / h[0] - 5.0) < 1e-12
    assert np.allclose(h[1:] / h[:-1], 5.0 ** (1 / 15), rtol=1e-12)
    _, _, zc = workloads.cell_centres(prm)
    assert np.allclose(np.unique(zc), 0.5 * (zf[1:] + zf[:-1]), rtol=1e-15)
    U, _, _ = workloads.fluid_fields(prm, z_bed=1e-3)
    z0 = workloads.D50 / 30
    above = zc - 1e-3 > z0
    assert np.allclose(U[above, 0], workloads.U_STAR / workloads.KAPPA *
                       np.log((zc[above] - 1e-3) / z0), rtol=1e-14)
    V = np.zeros((zc.size, 3))
    V[:, 0] = 0.3
    V[:, 2] = 0.01 + 2.0 * zc  # w grows linearly with z: w dw/dz = w * 2
    got = workloads.convective_derivative(prm, V)
    assert np.allclose(got[:, 2], V[:, 2] * 2.0, rtol=1e-12)
    # uniform meshes are unchanged by the option's default
    assert np.array_equal(workloads.z_faces(workloads.base_params()),
                          workloads.base_params()["Lz"] * np.arange(9) / 8)


def test_tiled_bed_copies_meet_without_overlap():
    """The 10M bed is an array of copies of one periodic deposited tile: the
    copies must meet at the seams without overlaps, keep the tile's size
    distribution and fill the whole domain."""
    n = 700
    d = workloads.lognormal_diameters(n, 9)
    tx, ty = 12 * workloads.D50, 9 * workloads.D50
    x = workloads.rsd_bed(n, d, tx, ty, 9)
    xt, dt = workloads.tile_bed(x, d, 3 * tx, 2 * ty, (3, 2))
    assert len(xt) == 6 * n and np.array_equal(dt[:n], d) and np.array_equal(dt[5 * n:], d)
    assert np.all((xt[:, 0] >= 0) & (xt[:, 0] < 3 * tx) & (xt[:, 1] >= 0) & (xt[:, 1] < 2 * ty))
    assert _min_gap(xt, dt, 3 * tx, 2 * ty) > -1e-12 * workloads.D50
    # copy (a, b) is the tile shifted by (a tx, b ty)
    k = (1 * 3 + 2) * n
    assert np.allclose(xt[k:k + n] - x, [2 * tx, ty, 0.0], rtol=0, atol=1e-15)
