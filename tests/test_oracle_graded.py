"""The oracle on a z mesh graded geometrically towards the bottom wall (the
channel case of Section 4 refines its mesh that way; read as cell heights
h_k = h_0 q^k with q^(nz-1) = z_grading).  Pins: the face geometry; the
deposition's cells and volumes; the finite-volume diffusion's conservation,
maximum principle, symmetry in the volume-weighted inner product and
convergence to the exact decay of the wall-normal cosine mode under mesh
refinement; interpolation that is exact for fields linear in z; the shear
lift's curl on the graded mesh; and z_grading = 1 reproducing the uniform
mesh exactly."""
import math

import numpy as np
import pytest

import workloads

D, RHO = workloads.D50, workloads.RHO_P


def graded_prm(nz=12, g=8.0, nx=6, ny=5, **kw):
    return workloads.base_params(Lx=3e-3, Ly=2.5e-3, Lz=4e-3, nx=nx, ny=ny, nz=nz,
                                 avg_bandwidth=1.0e-3, avg_ntau=4, cg_rtol=1e-14,
                                 z_grading=g, **kw)


def faces(prm):
    nz, g, Lz = prm["nz"], prm["z_grading"], prm["Lz"]
    q = g ** (1.0 / (nz - 1))
    h = q ** np.arange(nz)
    h *= Lz / h.sum()
    return np.concatenate([[0.0], np.cumsum(h)])


def cell_volumes(prm):
    zf = faces(prm)
    hz = np.diff(zf)
    hx, hy = prm["Lx"] / prm["nx"], prm["Ly"] / prm["ny"]
    return np.repeat(hz, prm["nx"] * prm["ny"]) * hx * hy


def test_deposit_on_graded_cells_conserves_volume(orc):
    prm = graded_prm()
    zf = faces(prm)
    assert abs(np.diff(zf)[-1] / np.diff(zf)[0] - 8.0) < 1e-12
    rng = np.random.default_rng(1)
    n = 3000
    d = rng.uniform(0.3e-3, 0.8e-3, n)
    x = rng.random((n, 3)) * [prm["Lx"], prm["Ly"], prm["Lz"]]
    raw = orc.deposit(prm, x, d)
    Vp = math.pi / 6 * d ** 3
    assert abs((raw[0] * cell_volumes(prm)).sum() - Vp.sum()) < 1e-12 * Vp.sum()
    # one sphere on a face of the graded mesh lands in the upper cell
    k = 5
    xp = np.array([[0.1e-3, 0.1e-3, zf[k]]])
    one = orc.deposit(prm, xp, np.array([D]))
    cell = k * prm["nx"] * prm["ny"]
    assert list(np.flatnonzero(one[0])) == [cell]
    assert one[0, cell] == pytest.approx(math.pi / 6 * D ** 3 / cell_volumes(prm)[cell], rel=1e-14)


def test_graded_diffusion_conserves_and_keeps_the_maximum_principle(orc):
    prm = graded_prm()
    n = prm["nx"] * prm["ny"] * prm["nz"]
    rng = np.random.default_rng(2)
    raw = np.zeros(n)
    raw[rng.choice(n, 25, replace=False)] = rng.random(25)
    out, iters = orc.diffuse(prm, raw[None])
    V = cell_volumes(prm)
    assert iters > 0
    assert abs((out[0] * V).sum() - (raw * V).sum()) < 1e-12 * (raw * V).sum()
    assert out.min() >= 0.0 and out.max() <= raw.max()
    uni, _ = orc.diffuse(prm, np.full((1, n), 0.42))
    assert np.max(np.abs(uni - 0.42)) < 1e-14
    # H (I - dtau L) is symmetric: <x, S y> = <S x, y>
    dtau = 1e-8
    hz = np.repeat(np.diff(faces(prm)), prm["nx"] * prm["ny"])
    a, b = rng.random(n), rng.random(n)
    Sa = hz * orc.apply_A(prm, dtau, a)
    Sb = hz * orc.apply_A(prm, dtau, b)
    assert abs(a @ Sb - Sa @ b) < 1e-13 * abs(a @ Sb)


def test_graded_diffusion_converges_to_the_cosine_mode_decay(orc):
    """A column (nx = ny = 1) holding cos(pi z / Lz) at its cell centres
    decays as exp(-(pi/Lz)^2 tau) under zero-flux walls; with BDF2 and many
    pseudo-time steps the remaining error is the mesh's, and it falls by at
    least 2.5x per halving of every cell on a graded mesh."""
    errs = []
    for nz in (16, 32, 64):
        prm = workloads.base_params(Lx=1e-3, Ly=1e-3, Lz=4e-3, nx=1, ny=1, nz=nz,
                                    avg_bandwidth=2e-3, avg_ntau=400, cg_rtol=1e-14,
                                    avg_scheme=1, z_grading=6.0)
        zf = faces(prm)
        zc = 0.5 * (zf[1:] + zf[:-1])
        f0 = np.cos(math.pi * zc / prm["Lz"])
        out, _ = orc.diffuse(prm, f0[None])
        tau = prm["avg_bandwidth"] ** 2 / 4
        exact = math.exp(-(math.pi / prm["Lz"]) ** 2 * tau) * f0
        errs.append(np.abs(out[0] - exact).max())
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5, errs
    assert errs[2] < 2e-3


def test_graded_interpolation_is_exact_for_fields_linear_in_z(orc):
    """With the Stokes drag and nothing else, a particle at rest feels
    3 pi mu d U(x_p): U = (a + b z, 0, 0) sampled at the graded centres is
    recovered exactly between the first and last centre, and held at the
    end values outside them."""
    prm = graded_prm(drag_law="stokes", lubrication=0, fluid_forces=0, bottom_wall=0,
                     top_wall=0)
    zf = faces(prm)
    zc = 0.5 * (zf[1:] + zf[:-1])
    a, b = 0.02, 15.0
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    U = np.zeros((ncell, 3))
    U[:, 0] = np.repeat(a + b * zc, prm["nx"] * prm["ny"])
    zs = np.array([0.5 * zc[0], zc[0], 0.3e-3, 1.234e-3, 2.9e-3, zc[-1], 0.5 * (zc[-1] + 4e-3)])
    x = np.stack([np.full(zs.size, 1.1e-3), np.full(zs.size, 0.7e-3), zs], axis=1)
    comps, _ = orc.forces(prm, x, np.zeros_like(x), np.zeros_like(x), np.full(zs.size, D),
                          np.full(zs.size, RHO), U=U)
    got = comps["drag"][:, 0] / (3 * math.pi * workloads.MU_F * D)
    want = a + b * np.clip(zs, zc[0], zc[-1])
    assert np.allclose(got, want, rtol=1e-13, atol=0)


def test_graded_lift_curl_of_a_linear_shear_is_exact(orc):
    """U = (g z, 0, 0) on the graded mesh: the centre differences, one-sided
    at the walls, give omega = (0, g, 0) exactly, so Saffman's lift holds."""
    g = 40.0
    prm = graded_prm(drag_law="none", lubrication=0, fluid_forces=0, bottom_wall=0,
                     top_wall=0, c_lift=1.6)
    zf = faces(prm)
    zc = 0.5 * (zf[1:] + zf[:-1])
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    U = np.zeros((ncell, 3))
    U[:, 0] = np.repeat(g * zc, prm["nx"] * prm["ny"])
    for zp in (0.5 * (zc[0] + zc[1]), 2.2e-3):
        x = np.array([[1.0e-3, 1.0e-3, zp]])
        comps, _ = orc.forces(prm, x, np.zeros((1, 3)), np.zeros((1, 3)), np.full(1, D),
                              np.full(1, RHO), U=U)
        f = comps["lift"][0]
        nu = workloads.MU_F / workloads.RHO_F
        want = 1.6 * workloads.RHO_F * math.sqrt(nu) * D * D * (g * zp) * math.sqrt(g)
        assert f[0] == 0 and abs(f[1]) < 1e-12 * want and abs(f[2] / want - 1) < 1e-12


def test_grading_one_is_the_uniform_mesh(orc):
    base = graded_prm(g=0.0)
    one = dict(base, z_grading=1.0)
    rng = np.random.default_rng(4)
    n = 500
    d = rng.uniform(0.3e-3, 0.8e-3, n)
    x = rng.random((n, 3)) * [base["Lx"], base["Ly"], base["Lz"]]
    r0, r1 = orc.deposit(base, x, d), orc.deposit(one, x, d)
    assert np.array_equal(r0, r1)
    s0, _ = orc.diffuse(base, r0[:1])
    s1, _ = orc.diffuse(one, r1[:1])
    assert np.array_equal(s0, s1)


@pytest.mark.parametrize("eps", [1e-6, 1e-9])
def test_grading_near_one_tends_to_the_uniform_mesh(orc, eps):
    """A grading of 1 + eps runs the graded branches (faces, per-cell
    volumes, the height-weighted operator) and must approach the uniform mesh
    as eps -> 0: faces within eps Lz, the bottom cell no taller than the top
    one, deposition and smoothing within a few eps."""
    base = graded_prm(g=0.0)
    near = dict(base, z_grading=1.0 + eps)
    zf = faces(near)
    nz = base["nz"]
    h = np.diff(zf)
    assert np.all(h[1:] >= h[:-1] * (1 - 1e-15)) and h[-1] / h[0] <= 1 + 2 * eps
    assert np.all(np.abs(zf - base["Lz"] * np.arange(nz + 1) / nz) < eps * base["Lz"])
    rng = np.random.default_rng(4)
    n = 500
    d = rng.uniform(0.3e-3, 0.8e-3, n)
    x = rng.random((n, 3)) * [base["Lx"], base["Ly"], base["Lz"]]
    r0, r1 = orc.deposit(base, x, d), orc.deposit(near, x, d)
    assert np.all(np.abs(r1 - r0) <= 4 * eps * np.abs(r0).max())
    s0, _ = orc.diffuse(base, r0[:1])
    s1, _ = orc.diffuse(near, r1[:1])
    assert np.all(np.abs(s1 - s0) <= 20 * eps * np.abs(s0).max())


def test_graded_run_with_averaging_conserves_the_solid_volume(orc):
    """A short velocity-Verlet run of a small bed on the graded mesh with
    averaging inside: the state stays finite and every averaging keeps the
    total solid volume sum(eps_s V_k) equal to the particles' volume."""
    w = workloads.workload("small")
    prm = dict(w["params"], z_grading=4.0, avg_ntau=2)
    st = orc.State(prm, w["x"], w["v"], w["w"], w["d"], w["rho"], U=w["U"], gradp=w["gradp"],
                   dudt=w["dudt"])
    st.average()
    st.init_accel()
    st.run(20, average_every=10)
    assert np.all(np.isfinite(st.x)) and np.all(np.isfinite(st.v))
    V = cell_volumes(prm)
    Vp = (math.pi / 6 * w["d"] ** 3).sum()
    assert abs((st.eps_s * V).sum() - Vp) < 1e-11 * Vp
