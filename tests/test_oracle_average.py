"""Pins of the oracle's averaging against the mathematics of Section 2.4 (CPU).

  - PCM deposition (Eq. 11) conserves the total particle volume exactly and
    puts each particle in exactly one cell;
  - the implicit diffusion solve (Eq. 12) equals the exact discrete solution
    obtained by diagonalising the operator with FFTs (periodic x, y) and a
    DCT-II (zero-flux z walls);
  - it conserves the integral (the no-flux wall condition), is positive, obeys
    the maximum principle and leaves a uniform field unchanged;
  - for a point source it converges to the Gaussian kernel with variance
    2 tau = b^2/2 per axis: first order in the pseudo-time step, second order
    in the mesh spacing.
"""
import math

import numpy as np
import pytest
from scipy import fft as sfft

import workloads


def mesh_prm(nx, ny, nz, L=(4e-3, 3e-3, 2.5e-3), b=1.5e-3, ntau=4, rtol=1e-14):
    return workloads.base_params(Lx=L[0], Ly=L[1], Lz=L[2], nx=nx, ny=ny, nz=nz,
                                 avg_bandwidth=b, avg_ntau=ntau, cg_rtol=rtol)


def spectral_solve(prm, raw, exact_time=False):
    """Diagonalise -L_h: FFT on the periodic axes, orthonormal DCT-II on z."""
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    hx, hy, hz = prm["Lx"] / nx, prm["Ly"] / ny, prm["Lz"] / nz
    tau = prm["avg_bandwidth"] ** 2 / 4
    bz = prm.get("avg_bandwidth_z", 0.0)
    kz = (bz / prm["avg_bandwidth"]) ** 2 if bz > 0 else 1.0  # diffusivity along z
    f = raw.reshape(nz, ny, nx)
    F = sfft.dct(np.fft.fft2(f, axes=(1, 2)), type=2, axis=0, norm="ortho")
    kx = 2 * np.pi * np.arange(nx) / nx
    ky = 2 * np.pi * np.arange(ny) / ny
    kzw = np.pi * np.arange(nz) / nz
    lam = (kz * (2 - 2 * np.cos(kzw))[:, None, None] / hz ** 2 +
           (2 - 2 * np.cos(ky))[None, :, None] / hy ** 2 +
           (2 - 2 * np.cos(kx))[None, None, :] / hx ** 2)
    N = prm["avg_ntau"]
    a = tau / N * lam
    if exact_time:
        G = np.exp(-tau * lam)
    elif prm.get("avg_scheme", 0) == 1:
        # BDF2 per mode: g1 = 1/(1+a), g_{m+1} = (4 g_m - g_{m-1}) / (3 + 2a)
        g0, g1 = np.ones_like(a), 1 / (1 + a)
        for _ in range(N - 1):
            g0, g1 = g1, (4 * g1 - g0) / (3 + 2 * a)
        G = g1
    else:
        G = (1 + a) ** (-N)
    out = np.fft.ifft2(sfft.idct(F * G, type=2, axis=0, norm="ortho"), axes=(1, 2))
    return out.real.ravel()


def test_pcm_conserves_volume(orc):
    w = workloads.workload("bed1m", n=20000)
    prm = w["params"]
    raw = orc.deposit(prm, w["x"], w["d"])
    Vc = prm["Lx"] / prm["nx"] * prm["Ly"] / prm["ny"] * prm["Lz"] / prm["nz"]
    total = (math.pi / 6 * w["d"] ** 3).sum()
    assert abs(raw[0].sum() * Vc - total) < 1e-12 * total
    assert np.all(raw[0] >= 0)


def test_pcm_single_particle_and_faces(orc):
    prm = mesh_prm(4, 4, 4, L=(4e-3, 4e-3, 4e-3))
    d = np.array([0.5e-3])
    Vc = 1e-9
    for pos, cell in (([0.5e-3, 0.5e-3, 0.5e-3], 0), ([1.0e-3, 0.5e-3, 0.5e-3], 1),
                      ([1.5e-3, 2.0e-3, 3.0e-3], (3 * 4 + 2) * 4 + 1)):
        raw = orc.deposit(prm, np.array([pos]), d, np.array([[1.0, 2.0, 3.0]]))
        nz = np.flatnonzero(raw[0])
        assert list(nz) == [cell]  # a centre on a face belongs to the upper cell
        assert raw[0, cell] == pytest.approx(math.pi / 6 * 0.5e-3 ** 3 / Vc, rel=1e-14)
        assert raw[1:, cell] == pytest.approx(np.array([1.0, 2.0, 3.0]) / Vc, rel=1e-14)


@pytest.mark.parametrize("shape,ntau,bz", [((8, 6, 5), 4, 0.0), ((16, 12, 10), 1, 0.0),
                                           ((10, 10, 24), 8, 0.0), ((12, 10, 16), 4, 0.6e-3)])
def test_diffusion_equals_spectral_solution(orc, shape, ntau, bz):
    prm = dict(mesh_prm(*shape, ntau=ntau), avg_bandwidth_z=bz)
    rng = np.random.default_rng(sum(shape))
    raw = rng.random((2, np.prod(shape))) ** 4
    out, iters = orc.diffuse(prm, raw)
    assert iters > 0
    for c in range(2):
        ref = spectral_solve(prm, raw[c])
        assert np.max(np.abs(out[c] - ref)) < 1e-12 * np.max(np.abs(raw[c]))


def test_diffusion_conservation_positivity_max_principle(orc):
    prm = mesh_prm(12, 10, 16)
    rng = np.random.default_rng(3)
    raw = np.zeros(12 * 10 * 16)
    raw[rng.choice(raw.size, 40, replace=False)] = rng.random(40)
    out, _ = orc.diffuse(prm, raw[None])
    assert abs(out.sum() - raw.sum()) < 1e-12 * raw.sum()
    assert out.min() >= 0.0
    assert out.max() <= raw.max()
    uni, _ = orc.diffuse(prm, np.full((1, raw.size), 0.37))
    assert np.max(np.abs(uni - 0.37)) < 1e-14


def gaussian_cells(prm, centre, mass):
    """Cell averages of a point source's heat kernel (variance 2 tau per axis),
    with periodic images in x, y (walls far away)."""
    from scipy.special import erf
    tau = prm["avg_bandwidth"] ** 2 / 4
    s = math.sqrt(4 * tau)
    out = []
    for ax, (L, n) in enumerate(((prm["Lx"], prm["nx"]), (prm["Ly"], prm["ny"]),
                                 (prm["Lz"], prm["nz"]))):
        edges = np.arange(n + 1) * (L / n)
        acc = np.zeros(n)
        shifts = (-1, 0, 1) if ax < 2 else (0,)
        for k in shifts:
            e = (edges - centre[ax] + k * L) / s
            acc += 0.5 * np.diff(erf(e))
        out.append(acc / (L / n))
    gx, gy, gz = out
    return mass * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]


def test_point_source_converges_to_gaussian(orc):
    b = 1.5e-3
    sigma = b / math.sqrt(2)
    L = 12 * sigma
    # pseudo-time: backward Euler -> semi-discrete (exact in time) at first order
    prm = mesh_prm(24, 24, 24, L=(L, L, L), b=b)
    src = np.zeros(24 ** 3)
    c = (12 * 24 + 12) * 24 + 12
    src[c] = 1.0
    semi = spectral_solve(prm, src, exact_time=True)
    errs = []
    for nt in (4, 8, 16, 32, 64):
        out, _ = orc.diffuse(dict(prm, avg_ntau=nt), src[None])
        errs.append(np.max(np.abs(out[0] - semi)))
    ratios = [errs[k] / errs[k + 1] for k in range(4)]
    assert all(r > 1.9 for r in ratios)  # monotone convergence
    assert 1.9 < ratios[-1] < 2.15 and ratios[-1] < ratios[-2]  # tends to first order
    # space: the semi-discrete solution -> cell-averaged Gaussian at second order
    errs = []
    for n in (24, 48, 96):
        p = mesh_prm(n, n, n, L=(L, L, L), b=b)
        h = L / n
        centre = (np.array([n // 2, n // 2, n // 2]) + 0.5) * h
        s = np.zeros(n ** 3)
        s[((n // 2) * n + n // 2) * n + n // 2] = 1.0
        sol = spectral_solve(p, s, exact_time=True)
        g = gaussian_cells(p, centre, h ** 3).ravel()  # unit value in one cell
        errs.append(np.max(np.abs(sol - g)) / g.max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r2 < 4.4 and r2 < r1 < 5.0  # tends to second order
    # and the oracle itself on the 48^3 mesh, Richardson-extrapolated in
    # pseudo-time from 16 and 32 steps, is within the mesh error (3.3%) of the
    # kernel (a wrong tau = b^2/2 would be off by ~60%)
    n = 48
    s = np.zeros(n ** 3)
    s[((n // 2) * n + n // 2) * n + n // 2] = 1.0
    o16, _ = orc.diffuse(mesh_prm(n, n, n, L=(L, L, L), b=b, ntau=16), s[None])
    o32, _ = orc.diffuse(mesh_prm(n, n, n, L=(L, L, L), b=b, ntau=32), s[None])
    p = mesh_prm(n, n, n, L=(L, L, L), b=b)
    g = gaussian_cells(p, (np.array([n // 2] * 3) + 0.5) * (L / n), (L / n) ** 3).ravel()
    ext = 2 * o32[0] - o16[0]
    assert np.max(np.abs(ext - g)) < 0.04 * g.max()


def test_diffusion_apply_matches_stencil_definition(orc):
    """orc_apply_A on a separable cosine mode returns (1 + dtau lambda) times it."""
    prm = mesh_prm(8, 6, 5)
    nx, ny, nz = 8, 6, 5
    hx, hy, hz = prm["Lx"] / nx, prm["Ly"] / ny, prm["Lz"] / nz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mode = (np.cos(2 * np.pi * 3 * i / nx) * np.cos(2 * np.pi * 1 * j / ny) *
            np.cos(np.pi * 2 * (k + 0.5) / nz)).ravel()
    lam = ((2 - 2 * math.cos(2 * math.pi * 3 / nx)) / hx ** 2 +
           (2 - 2 * math.cos(2 * math.pi / ny)) / hy ** 2 +
           (2 - 2 * math.cos(math.pi * 2 / nz)) / hz ** 2)
    dtau = 1e-7
    y = orc.apply_A(prm, dtau, mode)
    assert np.max(np.abs(y - (1 + dtau * lam) * mode)) < 1e-13


@pytest.mark.parametrize("bz_over_b", [1.0, 0.5])
def test_point_source_variance_grows_by_b2_over_2_per_axis(orc, bz_over_b):
    """Backward Euler with the discrete Laplacian raises the second moment of
    a point source by exactly 2 D_a dtau per step along each axis (sum by
    parts: the 3-point Laplacian of i^2 is 2), whatever the number of steps.
    So the variance after tau = b^2/4 is b^2/2 along x and y and, with the
    bandwidth b_z across the bed (diffusivity (b_z/b)^2), b_z^2/2 along z,
    up to the solver tolerance while the walls are far away."""
    n = 64
    b = 1.0e-3
    h = b / 4
    prm = dict(mesh_prm(n, n, n, L=(n * h, n * h, n * h), b=b, ntau=4),
               avg_bandwidth_z=(bz_over_b * b if bz_over_b != 1.0 else 0.0))
    src = np.zeros(n ** 3)
    src[((n // 2) * n + n // 2) * n + n // 2] = 1.0
    out, _ = orc.diffuse(prm, src[None])
    u = out[0].reshape(n, n, n)
    r = (np.arange(n) - n // 2) * h
    m0 = u.sum()
    assert abs(m0 - 1.0) < 1e-13
    var_x = (u.sum(axis=(0, 1)) * r ** 2).sum() / m0
    var_y = (u.sum(axis=(0, 2)) * r ** 2).sum() / m0
    var_z = (u.sum(axis=(1, 2)) * r ** 2).sum() / m0
    assert abs(var_x - b * b / 2) < 1e-9 * b * b
    assert abs(var_y - b * b / 2) < 1e-9 * b * b
    bz = bz_over_b * b
    assert abs(var_z - bz * bz / 2) < 1e-9 * b * b


def _us_case(seed, n=400, uniform=None):
    """A small bed of spheres in the lower half of a 12 x 10 x 16 mesh with
    random (or uniform) velocities."""
    prm = mesh_prm(12, 10, 16)
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3)) * [prm["Lx"], prm["Ly"], 0.5 * prm["Lz"]]
    d = rng.uniform(0.3e-3, 0.8e-3, n)
    v = np.tile(uniform, (n, 1)) if uniform is not None else rng.normal(size=(n, 3))
    return prm, x, d, v


def _smoothed_us(orc, prm, x, d, v):
    raw = np.concatenate([orc.deposit(prm, x, d)[:1], orc.deposit_flux(prm, x, d, v)])
    sm, _ = orc.diffuse(prm, raw)
    return raw, sm, orc.solid_velocity(sm[0], sm[1:])


def test_solid_velocity_of_a_uniform_motion_is_that_velocity(orc):
    """All particles moving with one velocity: the flux is that velocity
    times the solid fraction in every cell before and after the (linear)
    smoothing, so U_s equals it wherever there is solid; a transposed
    component or a wrong weight breaks the equality."""
    u0 = np.array([0.31, -0.07, 0.0123])
    prm, x, d, v = _us_case(5, uniform=u0)
    raw, sm, us = _smoothed_us(orc, prm, x, d, v)
    for e in range(3):
        assert np.max(np.abs(raw[1 + e] - u0[e] * raw[0])) < 1e-14 * raw[0].max()
    solid = sm[0] > 1e-6
    assert solid.sum() > 0.5 * solid.size
    for e in range(3):
        assert np.max(np.abs(us[e][solid] - u0[e])) < 1e-10 * abs(u0).max()
    assert np.all(us[:, sm[0] <= orc.US_EPS_MIN] == 0.0)


def test_solid_flux_conserves_momentum_and_stays_within_particle_velocities(orc):
    """sum over cells of flux V_c is the total particle volume flux, before
    and after the smoothing (zero-flux walls, periodic sides); the smoothing
    operator is a nonnegative matrix with unit column sums, so each cell's
    U_s is a convex combination of particle velocities."""
    prm, x, d, v = _us_case(6)
    raw, sm, us = _smoothed_us(orc, prm, x, d, v)
    Vc = prm["Lx"] / prm["nx"] * prm["Ly"] / prm["ny"] * prm["Lz"] / prm["nz"]
    Vp = math.pi / 6 * d ** 3
    total = (Vp[:, None] * v).sum(axis=0)
    scale = (Vp[:, None] * np.abs(v)).sum(axis=0)
    for e in range(3):
        assert abs(raw[1 + e].sum() * Vc - total[e]) < 1e-13 * scale[e]
        assert abs(sm[1 + e].sum() * Vc - total[e]) < 1e-12 * scale[e]
    solid = sm[0] > 1e-6
    for e in range(3):
        lo, hi = v[:, e].min(), v[:, e].max()
        assert np.all(us[e][solid] >= lo - 1e-9) and np.all(us[e][solid] <= hi + 1e-9)


def test_solid_velocity_single_particle_and_cell_sums(orc):
    """One sphere: the flux sits in its cell only, equal to V_p u / V_c; two
    spheres in one cell with opposite velocities and equal sizes cancel."""
    prm = mesh_prm(4, 4, 4, L=(4e-3, 4e-3, 4e-3))
    Vc = 1e-9
    d = np.array([0.5e-3])
    u = np.array([[0.2, -0.4, 1.5]])
    f = orc.deposit_flux(prm, np.array([[1.5e-3, 2.0e-3, 3.0e-3]]), d, u)
    cell = (3 * 4 + 2) * 4 + 1
    assert list(np.flatnonzero(f[0])) == [cell]
    Vp = math.pi / 6 * 0.5e-3 ** 3
    assert f[:, cell] == pytest.approx(Vp * u[0] / Vc, rel=1e-14)
    f2 = orc.deposit_flux(prm, np.array([[0.2e-3, 0.3e-3, 0.4e-3], [0.7e-3, 0.6e-3, 0.5e-3]]),
                          np.array([0.5e-3, 0.5e-3]), np.array([[1.0, 2.0, 3.0], [-1.0, -2.0, -3.0]]))
    assert np.all(f2 == 0.0)


@pytest.mark.parametrize("shape,ntau,bz", [((8, 6, 5), 4, 0.0), ((10, 10, 24), 7, 0.0),
                                           ((12, 10, 16), 3, 0.6e-3)])
def test_bdf2_equals_spectral_recurrence(orc, shape, ntau, bz):
    """BDF2 by CG in space equals the same scheme applied mode by mode after
    an FFT / DCT diagonalisation of the discrete Laplacian."""
    prm = dict(mesh_prm(*shape, ntau=ntau), avg_bandwidth_z=bz, avg_scheme=1)
    rng = np.random.default_rng(sum(shape) + 1)
    raw = rng.random((2, np.prod(shape))) ** 4
    out, _ = orc.diffuse(prm, raw)
    for c in range(2):
        ref = spectral_solve(prm, raw[c])
        assert np.max(np.abs(out[c] - ref)) < 1e-12 * np.max(np.abs(raw[c]))


def test_bdf2_is_second_order_and_euler_first_order(orc):
    """Against the exact semigroup exp(tau L_h) of the same discrete
    Laplacian, doubling the number of pseudo-time steps divides the error by
    about 4 for BDF2 and about 2 for backward Euler (a wrong BDF2
    coefficient leaves it first order or inconsistent); BDF2 also conserves the
    total and keeps a uniform field."""
    shape = (16, 12, 10)
    n = int(np.prod(shape))
    rng = np.random.default_rng(21)
    # a smooth field: a few low Fourier / cosine modes on top of a constant
    i, j, k = np.meshgrid(np.arange(16), np.arange(12), np.arange(10), indexing="ij")
    f = 1.0 + 0.3 * np.cos(2 * np.pi * i / 16) * np.cos(np.pi * (k + 0.5) / 10)
    f += 0.2 * np.sin(2 * np.pi * 2 * j / 12) + 0.1 * rng.random() * np.cos(3 * np.pi * (k + 0.5) / 10)
    raw = f.transpose(2, 1, 0).ravel()
    errs = {}
    for scheme in (0, 1):
        for N in (16, 32, 64):
            prm = dict(mesh_prm(*shape, ntau=N), avg_scheme=scheme)
            out, _ = orc.diffuse(prm, raw[None])
            exact = spectral_solve(prm, raw, exact_time=True)
            errs[scheme, N] = np.max(np.abs(out[0] - exact))
            if scheme == 1:
                assert abs(out.sum() - raw.sum()) < 1e-12 * raw.sum()
    # (the fastest mode has tau lambda ~ 5: the ratios reach 2 and 4 from
    # above as dtau lambda shrinks)
    for N in (16, 32):
        assert 1.8 < errs[0, N] / errs[0, 2 * N] < 2.2, errs
        assert 3.5 < errs[1, N] / errs[1, 2 * N] < 5.0, errs
    assert errs[1, 16] < 0.05 * errs[0, 16]
    uni, _ = orc.diffuse(dict(mesh_prm(*shape, ntau=5), avg_scheme=1), np.full((1, n), 0.37))
    assert np.max(np.abs(uni - 0.37)) < 1e-14


def test_zero_pseudo_time_steps_leave_the_field(orc):
    """avg_ntau = 0: no diffusion step is taken, the deposited field is
    returned unchanged (either scheme)."""
    prm = mesh_prm(6, 5, 4, ntau=0)
    raw = np.random.default_rng(2).random((2, 120))
    for scheme in (0, 1):
        out, iters = orc.diffuse(dict(prm, avg_scheme=scheme), raw)
        assert np.array_equal(out, raw) and iters == 0
