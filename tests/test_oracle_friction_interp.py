"""Pins of the oracle's pair friction and of its trilinear interpolation
(CPU only), each with planted errors that must make it fail.

Section 2.1 (Eq. 1b): contact forces carry tangential friction and torques on
both particles.  Section 2.3: the fluid velocity is taken at the particle
centre from the cell-centred mesh values.  What fixes the expected values:

  - rigid rotation of a pair in contact: with v = Omega x (x - c) and
    omega = Omega on both spheres, the contact points move together up to the
    overlap, so the relative tangential velocity is exactly
    delta Omega x n; a history vector in the plane of rotation then turns
    with the pair, keeps its length and grows by dt delta |Omega| per step;
  - an elastic oblique impact in gross sliding: the tangential impulse is the
    friction coefficient times the normal impulse 2 m_eff v_n, and each spin
    changes by r J_t / I about -n x t (same sense on both spheres);
  - trilinear interpolation reproduces any function a + bx + cy + dz + exy +
    fxz + gyz + hxyz between cell centres, and across a periodic seam it is
    the linear blend of the last and the first cell.
"""
import math

import numpy as np
import pytest

import workloads
from mutants import fails, mutant

D = workloads.D50
RHO = workloads.RHO_P


def _dry(**kw):
    p = workloads.base_params(nx=1, ny=1, nz=1, drag_law="none", lubrication=0,
                              fluid_forces=0, bottom_wall=0, top_wall=0, gz=0.0)
    p.update(kw)
    p["Lx"] = p["Ly"] = p["Lz"] = 8 * D
    return p


def _rec(i, j, xi):
    import oracle
    h = np.zeros(1, oracle.CONTACT_DTYPE)
    h[0]["i"], h[0]["j"], h[0]["xi"] = i, j, xi
    return h


# ---------------------------------------------------------------------------
# rigid rotation of a pair in contact
# ---------------------------------------------------------------------------
RI, RJ = 0.25e-3, 0.35e-3     # unequal radii: the torque on j must use r_j
DELTA = 1e-6                  # overlap
OMEGA = 50.0                  # rad/s about z
XI0 = 2e-8                    # initial history length (well below the Coulomb cap)


def _rigid_pair(theta):
    """Pair with its line of centres at angle theta in the xy plane, rotating
    rigidly about the centre c at OMEGA z."""
    c = np.array([4 * D, 4 * D, 4 * D])
    n = np.array([math.cos(theta), math.sin(theta), 0.0])
    dist = RI + RJ - DELTA
    xi_ = c - 0.4 * dist * n
    xj_ = c + 0.6 * dist * n
    Om = np.array([0.0, 0.0, OMEGA])
    x = np.array([xi_, xj_])
    v = np.array([np.cross(Om, xi_ - c), np.cross(Om, xj_ - c)])
    w = np.array([Om, Om])
    return x, v, w, n


def check_rigid_rotation(orc):
    prm = _dry(friction=1.0, dt=1e-5, restitution=0.9)
    kt = prm["kt_over_kn"] * prm["kn"]
    d = np.array([2 * RI, 2 * RJ])
    rho = np.full(2, RHO)
    dth = OMEGA * prm["dt"]
    th = 0.3
    # history perpendicular to the previous normal, in the plane of rotation
    t_prev = np.array([-math.sin(th - dth), math.cos(th - dth), 0.0])
    hist = _rec(0, 1, XI0 * t_prev)
    K = 400
    for k in range(K):
        x, v, w, n = _rigid_pair(th + k * dth)
        comps, hist = orc.forces(prm, x, v, w, d, rho, hist=hist)
        assert len(hist) == 1
        t = np.array([-n[1], n[0], 0.0])
        xi = hist[0]["xi"]
        want = (XI0 + (k + 1) * prm["dt"] * DELTA * OMEGA) * t
        # turns with the pair, keeps its length, grows by the slip delta Omega dt
        assert np.all(np.abs(xi - want) < 1e-9 * XI0), (k, xi, want)
        ft = comps["contact"][0] - np.dot(comps["contact"][0], n) * n
        assert np.all(np.abs(ft + kt * xi) < 1e-9 * kt * XI0)
        # torques: r_i n x F_t on i and r_j n x F_t on j, both about z
        tq_i = RI * np.cross(n, -kt * xi)
        assert np.all(np.abs(comps["torque"][0] - tq_i) < 1e-9 * np.abs(tq_i).max())
        assert np.all(np.abs(comps["torque"][1] - RJ / RI * tq_i) < 1e-9 * np.abs(tq_i).max())
    # the history has turned through K dtheta = 0.2 rad
    assert abs(math.atan2(-xi[0], xi[1]) - (th + (K - 1) * dth)) < 1e-9


def test_rigid_rotation_turns_the_history_with_the_pair(orc):
    check_rigid_rotation(orc)


# ---------------------------------------------------------------------------
# elastic oblique impact in gross sliding
# ---------------------------------------------------------------------------
def check_oblique_impact(orc):
    mu = 0.3
    di, dj = 0.5e-3, 0.7e-3
    ri, rj = 0.5 * di, 0.5 * dj
    mi, mj = RHO * math.pi / 6 * di ** 3, RHO * math.pi / 6 * dj ** 3
    meff = mi * mj / (mi + mj)
    kn = 1e3
    tc = math.pi * math.sqrt(meff / kn)
    prm = _dry(friction=mu, restitution=1.0, dt=tc / 2000, kn=kn)
    vn, vt = 2e-3, 8e-3   # v_t > 7 mu v_n: the contact slides from start to end
    gap = 2e-9
    c = 4 * D
    x = np.array([[c - 0.5 * (ri + rj + gap), c, c], [c + 0.5 * (ri + rj + gap), c, c]])
    v = np.array([[0.5 * vn, 0.5 * vt, 0.0], [-0.5 * vn, -0.5 * vt, 0.0]])
    st = orc.State(prm, x, v, np.zeros((2, 3)), np.array([di, dj]), np.full(2, RHO))
    st.init_accel()
    v0, w0 = st.v.copy(), st.w.copy()
    touched = False
    for _ in range(20000):
        st.run(1)
        if st.nhist.value > 0:
            touched = True
        elif touched:
            break
    assert touched and st.nhist.value == 0
    Jn = -mi * (st.v[0, 0] - v0[0, 0])    # along -x on i
    Jt = -mi * (st.v[0, 1] - v0[0, 1])    # along -y on i (opposes the slip)
    assert abs(Jn - 2 * meff * vn) < 1e-3 * 2 * meff * vn
    assert abs(Jt - mu * Jn) < 2e-3 * mu * Jn
    # momentum exchanged pairwise
    assert np.all(np.abs(mi * (st.v[0] - v0[0]) + mj * (st.v[1] - v0[1])) < 1e-12 * Jn)
    # spins: r J_t / I about -z (= -n x t with n = x, t = y) on both spheres
    Ii, Ij = 0.4 * mi * ri ** 2, 0.4 * mj * rj ** 2
    assert abs(st.w[0, 2] - w0[0, 2] + ri * Jt / Ii) < 2e-3 * ri * Jt / Ii
    assert abs(st.w[1, 2] - w0[1, 2] + rj * Jt / Ij) < 2e-3 * rj * Jt / Ij
    assert np.all(np.abs(st.w[:, :2]) < 1e-9 * ri * Jt / Ii)


def test_oblique_impact_impulse_and_spins(orc):
    check_oblique_impact(orc)


# ---------------------------------------------------------------------------
# trilinear interpolation (through the Stokes drag on particles at rest)
# ---------------------------------------------------------------------------
def _interp(orc, prm, Ucell, pts):
    """Interpolated U at pts: Stokes drag on tiny particles at rest is
    3 pi mu d U(x_p)."""
    dp = 1e-7
    n = len(pts)
    comps, _ = orc.forces(prm, pts, np.zeros((n, 3)), np.zeros((n, 3)), np.full(n, dp),
                          np.full(n, RHO), U=Ucell)
    return comps["drag"] / (3 * math.pi * prm["mu_f"] * dp)


def _trilinear_field(x, y, z):
    return (0.3 + 2.0 * x - 1.5 * y + 0.7 * z + 4.0 * x * y - 3.0 * x * z + 2.5 * y * z
            + 6.0 * x * y * z)


def _mesh(**kw):
    return workloads.base_params(nx=7, ny=5, nz=6, Lx=1.4, Ly=1.0, Lz=0.9, drag_law="stokes",
                                 lubrication=0, fluid_forces=0, bottom_wall=0, top_wall=0,
                                 **kw)


def check_trilinear_exact_inside(orc):
    prm = _mesh()
    xc, yc, zc = workloads.cell_centres(prm)
    U = np.zeros((len(xc), 3))
    U[:, 0] = _trilinear_field(xc, yc, zc)
    U[:, 1] = 1.0 + 3.0 * xc            # linear in x only
    U[:, 2] = 2.0 - 5.0 * yc            # linear in y only
    hx, hy, hz = prm["Lx"] / 7, prm["Ly"] / 5, prm["Lz"] / 6
    rng = np.random.default_rng(3)
    m = 200
    pts = np.stack([rng.uniform(0.5 * hx, prm["Lx"] - 0.5 * hx, m),
                    rng.uniform(0.5 * hy, prm["Ly"] - 0.5 * hy, m),
                    rng.uniform(0.5 * hz, prm["Lz"] - 0.5 * hz, m)], axis=1)
    got = _interp(orc, prm, U, pts)
    x, y, z = pts.T
    assert np.all(np.abs(got[:, 0] - _trilinear_field(x, y, z)) < 1e-12 * 20)
    assert np.all(np.abs(got[:, 1] - (1.0 + 3.0 * x)) < 1e-12 * 5)
    assert np.all(np.abs(got[:, 2] - (2.0 - 5.0 * y)) < 1e-12 * 5)
    # below the first and above the last centre the z profile is held flat
    pz = pts.copy()
    pz[:, 2] = np.where(np.arange(m) % 2 == 0, rng.uniform(0, 0.5 * hz, m),
                        rng.uniform(prm["Lz"] - 0.5 * hz, prm["Lz"], m))
    zc_clamp = np.where(np.arange(m) % 2 == 0, 0.5 * hz, prm["Lz"] - 0.5 * hz)
    got = _interp(orc, prm, U, pz)
    assert np.all(np.abs(got[:, 0] - _trilinear_field(pz[:, 0], pz[:, 1], zc_clamp)) < 2e-11)


def check_periodic_seams(orc):
    prm = _mesh()
    nx, ny, nz = 7, 5, 6
    hx, hy, hz = prm["Lx"] / nx, prm["Ly"] / ny, prm["Lz"] / nz
    rng = np.random.default_rng(4)
    F = rng.normal(size=(nz, ny, nx))
    U = np.zeros((nx * ny * nz, 3))
    U[:, 0] = F.ravel()
    m = 120
    k = rng.integers(0, nz, m)
    j = rng.integers(0, ny, m)
    i = rng.integers(0, nx, m)
    # x seam: points within half a cell of x = 0 or x = Lx, on cell centres in y and z
    t = rng.uniform(0, 1, m)
    xs = (prm["Lx"] - 0.5 * hx + t * hx) % prm["Lx"]
    pts = np.stack([xs, (j + 0.5) * hy, (k + 0.5) * hz], axis=1)
    got = _interp(orc, prm, U, pts)[:, 0]
    want = (1 - t) * F[k, j, nx - 1] + t * F[k, j, 0]
    assert np.all(np.abs(got - want) < 1e-12)
    # y seam
    ys = (prm["Ly"] - 0.5 * hy + t * hy) % prm["Ly"]
    pts = np.stack([(i + 0.5) * hx, ys, (k + 0.5) * hz], axis=1)
    got = _interp(orc, prm, U, pts)[:, 0]
    want = (1 - t) * F[k, ny - 1, i] + t * F[k, 0, i]
    assert np.all(np.abs(got - want) < 1e-12)


def test_trilinear_interpolation_is_exact_between_centres(orc):
    check_trilinear_exact_inside(orc)


def test_interpolation_wraps_across_the_x_and_y_seams(orc):
    check_periodic_seams(orc)


# ---------------------------------------------------------------------------
# planted errors: each must make its pin fail
# ---------------------------------------------------------------------------
F = "orc_forces.c"
PLANTED = {
    "sign of r_j omega_j in the contact-point velocity": (
        [(F, "+ rj * w[3 * j", "- rj * w[3 * j", 3)], [check_rigid_rotation]),
    "rotational term dropped from the relative velocity": (
        [(F, "cross3(rw, nv, rot);", "rot[0] = rot[1] = rot[2] = 0.0;")],
        [check_rigid_rotation]),
    "r_i used for the torque on j": (
        [(F, "add3(o.torque, j, r->tq, 0.5 * d[j]);", "add3(o.torque, j, r->tq, 0.5 * d[i]);")],
        [check_rigid_rotation, check_oblique_impact]),
    "history not rotated into the current tangent plane": (
        [(F, "xi[k] = xp[k] + vt[k] * p->dt;", "xi[k] = xi[k] + vt[k] * p->dt;")],
        [check_rigid_rotation]),
    "history projected but not rescaled to its length": (
        [(F, "double sc = old / pm;", "double sc = 1.0;")], [check_rigid_rotation]),
    "no Coulomb cap": (
        [(F, "if (fm > cap) {", "if (0 && fm > cap) {")], [check_oblique_impact]),
    "opposite torque sense on j": (
        [(F, "add3(o.torque, j, r->tq, 0.5 * d[j]);", "add3(o.torque, j, r->tq, -0.5 * d[j]);")],
        [check_rigid_rotation, check_oblique_impact]),
    "x cell-centre offset dropped": (
        [(F, "double sx = xp[0] / hx - 0.5,", "double sx = xp[0] / hx,")],
        [check_trilinear_exact_inside, check_periodic_seams]),
    "y cell-centre offset dropped": (
        [(F, "sy = xp[1] / hy - 0.5,", "sy = xp[1] / hy,")],
        [check_trilinear_exact_inside, check_periodic_seams]),
    "x seam clamped instead of periodic": (
        [(F, "i1 = (i0 + 1) % p->nx;", "i1 = i0 + 1 < p->nx ? i0 + 1 : i0;")],
        [check_periodic_seams]),
    "y seam clamped instead of periodic": (
        [(F, "j1 = (j0 + 1) % p->ny;", "j1 = j0 + 1 < p->ny ? j0 + 1 : j0;")],
        [check_periodic_seams]),
    "x and y weights swapped": (
        [(F, "(a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy)",
          "(a ? fy : 1.0 - fy) * (b ? fx : 1.0 - fx)")],
        [check_trilinear_exact_inside]),
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_error_fails_its_pin(tmp_path, name):
    edits, checks = PLANTED[name]
    mod = mutant(edits, tmp_path)
    for check in checks:
        assert fails(check, mod), f"{check.__name__} passes with: {name}"
