"""Pins of the oracle's particle step against closed-form physics (CPU only).

Each test isolates one model of Sections 2.1, 2.3 and 2.5 and checks the
oracle's time stepping against a result fixed by mechanics, not by the code:
  - restitution coefficient and contact duration of a linear spring-dashpot
    (two spheres head on, and a sphere on a wall);
  - a sliding sphere reaches rolling at v = 5/7 v0 after t = 2 v0/(7 mu g);
  - the lubrication squeeze force stops a sphere at h0 exp(-m v0/(6 pi mu r^2));
  - Stokes settling with buoyancy and added mass: v_t = (rho_p - rho_f) g d^2/(18 mu)
    reached with time constant (rho_p + C_add rho_f) d^2/(18 mu);
  - Di Felice drag tends to Stokes drag (within its 4% low-Re offset);
  - an elastic, frictionless gas conserves energy and momentum.
"""
import math

import numpy as np
import pytest

import workloads

D = workloads.D50
RHO = workloads.RHO_P


def dry(**kw):
    """No fluid, no gravity, no walls, no friction unless asked."""
    p = workloads.base_params(nx=1, ny=1, nz=1, drag_law="none", lubrication=0,
                              fluid_forces=0, bottom_wall=0, top_wall=0, gz=0.0,
                              friction=0.0)
    p.update(kw)
    return p


def mass(d=D, rho=RHO):
    return rho * math.pi / 6 * d ** 3


def analytic_e_tc(kn, e, meff):
    le = math.log(e)
    zeta = -le / math.sqrt(math.pi ** 2 + le ** 2)
    gam = 2 * zeta * math.sqrt(meff * kn)
    wd = math.sqrt(kn / meff - (gam / (2 * meff)) ** 2)
    return math.exp(-math.pi * zeta / math.sqrt(1 - zeta ** 2)), math.pi / wd


def head_on(orc, dt_frac, e=0.9):
    m = mass()
    _, tc = analytic_e_tc(1e3, e, m / 2)
    prm = dry(restitution=e, dt=tc * dt_frac)
    v0 = 0.05
    gap = 1e-6
    xc = 0.5 * prm["Lx"]
    x = np.array([[xc - 0.5 * D - gap, 1e-3, 2e-3], [xc + 0.5 * D + gap, 1e-3, 2e-3]])
    v = np.array([[v0, 0, 0], [-v0, 0, 0]])
    st = orc.State(prm, x, v, np.zeros((2, 3)), np.full(2, D), np.full(2, RHO))
    st.init_accel()
    steps_in = 0
    t_total = 0
    while True:
        st.run(1)
        t_total += 1
        dist = st.x[1, 0] - st.x[0, 0]
        if dist < D:
            steps_in += 1
        elif steps_in > 0:
            break
        assert t_total < 10 * tc / prm["dt"] + 1000
    vrel_after = st.v[1, 0] - st.v[0, 0]
    return vrel_after / (2 * v0), steps_in * prm["dt"]


def test_head_on_restitution_and_contact_time(orc):
    e_an, tc_an = analytic_e_tc(1e3, 0.9, mass() / 2)
    assert abs(tc_an - 2.927e-5) < 0.01e-5  # value quoted for d = 0.5 mm, k = 1e3 N/m
    errs = []
    for frac in (1 / 200, 1 / 400, 1 / 800):
        e_sim, tc_sim = head_on(orc, frac)
        errs.append(abs(e_sim - e_an))
        assert abs(tc_sim - tc_an) <= 2 * frac * tc_an
    assert errs[-1] < 2e-3
    # convergence in dt
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]


@pytest.mark.parametrize("e", [0.5, 0.97])
def test_head_on_other_restitution(orc, e):
    e_an, _ = analytic_e_tc(1e3, e, mass() / 2)
    e_sim, _ = head_on(orc, 1 / 1000, e=e)
    assert abs(e_sim - e_an) < 3e-3


def test_wall_bounce_restitution(orc):
    m = mass()
    e_an, tc_an = analytic_e_tc(1e3, 0.9, m)
    assert abs(tc_an - 4.140e-5) < 0.01e-5
    prm = dry(bottom_wall=1, dt=tc_an / 1000)
    v0 = 0.03
    x = np.array([[1e-3, 1e-3, 0.5 * D + 1e-7]])
    st = orc.State(prm, x, np.array([[0, 0, -v0]]), np.zeros((1, 3)), np.full(1, D),
                   np.full(1, RHO))
    st.init_accel()
    touched = False
    for _ in range(20000):
        st.run(1)
        if st.x[0, 2] < 0.5 * D:
            touched = True
        elif touched:
            break
    assert touched
    assert abs(st.v[0, 2] / v0 - e_an) < 3e-3


def test_sliding_to_rolling(orc):
    """Coulomb friction + rotation: a sphere launched sliding on a wall
    decelerates at mu g and rolls at 5/7 v0 from t* = 2 v0 / (7 mu g)."""
    mu, g, v0 = 0.3, 9.81, 0.1
    m = mass()
    prm = dry(bottom_wall=1, friction=mu, gz=-g, dt=1e-6)
    z0 = 0.5 * D - m * g / prm["kn"]  # static overlap
    st = orc.State(prm, np.array([[1e-3, 1e-3, z0]]), np.array([[v0, 0, 0]]),
                   np.zeros((1, 3)), np.full(1, D), np.full(1, RHO))
    st.init_accel()
    t_star = 2 * v0 / (7 * mu * g)
    n_half = int(0.5 * t_star / prm["dt"])
    st.run(n_half)
    v_half = st.v[0, 0]
    assert abs(v_half - (v0 - mu * g * n_half * prm["dt"])) < 2e-3 * v0
    st.run(int(1.5 * t_star / prm["dt"]) - n_half)
    vs, ws = [], []
    for _ in range(200):
        st.run(5)
        vs.append(st.v[0, 0])
        ws.append(st.w[0, 1])
    v_end, w_end = np.mean(vs), np.mean(ws)
    assert abs(v_end - 5 / 7 * v0) < 1e-3 * v0
    # rolling without slip: v = w r, with w about +y for motion along +x
    assert abs(w_end * 0.5 * D - v_end) < 2e-3 * v0


def test_lubrication_stop_distance(orc):
    """Squeeze-film approach to a wall: m dv/dt = -6 pi mu r^2 v / h
    integrates to h_f = h0 exp(-m v0 / (6 pi mu r^2))."""
    m = mass()
    r = 0.5 * D
    mu = workloads.MU_F
    v0 = 0.01
    prm = dry(bottom_wall=1, lubrication=1, dt=5e-7)
    h0 = prm["lub_out_frac"] * D * (1 - 1e-9)
    hf = h0 * math.exp(-m * v0 / (6 * math.pi * mu * r * r))
    assert abs(hf / h0 - 0.229) < 0.002  # value quoted for d = 0.5 mm, v0 = 1 cm/s
    assert hf > prm["lub_in_frac"] * D
    st = orc.State(prm, np.array([[1e-3, 1e-3, r + h0]]), np.array([[0, 0, -v0]]),
                   np.zeros((1, 3)), np.full(1, D), np.full(1, RHO))
    st.init_accel()
    st.run(80000)  # ~50 time constants of the final exponential approach
    h = st.x[0, 2] - r
    assert abs(st.v[0, 2]) < 1e-4 * v0
    assert abs(h - hf) < 2e-3 * h0


def stokes_setup(orc, c_add, dt):
    d = 50e-6
    g = 9.81
    prm = workloads.base_params(nx=1, ny=1, nz=1, drag_law="stokes", lubrication=0,
                                fluid_forces=1, bottom_wall=0, top_wall=0, c_add=c_add,
                                dt=dt, Lz=0.1)
    gradp = np.array([[0.0, 0.0, prm["rho_f"] * -g]])  # hydrostatic
    st = orc.State(prm, np.array([[1e-3, 1e-3, 0.09]]), np.zeros((1, 3)), np.zeros((1, 3)),
                   np.full(1, d), np.full(1, RHO), U=np.zeros((1, 3)), gradp=gradp,
                   dudt=np.zeros((1, 3)))
    st.init_accel()
    return st, d, g


def test_stokes_terminal_velocity_and_time_constant(orc):
    mu = workloads.MU_F
    rf = workloads.RHO_F
    vt = (RHO - rf) * 9.81 * (50e-6) ** 2 / (18 * mu)
    assert abs(vt - 2.248e-3) < 0.001e-3
    tau = (RHO + 0.5 * rf) * (50e-6) ** 2 / (18 * mu)
    errs = []
    for dt in (tau / 100, tau / 200):
        st, d, g = stokes_setup(orc, 0.5, dt)
        n1 = int(round(tau / dt))
        st.run(n1)
        v_tau = -st.v[0, 2]
        errs.append(abs(v_tau - vt * (1 - math.exp(-1))))
        st.run(20 * n1)
        assert abs(-st.v[0, 2] - vt) < 1e-9
    assert errs[-1] < 0.01 * vt
    assert errs[1] < 0.7 * errs[0]  # the lagged added mass converges with dt


def test_added_mass_slows_the_approach(orc):
    """Added mass raises the inertia (Section 4.1): the velocity after one
    Stokes time of the bare particle is lower with C_add = 0.5."""
    tau0 = RHO * (50e-6) ** 2 / (18 * workloads.MU_F)
    v = []
    for c in (0.0, 0.5):
        st, _, _ = stokes_setup(orc, c, tau0 / 200)
        st.run(200)
        v.append(-st.v[0, 2])
    vt = (RHO - workloads.RHO_F) * 9.81 * (50e-6) ** 2 / (18 * workloads.MU_F)
    assert abs(v[0] - vt * (1 - math.exp(-1))) < 0.01 * vt
    assert v[1] < v[0]


def test_difelice_tends_to_stokes_at_low_re(orc):
    """C_d = (0.63 + 4.8/sqrt(Re))^2 -> 23.04/Re as Re -> 0, i.e. 0.96 x Stokes."""
    prm = workloads.base_params(nx=1, ny=1, nz=1, drag_law="difelice", lubrication=0,
                                fluid_forces=0, bottom_wall=0, top_wall=0)
    d = 10e-6
    U = np.array([[1e-6, 0.0, 0.0]])  # Re = 1e-5
    x = np.array([[1e-3, 1e-3, 1e-3]])
    comps, _ = orc.forces(prm, x, np.zeros((1, 3)), np.zeros((1, 3)), np.full(1, d),
                          np.full(1, RHO), U=U)
    stokes = 3 * math.pi * workloads.MU_F * d * 1e-6
    ratio = comps["drag"][0, 0] / stokes
    assert abs(ratio - 0.96) < 0.005
    # drag points towards the fluid velocity (force on the particle)
    assert comps["drag"][0, 0] > 0


def test_difelice_terminal_velocity_matches_scalar_balance(orc):
    """d = 0.5 mm sand settling in still water: the stepped terminal velocity
    equals the root of (rho_p - rho_f) V g = f_drag(v) at eps_f = 1."""
    from scipy.optimize import brentq
    d = D
    rf, mu = workloads.RHO_F, workloads.MU_F
    V = math.pi / 6 * d ** 3

    def fd(v):
        Re = rf * d * v / mu
        cd = (0.63 + 4.8 / math.sqrt(Re)) ** 2
        return 0.5 * cd * rf * math.pi * d * d / 4 * v * v

    vt = brentq(lambda v: fd(v) - (RHO - rf) * V * 9.81, 1e-4, 1.0)
    assert 0.05 < vt < 0.09  # the usual 6-8 cm/s for medium sand
    prm = workloads.base_params(nx=1, ny=1, nz=1, drag_law="difelice", lubrication=0,
                                fluid_forces=1, bottom_wall=0, top_wall=0, dt=2e-5, Lz=1.0)
    st = orc.State(prm, np.array([[1e-3, 1e-3, 0.99]]), np.zeros((1, 3)), np.zeros((1, 3)),
                   np.full(1, d), np.full(1, RHO), U=np.zeros((1, 3)),
                   gradp=np.array([[0, 0, -rf * 9.81]]), dudt=np.zeros((1, 3)))
    st.init_accel()
    st.run(10000)
    assert abs(-st.v[0, 2] - vt) < 1e-6 * vt


def test_elastic_gas_conserves_energy_and_momentum(orc):
    n = 150
    prm = dry(restitution=1.0, bottom_wall=1, top_wall=1)
    m = mass()
    _, tc = analytic_e_tc(1e3, 0.999999, m / 2)
    prm["dt"] = tc / 100
    d = np.full(n, D)
    x = workloads.rsa(n, d, prm["Lx"], prm["Ly"], prm["Lz"], seed=5)
    rng = np.random.default_rng(5)
    v = rng.normal(scale=0.05, size=(n, 3))
    st = orc.State(prm, x, v, np.zeros((n, 3)), d, np.full(n, RHO))
    st.init_accel()

    def energy():
        ke = 0.5 * m * (st.v ** 2).sum()
        pe = 0.0
        pr = orc.pairs_brute(dict(prm, lub_out_frac=0.0), st.x, d)
        for i, j in pr:
            dx = st.x[j] - st.x[i]
            dx[0] -= prm["Lx"] * round(dx[0] / prm["Lx"])
            dx[1] -= prm["Ly"] * round(dx[1] / prm["Ly"])
            pe += 0.5 * prm["kn"] * (D - np.linalg.norm(dx)) ** 2
        for z in st.x[:, 2]:
            for dl in (0.5 * D - z, 0.5 * D - (prm["Lz"] - z)):
                if dl > 0:
                    pe += 0.5 * prm["kn"] * dl ** 2
        return ke + pe

    # energy is measured at synchronized velocities (after a full step)
    e0 = energy()
    p0 = m * st.v[:, :2].sum(axis=0)
    es = []
    for _ in range(10):
        st.run(300)
        es.append(energy())
    drift = max(abs(e - e0) for e in es) / e0
    assert drift < 2e-3
    p1 = m * st.v[:, :2].sum(axis=0)
    assert np.all(np.abs(p1 - p0) < 1e-12 * m * 0.05 * n)
    assert st.nhist.value >= 0


def test_pair_forces_are_antisymmetric(orc):
    """Contact + lubrication forces on a periodic, wall-free bed sum to zero."""
    w = workloads.workload("small")
    prm = dict(w["params"], bottom_wall=0, top_wall=0, drag_law="none", fluid_forces=0)
    x = w["x"].copy()
    # squeeze the spheres together to create contacts and lubrication pairs
    x[:, 2] *= 0.6
    rng = np.random.default_rng(1)
    v = rng.normal(scale=0.01, size=x.shape)
    wv = rng.normal(scale=10.0, size=x.shape)
    comps, hist = orc.forces(prm, x, v, wv, w["d"], w["rho"])
    s = comps["contact"].sum(axis=0) + comps["lub"].sum(axis=0)
    scale = np.abs(comps["contact"]).sum() + np.abs(comps["lub"]).sum()
    assert scale > 0
    assert np.all(np.abs(s) < 1e-13 * scale)


def _one_particle_drag(orc, law, U, eps_s, d=D):
    """Drag on one particle at rest in a uniform flow U on a one-cell mesh
    whose smoothed solid fraction is eps_s."""
    prm = workloads.base_params(nx=1, ny=1, nz=1, drag_law=law, lubrication=0,
                                fluid_forces=0, bottom_wall=0, top_wall=0, eps_s_max=0.7)
    x = np.array([[1e-3, 1e-3, 1e-3]])
    comps, _ = orc.forces(prm, x, np.zeros((1, 3)), np.zeros((1, 3)), np.full(1, d),
                          np.full(1, RHO), U=np.array([U]), eps_s=np.array([eps_s]))
    return comps["drag"][0]


def test_syamlal_single_sphere_is_dalla_valle(orc):
    """At eps_f = 1, A1 = A2 = 1 and V_r = 1: the correlation reduces to the
    single-sphere drag 1/2 C_d rho_f (pi d^2/4) |w| w, C_d = (0.63 + 4.8/sqrt(Re))^2."""
    rf, mu = workloads.RHO_F, workloads.MU_F
    for Re in (0.01, 1.0, 50.0, 2000.0):
        wm = Re * mu / (rf * D)
        f = _one_particle_drag(orc, "syamlal", [wm, 0.0, 0.0], 0.0)
        cd = (0.63 + 4.8 / math.sqrt(Re)) ** 2
        want = 0.5 * cd * rf * math.pi * D * D / 4 * wm * wm
        assert f[0] > 0 and f[1] == 0 and f[2] == 0
        assert abs(f[0] - want) < 1e-13 * want, Re


@pytest.mark.parametrize("eps_f", [0.5, 0.8, 0.95])
def test_syamlal_low_re_is_hindered_stokes(orc, eps_f):
    """Re -> 0: V_r -> A1 = eps_f^4.14 and C_d -> 23.04 V_r/Re, so the drag
    tends to 0.96 x Stokes / eps_f^4.14 (Richardson-Zaki hindering)."""
    rf, mu = workloads.RHO_F, workloads.MU_F
    wm = 1e-8 * mu / (rf * D)
    f = _one_particle_drag(orc, "syamlal", [0.0, wm, 0.0], 1.0 - eps_f)
    ratio = f[1] / (3 * math.pi * mu * D * wm)
    assert abs(ratio - 0.96 / eps_f ** 4.14) < 1e-3 * ratio


@pytest.mark.parametrize("eps_f", [0.5, 0.8, 0.9])
def test_syamlal_high_re_is_hindered_newton(orc, eps_f):
    """Re -> infinity: V_r -> A2 (0.8 eps_f^1.28 up to 0.85, eps_f^2.65 above)
    and C_d -> 0.63^2, so the drag tends to the Newton-regime drag / A2^2."""
    rf, mu = workloads.RHO_F, workloads.MU_F
    wm = 1e9 * mu / (rf * D)
    f = _one_particle_drag(orc, "syamlal", [0.0, 0.0, -wm], 1.0 - eps_f)
    A2 = 0.8 * eps_f ** 1.28 if eps_f <= 0.85 else eps_f ** 2.65
    newton = 0.5 * 0.63 ** 2 * rf * math.pi * D * D / 4 * wm * wm
    assert f[2] < 0
    assert abs(-f[2] / newton - 1.0 / A2 ** 2) < 2e-3 / A2 ** 2


def _lift_case(orc, Ufun, v=(0.0, 0.0, 0.0), zp=0.37e-3, c_lift=1.6):
    """One particle in a frozen field U(x, y, z) sampled at cell centres of a
    4 x 4 x 8 mesh (walls at z = 0 and 2 mm); only the lift is on."""
    prm = workloads.base_params(nx=4, ny=4, nz=8, Lx=2e-3, Ly=2e-3, Lz=2e-3, drag_law="none",
                                lubrication=0, fluid_forces=0, bottom_wall=0, top_wall=0,
                                c_lift=c_lift)
    h = 2e-3 / np.array([4, 4, 8])
    k, j, i = np.meshgrid(np.arange(8), np.arange(4), np.arange(4), indexing="ij")
    cx, cy, cz = (i + 0.5) * h[0], (j + 0.5) * h[1], (k + 0.5) * h[2]
    U = np.stack(Ufun(cx.ravel(), cy.ravel(), cz.ravel()), axis=1)
    x = np.array([[0.71e-3, 1.13e-3, 1e-3 + zp]])
    comps, _ = orc.forces(prm, x, np.array([v]), np.zeros((1, 3)), np.full(1, D), np.full(1, RHO),
                          U=U)
    return comps, x[0]


def test_lift_in_linear_shear_is_saffman(orc):
    """U = (g z, 0, 0): the discrete curl is exact, omega = (0, g, 0); a particle
    at rest lags the flow by s = g z and is lifted towards the faster fluid with
    Saffman's 6.46 mu a^2 s (g/nu)^(1/2) (C_l = 1.6 is its 1.615, rounded)."""
    g = 40.0
    comps, xp = _lift_case(orc, lambda x, y, z: (g * z, 0 * z, 0 * z))
    f = comps["lift"][0]
    s = g * xp[2]
    nu = workloads.MU_F / workloads.RHO_F
    saffman = 6.46 * workloads.MU_F * (D / 2) ** 2 * s * math.sqrt(g / nu)
    assert f[0] == 0 and f[1] == 0 and f[2] > 0
    assert abs(f[2] / saffman - 1.0) < 0.01
    assert abs(f[2] - 1.6 * workloads.RHO_F * math.sqrt(nu) * D * D * s * math.sqrt(g)) < 1e-12 * f[2]
    mg = RHO * math.pi / 6 * D ** 3 * 9.81
    assert np.allclose(comps["total"][0], f - np.array([0, 0, mg]), rtol=0, atol=1e-15 * mg)


def test_lift_is_perpendicular_to_slip_and_vorticity(orc):
    """U = (g1 z, g2 z, 0): omega = (-g2, g1, 0) exactly, perpendicular to the
    slip; the lift is perpendicular to both with magnitude
    C_l rho_f nu^(1/2) d^2 |w| |omega|^(1/2)."""
    g1, g2 = 30.0, -55.0
    comps, xp = _lift_case(orc, lambda x, y, z: (g1 * z, g2 * z, 0 * z))
    f = comps["lift"][0]
    w = np.array([g1, g2, 0.0]) * xp[2]
    om = np.array([-g2, g1, 0.0])
    nu = workloads.MU_F / workloads.RHO_F
    want = 1.6 * workloads.RHO_F * math.sqrt(nu) * D * D * np.linalg.norm(w) * math.sqrt(np.linalg.norm(om))
    assert abs(np.linalg.norm(f) - want) < 1e-12 * want
    assert abs(f @ w) < 1e-12 * want * np.linalg.norm(w)
    assert abs(f @ om) < 1e-12 * want * np.linalg.norm(om)


def test_lift_vanishes_without_vorticity_or_slip(orc):
    comps, _ = _lift_case(orc, lambda x, y, z: (0 * z + 0.3, 0 * z - 0.1, 0 * z))
    assert not comps["lift"].any()  # uniform flow: no vorticity
    g = 40.0
    zp = 0.37e-3
    comps, xp = _lift_case(orc, lambda x, y, z: (g * z, 0 * z, 0 * z), v=(g * (1e-3 + zp), 0, 0),
                           zp=zp)
    assert np.abs(comps["lift"]).max() < 1e-12 * RHO * D ** 3  # moving with the fluid
    comps, _ = _lift_case(orc, lambda x, y, z: (g * z, 0 * z, 0 * z), c_lift=0.0)
    assert not comps["lift"].any()


def test_lift_curl_wraps_periodically_and_takes_the_discrete_derivative(orc):
    """U = (A sin(2 pi y / Ly), 0, 0) on the 4-cell periodic y axis: at the
    cell centre next to the seam (j = 0) the central difference reaches
    across it, and the discrete curl is omega_z = -A sin(k h)/h cos(k y_c)
    (k = 2 pi / Ly), not the continuous -A k cos(k y_c).  A particle at rest
    at that centre lags the flow by s = A sin(k y_c), and the lift is
    C_l rho_f nu^(1/2) d^2 |omega_z|^(1/2) s along -sign(omega_z) y."""
    A, L, ny = 0.08, 2e-3, 4
    kk, h = 2 * math.pi / L, L / ny
    yc = 0.5 * h
    prm = workloads.base_params(nx=4, ny=ny, nz=8, Lx=L, Ly=L, Lz=2e-3, drag_law="none",
                                lubrication=0, fluid_forces=0, bottom_wall=0, top_wall=0,
                                c_lift=1.6)
    k, j, i = np.meshgrid(np.arange(8), np.arange(ny), np.arange(4), indexing="ij")
    cy = (j + 0.5) * h
    U = np.stack([A * np.sin(kk * cy.ravel()), 0 * cy.ravel(), 0 * cy.ravel()], axis=1)
    x = np.array([[2.5 * (L / 4), yc, 4.5 * (2e-3 / 8)]])  # a cell centre, j = 0
    comps, _ = orc.forces(prm, x, np.zeros((1, 3)), np.zeros((1, 3)), np.full(1, D),
                          np.full(1, RHO), U=U)
    f = comps["lift"][0]
    om = -A * math.sin(kk * h) / h * math.cos(kk * yc)
    s = A * math.sin(kk * yc)
    nu = workloads.MU_F / workloads.RHO_F
    want = 1.6 * workloads.RHO_F * math.sqrt(nu) * D * D / math.sqrt(abs(om)) * (-s * om)
    assert f[0] == 0 and f[2] == 0
    assert abs(f[1] - want) < 1e-12 * abs(want)
    # the continuous derivative would give a different value: the pin is sharp
    om_c = -A * kk * math.cos(kk * yc)
    want_c = 1.6 * workloads.RHO_F * math.sqrt(nu) * D * D / math.sqrt(abs(om_c)) * (-s * om_c)
    assert abs(want_c - want) > 1e-3 * abs(want)


def _difelice_force(orc, d, w, eps_f):
    prm = workloads.base_params(nx=1, ny=1, nz=1, drag_law="difelice", lubrication=0,
                                fluid_forces=0, bottom_wall=0, top_wall=0)
    comps, _ = orc.forces(prm, np.array([[1e-3, 1e-3, 1e-3]]), np.zeros((1, 3)), np.zeros((1, 3)),
                          np.full(1, d), np.full(1, RHO), U=np.array([[w, 0.0, 0.0]]),
                          eps_s=np.array([1.0 - eps_f]))
    return comps["drag"][0, 0]


def test_difelice_in_a_suspension_low_re_limit(orc):
    """eps_f < 1 as Re -> 0: chi -> 3.7 and C_d -> 23.04/Re with Re carrying
    eps_f, so the force tends to 0.96 eps_f^(-2.7) times the Stokes drag."""
    d, w = 10e-6, 1e-6
    for eps_f in (0.9, 0.6, 0.45):
        f = _difelice_force(orc, d, w, eps_f)
        ratio = f / (3 * math.pi * workloads.MU_F * d * w)
        assert abs(ratio / (0.96 * eps_f ** -2.7) - 1) < 2e-3, (eps_f, ratio)


def test_difelice_voidage_factor_at_fixed_reynolds_number(orc):
    """At a fixed particle Reynolds number (Re carries eps_f, so the slip is
    w = Re mu / (rho_f d eps_f)) C_d and chi are fixed and the force scales
    as eps_f^(2 - chi) w^2 ~ eps_f^(-chi); at log10 Re = 1.5 the exponent is
    exactly chi = 3.7 - 0.65 = 3.05."""
    d = D
    Re = 10 ** 1.5
    f = {}
    for eps_f in (0.9, 0.5):
        w = Re * workloads.MU_F / (workloads.RHO_F * d * eps_f)
        f[eps_f] = _difelice_force(orc, d, w, eps_f)
    assert abs(f[0.5] / f[0.9] / (0.5 / 0.9) ** -3.05 - 1) < 1e-12
