"""Graded z meshes on the GPU against the FP64 oracle (Section 4's channel
mesh, refined towards the bottom wall; cell heights growing geometrically
with z_grading = top / bottom cell height).

Bars, as on the uniform mesh: the deposited solid fraction bit-exact (the
same face search and per-cell volume, the same ID-order sums); the drag
density within 1e-12 of its largest value; smoothed fields within 1e-11 of
the deposited field's largest value with both solvers (the direct solve
diagonalises the graded z operator, the iterative one applies it), and the
solid volume sum(eps_s V_k) conserved; forces including the shear lift
(interpolated between the centres' own heights, curl over the centre
distances) within 1e-12 (FP64) and 1e-5 (FP32 forces) of the per-particle
force scale; a short coupled run following the oracle's trajectories.
"""
import math

import numpy as np
import pytest

import workloads
from gpu_helpers import dense_bed, gpu_context
from test_gpu_parity import _force_parity

pytestmark = pytest.mark.gpu


def graded_case(n, seed, grading, **kw):
    case = dense_bed(n, seed)
    prm = dict(case["params"], z_grading=grading, **kw)
    zb = workloads.bed_top(case["x"], case["d"], prm["Lx"], prm["Ly"])
    U, gradp, dudt = workloads.fluid_fields(prm, z_bed=zb, fluct=0.05, seed=seed + 11)
    return dict(case, params=prm, U=U, gradp=gradp, dudt=dudt)


def cell_volumes(prm):
    zf = workloads.z_faces(prm)
    hx, hy = prm["Lx"] / prm["nx"], prm["Ly"] / prm["ny"]
    return np.repeat(np.diff(zf), prm["nx"] * prm["ny"]) * hx * hy


@pytest.mark.parametrize("solver", ["direct", "iterative"])
@pytest.mark.parametrize("grading", [4.0, 6.0])
def test_graded_deposit_bit_exact_and_smooth(orc, grading, solver):
    case = graded_case(4000, 21, grading)
    prm = case["params"]
    comps, _ = orc.forces(prm, case["x"], case["v"], case["w"], case["d"], case["rho"],
                          U=case["U"], gradp=case["gradp"], dudt=case["dudt"])
    raw_o = orc.deposit(prm, case["x"], case["d"], comps["drag"])
    sm_o, _ = orc.diffuse(prm, raw_o)
    g = gpu_context(case, solver=solver)
    g.compute_forces()
    g.average()
    raw_g, sm_g = g.get_field(0), g.get_field(1)
    assert np.array_equal(raw_g[0], raw_o[0])
    dscale = np.abs(raw_o[1:]).max()
    assert np.abs(raw_g[1:] - raw_o[1:]).max() < 1e-12 * dscale
    err0 = np.abs(sm_g[0] - sm_o[0]).max()
    err1 = np.abs(sm_g[1:] - sm_o[1:]).max()
    print(f"grading {grading} {solver}: eps_s {err0:.2e}, drag {err1 / dscale:.2e} (rel)")
    assert err0 < 1e-11 * raw_o[0].max()
    assert err1 < 1e-11 * dscale
    V = cell_volumes(prm)
    Vp = (math.pi / 6 * case["d"] ** 3).sum()
    assert abs((raw_g[0] * V).sum() - Vp) < 1e-12 * Vp
    assert abs((sm_g[0] * V).sum() - Vp) < 1e-11 * Vp
    st = g.stats()
    assert st["solve_residual"] < 1e-11
    assert (st["solve_iters"] == 0) == (solver == "direct")


@pytest.mark.parametrize("solver", ["direct", "iterative"])
@pytest.mark.parametrize("shape,ntau,bz,grading,scheme",
                         [((16, 16, 8), 4, 0.0, 5.0, 0), ((33, 20, 17), 3, 0.0, 4.0, 0),
                          ((24, 16, 40), 2, 3.0e-3, 6.0, 0), ((20, 12, 64), 4, 0.5e-3, 5.0, 0),
                          ((16, 16, 8), 3, 0.0, 0.2, 0), ((33, 20, 17), 4, 0.0, 5.0, 1),
                          ((5, 4, 2), 3, 0.0, 4.0, 0)])
def test_graded_smooth_matches_oracle(orc, shape, ntau, bz, grading, scheme, solver):
    """Random fields on graded meshes, refined towards the bottom (grading >
    1) and, once, towards the top (0.2); z bandwidths below and above the
    horizontal one; BDF2 once; two planes only once."""
    prm = workloads.base_params(Lx=max(shape[0] * 0.3e-3, 5e-3), Ly=max(shape[1] * 0.3e-3, 5e-3),
                                Lz=shape[2] * 0.2e-3, nx=shape[0], ny=shape[1], nz=shape[2],
                                avg_ntau=ntau, avg_bandwidth_z=bz, z_grading=grading,
                                avg_scheme=scheme)
    rng = np.random.default_rng(sum(shape) + int(10 * grading))
    raw = rng.random((4, np.prod(shape))) ** 3
    want, _ = orc.diffuse(prm, raw)
    case = dict(params=prm, x=np.zeros((0, 3)), v=np.zeros((0, 3)), w=np.zeros((0, 3)),
                d=np.zeros(0), rho=np.zeros(0))
    g = gpu_context(case, cap=1, solver=solver)
    g.set_field(0, raw)
    g.smooth(4)
    got = g.get_field(1)
    st = g.stats()
    err = np.abs(got - want).max() / raw.max()
    print(f"{solver} {shape} grading {grading} scheme {scheme}: rel err {err:.2e}, "
          f"iterations {st['solve_iters']}, residual {st['solve_residual']:.2e}")
    assert err < 1e-11
    V = cell_volumes(prm)
    assert np.all(np.abs((got * V).sum(axis=1) - (raw * V).sum(axis=1)) <
                  1e-11 * (raw * V).sum(axis=1))
    if solver == "direct":
        assert st["solve_iters"] == 0


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
@pytest.mark.parametrize("grading", [4.0, 6.0])
def test_graded_forces_with_lift(orc, grading, precision, tol):
    """Every force component with the shear lift on the graded mesh: the
    fluid fields interpolated between the graded centres and the curl's z
    differences over the centre distances."""
    case = graded_case(3000, 22, grading, c_lift=1.6)
    worst = _force_parity(orc, case, precision, tol, 22)
    assert worst["lift"] < tol and worst["drag"] < tol


def test_graded_short_run_follows_the_oracle(orc):
    case = graded_case(2000, 23, 5.0, avg_ntau=2)
    prm = case["params"]
    st = orc.State(prm, case["x"], case["v"], case["w"], case["d"], case["rho"], U=case["U"],
                   gradp=case["gradp"], dudt=case["dudt"])
    st.average()
    st.init_accel()
    g = gpu_context(case)
    g.average()
    g.compute_forces(update_history=False)
    st.run(20, average_every=10)
    g.step(20, average_every=10)
    p = g.get_particles()
    dx = p["x"] - st.x
    dx[:, 0] -= prm["Lx"] * np.round(dx[:, 0] / prm["Lx"])
    dx[:, 1] -= prm["Ly"] * np.round(dx[:, 1] / prm["Ly"])
    err = np.abs(dx).max() / workloads.D50
    print(f"graded run: max |dx|/d {err:.2e}")
    assert err < 1e-9
    assert np.abs(g.get_field(1)[0] - st.avg[0]).max() < 1e-9
