"""Shared set-up for the GPU parity tests: seeded inputs fed to both the HIP
library (through its C ABI) and the oracle."""
import math

import numpy as np

import workloads


def dense_bed(n, seed, poly=True, jitter=0.002, Lfac=1.0):
    """A deposited bed jittered so that it has overlaps, with random
    translational and angular velocities."""
    d = workloads.lognormal_diameters(n, seed) if poly else np.full(n, workloads.D50)
    L = math.sqrt(n / 2000) * 20 * workloads.D50 * Lfac
    prm = workloads.base_params(Lx=L, Ly=L, Lz=14 * workloads.D50, nx=max(3, int(L / (1.25 * workloads.D50))),
                                ny=max(3, int(L / (1.25 * workloads.D50))), nz=11)
    x = workloads.rsd_bed(n, d, L, L, seed)
    rng = np.random.default_rng(seed + 7)
    x = x + rng.normal(scale=jitter * workloads.D50, size=x.shape)
    x[:, 0] %= L
    x[:, 1] %= L
    x[:, 2] = np.clip(x[:, 2], 0.3 * d, prm["Lz"] - 0.5 * d)
    v = rng.normal(scale=0.01, size=(n, 3))
    w = rng.normal(scale=20.0, size=(n, 3))
    zb = workloads.bed_top(x, d, L, L)
    U, gradp, dudt = workloads.fluid_fields(prm, z_bed=zb, fluct=0.05, seed=seed + 11)
    return dict(params=prm, x=x, v=v, w=w, d=d, rho=np.full(n, workloads.RHO_P), U=U,
                gradp=gradp, dudt=dudt)


def gpu_context(case, precision="fp64", skin_frac=0.1, max_neighbors=24, cap=None,
                solver="auto"):
    import paper_1601_03801_amd as sm
    prm = dict(case["params"])
    dmax = float(np.max(case["d"])) if len(case["d"]) else workloads.D50
    n = len(case["d"])
    g = sm.Sedimi(prm, cap if cap is not None else max(n, 1), precision=precision,
                  d_max=dmax, skin=skin_frac * dmax, max_neighbors=max_neighbors,
                  solver=solver)
    g.set_fluid(case.get("U"), case.get("gradp"), case.get("dudt"))
    g.set_particles(case["x"], case["v"], case["d"], case["rho"], omega=case.get("w"))
    return g


def rel_err(a, b, scale):
    """Per-particle |a - b| / scale, scale a per-particle magnitude."""
    return np.linalg.norm(a - b, axis=1) / np.maximum(scale, 1e-300)
