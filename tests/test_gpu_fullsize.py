"""Parity at the full workload sizes (the 1M-sphere bed in FP64, the
10M-sphere bed in mixed precision), in the launch configuration bench.py
times: skin 0.1 d_max, 24 neighbour slots, whole bed resident.

The oracle cannot evaluate a whole bed quickly, so it evaluates local
patches: every particle within reach of a sample of particles.  A sampled
particle's pair set, forces and contact history depend only on particles
within its pair range, so its outputs from the patch equal those from the
whole bed.  All inputs (velocities, spins, the previous acceleration, the
smoothed solid fraction) are seeded and synthetic; nothing fed to the oracle
comes from the GPU.
"""
import math

import numpy as np
import pytest

import workloads
from gpu_helpers import rel_err

pytestmark = pytest.mark.gpu

_BEDS = {}


def _bed(name):
    if name not in _BEDS:
        print(f"generating {name}", flush=True)
        w = workloads.workload(name)
        n = len(w["d"])
        rng = np.random.default_rng(77)
        w["v"] = rng.normal(scale=0.01, size=(n, 3))
        w["w"] = rng.normal(scale=20.0, size=(n, 3))
        w["a_prev"] = rng.normal(scale=1.0, size=(n, 3))
        ncell = np.prod(w["meta"]["mesh"])
        sm = np.zeros((4, ncell))
        sm[0] = 0.6 * rng.random(ncell)
        w["smooth"] = sm
        _BEDS[name] = w
    return _BEDS[name]


def _samples(w, count, seed):
    """Random particles plus some at the periodic seams and at the walls."""
    prm = w["params"]
    x, d = w["x"], w["d"]
    rng = np.random.default_rng(seed)
    n = len(d)
    pick = list(rng.choice(n, count, replace=False))
    for mask in (x[:, 0] < d, x[:, 0] > prm["Lx"] - d, x[:, 1] < d, x[:, 1] > prm["Ly"] - d,
                 x[:, 2] < 0.6 * d):
        idx = np.flatnonzero(mask)
        if len(idx):
            pick += list(rng.choice(idx, min(10, len(idx)), replace=False))
    return np.unique(np.array(pick, dtype=np.int64))


def _patch(w, samples, reach):
    """Indices of every particle within `reach` (minimum image in x, y) of a
    sample, the samples included."""
    prm = w["params"]
    x = w["x"]
    Lx, Ly = prm["Lx"], prm["Ly"]
    nbx, nby = int(Lx // reach), int(Ly // reach)
    nbz = max(1, int(prm["Lz"] // reach))
    bx = np.minimum((x[:, 0] / Lx * nbx).astype(np.int64), nbx - 1)
    by = np.minimum((x[:, 1] / Ly * nby).astype(np.int64), nby - 1)
    bz = np.clip((x[:, 2] / prm["Lz"] * nbz).astype(np.int64), 0, nbz - 1)
    key = (bz * nby + by) * nbx + bx
    order = np.argsort(key, kind="stable")
    skey = key[order]
    keep = [samples]
    for s in samples:
        cand = []
        for dz in (-1, 0, 1):
            cz = bz[s] + dz
            if cz < 0 or cz >= nbz:
                continue
            for dy in (-1, 0, 1):
                cy = (by[s] + dy) % nby
                for dx in (-1, 0, 1):
                    cx = (bx[s] + dx) % nbx
                    k = (cz * nby + cy) * nbx + cx
                    lo, hi = np.searchsorted(skey, [k, k + 1])
                    cand.append(order[lo:hi])
        cand = np.concatenate(cand)
        dxy = x[cand] - x[s]
        dxy[:, 0] -= Lx * np.round(dxy[:, 0] / Lx)
        dxy[:, 1] -= Ly * np.round(dxy[:, 1] / Ly)
        keep.append(cand[np.einsum("ij,ij->i", dxy, dxy) < reach * reach])
    return np.unique(np.concatenate(keep))


def _context(w, precision, prm=None):
    import paper_1601_03801_amd as sm
    dmax = float(w["d"].max())
    g = sm.Sedimi(prm or w["params"], len(w["d"]), precision=precision, d_max=dmax,
                  skin=0.1 * dmax, max_neighbors=24)
    g.set_fluid(w["U"], w["gradp"], w["dudt"])
    g.set_particles(w["x"], w["v"], w["d"], w["rho"], omega=w["w"])
    return g


@pytest.mark.parametrize("name,precision,tol,opts", [
    ("bed1m", "fp64", 1e-12, {}),
    ("bed10m", "mixed", 1e-5, {}),
    ("bed1m", "fp64", 1e-12, {"c_lift": 1.6, "drag_law": "syamlal"})])
def test_fullsize_forces_on_sampled_particles(orc, name, precision, tol, opts):
    """opts: the shear lift and the Syamlal-O'Brien drag (bench.py --lift 1.6
    --drag syamlal)."""
    w = _bed(name)
    prm = dict(w["params"], **opts)
    print(f"{name}: {len(w['d'])} spheres, context ({precision}, {opts})", flush=True)
    g = _context(w, precision, prm)
    g.set_field(1, w["smooth"])
    g.set_accel(w["a_prev"])
    g.compute_forces(update_history=True)
    samples = _samples(w, 300, 5)
    reach = 1.3 * float(w["d"].max())
    patch = _patch(w, samples, reach)
    print(f"{len(samples)} samples, patch of {len(patch)} spheres", flush=True)
    sub = lambda a: a[patch]  # noqa: E731
    comps, hout = orc.forces(prm, sub(w["x"]), sub(w["v"]), sub(w["w"]), sub(w["d"]),
                             sub(w["rho"]), a_prev=sub(w["a_prev"]), U=w["U"],
                             gradp=w["gradp"], dudt=w["dudt"], eps_s=w["smooth"][0])
    loc = np.searchsorted(patch, samples)
    m = w["rho"][samples] * math.pi / 6 * w["d"][samples] ** 3
    scale = sum(np.linalg.norm(comps[k][loc], axis=1) for k in
                ("contact", "lub", "drag", "pressure", "added", "lift")) + m * 9.81
    if opts.get("c_lift"):
        assert np.abs(comps["lift"][loc]).max() > 0.0
    table = {}
    for k in ("contact", "lub", "drag", "pressure", "added", "lift", "total"):
        e = rel_err(g.get_forces(k)[samples], comps[k][loc], scale)
        table[k] = (float(e.max()), float(np.quantile(e, 0.99)))
    r = 0.5 * w["d"][samples]
    tscale = np.linalg.norm(comps["torque"][loc], axis=1) + r * scale
    e = rel_err(g.get_forces("torque")[samples], comps["torque"][loc], tscale)
    table["torque"] = (float(e.max()), float(np.quantile(e, 0.99)))
    print(f"{name} {precision} per-component error (max, p99):", table, flush=True)
    for k, (mx, _) in table.items():
        assert mx < tol, (k, mx)
    # pair sets and contact history of the sampled particles
    sset = set(samples.tolist())
    pairs = g.get_pairs()
    mine = pairs[np.isin(pairs[:, 0], samples) | np.isin(pairs[:, 1], samples)]
    want = orc.pairs_cells(prm, sub(w["x"]), sub(w["d"]))
    want = patch[want]
    want = want[np.isin(want[:, 0], samples) | np.isin(want[:, 1], samples)]
    assert len(want) > 2 * len(samples)
    assert np.array_equal(np.unique(mine, axis=0), np.unique(want, axis=0))
    gh = g.get_history()
    gsel = [t for t in range(len(gh)) if gh["i"][t] in sset or (gh["j"][t] >= 0 and gh["j"][t] in sset)]
    oi = np.where(hout["i"] >= 0, patch[np.maximum(hout["i"], 0)], hout["i"])
    oj = np.where(hout["j"] >= 0, patch[np.maximum(hout["j"], 0)], hout["j"])
    osel = [t for t in range(len(hout)) if oi[t] in sset or (oj[t] >= 0 and oj[t] in sset)]
    ga = sorted((int(gh["i"][t]), int(gh["j"][t])) for t in gsel)
    oa = sorted((int(oi[t]), int(oj[t])) for t in osel)
    assert ga == oa
    gx = {(int(gh["i"][t]), int(gh["j"][t])): gh["xi"][t] for t in gsel}
    ox = {(int(oi[t]), int(oj[t])): hout["xi"][t] for t in osel}
    xs = max(np.abs(np.array(list(ox.values()))).max(), 1e-30)
    herr = max(np.abs(gx[k] - ox[k]).max() for k in ox) / xs
    print(f"{name} history pairs {len(oa)}, max rel error {herr:.3e}", flush=True)
    assert herr < tol


@pytest.mark.parametrize("name", ["bed1m", "bed10m"])
def test_fullsize_deposit_bit_exact_and_smooth(orc, name):
    w = _bed(name)
    prm = w["params"]
    g = _context(w, "fp64" if name == "bed1m" else "mixed")
    g.average()  # drag channels are zero: no force evaluation yet
    raw_g, sm_g = g.get_field(0), g.get_field(1)
    raw_o = orc.deposit(prm, w["x"], w["d"])
    assert np.array_equal(raw_g, raw_o)
    print(f"{name}: oracle diffusion of the solid fraction", flush=True)
    sm_o, _ = orc.diffuse(prm, raw_o[:1])
    err = np.abs(sm_g[0] - sm_o[0]).max()
    print(f"{name}: smoothed solid fraction max abs error {err:.3e}", flush=True)
    assert err < 1e-11 * raw_o[0].max()
    assert not sm_g[1:].any()


def test_fullsize_solid_velocity_and_bdf2(orc):
    """The 1M bed with the solid volume flux and BDF2 pseudo-time, both
    solvers' default for this mesh (direct): flux deposited bit-identically,
    smoothed solid fraction and flux against the oracle's BDF2 CG solves,
    and U_s on every solid cell."""
    w = _bed("bed1m")
    prm = dict(w["params"], avg_solid_velocity=1, avg_scheme=1)
    g = _context(w, "fp64", prm)
    g.average()
    raw_g, sm_g, us_g = g.get_field(0), g.get_field(1), g.get_field(2)
    raw_o = orc.deposit(prm, w["x"], w["d"])
    flux_o = orc.deposit_flux(prm, w["x"], w["d"], w["v"])
    assert np.array_equal(raw_g[0], raw_o[0]) and np.array_equal(raw_g[4:], flux_o)
    print("bed1m: oracle BDF2 diffusion of the solid fraction and flux", flush=True)
    sm_o, _ = orc.diffuse(prm, np.concatenate([raw_o[:1], flux_o]))
    err = np.abs(sm_g[0] - sm_o[0]).max()
    qscale = np.abs(flux_o).max()
    qerr = np.abs(sm_g[4:] - sm_o[1:]).max()
    print(f"bed1m: eps_s max abs error {err:.3e}, flux max error {qerr / qscale:.3e}", flush=True)
    assert err < 1e-11 * raw_o[0].max()
    assert qerr < 1e-10 * qscale
    us_o = orc.solid_velocity(sm_o[0], sm_o[1:])
    solid = sm_o[0] > 1e-6
    vmax = np.abs(w["v"]).max()
    assert solid.sum() > 1000
    assert np.abs(us_g[:, solid] - us_o[:, solid]).max() < 1e-8 * vmax
