"""Seeded synthetic inputs shaped like the paper's sediment-transport workloads.

This package is shared by the GPU path's tests/benchmark and by the oracle's
tests.  It holds no part of the particle method (no forces, integration or
averaging): it only produces parameters, particle beds and frozen fluid fields.

Conventions: SI units; x streamwise and y spanwise (both periodic), z
wall-normal with a wall at z = 0 (and z = Lz); mesh cell (i, j, k) has index
(k*ny + j)*nx + i; particle arrays are [n, 3] / [n] float64 in particle-ID order.

Workloads (sizes of the paper's cases, Table 1 and Section 5.2):
  small       2,000 monodisperse d = 0.5 mm spheres, random sequential insertion
              in a periodic 20d x 20d x 10d box, 16 x 16 x 8 mesh, log-law flow
  bed1m       1,000,000 log-normal spheres (median 0.5 mm, sigma 0.2, truncated
              to [0.3, 0.8] mm) deposited in a 400d x 200d x 60d channel,
              128 x 64 x 48 mesh, log-law + 5% rms fluctuations
  bed10m      10,000,000 spheres in 1200d x 600d x 60d, 384 x 192 x 48 mesh: a
              5 x 2 array of copies of one seeded 1M-sphere deposited tile of
              240d x 300d (the tile is periodic, so its copies meet without
              overlaps; same size distribution, packing and depth as one
              deposition of 10M spheres, generated in a tenth of the time)
  fine2m/4m   2M / 4M spheres, 256 x 128 x 128 mesh with cells of
              (3.125d, 3.125d, 0.5d) in an 800d x 400d x 64d channel; 4 x 4
              copies of a 125k-sphere tile (2M) and 2 x 2 of a 1M tile (4M)
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbedgen.so")

D50 = 0.5e-3          # median diameter (m)
RHO_P = 2650.0        # particle density (kg/m^3)
RHO_F = 1000.0        # water (Table 1)
NU_F = 1.0e-6
MU_F = RHO_F * NU_F
KAPPA = 0.41
U_STAR = 0.0284       # friction velocity: Shields number 0.1 for d = 0.5 mm sand


def build(verbose=False):
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-o", tmp,
           os.path.join(_HERE, "bedgen.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _bedlib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.bedgen_rsd.argtypes = [C.c_int, C.c_void_p, C.c_double, C.c_double, C.c_uint64,
                                 C.c_void_p]
        L.bedgen_rsa.argtypes = [C.c_int, C.c_void_p, C.c_double, C.c_double, C.c_double,
                                 C.c_uint64, C.c_int, C.c_void_p]
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------

def contact_time(kn, e, m_eff):
    """Duration of a linear spring-dashpot contact (used for the dt rule)."""
    le = math.log(e) if e < 1 else 0.0
    zeta = -le / math.sqrt(math.pi ** 2 + le ** 2)
    gamma = 2 * zeta * math.sqrt(m_eff * kn)
    return math.pi / math.sqrt(kn / m_eff - (gamma / (2 * m_eff)) ** 2)


def base_params(**kw):
    """Default parameter dict (the small workload); keys follow the C structs."""
    p = dict(
        Lx=20 * D50, Ly=20 * D50, Lz=10 * D50, nx=16, ny=16, nz=8,
        kn=1.0e3, restitution=0.9, friction=0.3, kt_over_kn=2.0 / 7.0,
        gammat_over_gamman=0.0, lub_out_frac=0.05, lub_in_frac=0.001,
        rho_f=RHO_F, mu_f=MU_F, c_add=0.5, gx=0.0, gy=0.0, gz=-9.81, dt=1.0e-5,
        drag_law="difelice", lubrication=1, fluid_forces=1, bottom_wall=1, top_wall=1,
        eps_s_max=0.7, avg_bandwidth=3 * D50, avg_ntau=4, cg_rtol=1e-14,
        avg_bandwidth_z=0.0, c_lift=0.0, avg_scheme=0,
        z_grading=0.0,
    )
    p.update(kw)
    return p


# ----------------------------------------------------------------------------
# particles
# ----------------------------------------------------------------------------

def lognormal_diameters(n, seed, median=D50, sigma=0.2, lo=0.3e-3, hi=0.8e-3):
    """ln d ~ N(ln median, sigma^2), truncated to [lo, hi] by resampling."""
    rng = np.random.default_rng(seed)
    out = np.empty(0)
    while out.size < n:
        draw = np.exp(rng.normal(math.log(median), sigma, size=int(1.1 * (n - out.size)) + 16))
        draw = draw[(draw >= lo) & (draw <= hi)]
        out = np.concatenate([out, draw])
    return out[:n].copy()


def rsa(n, d, Lx, Ly, Lz, seed, max_trials=100000):
    """Random sequential insertion (no overlaps), z in [r, Lz - r]."""
    d = np.ascontiguousarray(d, np.float64)
    r = 0.5 * d
    x = np.zeros((n, 3))
    rc = _bedlib().bedgen_rsa(n, r.ctypes.data, Lx, Ly, Lz, seed, max_trials, x.ctypes.data)
    if rc != 0:
        raise RuntimeError("random sequential insertion failed to place all spheres")
    return x


def rsd_bed(n, d, Lx, Ly, seed):
    """Random sequential deposition bed on the floor z = 0."""
    d = np.ascontiguousarray(d, np.float64)
    r = 0.5 * d
    x = np.zeros((n, 3))
    _bedlib().bedgen_rsd(n, r.ctypes.data, Lx, Ly, seed, x.ctypes.data)
    return x


def tile_bed(x, d, Lx, Ly, tiles):
    """Copies of a bed that is periodic on [0, Lx/tiles[0]) x [0, Ly/tiles[1])
    laid side by side over [0, Lx) x [0, Ly); copy (a, b) holds IDs
    (b * tiles[0] + a) * n + i."""
    tx, ty = Lx / tiles[0], Ly / tiles[1]
    x = np.concatenate([x + [a * tx, b * ty, 0.0]
                        for b in range(tiles[1]) for a in range(tiles[0])])
    x[:, 0] = np.where(x[:, 0] >= Lx, x[:, 0] - Lx, x[:, 0])
    x[:, 1] = np.where(x[:, 1] >= Ly, x[:, 1] - Ly, x[:, 1])
    return x, np.tile(d, tiles[0] * tiles[1])


def bed_top(x, d, Lx, Ly, nbins=16):
    """Mean height of the highest sphere tops over a coarse horizontal grid."""
    if len(x) == 0:
        return 0.0
    a = np.minimum((x[:, 0] / Lx * nbins).astype(int), nbins - 1)
    b = np.minimum((x[:, 1] / Ly * nbins).astype(int), nbins - 1)
    top = np.zeros(nbins * nbins)
    np.maximum.at(top, a * nbins + b, x[:, 2] + 0.5 * d)
    return float(top.mean())


# ----------------------------------------------------------------------------
# frozen fluid fields (stand-in for the CFD solution)
# ----------------------------------------------------------------------------

def z_faces(prm):
    """Cell faces along z: uniform, or graded geometrically towards the
    bottom with z_grading = top / bottom cell height (0 or 1: uniform)."""
    nz, Lz, g = prm["nz"], prm["Lz"], prm.get("z_grading", 0.0)
    if not _graded(prm):
        return Lz * np.arange(nz + 1) / nz
    h = g ** (np.arange(nz) / (nz - 1))
    zf = np.concatenate([[0.0], np.cumsum(h * (Lz / h.sum()))])
    zf[-1] = Lz
    return zf


def cell_centres(prm):
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    hx, hy, hz = prm["Lx"] / nx, prm["Ly"] / ny, prm["Lz"] / nz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    if _graded(prm):
        zf = z_faces(prm)
        zc = (0.5 * (zf[1:] + zf[:-1]))[k]
    else:
        zc = (k + 0.5) * hz
    return ((i + 0.5) * hx).ravel(), ((j + 0.5) * hy).ravel(), zc.ravel()


def _graded(prm):
    g = prm.get("z_grading", 0.0)
    return prm["nz"] > 1 and g > 0.0 and g != 1.0


def fluid_fields(prm, z_bed=0.0, d=D50, u_star=U_STAR, fluct=0.0, seed=0):
    """Log-law streamwise velocity over the bed, optional white fluctuations,
    hydrostatic + driving pressure gradient and the convective derivative
    U . grad U (the field is frozen, so dU/dt = 0).  Returns U, gradp, dudt
    as [ncell, 3] arrays."""
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    _, _, zc = cell_centres(prm)
    z0 = d / 30.0
    h = zc - z_bed
    u = np.where(h > z0, u_star / KAPPA * np.log(np.maximum(h, z0) / z0), 0.0)
    U = np.zeros((nx * ny * nz, 3))
    U[:, 0] = u
    if fluct > 0.0:
        rng = np.random.default_rng(seed)
        U += fluct * u[:, None] * rng.standard_normal(U.shape)
    H = prm["Lz"] - z_bed
    gradp = np.zeros_like(U)
    gradp[:, 0] = -prm["rho_f"] * u_star ** 2 / max(H, 1e-30)
    gradp[:, 0] += prm["rho_f"] * prm["gx"]
    gradp[:, 1] += prm["rho_f"] * prm["gy"]
    gradp[:, 2] += prm["rho_f"] * prm["gz"]
    dudt = convective_derivative(prm, U)
    return U, gradp, dudt


def convective_derivative(prm, U):
    """U . grad U by second-order central differences of the cell field
    (periodic x, y; one-sided at the z walls)."""
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    hx, hy, hz = prm["Lx"] / nx, prm["Ly"] / ny, prm["Lz"] / nz
    F = U.reshape(nz, ny, nx, 3)
    dfx = (np.roll(F, -1, axis=2) - np.roll(F, 1, axis=2)) / (2 * hx)
    dfy = (np.roll(F, -1, axis=1) - np.roll(F, 1, axis=1)) / (2 * hy)
    if nz > 1:
        if _graded(prm):
            zf = z_faces(prm)
            dfz = np.gradient(F, 0.5 * (zf[1:] + zf[:-1]), axis=0)
        else:
            dfz = np.gradient(F, hz, axis=0)
    else:
        dfz = np.zeros_like(F)
    out = F[..., 0:1] * dfx + F[..., 1:2] * dfy + F[..., 2:3] * dfz
    return out.reshape(-1, 3).copy()


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def dt_rule(prm, dmin, rho=RHO_P):
    """The paper's rule: 1/50 of the shortest pair contact time (Section 2.5)."""
    m = rho * math.pi / 6 * dmin ** 3
    return contact_time(prm["kn"], prm["restitution"], 0.5 * m) / 50.0


DEFAULT_TILES = {"bed10m": (5, 2), "fine2m": (4, 4), "fine4m": (2, 2)}


def workload(name, seed=None, n=None, tiles=None):
    """Build a named workload.  Returns dict(params, x, v, w, d, rho, U, gradp,
    dudt, meta).  tiles = (a, b): the bed is an a x b array of copies of one
    seeded deposited tile (default DEFAULT_TILES, (1, 1) when n is given)."""
    if name == "small":
        s = 0 if seed is None else seed
        n = 2000 if n is None else n
        prm = base_params()
        d = np.full(n, D50)
        x = rsa(n, d, prm["Lx"], prm["Ly"], prm["Lz"], seed=s + 1)
        U, gradp, dudt = fluid_fields(prm, z_bed=0.0)
        meta = dict(workload="small", n=n, mesh=[16, 16, 8], seed=s)
    elif name in ("bed1m", "bed10m", "fine2m", "fine4m"):
        spec = {
            "bed1m": (1_000_000, 400, 200, 60, (128, 64, 48), 1, 101),
            "bed10m": (10_000_000, 1200, 600, 60, (384, 192, 48), 2, 102),
            "fine2m": (2_000_000, 800, 400, 64, (256, 128, 128), 1000, 1100),
            "fine4m": (4_000_000, 800, 400, 64, (256, 128, 128), 4, 104),
        }[name]
        N, lx, ly, lz, mesh, bseed, fseed = spec
        if seed is not None:
            bseed, fseed = seed, seed + 100
        N = N if n is None else n
        scale = math.sqrt(N / spec[0])  # shrink the footprint for reduced test sizes
        prm = base_params(Lx=lx * D50 * scale, Ly=ly * D50 * scale, Lz=lz * D50,
                          nx=max(2, int(round(mesh[0] * scale))),
                          ny=max(2, int(round(mesh[1] * scale))), nz=mesh[2])
        if tiles is None:
            tiles = DEFAULT_TILES.get(name, (1, 1)) if n is None else (1, 1)
        nt = tiles[0] * tiles[1]
        d = lognormal_diameters(N // nt, bseed)
        x = rsd_bed(N // nt, d, prm["Lx"] / tiles[0], prm["Ly"] / tiles[1], seed=bseed)
        if nt > 1:
            x, d = tile_bed(x, d, prm["Lx"], prm["Ly"], tiles)
        prm["dt"] = dt_rule(prm, float(d.min()))
        zb = bed_top(x, d, prm["Lx"], prm["Ly"])
        U, gradp, dudt = fluid_fields(prm, z_bed=zb, fluct=0.05, seed=fseed)
        meta = dict(workload=name, n=N, mesh=[prm["nx"], prm["ny"], prm["nz"]],
                    bed_seed=bseed, field_seed=fseed, bed_top=zb, tiles=list(tiles))
    else:
        raise KeyError(name)
    n = len(d)
    return dict(params=prm, x=x, v=np.zeros((n, 3)), w=np.zeros((n, 3)), d=d,
                rho=np.full(n, RHO_P), U=U, gradp=gradp, dudt=dudt, meta=meta)
