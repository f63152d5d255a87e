"""Plain FP64 CPU oracle for the SediFoam particle step and diffusion averaging.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; the product library never uses it.  The C
sources in this folder share no code with the GPU path.  This module builds
``liborc.so`` with gcc and wraps it with ctypes over numpy arrays.

Parameters are passed as a plain dict (keys = ``orc_params`` field names); the
seeded input generators in ``workloads`` produce such dicts.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_SOURCES = ["orc_pairs.c", "orc_forces.c", "orc_average.c", "orc_cnn.c", "orc_mesh.c"]

DRAG = {"none": 0, "difelice": 1, "stokes": 2, "syamlal": 3}
WALL_BOTTOM = -1
WALL_TOP = -2


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-Wall", "-Wno-unused-function", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class orc_params(C.Structure):
    _fields_ = [
        ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("kn", C.c_double), ("restitution", C.c_double), ("friction", C.c_double),
        ("kt_over_kn", C.c_double), ("gammat_over_gamman", C.c_double),
        ("lub_out_frac", C.c_double), ("lub_in_frac", C.c_double),
        ("rho_f", C.c_double), ("mu_f", C.c_double), ("c_add", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double),
        ("dt", C.c_double),
        ("drag_law", C.c_int), ("lubrication", C.c_int), ("fluid_forces", C.c_int),
        ("bottom_wall", C.c_int), ("top_wall", C.c_int),
        ("eps_s_max", C.c_double),
        ("avg_bandwidth", C.c_double), ("avg_ntau", C.c_int), ("cg_rtol", C.c_double),
        ("avg_bandwidth_z", C.c_double), ("c_lift", C.c_double),
        ("avg_scheme", C.c_int), ("z_grading", C.c_double),
    ]


class orc_contact(C.Structure):
    _fields_ = [("i", C.c_int64), ("j", C.c_int64), ("xi", C.c_double * 3)]


class orc_fields(C.Structure):
    _fields_ = [("U", C.c_void_p), ("gradp", C.c_void_p), ("dudt", C.c_void_p),
                ("eps_s", C.c_void_p)]


class orc_forces_out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("contact", "lub", "drag", "pressure", "added", "total", "torque", "lift")]


CONTACT_DTYPE = np.dtype([("i", np.int64), ("j", np.int64), ("xi", np.float64, (3,))])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i64 = C.c_int64
        pp = C.POINTER(orc_params)
        L.orc_pairs_brute.argtypes = [pp, i64, P, P, i64, P, C.POINTER(i64)]
        L.orc_pairs_cells.argtypes = [pp, i64, P, P, i64, P, C.POINTER(i64)]
        L.orc_forces.argtypes = [pp, i64, P, P, P, P, P, P, C.POINTER(orc_fields), P, i64, P,
                                 i64, C.POINTER(i64), C.POINTER(orc_forces_out)]
        L.orc_run.argtypes = [pp, i64, P, P, P, P, P, P, P, P, P, P, P, P, P, P, i64,
                              C.POINTER(i64), C.POINTER(i64), C.c_int, C.c_int]
        L.orc_init_accel.argtypes = [pp, i64, P, P, P, P, P, P, P, P, P, P, P, P, P, i64]
        L.orc_deposit.argtypes = [pp, i64, P, P, P, P]
        L.orc_diffuse.argtypes = [pp, C.c_int, P, P, C.POINTER(i64)]
        L.orc_deposit_flux.argtypes = [pp, i64, P, P, P, P]
        L.orc_solid_velocity.argtypes = [i64, P, P, P]
        L.orc_solid_velocity.restype = None
        L.orc_apply_A.argtypes = [pp, C.c_double, P, P]
        L.orc_apply_A.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = C.c_int
        # one thread unless a caller asks for more (set_threads)
        L.orc_set_threads(1)
        if hasattr(L, "orc_conv3d_fwd"):
            _declare_cnn(L)
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops (results do not depend
    on it: every sum keeps its order)."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def _declare_cnn(L):
    P, i, d, i64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
    L.orc_conv3d_fwd.argtypes = [i, i, i, i, i, i, P, P, P, P]
    L.orc_conv3d_fwd.restype = None
    L.orc_conv3d_bwd.argtypes = [i, i, i, i, i, i, P, P, P, P, P, P]
    L.orc_conv3d_bwd.restype = None
    L.orc_nn_param_count.argtypes = [i]
    L.orc_nn_param_count.restype = i64
    L.orc_nn_forward.argtypes = [i, i, i, i, d, i, P, P, P, P, P]
    L.orc_nn_forward.restype = None
    L.orc_nn_loss_grad.argtypes = [i, i, i, i, d, i, P, P, P, P, P, P]
    L.orc_nn_loss_grad.restype = d
    L.orc_split_smooth.argtypes = [i, i, i, i, P, P, P]
    L.orc_split_smooth.restype = None
    L.orc_adam.argtypes = [i64, P, P, P, P, d, d, d, d, i64]
    L.orc_adam.restype = None


def make_params(prm: dict) -> orc_params:
    p = orc_params()
    for name, _ in orc_params._fields_:
        val = prm[name]
        if name == "drag_law" and isinstance(val, str):
            val = DRAG[val]
        setattr(p, name, val)
    return p


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def pairs_brute(prm, x, d):
    p = make_params(prm)
    x = _f64(x, (-1, 3))
    d = _f64(d)
    n = x.shape[0]
    cnt = C.c_int64(0)
    lib().orc_pairs_brute(C.byref(p), n, _ptr(x), _ptr(d), 0, None, C.byref(cnt))
    out = np.zeros((max(cnt.value, 1), 2), np.int64)
    _check(lib().orc_pairs_brute(C.byref(p), n, _ptr(x), _ptr(d), cnt.value, _ptr(out),
                                 C.byref(cnt)), "pairs_brute")
    return out[:cnt.value]


def pairs_cells(prm, x, d):
    p = make_params(prm)
    x = _f64(x, (-1, 3))
    d = _f64(d)
    n = x.shape[0]
    cnt = C.c_int64(0)
    rc = lib().orc_pairs_cells(C.byref(p), n, _ptr(x), _ptr(d), 0, None, C.byref(cnt))
    if rc == -2:
        raise MemoryError("oracle pairs_cells")
    out = np.zeros((max(cnt.value, 1), 2), np.int64)
    _check(lib().orc_pairs_cells(C.byref(p), n, _ptr(x), _ptr(d), cnt.value, _ptr(out),
                                 C.byref(cnt)), "pairs_cells")
    return out[:cnt.value]


def empty_history(cap=0):
    return np.zeros(cap, CONTACT_DTYPE)


def _fields_struct(U=None, gradp=None, dudt=None, eps_s=None):
    keep = [None if a is None else _f64(a) for a in (U, gradp, dudt, eps_s)]
    fl = orc_fields(*[_ptr(a) for a in keep])
    return fl, keep


def forces(prm, x, v, w, d, rho, a_prev=None, U=None, gradp=None, dudt=None, eps_s=None,
           hist=None):
    """One force evaluation.  Returns (dict of [n,3] components, new history)."""
    p = make_params(prm)
    x, v, w = _f64(x, (-1, 3)), _f64(v, (-1, 3)), _f64(w, (-1, 3))
    d, rho = _f64(d), _f64(rho)
    n = x.shape[0]
    ap = None if a_prev is None else _f64(a_prev, (-1, 3))
    fl, keep = _fields_struct(U, gradp, dudt, eps_s)
    hin = empty_history() if hist is None else np.ascontiguousarray(hist, CONTACT_DTYPE)
    cap = 16 * n + 64
    hout = np.zeros(cap, CONTACT_DTYPE)
    nh = C.c_int64(0)
    comps = {k: np.zeros((n, 3)) for k in
             ("contact", "lub", "drag", "pressure", "added", "total", "torque", "lift")}
    o = orc_forces_out(*[_ptr(comps[k]) for k, _ in orc_forces_out._fields_])
    _check(lib().orc_forces(C.byref(p), n, _ptr(x), _ptr(v), _ptr(w), _ptr(d), _ptr(rho),
                            _ptr(ap), C.byref(fl), _ptr(hin) if len(hin) else None, len(hin),
                            _ptr(hout), cap, C.byref(nh), C.byref(o)), "forces")
    del keep
    return comps, hout[:nh.value].copy()


class State:
    """Mutable particle state for oracle time stepping (arrays indexed by ID)."""

    def __init__(self, prm, x, v, w, d, rho, U=None, gradp=None, dudt=None, eps_s=None,
                 hist_cap=None):
        self.prm = dict(prm)
        self.p = make_params(prm)
        self.x = _f64(x, (-1, 3)).copy()
        n = self.x.shape[0]
        self.n = n
        self.v = _f64(v, (-1, 3)).copy()
        self.w = _f64(w, (-1, 3)).copy()
        self.d = _f64(d).copy()
        self.rho = _f64(rho).copy()
        self.a = np.zeros((n, 3))
        self.alpha = np.zeros((n, 3))
        self.fdrag = np.zeros((n, 3))
        ncell = prm["nx"] * prm["ny"] * prm["nz"]
        self.U = None if U is None else _f64(U, (-1, 3)).copy()
        self.gradp = None if gradp is None else _f64(gradp, (-1, 3)).copy()
        self.dudt = None if dudt is None else _f64(dudt, (-1, 3)).copy()
        self.eps_s = np.zeros(ncell) if eps_s is None else _f64(eps_s).copy()
        self.avg = np.zeros((4, ncell))
        cap = hist_cap if hist_cap is not None else 16 * n + 64
        self.hist = np.zeros(cap, CONTACT_DTYPE)
        self.nhist = C.c_int64(0)
        self.step = C.c_int64(0)

    def history(self):
        return self.hist[:self.nhist.value].copy()

    def init_accel(self):
        _check(lib().orc_init_accel(
            C.byref(self.p), self.n, _ptr(self.x), _ptr(self.v), _ptr(self.w), _ptr(self.a),
            _ptr(self.alpha), _ptr(self.d), _ptr(self.rho), _ptr(self.fdrag), _ptr(self.U),
            _ptr(self.gradp), _ptr(self.dudt), _ptr(self.eps_s),
            _ptr(self.hist) if self.nhist.value else None, self.nhist.value), "init_accel")

    def average(self):
        raw = deposit(self.prm, self.x, self.d, self.fdrag)
        sm, _ = diffuse(self.prm, raw)
        self.eps_s[:] = sm[0]
        self.avg[:] = sm
        return raw, sm

    def run(self, nsteps, average_every=0):
        _check(lib().orc_run(
            C.byref(self.p), self.n, _ptr(self.x), _ptr(self.v), _ptr(self.w), _ptr(self.a),
            _ptr(self.alpha), _ptr(self.d), _ptr(self.rho), _ptr(self.fdrag), _ptr(self.U),
            _ptr(self.gradp), _ptr(self.dudt), _ptr(self.eps_s), _ptr(self.avg),
            _ptr(self.hist), len(self.hist), C.byref(self.nhist), C.byref(self.step),
            int(nsteps), int(average_every)), "run")


def deposit(prm, x, d, fdrag=None):
    p = make_params(prm)
    x = _f64(x, (-1, 3))
    d = _f64(d)
    fd = None if fdrag is None else _f64(fdrag, (-1, 3))
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    raw = np.zeros((4, ncell))
    _check(lib().orc_deposit(C.byref(p), x.shape[0], _ptr(x), _ptr(d), _ptr(fd), _ptr(raw)),
           "deposit")
    return raw


def deposit_flux(prm, x, d, v):
    """Solid volume flux [3, ncell]: sum V_p u_p / V_c per cell."""
    p = make_params(prm)
    x = _f64(x, (-1, 3))
    d = _f64(d)
    v = _f64(v, (-1, 3))
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    flux = np.zeros((3, ncell))
    _check(lib().orc_deposit_flux(C.byref(p), x.shape[0], _ptr(x), _ptr(d), _ptr(v),
                                  _ptr(flux)), "deposit_flux")
    return flux


US_EPS_MIN = 1e-9


def solid_velocity(eps_s, flux):
    """U_s [3, ncell] = flux / eps_s where eps_s > US_EPS_MIN, else 0."""
    eps_s = _f64(eps_s)
    flux = _f64(flux).reshape(3, -1)
    us = np.zeros_like(flux)
    lib().orc_solid_velocity(eps_s.size, _ptr(eps_s), _ptr(flux), _ptr(us))
    return us


def diffuse(prm, raw):
    p = make_params(prm)
    raw = _f64(raw)
    ncell = prm["nx"] * prm["ny"] * prm["nz"]
    raw = raw.reshape(-1, ncell)
    out = np.zeros_like(raw)
    it = C.c_int64(0)
    _check(lib().orc_diffuse(C.byref(p), raw.shape[0], _ptr(raw), _ptr(out), C.byref(it)),
           "diffuse")
    return out, it.value


def apply_A(prm, dtau, x):
    p = make_params(prm)
    x = _f64(x)
    y = np.zeros_like(x)
    lib().orc_apply_A(C.byref(p), float(dtau), _ptr(x), _ptr(y))
    return y


# ---------------------------------------------------------------------------
# learned stand-in for the diffusion averaging (orc_cnn.c)
# ---------------------------------------------------------------------------
NN_DILATIONS = (1, 2, 4, 4, 2, 1)


def conv3d_fwd(shape, x, w, b, dil):
    """shape = (nx, ny, nz); x [n, cin]; w [27, cin, cout]; b [cout] or None."""
    nx, ny, nz = shape
    x = _f64(x)
    w = _f64(w)
    cin, cout = w.shape[1], w.shape[2]
    y = np.zeros((nx * ny * nz, cout))
    bb = None if b is None else _f64(b)
    lib().orc_conv3d_fwd(nx, ny, nz, cin, cout, dil, _ptr(x), _ptr(w), _ptr(bb), _ptr(y))
    return y


def conv3d_bwd(shape, x, w, dy, dil):
    nx, ny, nz = shape
    x, w, dy = _f64(x), _f64(w), _f64(dy)
    cin, cout = w.shape[1], w.shape[2]
    dx = np.zeros((nx * ny * nz, cin))
    dw = np.zeros_like(w)
    db = np.zeros(cout)
    lib().orc_conv3d_bwd(nx, ny, nz, cin, cout, dil, _ptr(x), _ptr(w), _ptr(dy), _ptr(dx),
                         _ptr(dw), _ptr(db))
    return dx, dw, db


def nn_param_count(C=32):
    return int(lib().orc_nn_param_count(C))


def split_coefficients(prm):
    """{c_x, c_y, c_z, N} of the network's skip S for a parameter dict:
    c_a = dtau D_a / h_a^2 with dtau = b^2 / (4 N) and D_z = (b_z / b)^2."""
    N = max(1, int(prm["avg_ntau"]))
    b = prm["avg_bandwidth"]
    bz = prm.get("avg_bandwidth_z", 0.0) or b
    dtau = 0.25 * b * b / N
    hx, hy, hz = prm["Lx"] / prm["nx"], prm["Ly"] / prm["ny"], prm["Lz"] / prm["nz"]
    kz = (bz / b) ** 2 if b > 0 else 1.0
    return np.array([dtau / hx ** 2, dtau / hy ** 2, dtau * kz / hz ** 2, float(N)])


def split_smooth(shape, split, x):
    """S x for channel-last x [n, nchan] (the network's skip)."""
    nx, ny, nz = shape
    x = _f64(x)
    nchan = x.shape[1] if x.ndim == 2 else 1
    out = np.zeros_like(x)
    lib().orc_split_smooth(nx, ny, nz, nchan, _ptr(_f64(split)), _ptr(x), _ptr(out))
    return out


def nn_forward(shape, params, x, C=32, alpha=0.1, bf16=False, split=None):
    nx, ny, nz = shape
    params, x = _f64(params), _f64(x)
    sp = None if split is None else _f64(split)
    y = np.zeros((nx * ny * nz, 4))
    lib().orc_nn_forward(nx, ny, nz, C, alpha, 1 if bf16 else 0, _ptr(params), _ptr(sp),
                         _ptr(x), _ptr(y), None)
    return y


def nn_loss_grad(shape, params, x, target, C=32, alpha=0.1, bf16=False, split=None,
                 loss_weights=None):
    nx, ny, nz = shape
    params, x, target = _f64(params), _f64(x), _f64(target)
    sp = None if split is None else _f64(split)
    lw = None if loss_weights is None else _f64(loss_weights)
    g = np.zeros_like(params)
    loss = lib().orc_nn_loss_grad(nx, ny, nz, C, alpha, 1 if bf16 else 0, _ptr(params),
                                  _ptr(sp), _ptr(lw), _ptr(x), _ptr(target), _ptr(g))
    return loss, g


def adam(w, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays w, m, v."""
    g = _f64(g)
    lib().orc_adam(len(w), _ptr(w), _ptr(m), _ptr(v), _ptr(g), lr, b1, b2, eps, int(t))
