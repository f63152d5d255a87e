"""MI355X-native SediFoam particle step and diffusion averaging (libsedimi).

A thin ctypes binding over the C ABI declared in ``include/sedimi.h``: every
function here marshals arguments and calls the library of the same name; all
computation runs in the HIP kernels of ``libsedimi.so``.  PyTorch provides the
device workspace (one uint8 tensor) and the stream.  Importing works without
a GPU; creating a :class:`Sedimi` requires the built library and a GPU and
raises otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsedimi.so")

OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW, EUNSTABLE, EESCAPE, ENOCONV, ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
DRAG = {"none": 0, "difelice": 1, "stokes": 2, "syamlal": 3}
FP64, MIXED = 0, 1
SOLVERS = {"auto": 0, "direct": 1, "iterative": 2}
FORCE = {"contact": 0, "lub": 1, "drag": 2, "pressure": 3, "added": 4, "total": 5,
         "torque": 6, "lift": 7}
FIELD_RAW, FIELD_SMOOTH, FIELD_US = 0, 1, 2

HISTORY_DTYPE = np.dtype([("i", np.int64), ("j", np.int64), ("xi", np.float64, (3,))])


class SedimiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sedimi error {code}: {msg}")
        self.code = code


class sedimi_params(C.Structure):
    _fields_ = [
        ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("kn", C.c_double), ("restitution", C.c_double), ("friction", C.c_double),
        ("kt_over_kn", C.c_double), ("gammat_over_gamman", C.c_double),
        ("lub_out_frac", C.c_double), ("lub_in_frac", C.c_double),
        ("rho_f", C.c_double), ("mu_f", C.c_double), ("c_add", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double), ("dt", C.c_double),
        ("drag_law", C.c_int), ("lubrication", C.c_int), ("fluid_forces", C.c_int),
        ("bottom_wall", C.c_int), ("top_wall", C.c_int),
        ("eps_s_max", C.c_double),
        ("avg_bandwidth", C.c_double), ("avg_ntau", C.c_int), ("avg_rtol", C.c_double),
        ("precision", C.c_int),
        ("d_max", C.c_double), ("skin", C.c_double), ("max_neighbors", C.c_int),
        ("nn_enable", C.c_int), ("nn_alpha", C.c_double), ("nn_bound", C.c_double),
        ("nn_sample", C.c_double), ("nn_seed", C.c_uint64),
        ("avg_solver", C.c_int),
        ("avg_bandwidth_z", C.c_double), ("c_lift", C.c_double),
        ("avg_solid_velocity", C.c_int), ("avg_scheme", C.c_int), ("z_grading", C.c_double),
    ]


class sedimi_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rebuilds", C.c_int64), ("max_neighbors", C.c_int32),
                ("flags", C.c_int32), ("solve_iters", C.c_int64),
                ("solve_residual", C.c_double), ("mean_neighbors", C.c_double),
                ("mean_contacts", C.c_double), ("nn_calls", C.c_int64),
                ("nn_fallbacks", C.c_int64), ("nn_last_check", C.c_double),
                ("particles", C.c_int64), ("nn_check_trunc", C.c_double),
                ("nn_check_window", C.c_int32 * 3), ("nn_check_columns", C.c_int32),
                ("graph_steps", C.c_int64)]


NPHASES = 6
PHASES = ("drift", "rebuild", "forces", "deposit", "smooth", "nn_train")
AVG_PLAIN, AVG_SURROGATE_CHECKED, AVG_SURROGATE = 0, 1, 2
NN_TENSORS = {"x": 0, "xb": 1, "sx": 2, "z": 3, "h": 4, "y": 5, "dy": 6, "dh": 7, "dz": 8}


class sedimi_profile(C.Structure):
    _fields_ = [("ms", C.c_double * NPHASES), ("count", C.c_int64 * NPHASES)]


_lib = None


def lib():
    """Load libsedimi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "paper_1601_03801_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P, i64, I = C.c_void_p, C.c_int64, C.c_int
        ctxp = C.POINTER(C.c_void_p)
        L.sedimi_create.argtypes = [C.POINTER(sedimi_params), i64, ctxp]
        L.sedimi_destroy.argtypes = [P]
        L.sedimi_destroy.restype = None
        L.sedimi_last_error.argtypes = [P]
        L.sedimi_last_error.restype = C.c_char_p
        L.sedimi_workspace_bytes.argtypes = [P]
        L.sedimi_workspace_bytes.restype = C.c_size_t
        L.sedimi_bind_workspace.argtypes = [P, P, C.c_size_t]
        L.sedimi_set_stream.argtypes = [P, P]
        L.sedimi_set_particles.argtypes = [P, i64, P, P, P, P, P]
        L.sedimi_set_fluid.argtypes = [P, P, P, P]
        L.sedimi_set_field.argtypes = [P, I, P]
        L.sedimi_set_accel.argtypes = [P, P, P]
        L.sedimi_translate.argtypes = [P, C.c_double, C.c_double]
        L.sedimi_compute_forces.argtypes = [P, I]
        L.sedimi_step.argtypes = [P, I, I]
        L.sedimi_rebuild.argtypes = [P]
        L.sedimi_smooth_static.argtypes = [C.POINTER(sedimi_params), I, P, P, P]
        L.sedimi_average.argtypes = [P]
        L.sedimi_deposit.argtypes = [P]
        L.sedimi_smooth.argtypes = [P, I]
        L.sedimi_get_particles.argtypes = [P, P, P, P, P]
        L.sedimi_get_accel.argtypes = [P, P, P]
        L.sedimi_get_state.argtypes = [P, P, C.c_size_t, C.POINTER(C.c_size_t)]
        L.sedimi_set_state.argtypes = [P, P, C.c_size_t]
        L.sedimi_get_forces.argtypes = [P, I, P]
        L.sedimi_get_field.argtypes = [P, I, P]
        L.sedimi_get_pairs.argtypes = [P, i64, P, C.POINTER(i64)]
        L.sedimi_get_history.argtypes = [P, i64, P, C.POINTER(i64)]
        L.sedimi_set_history.argtypes = [P, i64, P]
        L.sedimi_get_stats.argtypes = [P, C.POINTER(sedimi_stats)]
        L.sedimi_set_profiling.argtypes = [P, I]
        L.sedimi_set_avg_mode.argtypes = [P, I]
        L.sedimi_nn_param_count.argtypes = [P, C.POINTER(i64)]
        L.sedimi_nn_init.argtypes = [P, C.c_uint64]
        L.sedimi_nn_set_groups.argtypes = [P, C.c_int]
        L.sedimi_set_step_graphs.argtypes = [P, C.c_int]
        L.sedimi_nn_set_params.argtypes = [P, P, i64]
        L.sedimi_nn_get_params.argtypes = [P, P, i64]
        L.sedimi_nn_get_grads.argtypes = [P, P, i64]
        L.sedimi_nn_set_norm.argtypes = [P, P, P]
        L.sedimi_nn_forward.argtypes = [P]
        L.sedimi_nn_set_loss_weights.argtypes = [P, P]
        L.sedimi_nn_save.argtypes = [P, P, C.c_size_t, C.POINTER(C.c_size_t)]
        L.sedimi_nn_load.argtypes = [P, P, C.c_size_t]
        L.sedimi_nn_train_step.argtypes = [P, C.c_double, C.POINTER(C.c_double)]
        L.sedimi_nn_check.argtypes = [P, P]
        L.sedimi_nn_get_tensor.argtypes = [P, I, I, P, i64]
        L.sedimi_get_profile.argtypes = [P, C.POINTER(sedimi_profile)]
        _lib = L
    return _lib


def make_params(prm: dict, precision="fp64", skin=None, max_neighbors=24, d_max=None,
                avg_rtol=1e-12, nn=False, nn_alpha=0.1, nn_bound=1e-3, nn_sample=0.01,
                nn_seed=12345, solver="auto") -> sedimi_params:
    """sedimi_params from a parameter dict (the oracle's keys plus options)."""
    p = sedimi_params()
    for name, _ in sedimi_params._fields_:
        if name in prm:
            val = prm[name]
            if name == "drag_law" and isinstance(val, str):
                val = DRAG[val]
            setattr(p, name, val)
    p.avg_rtol = prm.get("avg_rtol", avg_rtol)
    p.precision = {"fp64": FP64, "mixed": MIXED}[prm.get("precision", precision)]
    dm = prm.get("d_max", d_max)
    if dm is None:
        raise ValueError("d_max (largest particle diameter) is required")
    p.d_max = dm
    p.skin = prm.get("skin", 0.1 * dm if skin is None else skin)
    p.max_neighbors = prm.get("max_neighbors", max_neighbors)
    p.nn_enable = 1 if prm.get("nn", nn) else 0
    p.nn_alpha = prm.get("nn_alpha", nn_alpha)
    p.nn_bound = prm.get("nn_bound", nn_bound)
    p.nn_sample = prm.get("nn_sample", nn_sample)
    p.nn_seed = prm.get("nn_seed", nn_seed)
    p.avg_solver = SOLVERS[prm.get("solver", solver)]
    return p


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _ptr(a):
    return None if a is None else a.ctypes.data


class Sedimi:
    """One sedimi context with its device workspace on the current GPU."""

    def __init__(self, prm: dict, max_particles: int, stream=None, **opts):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Sedimi needs a GPU (no CPU fallback)")
        self._L = lib()
        self.prm = dict(prm)
        self.params = make_params(prm, **opts)
        self._ctx = C.c_void_p()
        rc = self._L.sedimi_create(C.byref(self.params), int(max_particles), C.byref(self._ctx))
        if rc != OK:
            raise SedimiError(rc, "sedimi_create rejected the parameters (see stderr)")
        nbytes = self._L.sedimi_workspace_bytes(self._ctx)
        self.workspace = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._chk(self._L.sedimi_set_stream(self._ctx, C.c_void_p(self.stream.cuda_stream)))
        self._chk(self._L.sedimi_bind_workspace(self._ctx, C.c_void_p(aligned), nbytes))
        self.ncell = prm["nx"] * prm["ny"] * prm["nz"]
        self.nch = 7 if self.params.avg_solid_velocity else 4  # averaged channels
        self.n = 0

    # -- plumbing --
    def _chk(self, rc):
        if rc != OK:
            msg = self._L.sedimi_last_error(self._ctx).decode()
            raise SedimiError(rc, msg)
        return rc

    def close(self):
        if self._ctx:
            self._L.sedimi_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self):
        return int(self._L.sedimi_workspace_bytes(self._ctx))

    # -- calls of the C ABI --
    def set_particles(self, x, v, d, rho, omega=None):
        x = _f64(x, (-1, 3))
        n = x.shape[0]
        v, d, rho, w = _f64(v, (-1, 3)), _f64(d), _f64(rho), _f64(omega, (-1, 3))
        self._chk(self._L.sedimi_set_particles(self._ctx, n, _ptr(x), _ptr(v), _ptr(w),
                                               _ptr(d), _ptr(rho)))
        self.n = n

    def set_fluid(self, U=None, gradp=None, dudt=None):
        U, gradp, dudt = (_f64(a, (-1, 3)) for a in (U, gradp, dudt))
        self._chk(self._L.sedimi_set_fluid(self._ctx, _ptr(U), _ptr(gradp), _ptr(dudt)))

    def set_field(self, which, arr):
        arr = _f64(arr).reshape(self.nch, self.ncell)
        self._chk(self._L.sedimi_set_field(self._ctx, which, _ptr(arr)))

    def translate(self, dx, dy):
        self._chk(self._L.sedimi_translate(self._ctx, float(dx), float(dy)))

    def set_accel(self, a=None, alpha=None):
        a, alpha = _f64(a, (-1, 3)), _f64(alpha, (-1, 3))
        self._chk(self._L.sedimi_set_accel(self._ctx, _ptr(a), _ptr(alpha)))

    def compute_forces(self, update_history=False):
        self._chk(self._L.sedimi_compute_forces(self._ctx, 1 if update_history else 0))

    def step(self, nsteps, average_every=0):
        self._chk(self._L.sedimi_step(self._ctx, int(nsteps), int(average_every)))

    def rebuild(self):
        self._chk(self._L.sedimi_rebuild(self._ctx))

    def average(self):
        self._chk(self._L.sedimi_average(self._ctx))

    def deposit(self):
        self._chk(self._L.sedimi_deposit(self._ctx))

    def smooth(self, nch=None):
        self._chk(self._L.sedimi_smooth(self._ctx, int(self.nch if nch is None else nch)))

    def get_particles(self):
        out = [np.zeros((self.n, 3)) for _ in range(4)]
        self._chk(self._L.sedimi_get_particles(self._ctx, *[_ptr(o) for o in out]))
        return dict(zip(("x", "v", "omega", "a"), out))

    def get_state(self):
        """Opaque checkpoint blob (numpy uint8) of the whole context."""
        size = C.c_size_t(0)
        self._chk(self._L.sedimi_get_state(self._ctx, None, 0, C.byref(size)))
        blob = np.empty(size.value, np.uint8)
        self._chk(self._L.sedimi_get_state(self._ctx, _ptr(blob), blob.size, C.byref(size)))
        return blob

    def set_state(self, blob):
        blob = np.ascontiguousarray(blob, np.uint8)
        self._chk(self._L.sedimi_set_state(self._ctx, _ptr(blob), blob.size))
        self.n = int(self.stats()["particles"])

    def get_accel(self):
        out = [np.zeros((self.n, 3)) for _ in range(2)]
        self._chk(self._L.sedimi_get_accel(self._ctx, *[_ptr(o) for o in out]))
        return dict(zip(("a", "alpha"), out))

    def get_forces(self, component):
        f = np.zeros((self.n, 3))
        comp = FORCE[component] if isinstance(component, str) else component
        self._chk(self._L.sedimi_get_forces(self._ctx, comp, _ptr(f)))
        return f

    def get_field(self, which):
        out = np.zeros((3 if which == FIELD_US else self.nch, self.ncell))
        self._chk(self._L.sedimi_get_field(self._ctx, which, _ptr(out)))
        return out

    def get_pairs(self):
        cnt = C.c_int64(0)
        cap = 16 * max(self.n, 1)
        while True:
            buf = np.zeros((cap, 2), np.int64)
            rc = self._L.sedimi_get_pairs(self._ctx, cap, _ptr(buf), C.byref(cnt))
            if rc == EOVERFLOW and cnt.value > cap:
                cap = cnt.value
                continue
            self._chk(rc)
            return buf[:cnt.value].copy()

    def get_history(self):
        cnt = C.c_int64(0)
        cap = 16 * max(self.n, 1)
        while True:
            buf = np.zeros(cap, HISTORY_DTYPE)
            rc = self._L.sedimi_get_history(self._ctx, cap, _ptr(buf), C.byref(cnt))
            if rc == EOVERFLOW and cnt.value > cap:
                cap = cnt.value
                continue
            self._chk(rc)
            return buf[:cnt.value].copy()

    def set_history(self, records):
        rec = np.ascontiguousarray(records, HISTORY_DTYPE)
        self._chk(self._L.sedimi_set_history(self._ctx, len(rec), _ptr(rec) if len(rec) else None))

    def set_step_graphs(self, enable=True):
        """Replay step() from captured HIP graphs (on by default)."""
        self._chk(self._L.sedimi_set_step_graphs(self._ctx, 1 if enable else 0))

    def set_avg_mode(self, mode):
        self._chk(self._L.sedimi_set_avg_mode(self._ctx, int(mode)))

    # -- learned stand-in for the averaging --
    def nn_param_count(self):
        n = C.c_int64(0)
        self._chk(self._L.sedimi_nn_param_count(self._ctx, C.byref(n)))
        return n.value

    def nn_init(self, seed=0):
        self._chk(self._L.sedimi_nn_init(self._ctx, int(seed)))

    def nn_set_groups(self, groups):
        """1: hidden channels shared by all fields; 4: one group of 8 per field."""
        self._chk(self._L.sedimi_nn_set_groups(self._ctx, int(groups)))

    def nn_set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self._chk(self._L.sedimi_nn_set_params(self._ctx, _ptr(p), len(p)))

    def nn_get_params(self):
        p = np.zeros(self.nn_param_count(), np.float32)
        self._chk(self._L.sedimi_nn_get_params(self._ctx, _ptr(p), len(p)))
        return p

    def nn_save(self):
        """The trained network (parameters, Adam moments and step, standardisation,
        loss weights) as bytes."""
        size = C.c_size_t(0)
        self._chk(self._L.sedimi_nn_save(self._ctx, None, 0, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        self._chk(self._L.sedimi_nn_save(self._ctx, buf, size.value, C.byref(size)))
        return buf.raw

    def nn_load(self, blob):
        self._chk(self._L.sedimi_nn_load(self._ctx, blob, len(blob)))

    def nn_get_grads(self):
        g = np.zeros(self.nn_param_count(), np.float32)
        self._chk(self._L.sedimi_nn_get_grads(self._ctx, _ptr(g), len(g)))
        return g

    def nn_set_norm(self, mean, std):
        mean, std = _f64(mean), _f64(std)
        self._chk(self._L.sedimi_nn_set_norm(self._ctx, _ptr(mean), _ptr(std)))

    def nn_set_loss_weights(self, w):
        w = _f64(w)
        self._chk(self._L.sedimi_nn_set_loss_weights(self._ctx, _ptr(w)))

    def nn_forward(self):
        self._chk(self._L.sedimi_nn_forward(self._ctx))

    def nn_train_step(self, lr):
        loss = C.c_double(0.0)
        self._chk(self._L.sedimi_nn_train_step(self._ctx, float(lr), C.byref(loss)))
        return loss.value

    def nn_tensor(self, which, layer=0):
        """A stored network tensor (NN_* names) as float32 [ncell, channels]."""
        which = NN_TENSORS[which] if isinstance(which, str) else which
        ch = 32 if which in (NN_TENSORS["z"], NN_TENSORS["h"], NN_TENSORS["dh"],
                             NN_TENSORS["dz"]) else 4
        out = np.zeros((self.ncell, ch), np.float32)
        self._chk(self._L.sedimi_nn_get_tensor(self._ctx, int(which), int(layer), _ptr(out),
                                               out.size))
        return out

    def nn_check(self):
        rel = np.zeros(4)
        self._chk(self._L.sedimi_nn_check(self._ctx, _ptr(rel)))
        return rel

    def set_profiling(self, on=True):
        self._chk(self._L.sedimi_set_profiling(self._ctx, 1 if on else 0))

    def profile(self):
        """{phase: (total ms, launches)} since profiling was turned on."""
        p = sedimi_profile()
        self._chk(self._L.sedimi_get_profile(self._ctx, C.byref(p)))
        return {PHASES[k]: (p.ms[k], p.count[k]) for k in range(NPHASES)}

    def stats(self):
        s = sedimi_stats()
        self._chk(self._L.sedimi_get_stats(self._ctx, C.byref(s)))
        out = {k: getattr(s, k) for k, _ in sedimi_stats._fields_}
        out["nn_check_window"] = list(s.nn_check_window)
        return out


def smooth_static(prm: dict, raw, smooth, nch=None, stream=None, **opts):
    """sedimi_smooth_static on torch float64 device tensors raw and smooth
    ([nch, ncell], contiguous); enqueued on `stream` (default: the current
    torch stream)."""
    import torch
    L = lib()
    p = make_params(prm, d_max=opts.pop("d_max", 1.0), **opts)
    for t in (raw, smooth):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("raw and smooth must be contiguous float64 device tensors")
    nch = raw.shape[0] if nch is None else nch
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = L.sedimi_smooth_static(C.byref(p), int(nch), C.c_void_p(raw.data_ptr()),
                                C.c_void_p(smooth.data_ptr()), C.c_void_p(s.cuda_stream))
    if rc != OK:
        raise SedimiError(rc, L.sedimi_last_error(None).decode())


def exported_symbols():
    """Names of the C ABI entry points declared in include/sedimi.h."""
    hdr = os.path.join(os.path.dirname(_HERE), "include", "sedimi.h")
    import re
    names = re.findall(r"^\s*(?:int|void|size_t|const char\*)\s+(sedimi_\w+)\s*\(",
                       open(hdr).read(), re.M)
    return sorted(set(names))
