"""The C ABI on the host, without a GPU: the built library loads, exports
every entry point include/sedimi.h declares (and no other sedimi_ symbol),
and its host-side logic (parameter checks, workspace sizing, calls made
before a workspace is bound) answers with the documented codes.  No call
here reaches a kernel or the HIP runtime."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

import paper_1601_03801_amd as sm
import workloads

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "sedimi.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sm.LIB_PATH):
        from paper_1601_03801_amd import build
        build.build()
    return sm.lib()


def declared():
    names = sm.exported_symbols()
    # every prototype of the header, counted independently of the helper
    text = open(HEADER).read()
    protos = set(re.findall(r"\b(sedimi_\w+)\s*\(", text))
    assert set(names) == protos, sorted(protos ^ set(names))
    return names


def test_library_exports_every_declared_entry_point(L):
    names = declared()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_no_undeclared_sedimi_exports(L):
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm is not available")
    out = subprocess.run([nm, "-D", "--defined-only", sm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines()
                if ln.split() and ln.split()[-1].startswith("sedimi_")}
    assert exported == set(declared()), sorted(exported ^ set(declared()))


def create(L, prm, cap=1000, **kw):
    p = sm.make_params(prm, d_max=kw.pop("d_max", workloads.D50), **kw)
    ctx = C.c_void_p()
    rc = L.sedimi_create(C.byref(p), cap, C.byref(ctx))
    return rc, ctx


def test_create_checks_parameters(L):
    prm = workloads.base_params()
    rc, ctx = create(L, prm)
    assert rc == sm.OK and ctx.value
    n1 = L.sedimi_workspace_bytes(ctx)
    L.sedimi_destroy(ctx)
    rc, ctx = create(L, prm, cap=100000)
    n2 = L.sedimi_workspace_bytes(ctx)
    L.sedimi_destroy(ctx)
    # per-particle arrays grow with the capacity, the mesh part does not
    assert 0 < n1 < n2
    bad = [dict(prm, nx=0), dict(prm, Lx=-1.0), dict(prm, restitution=1.5),
           dict(prm, Lx=2 * workloads.D50)]  # fewer than 3 neighbour bins across x
    for b in bad:
        rc, ctx = create(L, b)
        assert rc == sm.EINVAL and not ctx.value, b
    rc, ctx = create(L, prm, max_neighbors=0)
    assert rc == sm.EINVAL
    # the network covers the 4 standard channels only
    rc, ctx = create(L, dict(prm, avg_solid_velocity=1), nn=True)
    assert rc == sm.EINVAL and not ctx.value
    rc, ctx = create(L, dict(prm, avg_solid_velocity=1))
    assert rc == sm.OK
    n3 = L.sedimi_workspace_bytes(ctx)
    L.sedimi_destroy(ctx)
    assert n3 > n1  # three more averaged channels and the solid velocity
    # BDF2 pseudo-time: either solver, not with the network
    rc, ctx = create(L, dict(prm, avg_scheme=1))
    assert rc == sm.OK
    L.sedimi_destroy(ctx)
    rc, ctx = create(L, dict(prm, avg_scheme=1), solver="iterative")
    assert rc == sm.OK
    L.sedimi_destroy(ctx)
    rc, ctx = create(L, dict(prm, avg_scheme=1), nn=True)
    assert rc == sm.EINVAL and not ctx.value
    rc, ctx = create(L, dict(prm, avg_scheme=2))
    assert rc == sm.EINVAL
    # graded z meshes: any finite grading >= 0; not with the network
    for g in (0.0, 1.0, 4.0, 0.25):
        rc, ctx = create(L, dict(prm, z_grading=g))
        assert rc == sm.OK
        L.sedimi_destroy(ctx)
    for g in (-1.0, float("inf"), float("nan")):
        rc, ctx = create(L, dict(prm, z_grading=g))
        assert rc == sm.EINVAL and not ctx.value
    rc, ctx = create(L, dict(prm, z_grading=4.0), nn=True)
    assert rc == sm.EINVAL and not ctx.value
    # the direct solve on a graded mesh: nz <= 512
    rc, ctx = create(L, dict(prm, z_grading=4.0, nz=600, Lz=600 * 1e-4, solver="direct"))
    assert rc == sm.EINVAL and not ctx.value
    rc, ctx = create(L, prm, cap=-1)
    assert rc == sm.EINVAL


def test_calls_before_a_workspace_fail_cleanly(L):
    rc, ctx = create(L, workloads.base_params())
    assert rc == sm.OK
    try:
        assert L.sedimi_step(ctx, 1, 0) == sm.ENOMEM
        assert b"workspace" in L.sedimi_last_error(ctx)
        assert L.sedimi_average(ctx) == sm.ENOMEM
        assert L.sedimi_smooth(ctx, 1) == sm.ENOMEM
        size = C.c_size_t(0)
        assert L.sedimi_get_state(ctx, None, 0, C.byref(size)) == sm.ENOMEM
        assert L.sedimi_set_state(ctx, None, 0) == sm.ENOMEM
        # a misaligned workspace is refused before any device call
        assert L.sedimi_bind_workspace(ctx, C.c_void_p(0x1001), 1 << 30) == sm.EINVAL
        assert b"aligned" in L.sedimi_last_error(ctx)
    finally:
        L.sedimi_destroy(ctx)
    assert L.sedimi_step(None, 1, 0) == sm.EINVAL
    assert L.sedimi_last_error(None) == b"null context"


STRUCTS = (("sedimi_params", sm.sedimi_params), ("sedimi_stats", sm.sedimi_stats),
           ("sedimi_profile", sm.sedimi_profile))


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors of sedimi_params, sedimi_stats and sedimi_profile have the C
    header's size and field offsets (a drift would pass garbage across the
    boundary)."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sedimi.h"', 'int main(void) {']
    for struct, cls in STRUCTS:
        lines.append(f'  printf("{struct} %zu\\n", sizeof({struct}));')
        for name, _ in cls._fields_:
            lines.append(f'  printf("{struct}.{name} %zu\\n", offsetof({struct}, {name}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = str(tmp_path / "layout")
    subprocess.run([gcc, "-I", os.path.dirname(HEADER), str(src), "-o", exe], check=True,
                   capture_output=True, timeout=120)
    got = dict(ln.split() for ln in subprocess.run([exe], capture_output=True, text=True,
                                                    check=True).stdout.splitlines())
    for struct, cls in STRUCTS:
        assert int(got[struct]) == C.sizeof(cls), struct
        for name, _ in cls._fields_:
            assert int(got[f"{struct}.{name}"]) == getattr(cls, name).offset, (struct, name)
