"""sedimi_smooth_static (the direct solve for callers that cannot allocate:
tables and intermediate field in the library's static device scratch)
against sedimi_smooth of a context on the same field: two calls in a row,
the second on a smaller mesh, so the second runs on scratch still holding
the first call's tables and products.  Both sides run the same six-pass
transform, the static one with tables computed on the device instead of the
host, so they agree to rounding."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _plain(prm, raw, nch):
    import paper_1601_03801_amd as sm
    g = sm.Sedimi(prm, 1, d_max=workloads.D50, solver="direct")
    full = np.zeros((g.nch, g.ncell))
    full[:nch] = raw
    g.set_field(0, full)
    g.smooth(nch)
    out = g.get_field(1)[:nch].copy()
    g.close()
    return out


def _static(prm, raw, nch):
    import torch

    import paper_1601_03801_amd as sm
    r = torch.tensor(raw, dtype=torch.float64, device="cuda").contiguous()
    s = torch.full_like(r, float("nan"))
    sm.smooth_static(prm, r, s, nch=nch)
    torch.cuda.synchronize()
    return s.cpu().numpy()


CASES = [
    # (mesh, nch, scheme, ntau, b_z / b): the 1M-bed mesh, then smaller inputs
    ((128, 64, 48), 4, 0, 4, 1.0),
    ((20, 12, 10), 3, 0, 4, 0.5),
    ((17, 9, 30), 7, 1, 3, 1.0),
    ((6, 5, 4), 1, 0, 0, 1.0),
]


@pytest.mark.parametrize("order", [(0, 1), (2, 3), (0, 2)])
def test_static_solve_matches_the_context_solve_twice(order):
    for case in order:
        (nx, ny, nz), nch, scheme, ntau, bz = CASES[case]
        d = workloads.D50
        prm = workloads.base_params(Lx=nx * 3.125 * d, Ly=ny * 3.125 * d, Lz=nz * 1.25 * d, nx=nx,
                                    ny=ny, nz=nz, avg_scheme=scheme, avg_ntau=ntau,
                                    avg_bandwidth=3 * d, avg_bandwidth_z=3 * d * bz)
        if nch == 7:
            prm["avg_solid_velocity"] = 1
        rng = np.random.default_rng(case + 40)
        raw = rng.random((nch, nx * ny * nz)) ** 3
        print(f"static solve: mesh {(nx, ny, nz)}, nch {nch}, scheme {scheme}, ntau {ntau}",
              flush=True)
        got = _static(prm, raw, nch)
        want = _plain(prm, raw, nch)
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"static solve: max rel error {err:.2e}", flush=True)
        assert np.all(np.isfinite(got))
        assert err < 1e-12
        if ntau == 0:
            assert np.array_equal(got, raw)


def test_static_solve_refuses_what_does_not_fit():
    import torch

    import paper_1601_03801_amd as sm
    d = workloads.D50
    # tables alone: 2 x 2048^2 doubles = 64 MiB, above the scratch with the field
    prm = workloads.base_params(Lx=2048 * d, Ly=2048 * d, Lz=d, nx=2048, ny=2048, nz=1)
    r = torch.zeros((1, 2048 * 2048), dtype=torch.float64, device="cuda")
    s = torch.zeros_like(r)
    with pytest.raises(sm.SedimiError) as e:
        sm.smooth_static(prm, r, s)
    assert e.value.code == sm.ENOMEM and "static scratch" in str(e.value)
    with pytest.raises(sm.SedimiError):
        sm.smooth_static(dict(prm, nx=4096), r, s)
    with pytest.raises(sm.SedimiError):
        sm.smooth_static(prm, r, r)  # overlapping fields
    torch.cuda.synchronize()
    assert not s.any()  # nothing was enqueued
