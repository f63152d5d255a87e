"""The learned stand-in for the averaging on the GPU: Adam against the
oracle's closed form, training on targets from the plain solver, the
sampled error check and the fallback.  The forward and backward kernels are
compared with the oracle element by element, layer by layer, in
test_gpu_nn_elementwise.py."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

ALPHA = 0.1


def bf16(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def mesh_ctx(shape, **kw):
    import paper_1601_03801_amd as sm
    nx, ny, nz = shape
    prm = workloads.base_params(Lx=nx * 1e-3, Ly=ny * 1e-3, Lz=nz * 0.4e-3, nx=nx, ny=ny, nz=nz)
    g = sm.Sedimi(prm, 1, d_max=0.5e-3, nn=True, nn_alpha=ALPHA, **kw)
    return g, prm


def setup(orc, shape, seed, scale=0.08):
    g, prm = mesh_ctx(shape)
    n = shape[0] * shape[1] * shape[2]
    rng = np.random.default_rng(seed)
    P = g.nn_param_count()
    assert P == orc.nn_param_count(32) == 117668
    params = bf16(rng.normal(scale=scale, size=P))
    raw = rng.random((4, n)) ** 2
    mean = np.array([0.3, 0.1, -0.05, 0.2])
    std = np.array([0.25, 0.5, 0.4, 0.3])
    g.set_field(0, raw)
    g.nn_set_norm(mean, std)
    g.nn_set_params(params)
    xh = ((raw.T - mean) / std).astype(np.float32).astype(np.float64)
    g.split = orc.split_coefficients(prm)  # the skip S of this mesh
    return g, params.astype(np.float64), raw, mean, std, xh


def test_adam_step_matches_oracle(orc):
    shape = (16, 8, 12)
    g, params, raw, mean, std, xh = setup(orc, shape, 4)
    target = raw * 0.9 + 0.01
    g.set_field(1, target)
    g.nn_train_step(1e-3)
    got = g.nn_get_params().astype(np.float64)
    gr = g.nn_get_grads().astype(np.float64)
    w = params.copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    orc.adam(w, m, v, gr, 1e-3, 1)
    assert np.abs(got - w).max() < 1e-6


def test_training_reduces_loss():
    g, prm = mesh_ctx((16, 16, 16))
    n = 16 ** 3
    rng = np.random.default_rng(5)
    g.nn_init(7)
    raws = [rng.random((4, n)) ** 4 for _ in range(4)]
    losses = []
    for it in range(60):
        raw = raws[it % 4]
        g.set_field(0, raw)
        g.smooth(4)  # the target comes from the plain solver itself
        losses.append(g.nn_train_step(2e-3))
    first, last = np.mean(losses[:4]), np.mean(losses[-4:])
    print("loss", first, "->", last)
    assert last < 0.5 * first


def test_check_and_fallback():
    """Checked averaging on a small bed on the fine mesh's cells (3.125d x
    3.125d x 0.5d): the plain field passes the check, an untrained network
    fails it and the averaging falls back to the plain solve; a bound every
    field passes keeps the network's field."""
    import paper_1601_03801_amd as sm
    w = workloads.workload("fine2m", n=20000)
    prm = w["params"]
    n = len(w["d"])

    def ctx(bound):
        g = sm.Sedimi(prm, n, d_max=float(w["d"].max()), nn=True, nn_alpha=ALPHA,
                      nn_bound=bound, nn_sample=0.05)
        g.set_fluid(w["U"], w["gradp"], w["dudt"])
        g.set_particles(w["x"], w["v"], w["d"], w["rho"])
        g.compute_forces()
        g.nn_init(3)
        return g

    g = ctx(1e-3)
    st = g.stats()
    print("check window", st["nn_check_window"], "mass outside", st["nn_check_trunc"],
          "columns", st["nn_check_columns"])
    assert st["nn_check_trunc"] <= 1e-4 and st["nn_check_columns"] >= 1
    g.average()  # plain
    plain = g.get_field(1)
    # the estimate of the plain solution misses at most 1e-4 of G's mass
    assert g.nn_check()[0] < 3e-4
    g.nn_forward()
    assert g.nn_check()[0] > 1e-3  # an untrained network is far off
    g.set_avg_mode(sm.AVG_SURROGATE_CHECKED)
    g.average()
    st = g.stats()
    assert st["nn_calls"] == 1 and st["nn_fallbacks"] == 1
    assert st["nn_last_check"] > 1e-3
    assert np.array_equal(g.get_field(1), plain)  # the fallback is the plain solve

    g2 = ctx(1e9)  # a bound every field passes
    g2.set_avg_mode(sm.AVG_SURROGATE_CHECKED)
    g2.average()
    st2 = g2.stats()
    assert st2["nn_calls"] == 1 and st2["nn_fallbacks"] == 0
    assert not np.array_equal(g2.get_field(1), plain)
    g2.set_avg_mode(sm.AVG_SURROGATE)
    g2.step(2, average_every=1)
    assert g2.stats()["nn_calls"] == 3


@pytest.mark.parametrize("bz", [1.0, 0.4])
def test_check_estimates_the_error_against_the_plain_solve(bz):
    """The check's estimate |y - G*raw| / |G*raw| on the sampled columns:
    within the window's missing mass for the plain field itself, and for
    y = plain + white noise of known size the full-field relative error up to
    sampling (5% of the columns here); isotropic and anisotropic bandwidth
    (b_z / b = 0.4)."""
    import paper_1601_03801_amd as sm
    nx, ny, nz = 40, 24, 64
    d = workloads.D50
    prm = workloads.base_params(Lx=nx * 3.125 * d, Ly=ny * 3.125 * d, Lz=nz * 0.5 * d, nx=nx,
                                ny=ny, nz=nz, avg_bandwidth=3 * d, avg_bandwidth_z=3 * d * bz)
    g = sm.Sedimi(prm, 1, d_max=d, nn=True, nn_alpha=ALPHA, nn_sample=0.05)
    rng = np.random.default_rng(9)
    n = nx * ny * nz
    raw = rng.random((4, n)) ** 3
    raw[0, n // 2:] = 0.0  # an empty upper half, as above a bed
    g.set_field(0, raw)
    g.smooth(4)
    plain = g.get_field(1)
    st = g.stats()
    assert st["nn_check_trunc"] <= 1e-4
    floor = g.nn_check()
    print("check of the plain field", floor, "window", st["nn_check_window"])
    assert np.all(floor < 3e-4)
    for eps in (1e-2, 3e-3):
        noise = rng.normal(size=plain.shape)
        y = plain + eps * noise * np.abs(plain).mean(axis=1, keepdims=True)
        g.set_field(1, y)
        est = g.nn_check()
        full = np.linalg.norm(y - plain, axis=1) / np.linalg.norm(plain, axis=1)
        print("check estimate", est, "full-field error", full)
        assert np.all(np.abs(est - full) < 0.2 * full + floor), (est, full)


def test_save_load_resumes_training_exactly():
    """sedimi_nn_save / sedimi_nn_load carry the parameters, Adam's moments
    and step, the standardisation and the loss weights: a context loaded
    from a blob takes the same next training step, bit for bit, as the one
    that saved it; blobs of another slope or truncated ones are refused."""
    shape = (16, 12, 10)
    n = int(np.prod(shape))
    rng = np.random.default_rng(8)
    raws = [rng.random((4, n)) ** 3 for _ in range(3)]
    a, _ = mesh_ctx(shape)
    a.nn_init(5)
    a.nn_set_norm(np.zeros(4), np.array([0.3, 0.2, 0.25, 0.1]))
    a.nn_set_loss_weights(np.array([1.0, 0.5, 2.0, 1.5]))
    for r in raws[:2]:
        a.set_field(0, r)
        a.smooth(4)
        a.nn_train_step(1e-3)
    blob = a.nn_save()
    b, _ = mesh_ctx(shape)
    b.nn_load(blob)
    for g in (a, b):
        g.set_field(0, raws[2])
        g.smooth(4)
        g.nn_train_step(1e-3)
    assert np.array_equal(a.nn_get_params(), b.nn_get_params())
    assert np.array_equal(a.nn_save(), b.nn_save())
    import paper_1601_03801_amd as sm
    c, _ = mesh_ctx(shape)
    with pytest.raises(sm.SedimiError):
        c.nn_load(blob[:-4])
    nx, ny, nz = shape
    prm = workloads.base_params(Lx=nx * 1e-3, Ly=ny * 1e-3, Lz=nz * 0.4e-3, nx=nx, ny=ny, nz=nz)
    other = sm.Sedimi(prm, 1, d_max=0.5e-3, nn=True, nn_alpha=0.5)
    with pytest.raises(sm.SedimiError):
        other.nn_load(blob)


def test_channel_groups_keep_fields_apart():
    """With 4 channel groups (sedimi_nn_set_groups) each field's output depends
    on that field's input alone, as the averaging's does: the weights joining
    two groups are zero after the initialisation and stay zero through
    training steps, new drag inputs leave the solid fraction's output
    bit-identical, and the setting travels in the network blob."""
    import paper_1601_03801_amd as sm
    shape = (16, 12, 10)
    n = int(np.prod(shape))
    rng = np.random.default_rng(9)
    g, _ = mesh_ctx(shape)
    with pytest.raises(sm.SedimiError):
        g.nn_set_groups(3)
    g.nn_set_groups(4)
    g.nn_init(5)
    g.nn_set_norm(np.zeros(4), np.array([0.3, 0.2, 0.25, 0.1]))

    def check_mask(p):
        off = 0
        for ci, co in [(4, 32)] + [(32, 32)] * 4 + [(32, 4)]:
            w = p[off:off + 27 * ci * co].reshape(27, ci, co)
            gi = np.arange(ci) if ci == 4 else np.arange(ci) // (ci // 4)
            go = np.arange(co) if co == 4 else np.arange(co) // (co // 4)
            cross = gi[:, None] != go[None, :]
            assert np.all(w[:, cross] == 0), (ci, co)
            assert np.any(w[:, ~cross] != 0), (ci, co)
            off += 27 * ci * co + co

    for _ in range(3):
        g.set_field(0, rng.random((4, n)) ** 3)
        g.smooth(4)
        g.nn_train_step(1e-3)
    check_mask(g.nn_get_params())
    raw = rng.random((4, n)) ** 3
    g.set_field(0, raw)
    g.nn_forward()
    y1 = g.get_field(1)
    raw2 = raw.copy()
    raw2[1:] = rng.random((3, n))
    g.set_field(0, raw2)
    g.nn_forward()
    y2 = g.get_field(1)
    assert np.array_equal(y1[0], y2[0])
    assert not np.array_equal(y1[1], y2[1])
    b, _ = mesh_ctx(shape)
    b.nn_load(g.nn_save())
    b.set_field(0, raw2)
    b.nn_forward()
    assert np.array_equal(b.get_field(1), y2)
    b.set_field(0, raw)
    b.smooth(4)
    b.nn_train_step(1e-3)
    check_mask(b.nn_get_params())
