"""The learned stand-in for the averaging on the GPU (BF16 MFMA kernels)
against the FP64 oracle fed the same BF16-rounded weights and inputs, with the
oracle storing activations in BF16 at the same points as the kernels.  What
remains is FP32-vs-FP64 accumulation order and the rare BF16 tie it flips."""
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
    return g, params.astype(np.float64), raw, mean, std, xh


# (70, 20, 5): two ragged tiles of 64 x 16 cells in x and y, and z-taps of
# dilation 4 that mostly fall outside the mesh
@pytest.mark.parametrize("shape", [(16, 8, 12), (10, 7, 9), (70, 20, 5)])
def test_forward_matches_oracle(orc, shape):
    g, params, raw, mean, std, xh = setup(orc, shape, 1)
    g.nn_forward()
    got = g.get_field(1)
    y = orc.nn_forward(shape, params, xh, C=32, alpha=ALPHA, bf16=True)
    want = (y * std + mean).T
    net = np.abs(want - raw).max()  # size of the network's contribution
    err = np.abs(got - want)
    print("forward: max err / max net", err.max() / net, "mean", err.mean() / net)
    assert net > 1e-2
    assert err.max() < 5e-3 * net
    assert err.mean() < 3e-4 * net


def test_gradients_match_oracle(orc):
    shape = (16, 8, 12)
    g, params, raw, mean, std, xh = setup(orc, shape, 2)
    n = np.prod(shape)
    rng = np.random.default_rng(3)
    target = raw + 0.05 * rng.normal(size=raw.shape)
    g.set_field(1, target)
    loss = g.nn_train_step(0.0)  # lr 0: gradient only
    gg = g.nn_get_grads().astype(np.float64)
    th = ((target.T - mean) / std).astype(np.float32).astype(np.float64)
    lo, go = orc.nn_loss_grad(shape, params, xh, th, C=32, alpha=ALPHA, bf16=True)
    assert abs(loss - lo) < 1e-3 * lo
    off = 0
    for l in range(6):
        cin = 4 if l == 0 else 32
        cout = 4 if l == 5 else 32
        nw = 27 * cin * cout
        for part, sl in (("w", slice(off, off + nw)), ("b", slice(off + nw, off + nw + cout))):
            rel = np.linalg.norm(gg[sl] - go[sl]) / (np.linalg.norm(go[sl]) + 1e-30)
            print(f"layer {l + 1} {part}: rel grad err {rel:.2e}")
            assert rel < 2e-3, (l, part, rel)
        off += nw + cout
    # lr = 0 leaves the parameters unchanged
    assert np.array_equal(g.nn_get_params().astype(np.float64), params)


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


def test_residual_check_and_fallback():
    import paper_1601_03801_amd as sm
    w = workloads.workload("small")
    prm = w["params"]
    n = len(w["d"])

    def ctx(bound):
        g = sm.Sedimi(prm, n, d_max=float(w["d"].max()), nn=True, nn_alpha=ALPHA,
                      nn_bound=bound, nn_sample=0.25)
        g.set_fluid(w["U"], w["gradp"], w["dudt"])
        g.set_particles(w["x"], w["v"], w["d"], w["rho"])
        g.compute_forces()
        g.nn_init(3)
        return g

    g = ctx(1e-3)
    g.average()  # plain
    plain = g.get_field(1)
    assert np.all(g.nn_check() < 1e-10)  # A^ntau y = raw holds for the plain solve
    g.nn_forward()
    assert g.nn_check().max() > 1e-3  # an untrained network is far off
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


@pytest.mark.parametrize("shape", [(10, 7, 9), (70, 20, 5)])
def test_gradients_ragged_mesh(orc, shape):
    """x-rows shorter than, or not a multiple of, the 32-cell weight-gradient
    chunk; several ragged 64 x 16 convolution tiles."""
    g, params, raw, mean, std, xh = setup(orc, shape, 8)
    target = raw * 0.8 + 0.05
    g.set_field(1, target)
    g.nn_train_step(0.0)
    gg = g.nn_get_grads().astype(np.float64)
    th = ((target.T - mean) / std).astype(np.float32).astype(np.float64)
    _, go = orc.nn_loss_grad(shape, params, xh, th, C=32, alpha=ALPHA, bf16=True)
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    assert rel < 2e-3, rel
