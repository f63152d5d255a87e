"""Pins of the oracle's convolutional stand-in (CPU only): the convolution's
impulse response and adjoint identity, finite-difference gradients of the
convolution and of the whole network's loss, and Adam's closed-form first
step."""
import numpy as np
import pytest

SHAPE = (6, 5, 9)  # nx, ny, nz
N = SHAPE[0] * SHAPE[1] * SHAPE[2]


def cell(i, j, k):
    return (k * SHAPE[1] + j) * SHAPE[0] + i


@pytest.mark.parametrize("dil", [1, 2, 4])
def test_conv_impulse_response(orc, dil):
    """A unit impulse at (i0, j0, k0) in channel 1 makes output cell
    (i0 - dx, j0 - dy, k0 - dil*dz) equal to w[t][1][:], wrapped in x and y,
    and nothing where k0 - dil*dz leaves the mesh."""
    rng = np.random.default_rng(dil)
    cin, cout = 3, 2
    w = rng.normal(size=(27, cin, cout))
    for (i0, j0, k0) in ((0, 4, 0), (5, 0, 8), (2, 2, 4)):
        x = np.zeros((N, cin))
        x[cell(i0, j0, k0), 1] = 1.0
        y = orc.conv3d_fwd(SHAPE, x, w, None, dil)
        want = np.zeros((N, cout))
        for t in range(27):
            dz, dy, dx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
            k = k0 - dil * dz
            if not 0 <= k < SHAPE[2]:
                continue
            want[cell((i0 - dx) % SHAPE[0], (j0 - dy) % SHAPE[1], k)] += w[t, 1]
        assert np.allclose(y, want, rtol=0, atol=1e-15)


def test_conv_adjoint_identity(orc):
    rng = np.random.default_rng(3)
    cin, cout = 4, 3
    w = rng.normal(size=(27, cin, cout))
    x = rng.normal(size=(N, cin))
    g = rng.normal(size=(N, cout))
    y = orc.conv3d_fwd(SHAPE, x, w, None, 2)
    dx, _, _ = orc.conv3d_bwd(SHAPE, x, w, g, 2)
    assert abs((y * g).sum() - (x * dx).sum()) < 1e-11 * np.abs(y * g).sum()


def test_conv_gradients_finite_difference(orc):
    rng = np.random.default_rng(4)
    cin, cout, dil = 2, 3, 4
    w = rng.normal(size=(27, cin, cout))
    b = rng.normal(size=cout)
    x = rng.normal(size=(N, cin))
    g = rng.normal(size=(N, cout))

    def L(w_, b_, x_):
        return (orc.conv3d_fwd(SHAPE, x_, w_, b_, dil) * g).sum()

    dx, dw, db = orc.conv3d_bwd(SHAPE, x, w, g, dil)
    h = 1e-6
    for idx in [(0, 0, 0), (13, 1, 2), (26, 0, 1), (4, 1, 0)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        assert abs((L(wp, b, x) - L(wm, b, x)) / (2 * h) - dw[idx]) < 1e-6 * (1 + abs(dw[idx]))
    for o in range(cout):
        bp, bm = b.copy(), b.copy()
        bp[o] += h
        bm[o] -= h
        assert abs((L(w, bp, x) - L(w, bm, x)) / (2 * h) - db[o]) < 1e-6 * (1 + abs(db[o]))
    for idx in [(0, 0), (cell(5, 4, 8), 1), (cell(2, 2, 2), 0)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        assert abs((L(w, b, xp) - L(w, b, xm)) / (2 * h) - dx[idx]) < 1e-6 * (1 + abs(dx[idx]))


def test_network_gradient_finite_difference(orc):
    C = 4
    rng = np.random.default_rng(5)
    npar = orc.nn_param_count(C)
    params = rng.normal(scale=0.3, size=npar)
    x = rng.normal(size=(N, 4))
    target = rng.normal(size=(N, 4))
    loss, grad = orc.nn_loss_grad(SHAPE, params, x, target, C=C, alpha=0.1)
    y = orc.nn_forward(SHAPE, params, x, C=C, alpha=0.1)
    assert abs(loss - ((y - target) ** 2).mean()) < 1e-12 * loss
    h = 1e-6
    picks = rng.choice(npar, 25, replace=False)
    for k in picks:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        lp, _ = orc.nn_loss_grad(SHAPE, pp, x, target, C=C, alpha=0.1)
        lm, _ = orc.nn_loss_grad(SHAPE, pm, x, target, C=C, alpha=0.1)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[k]) < 2e-6 * (abs(grad[k]) + 1e-3), (k, fd, grad[k])


def test_network_identity_at_zero_weights(orc):
    """With all parameters zero the network is the global residual alone."""
    x = np.random.default_rng(6).normal(size=(N, 4))
    y = orc.nn_forward(SHAPE, np.zeros(orc.nn_param_count(8)), x, C=8)
    assert np.array_equal(y, x)


def test_adam_first_steps_closed_form(orc):
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    orc.adam(w, m, v, g, lr, 1, eps=eps)
    # first step: bias-corrected m = g, v = g^2
    assert np.allclose(w, 1.0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    w2 = w.copy()
    orc.adam(w, m, v, g, lr, 2, eps=eps)
    # same gradient twice: bias-corrected moments are again g and g^2
    assert np.allclose(w, w2 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)
