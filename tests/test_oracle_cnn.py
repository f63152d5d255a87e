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


def mirror_extended_conv(shape, x, w, dil):
    """The convolution written as the textbook recipe: extend the field along
    z by reflection about the wall faces (numpy's 'symmetric' padding, the
    even extension), wrap it periodically in x and y, then take the plain
    correlation over the extended array."""
    nx, ny, nz = shape
    cin, cout = w.shape[1], w.shape[2]
    f = x.reshape(nz, ny, nx, cin)
    pad = dil
    while True:  # numpy reflects once per call: repeat for thin meshes
        reps = min(pad, f.shape[0])
        f = np.pad(f, ((reps, reps), (0, 0), (0, 0), (0, 0)), mode="symmetric")
        pad -= reps
        if pad == 0:
            break
    f = np.pad(f, ((0, 0), (1, 1), (1, 1), (0, 0)), mode="wrap")
    y = np.zeros((nz, ny, nx, cout))
    for t in range(27):
        dz, dy, dx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
        sl = f[dil + dil * dz: dil + dil * dz + nz, 1 + dy: 1 + dy + ny, 1 + dx: 1 + dx + nx]
        y += sl @ w[t]
    return y.reshape(-1, cout)


@pytest.mark.parametrize("dil", [1, 2, 4])
@pytest.mark.parametrize("shape", [SHAPE, (4, 3, 3), (3, 4, 1)])
def test_conv_is_the_mirror_extended_correlation(orc, dil, shape):
    """conv3d equals the correlation over the field extended by reflection
    in z (several reflections on meshes thinner than the dilation) and
    periodically in x and y."""
    rng = np.random.default_rng(dil)
    cin, cout = 3, 2
    n = shape[0] * shape[1] * shape[2]
    w = rng.normal(size=(27, cin, cout))
    x = rng.normal(size=(n, cin))
    y = orc.conv3d_fwd(shape, x, w, None, dil)
    assert np.allclose(y, mirror_extended_conv(shape, x, w, dil), rtol=0, atol=1e-12)


@pytest.mark.parametrize("dil", [1, 2, 4])
def test_conv_impulse_response(orc, dil):
    """A unit impulse at (i0, j0, k0) in channel 1 makes output cell
    (i0 - dx, j0 - dy, k) equal to w[t][1][:] for every k whose tap
    k + dil*dz lands on k0 or on its mirror image about a wall face."""
    rng = np.random.default_rng(dil)
    cin, cout = 3, 2
    nz = SHAPE[2]
    w = rng.normal(size=(27, cin, cout))
    for (i0, j0, k0) in ((0, 4, 0), (5, 0, 8), (2, 2, 4), (1, 1, 1)):
        x = np.zeros((N, cin))
        x[cell(i0, j0, k0), 1] = 1.0
        y = orc.conv3d_fwd(SHAPE, x, w, None, dil)
        want = np.zeros((N, cout))
        for t in range(27):
            dz, dy, dx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
            for k in range(nz):
                src = k + dil * dz
                img = -src - 1 if src < 0 else (2 * nz - 1 - src if src >= nz else src)
                if img == k0:
                    want[cell((i0 - dx) % SHAPE[0], (j0 - dy) % SHAPE[1], k)] += w[t, 1]
        assert np.allclose(y, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dil,shape", [(2, SHAPE), (4, SHAPE), (4, (5, 4, 3)), (1, (4, 4, 1))])
def test_conv_adjoint_identity(orc, dil, shape):
    rng = np.random.default_rng(3)
    cin, cout = 4, 3
    n = shape[0] * shape[1] * shape[2]
    w = rng.normal(size=(27, cin, cout))
    x = rng.normal(size=(n, cin))
    g = rng.normal(size=(n, cout))
    y = orc.conv3d_fwd(shape, x, w, None, dil)
    dx, _, _ = orc.conv3d_bwd(shape, x, w, g, dil)
    assert abs((y * g).sum() - (x * dx).sum()) < 1e-11 * np.abs(y * g).sum()


def test_network_keeps_a_field_even_about_the_walls(orc):
    """With taps symmetric in z, mirror padding makes each layer commute with
    the reflection of the column about its centre: a field symmetric in z
    stays symmetric through the whole network (zero padding would not keep
    the planes next to the walls equal to their mirror images' values)."""
    C = 4
    rng = np.random.default_rng(8)
    params = rng.normal(scale=0.3, size=orc.nn_param_count(C))
    off = 0
    for l in range(6):
        cin = 4 if l == 0 else C
        cout = 4 if l == 5 else C
        w = params[off:off + 27 * cin * cout].reshape(3, 9, cin, cout)
        w[2] = w[0]  # taps dz = +1 equal taps dz = -1
        params[off:off + 27 * cin * cout] = w.ravel()
        off += 27 * cin * cout + cout
    nx, ny, nz = SHAPE
    x = rng.normal(size=(nz, ny, nx, 4))
    x = 0.5 * (x + x[::-1])
    y = orc.nn_forward(SHAPE, params, x.reshape(-1, 4), C=C, alpha=0.1).reshape(nz, ny, nx, 4)
    assert np.allclose(y, y[::-1], rtol=0, atol=1e-12)


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
    split = np.array([0.1, 0.2, 1.5, 3.0])
    loss, grad = orc.nn_loss_grad(SHAPE, params, x, target, C=C, alpha=0.1, split=split)
    y = orc.nn_forward(SHAPE, params, x, C=C, alpha=0.1, split=split)
    assert abs(loss - ((y - target) ** 2).mean()) < 1e-12 * loss
    h = 1e-6
    picks = rng.choice(npar, 25, replace=False)
    for k in picks:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        lp, _ = orc.nn_loss_grad(SHAPE, pp, x, target, C=C, alpha=0.1, split=split)
        lm, _ = orc.nn_loss_grad(SHAPE, pm, x, target, C=C, alpha=0.1, split=split)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[k]) < 2e-6 * (abs(grad[k]) + 1e-3), (k, fd, grad[k])


def test_weighted_loss_gradient_finite_difference(orc):
    C = 4
    rng = np.random.default_rng(15)
    npar = orc.nn_param_count(C)
    params = rng.normal(scale=0.3, size=npar)
    x = rng.normal(size=(N, 4))
    target = rng.normal(size=(N, 4))
    lw = np.array([2.0, 0.5, 0.0, 1.5])
    split = np.array([0.1, 0.2, 1.5, 3.0])
    loss, grad = orc.nn_loss_grad(SHAPE, params, x, target, C=C, split=split, loss_weights=lw)
    y = orc.nn_forward(SHAPE, params, x, C=C, split=split)
    assert abs(loss - (lw * (y - target) ** 2).mean()) < 1e-12 * loss
    h = 1e-6
    for k in rng.choice(npar, 12, replace=False):
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        lp, _ = orc.nn_loss_grad(SHAPE, pp, x, target, C=C, split=split, loss_weights=lw)
        lm, _ = orc.nn_loss_grad(SHAPE, pm, x, target, C=C, split=split, loss_weights=lw)
        assert abs((lp - lm) / (2 * h) - grad[k]) < 2e-6 * (abs(grad[k]) + 1e-3)


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


def split_symbol_apply(shape, c, x):
    """The split skip S through its Fourier / cosine symbol: periodic FFT in x
    and y, the even extension about the wall faces in z (DCT-II), each axis
    multiplied by (1 + c_a (2 - 2 cos k_a))^-N."""
    nx, ny, nz = shape
    N = int(c[3])
    f = x.reshape(nz, ny, nx, -1)
    f = np.concatenate([f, f[::-1]], axis=0)
    F = np.fft.fftn(f, axes=(0, 1, 2))
    kz = 2 * np.pi * np.fft.fftfreq(2 * nz)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    sym = ((1 + c[2] * (2 - 2 * np.cos(kz)))[:, None, None] *
           (1 + c[1] * (2 - 2 * np.cos(ky)))[None, :, None] *
           (1 + c[0] * (2 - 2 * np.cos(kx)))[None, None, :]) ** (-N)
    out = np.real(np.fft.ifftn(F * sym[..., None], axes=(0, 1, 2)))[:nz]
    return out.reshape(-1, x.shape[1])


@pytest.mark.parametrize("shape,c", [
    ((6, 5, 9), (0.06, 0.3, 2.25, 4)), ((3, 4, 1), (1.5, 0.2, 0.7, 2)),
    ((2, 7, 5), (0.5, 0.05, 3.0, 3)), ((1, 3, 4), (0.4, 0.9, 0.1, 1)),
    ((16, 8, 32), (0.0576, 0.0576, 2.25, 4))])
def test_split_skip_is_the_product_of_one_dimensional_implicit_steps(orc, shape, c):
    """S from the exact per-line solves (cyclic tridiagonal in x and y,
    Thomas with zero-flux ends in z) equals the separable symbol applied in
    Fourier / cosine space; it conserves each channel's sum."""
    n = shape[0] * shape[1] * shape[2]
    x = np.random.default_rng(len(shape) + shape[0]).random((n, 3))
    got = orc.split_smooth(shape, np.array(c, float), x)
    want = split_symbol_apply(shape, c, x)
    assert np.allclose(got, want, rtol=0, atol=1e-13)
    assert np.allclose(got.sum(axis=0), x.sum(axis=0), rtol=1e-13)


def test_split_skip_is_close_to_the_exact_steps_on_a_fine_mesh(orc):
    """On cells small along z against the bandwidth (3.125d x 3.125d x 0.5d,
    b = 3d) the split differs from the exact backward-Euler steps only by
    their cross terms: well under 1% of a deposited bed's smoothed field."""
    import workloads
    w = workloads.workload("fine2m", n=12000)
    prm = w["params"]
    shape = (prm["nx"], prm["ny"], prm["nz"])
    raw = orc.deposit(prm, w["x"], w["d"])[:1]
    exact, _ = orc.diffuse(prm, raw)
    s = orc.split_smooth(shape, orc.split_coefficients(prm), raw.T)[:, 0]
    rel = np.linalg.norm(s - exact[0]) / np.linalg.norm(exact[0])
    assert rel < 1e-2
    # and it carries most of the smoothing: the deposited field is far off
    assert np.linalg.norm(raw[0] - exact[0]) / np.linalg.norm(exact[0]) > 0.2


def test_network_with_split_skip_at_zero_weights_is_the_split(orc):
    x = np.random.default_rng(7).normal(size=(N, 4))
    c = np.array([0.1, 0.2, 1.5, 3.0])
    y = orc.nn_forward(SHAPE, np.zeros(orc.nn_param_count(8)), x, C=8, split=c)
    assert np.allclose(y, orc.split_smooth(SHAPE, c, x), rtol=0, atol=1e-15)
