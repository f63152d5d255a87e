"""The network's kernels element by element, one layer at a time.

Each layer is checked on the GPU's own stored inputs (read back through
sedimi_nn_get_tensor after a training step with learning rate 0), so a BF16
rounding that went the other way in an earlier layer cannot spread into the
comparison.  Per element, a tensor the GPU rounds to BF16 from an FP32 sum
must satisfy

    |gpu - exact| <= 2^-8 |exact| + (K + 2) 2^-24 S_abs,

where exact is the FP64 sum of the oracle's convolution on the same inputs,
2^-8 |exact| bounds half a BF16 unit in the last place (8 significant bits),
and the second term bounds the FP32 accumulation of K products (S_abs the
same sum of absolute values, from the oracle on |w| and |inputs|).  The
element-wise products and sums the kernels do in FP32 before a BF16 rounding
(leaky ReLU, residual add, loss gradient, the gradient through the
activation) are reproduced in float32 here and must match bit for bit
(allowing for a fused multiply-add in the residual layers).  The weight
gradients are sums over all cells: their bound takes K = the cell count.
No element may exceed its bound: the allowed count is zero.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

DIL = (1, 2, 4, 4, 2, 1)
U32 = 2.0 ** -24


def bf16(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def layer_slices(params):
    out, off = [], 0
    for l in range(6):
        cin = 4 if l == 0 else 32
        cout = 4 if l == 5 else 32
        nw = 27 * cin * cout
        out.append((params[off:off + nw].reshape(27, cin, cout), params[off + nw:off + nw + cout]))
        off += nw + cout
    return out


def within(gpu, exact, sabs, K, what, rel=2.0 ** -8):
    tol = rel * np.abs(exact) + (K + 2) * U32 * sabs + 1e-30
    bad = np.abs(gpu.astype(np.float64) - exact) > tol
    worst = float((np.abs(gpu - exact) / tol).max())
    print(f"{what}: {bad.sum()} of {bad.size} above the bound, worst ratio {worst:.3f}")
    assert not bad.any(), (what, np.argwhere(bad)[:5])


def leaky_variants(z, a, hin=None):
    """float32 leaky ReLU (+ residual), unfused and with a fused multiply-add."""
    a32 = np.float32(a)
    lz = np.where(z > 0, z, (a32 * z).astype(np.float32)).astype(np.float32)
    if hin is None:
        return [lz]
    plain = (lz + hin).astype(np.float32)
    fused = np.where(z > 0, plain,
                     (a32.astype(np.float64) * z.astype(np.float64) + hin).astype(np.float32))
    return [plain, fused]


@pytest.mark.parametrize("shape,alpha", [((16, 8, 12), 0.1), ((70, 20, 5), 1.0),
                                         ((10, 7, 9), 0.3)])
def test_every_layer_element_by_element(orc, shape, alpha):
    import paper_1601_03801_amd as sm
    nx, ny, nz = shape
    n = nx * ny * nz
    prm = workloads.base_params(Lx=nx * 1e-3, Ly=ny * 1e-3, Lz=nz * 0.4e-3, nx=nx, ny=ny, nz=nz)
    g = sm.Sedimi(prm, 1, d_max=0.5e-3, nn=True, nn_alpha=alpha)
    rng = np.random.default_rng(sum(shape))
    P = g.nn_param_count()
    params = bf16(rng.normal(scale=0.08, size=P)).astype(np.float64)
    raw = rng.random((4, n)) ** 2
    target = raw * 0.8 + 0.05 * rng.random((4, n))
    mean = np.array([0.3, 0.1, -0.05, 0.2])
    std = np.array([0.25, 0.5, 0.4, 0.3])
    g.set_field(0, raw)
    g.set_field(1, target)
    g.nn_set_norm(mean, std)
    lw = np.array([1.0, 0.5, 3.0, 1.25])
    g.nn_set_loss_weights(lw)
    g.nn_set_params(params)
    g.nn_train_step(0.0)
    T = {k: g.nn_tensor(k) for k in ("x", "xb", "sx", "y", "dy")}
    z = [g.nn_tensor("z", l) for l in range(5)]
    h = [g.nn_tensor("h", l) for l in range(5)]
    dh = [g.nn_tensor("dh", l) for l in range(5)]
    dz = [g.nn_tensor("dz", l) for l in range(5)]
    grads = g.nn_get_grads().astype(np.float64)
    W = layer_slices(params)
    Gr = layer_slices(grads)

    # input, its BF16 copy and the skip
    xf = T["x"].astype(np.float64)
    want_x = ((raw.T - mean) / std).astype(np.float32)
    assert np.array_equal(T["x"], want_x)
    split = orc.split_coefficients(prm)
    sx = orc.split_smooth(shape, split, xf)
    within(T["sx"], sx, orc.split_smooth(shape, split, np.abs(xf)), 4 * nz, "skip S x",
           rel=2 * U32)
    # the first layer reads x - S x in BF16
    assert np.array_equal(T["xb"], bf16((T["x"] - T["sx"]).astype(np.float32)))

    # forward, layer by layer on the GPU's own inputs
    for l in range(5):
        inp = (T["xb"] if l == 0 else h[l - 1]).astype(np.float64)
        w, b = W[l]
        ex = orc.conv3d_fwd(shape, inp, w, b, DIL[l])
        sa = orc.conv3d_fwd(shape, np.abs(inp), np.abs(w), np.abs(b), DIL[l])
        within(z[l], ex, sa, 27 * w.shape[1], f"z{l + 1}")
        cand = leaky_variants(z[l], alpha, None if l == 0 else h[l - 1])
        ok = np.zeros(z[l].shape, bool)
        for c in cand:
            ok |= bf16(c) == h[l]
        assert ok.all(), (f"h{l + 1}", int((~ok).sum()))
    w, b = W[5]
    ex = T["sx"].astype(np.float64) + orc.conv3d_fwd(shape, h[4], w, b, DIL[5])
    sa = np.abs(T["sx"]) + orc.conv3d_fwd(shape, np.abs(h[4]), np.abs(w), np.abs(b), DIL[5])
    within(T["y"], ex, sa, 27 * 32 + 1, "y", rel=2 * U32)

    # loss gradient at the output, reproduced in float32
    t = ((target.T - mean) / std).astype(np.float32)
    scale = np.float32(2.0) / (np.float32(4.0) * np.float32(n))
    sw = (scale * lw.astype(np.float32)).astype(np.float32)
    d = (T["y"] - t).astype(np.float32)
    assert np.array_equal(T["dy"], bf16((sw * d).astype(np.float32)))

    # backward: the adjoint of layer 6, then layers 5..2, each on the GPU's inputs
    dx6, _, _ = orc.conv3d_bwd(shape, h[4], w, T["dy"], DIL[5])
    sa6, _, _ = orc.conv3d_bwd(shape, np.abs(h[4]), np.abs(w), np.abs(T["dy"]), DIL[5])
    within(dh[4], dx6, sa6, 54 * 4, "dh5")
    for l in range(4, -1, -1):
        dphi = np.where(z[l] > 0, np.float32(1.0), np.float32(alpha)).astype(np.float32)
        assert np.array_equal(dz[l], bf16((dh[l] * dphi).astype(np.float32))), f"dz{l + 1}"
        if l == 0:
            break
        w, b = W[l]
        dx, _, _ = orc.conv3d_bwd(shape, h[l - 1], w, dz[l], DIL[l])
        sa, _, _ = orc.conv3d_bwd(shape, np.abs(h[l - 1]), np.abs(w), np.abs(dz[l]), DIL[l])
        within(dh[l - 1], dh[l].astype(np.float64) + dx, np.abs(dh[l]) + sa, 54 * 32,
               f"dh{l}")

    # weight and bias gradients: sums over every cell
    for l in range(6):
        w, b = W[l]
        inp = (T["xb"] if l == 0 else h[l - 1]).astype(np.float64)
        gy = (T["dy"] if l == 5 else dz[l]).astype(np.float64)
        _, dw, db = orc.conv3d_bwd(shape, inp, w, gy, DIL[l])
        _, sw, sb = orc.conv3d_bwd(shape, np.abs(inp), np.abs(w), np.abs(gy), DIL[l])
        within(Gr[l][0], dw, sw, n, f"dW{l + 1}", rel=0.0)
        within(Gr[l][1], db, sb, n, f"db{l + 1}", rel=0.0)
