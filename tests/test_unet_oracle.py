"""Pins of the surrogate's FP64 CPU oracle: the convolution against a direct loop over the
definition, the pool / upsample gradients as adjoints, and the full analytic gradient of the
loss against central finite differences."""
import numpy as np

from oracle import unet_oracle as U

RNG = np.random.default_rng(7)


def test_conv_matches_direct_definition():
    n, h, w, cin, cout = 2, 5, 4, 3, 2
    x = RNG.normal(size=(n, h, w, cin))
    for ks in (1, 3):
        wt = RNG.normal(size=(cout, ks * ks, cin))
        b = RNG.normal(size=cout)
        y = U.conv(x, wt, b)
        ref = np.zeros_like(y)
        for nn in range(n):
            for yy in range(h):
                for xx in range(w):
                    for co in range(cout):
                        s = b[co]
                        for t in range(ks * ks):
                            dy, dx = (t // 3 - 1, t % 3 - 1) if ks == 3 else (0, 0)
                            for ci in range(cin):
                                s += x[nn, (yy + dy) % h, (xx + dx) % w, ci] * wt[co, t, ci]
                        ref[nn, yy, xx, co] = s
        np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv_backward_is_adjoint():
    x = RNG.normal(size=(2, 6, 4, 3))
    wt = RNG.normal(size=(5, 9, 3))
    g = RNG.normal(size=(2, 6, 4, 5))
    gx, gw, gb = U.conv_backward(x, wt, g)
    # <conv(x) - b, g> is bilinear in (x, w): check both partial derivatives and the bias
    dx = RNG.normal(size=x.shape)
    dw = RNG.normal(size=wt.shape)
    z = np.zeros(5)
    assert abs((U.conv(dx, wt, z) * g).sum() - (gx * dx).sum()) < 1e-10
    assert abs((U.conv(x, dw, z) * g).sum() - (gw * dw).sum()) < 1e-10
    np.testing.assert_allclose(gb, g.sum(axis=(0, 1, 2)))


def test_pool_and_upsample_backward_are_adjoints():
    x = RNG.normal(size=(2, 8, 6, 3))
    g = RNG.normal(size=(2, 4, 3, 3))
    assert abs((U.pool(x) * g).sum() - (x * U.pool_backward(g)).sum()) < 1e-12
    y = RNG.normal(size=(2, 4, 3, 3))
    G = RNG.normal(size=(2, 8, 6, 3))
    assert abs((U.up(y) * G).sum() - (y * U.up_backward(G)).sum()) < 1e-12


def test_loss_gradient_matches_finite_differences():
    base = 16
    L, npar = U.layers(base)
    params = np.zeros(npar)
    for i, l in enumerate(L):
        nw = l["cout"] * l["ks"] ** 2 * l["cin"]
        params[l["woff"]:l["woff"] + nw] = RNG.normal(size=nw) * np.sqrt(2.0 / (l["ks"] ** 2 * l["cin"]))
        params[l["boff"]:l["boff"] + l["cout"]] = RNG.normal(size=l["cout"]) * 0.1
    xin = RNG.normal(size=(1, 8, 8, 4))
    target = RNG.normal(size=(1, 8, 8, 4))
    wch = np.array([1.0, 2.0, 0.5, 1.5])
    lval, grad = U.loss_grad(params, xin, target, wch, base)
    assert abs(lval - U.loss(params, xin, target, wch, base)) < 1e-14
    eps = 1e-6
    for i, l in enumerate(L):
        nw = l["cout"] * l["ks"] ** 2 * l["cin"]
        idx = list(RNG.choice(nw, size=6, replace=False) + l["woff"]) + [l["boff"]]
        for k in idx:
            p = params.copy()
            p[k] += eps
            lp = U.loss(p, xin, target, wch, base)
            p[k] -= 2 * eps
            lm = U.loss(p, xin, target, wch, base)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(grad[k])) + 1e-9, (i, k, fd, grad[k])


def test_bf16_rounding():
    # ties to even and ordinary rounding of the 8-bit significand
    assert U.bf16_round(1.0) == 1.0
    assert U.bf16_round(1.0 + 2 ** -8) == 1.0          # tie, round to even
    assert U.bf16_round(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7      # nearest
    assert U.bf16_round(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
