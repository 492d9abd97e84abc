"""FP64 CPU oracle of the surrogate network (test infrastructure only).

A plain numpy forward pass and a hand-written backward pass of the 4-level U-Net that the HIP
library trains: 3x3 convolutions with circular padding, 2x2 average pooling, nearest 2x
upsampling, skip concatenation, ReLU, a 1x1 head, prediction = input + head[:in_ch], loss =
mean over pixels and channels of w_c (prediction - target)^2. It shares no code with the HIP
path; only the flat parameter order is common (an interface): layer by layer (encoder 0..3,
decoder 2, 1, 0, head), weights [cout][ks*ks][cin] then bias [cout].

Pinned by tests/test_unet_oracle.py: the convolution against a direct quadruple loop, and every
gradient against central finite differences of the oracle's own loss.
"""
import numpy as np


def layers(base=32, in_pad=16):
    c = [base << l for l in range(4)]
    spec = [(in_pad, c[0], 3), (c[0], c[1], 3), (c[1], c[2], 3), (c[2], c[3], 3),
            (c[3] + c[2], c[2], 3), (c[2] + c[1], c[1], 3), (c[1] + c[0], c[0], 3), (c[0], 16, 1)]
    out, off = [], 0
    for cin, cout, ks in spec:
        nw = cout * ks * ks * cin
        out.append(dict(cin=cin, cout=cout, ks=ks, woff=off, boff=off + nw))
        off += nw + cout
    return out, off


def unpack(params, base=32):
    L, n = layers(base)
    assert params.size == n
    ws = []
    for l in L:
        w = params[l["woff"]:l["woff"] + l["cout"] * l["ks"] ** 2 * l["cin"]]
        ws.append((w.reshape(l["cout"], l["ks"] ** 2, l["cin"]), params[l["boff"]:l["boff"] + l["cout"]]))
    return ws


def offsets(ks):
    if ks == 1:
        return [(0, 0)]
    return [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def shift(x, dy, dx):
    """x[n, (y + dy) mod H, (x + dx) mod W, c]"""
    return np.roll(x, shift=(-dy, -dx), axis=(1, 2))


def conv(x, w, b):
    """y[p, co] = b[co] + sum_{tap, ci} x[p + off(tap), ci] w[co, tap, ci] (circular)"""
    ks = int(round(np.sqrt(w.shape[1])))
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (dy, dx) in enumerate(offsets(ks)):
        y += shift(x, dy, dx) @ w[:, t, :].T
    return y + b


def conv_backward(x, w, gy):
    """gradients of conv with respect to x, w, b given the output gradient gy"""
    ks = int(round(np.sqrt(w.shape[1])))
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for t, (dy, dx) in enumerate(offsets(ks)):
        xs = shift(x, dy, dx)
        gw[:, t, :] = np.einsum("nhwo,nhwi->oi", gy, xs)
        gx += shift(gy @ w[:, t, :], -dy, -dx)
    return gx, gw, gy.sum(axis=(0, 1, 2))


def pool(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(g):
    n, h, w, c = g.shape
    return g.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def forward(params, xin, base=32):
    """prediction and the activations the backward pass needs; xin [n, h, w, in_ch]"""
    ws = unpack(params, base)
    n, h, w, cin = xin.shape
    x0 = np.zeros((n, h, w, 16))
    x0[..., :cin] = xin
    A = {"x0": x0}
    relu = lambda z: np.maximum(z, 0.0)
    A["e0"] = relu(conv(x0, *ws[0]))
    A["p1"] = pool(A["e0"])
    A["e1"] = relu(conv(A["p1"], *ws[1]))
    A["p2"] = pool(A["e1"])
    A["e2"] = relu(conv(A["p2"], *ws[2]))
    A["p3"] = pool(A["e2"])
    A["e3"] = relu(conv(A["p3"], *ws[3]))
    A["u2"] = np.concatenate([up(A["e3"]), A["e2"]], axis=-1)
    A["d2"] = relu(conv(A["u2"], *ws[4]))
    A["u1"] = np.concatenate([up(A["d2"]), A["e1"]], axis=-1)
    A["d1"] = relu(conv(A["u1"], *ws[5]))
    A["u0"] = np.concatenate([up(A["d1"]), A["e0"]], axis=-1)
    A["d0"] = relu(conv(A["u0"], *ws[6]))
    A["y"] = conv(A["d0"], *ws[7])
    pred = xin + A["y"][..., :cin]
    return pred, A


def loss(params, xin, target, wch=None, base=32):
    pred, _ = forward(params, xin, base)
    wc = np.ones(xin.shape[-1]) if wch is None else np.asarray(wch)[:xin.shape[-1]]
    return float((wc * (pred - target) ** 2).sum() / pred.size)


def loss_grad(params, xin, target, wch=None, base=32):
    """loss and its gradient with respect to the flat parameter vector"""
    ws = unpack(params, base)
    L, _ = layers(base)
    pred, A = forward(params, xin, base)
    cin = xin.shape[-1]
    wc = np.ones(cin) if wch is None else np.asarray(wch)[:cin]
    d = pred - target
    lval = float((wc * d ** 2).sum() / pred.size)
    grad = np.zeros_like(params)

    def put(i, gw, gb):
        l = L[i]
        grad[l["woff"]:l["woff"] + gw.size] = gw.ravel()
        grad[l["boff"]:l["boff"] + gb.size] = gb

    gy = np.zeros(A["y"].shape)
    gy[..., :cin] = 2.0 * wc * d / pred.size
    gd0, gw, gb = conv_backward(A["d0"], ws[7][0], gy)
    put(7, gw, gb)
    gd0 = gd0 * (A["d0"] > 0)
    gu0, gw, gb = conv_backward(A["u0"], ws[6][0], gd0)
    put(6, gw, gb)
    c1 = A["d1"].shape[-1]
    gd1 = up_backward(gu0[..., :c1]) * (A["d1"] > 0)
    ge0 = gu0[..., c1:]
    gu1, gw, gb = conv_backward(A["u1"], ws[5][0], gd1)
    put(5, gw, gb)
    c2 = A["d2"].shape[-1]
    gd2 = up_backward(gu1[..., :c2]) * (A["d2"] > 0)
    ge1 = gu1[..., c2:]
    gu2, gw, gb = conv_backward(A["u2"], ws[4][0], gd2)
    put(4, gw, gb)
    c3 = A["e3"].shape[-1]
    ge3 = up_backward(gu2[..., :c3]) * (A["e3"] > 0)
    ge2 = gu2[..., c3:]
    gp3, gw, gb = conv_backward(A["p3"], ws[3][0], ge3)
    put(3, gw, gb)
    ge2 = (ge2 + pool_backward(gp3)) * (A["e2"] > 0)
    gp2, gw, gb = conv_backward(A["p2"], ws[2][0], ge2)
    put(2, gw, gb)
    ge1 = (ge1 + pool_backward(gp2)) * (A["e1"] > 0)
    gp1, gw, gb = conv_backward(A["p1"], ws[1][0], ge1)
    put(1, gw, gb)
    ge0 = (ge0 + pool_backward(gp1)) * (A["e0"] > 0)
    _, gw, gb = conv_backward(A["x0"], ws[0][0], ge0)
    put(0, gw, gb)
    return lval, grad


def bf16_round(a):
    """round float64 values to the nearest BF16 (ties to even), returned as float64"""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
