"""FP64 reference of the warm-start network (test infrastructure only).

Same layers, parameter layout and loss as the library's warm-start network.
Every convolution operand can be rounded to bfloat16 first (round to nearest,
ties to even, on the float32 bit pattern), which is how the matrix-core
kernels consume them; products are then summed in FP64.  With ``bf16=False``
the network is plain FP64 (used for the finite-difference pins).
"""
from __future__ import annotations

import numpy as np

LAYERS = [(3, 16), (16, 32), (32, 64), (80, 32), (32, 6)]


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), via float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layout(K: int):
    """Offsets of (W_i, b_i) for the 5 convolutions, then (Wl, bl); total size."""
    offs, o = [], 0
    for cin, cout in LAYERS:
        offs.append((o, o + 9 * cin * cout))
        o += 9 * cin * cout + cout
    wl, bl = o, o + 64 * 2 * K
    return offs, wl, bl, bl + 2 * K


def unpack(params, K):
    offs, wl, bl, n = layout(K)
    p = np.asarray(params, dtype=np.float64)
    assert p.size == n
    Ws = [p[a:b].reshape(9 * cin, cout) for (a, b), (cin, cout) in zip(offs, LAYERS)]
    bs = [p[b:b + cout] for (a, b), (cin, cout) in zip(offs, LAYERS)]
    return Ws, bs, p[wl:bl].reshape(64, 2 * K), p[bl:n]


def im2col(x):
    """(B, H, W, C) -> (B*H*W, 9*C) with zero padding; column (kh*3 + kw)*C + c."""
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1] = x
    cols = [xp[:, kh:kh + H, kw:kw + W, :] for kh in range(3) for kw in range(3)]
    return np.concatenate(cols, axis=3).reshape(B * H * W, 9 * C)


def col2im(cols, shape):
    """Adjoint of im2col."""
    B, H, W, C = shape
    c = cols.reshape(B, H, W, 9, C)
    xp = np.zeros((B, H + 2, W + 2, C))
    for t in range(9):
        kh, kw = divmod(t, 3)
        xp[:, kh:kh + H, kw:kw + W, :] += c[:, :, :, t, :]
    return xp[:, 1:H + 1, 1:W + 1]


def conv(x, Wm, b, rnd):
    B, H, W, _ = x.shape
    r = bf16_round if rnd else (lambda a: a)
    y = r(im2col(x)) @ r(Wm) + b
    return y.reshape(B, H, W, -1)


def pool(x):
    return 0.25 * (x[:, 0::2, 0::2] + x[:, 1::2, 0::2] + x[:, 0::2, 1::2] + x[:, 1::2, 1::2])


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def forward(params, x, K, eps_min, eps_max, bf16=True):
    Ws, bs, Wl, bl = unpack(params, K)
    x = np.asarray(x, dtype=np.float64)
    a1 = np.maximum(conv(x, Ws[0], bs[0], bf16), 0)
    p1 = pool(a1)
    a2 = np.maximum(conv(p1, Ws[1], bs[1], bf16), 0)
    a3 = np.maximum(conv(a2, Ws[2], bs[2], bf16), 0)
    cat = np.concatenate([up(a3), a1], axis=3)
    a4 = np.maximum(conv(cat, Ws[3], bs[3], bf16), 0)
    z = conv(a4, Ws[4], bs[4], bf16)
    nz = np.sqrt(np.sum(z * z, axis=3, keepdims=True))
    mu = z / np.maximum(1.0, nz)
    g = a3.mean(axis=(1, 2))
    e = 1.0 / (1.0 + np.exp(-(g @ Wl + bl)))
    # the box E on a log scale: eps = eps_min (eps_max / eps_min)^e
    lo = np.tile(np.asarray(eps_min, dtype=np.float64), K)
    hi = np.tile(np.asarray(eps_max, dtype=np.float64), K)
    eps = lo * np.exp(e * np.log(hi / lo))
    cache = dict(x=x, a1=a1, p1=p1, a2=a2, a3=a3, cat=cat, a4=a4, z=z, nz=nz, mu=mu, g=g, e=e, lo=lo, hi=hi)
    return mu, eps.reshape(-1, K, 2), cache


def loss_grad(params, x, mu_t, eps_t, K, eps_min, eps_max, w_eps, bf16=True):
    """Loss and its gradient (backward written out layer by layer)."""
    Ws, bs, Wl, bl = unpack(params, K)
    mu, eps, c = forward(params, x, K, eps_min, eps_max, bf16)
    r = bf16_round if bf16 else (lambda a: a)
    B, H, W, _ = c["x"].shape
    P = B * H * W
    et = np.log(np.asarray(eps_t, dtype=np.float64).reshape(B, 2 * K) / c["lo"]) / np.log(c["hi"] / c["lo"])
    diff = mu - np.asarray(mu_t, dtype=np.float64)
    loss = np.sum(diff ** 2) / P + w_eps * np.mean((c["e"] - et) ** 2)
    grads = [None] * 5, [None] * 5
    gW, gb = grads
    # mu head: mu = z / max(1, |z|)
    dmu = 2.0 * diff / P
    nz = c["nz"]
    inside = nz <= 1.0
    dz = np.where(inside, dmu, (dmu - mu * np.sum(mu * dmu, axis=3, keepdims=True)) / np.maximum(nz, 1.0))

    def conv_back(i, xin, dy):
        cols = r(im2col(xin))
        dyf = dy.reshape(-1, dy.shape[3])
        gW[i] = cols.T @ r(dyf)
        gb[i] = dyf.sum(axis=0)
        return col2im(r(dyf) @ r(Ws[i]).T, xin.shape)

    d4 = conv_back(4, c["a4"], dz) * (c["a4"] > 0)
    dcat = conv_back(3, c["cat"], d4)
    # control head
    de = 2.0 * w_eps * (c["e"] - et) / (B * 2 * K)
    dpre = de * c["e"] * (1.0 - c["e"])
    gWl = c["g"].T @ dpre
    gbl = dpre.sum(axis=0)
    dg = dpre @ Wl.T
    du = dcat[..., :64]
    d3 = du[:, 0::2, 0::2] + du[:, 0::2, 1::2] + du[:, 1::2, 0::2] + du[:, 1::2, 1::2]
    d3 = d3 + dg[:, None, None, :] / (H // 2 * W // 2)
    d3 = d3 * (c["a3"] > 0)
    d2 = conv_back(2, c["a2"], d3) * (c["a2"] > 0)
    dp1 = conv_back(1, c["p1"], d2)
    d1 = (dcat[..., 64:] + 0.25 * up(dp1)) * (c["a1"] > 0)
    conv_back(0, c["x"], d1)
    offs, wl, bl_off, n = layout(K)
    g = np.zeros(n)
    for i, ((a, b), (cin, cout)) in enumerate(zip(offs, LAYERS)):
        g[a:b] = gW[i].ravel()
        g[b:b + cout] = gb[i]
    g[wl:bl_off] = gWl.ravel()
    g[bl_off:n] = gbl
    return loss, g
