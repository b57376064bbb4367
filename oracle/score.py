"""FP64 reference of the score network (TEST INFRASTRUCTURE ONLY).

Only the tests may import this module.  It is the plain numpy statement of
the noise-prediction network eps_theta(x_t, t) that the HIP kernels
implement, layer by layer, with its backward pass written out by the chain
rule.  The network plays the role of the score model of Sec. 3 (denoising
score matching, Eqs. L1 / L2_rewrite, in the noise-prediction form
s = -eps / sqrt(1 - abar)), on which Algorithm 2's clean estimator
(Eq. v0hat) and the chain rule of Eq. chain_rule operate.

``rounding=True`` rounds to BF16 exactly where the GPU stores BF16
(activations, GEMM weights, and gradient streams where they feed a GEMM), so
GPU and reference see the same numbers; ``rounding=False`` is pure FP64 (used
for the finite-difference pins of the backward pass).

Network (x [B, 70, 70] in the normalised diffusion state, t in [0, 1]):
  time      e = [sin(1000 t f_k), cos(1000 t f_k)], f_k = 10000^(-k/16), k < 16;
            tb = W_t2^T gelu(W_t1^T e + b_t1) + b_t2     (320 per-channel biases, FP32)
  lift      on a 72 x 72 grid (the 70 x 70 state in rows/columns 1..70, zero
            ring): h = R(W_l^T [x, (i - 35.5)/36, (j - 35.5)/36] + b_l), 32 channels
  block(C)  p = R(conv3(h; W1) + b1 + tb_block); q = R(gelu(p));
            h' = R(h + R(conv3(q; W2) + b2))          (3 x 3, zero padding)
  U-Net     L0a(32) 72^2 -> pool, 1x1 32->64 -> L1a(64) 36^2 -> pool, 1x1 64->128 ->
            L2(128) 18^2 -> 1x1 128->64, nearest x2, + L1a -> L1b(64) ->
            1x1 64->32, nearest x2, + L0a -> L0b(32) -> head 1x1 32->1 (FP32)
  output    out = skip_b x + scale_b eps[1:71, 1:71] (per-sample affine map:
            eps itself, the score, or the clean estimate of Eq. v0hat)
Convolutions are written as im2col products: column tap * C + c with
tap = 3 dy + dx holds the input at (i + dy - 1, j + dx - 1).
"""
from __future__ import annotations

import numpy as np

from .surrogate import bf, gelu, gelu_grad

G = 72            # padded grid
NZ = NX = 70
C0, C1, C2 = 32, 64, 128
NF = 16           # time frequencies
TH = 128          # time MLP width
# (name, channels, grid) in forward order, and each block's offset in the time-bias vector
BLOCKS = (("b0a", C0, 72), ("b1a", C1, 36), ("b2", C2, 18), ("b1b", C1, 36), ("b0b", C0, 72))
TB_OFF = {}
_o = 0
for _n, _c, _g in BLOCKS:
    TB_OFF[_n] = _o
    _o += _c
NTB = _o          # 320
# weights that are matrix-core GEMM operands (held as BF16 on the GPU)
GEMM_WEIGHTS = frozenset([f"{n}_w{k}" for n, _, _ in BLOCKS for k in (1, 2)] +
                         ["down0_w", "down1_w", "up1_w", "up0_w"])


def layout():
    """[(name, shape)] in the order of the FP32 parameter vector (the C ABI's order)."""
    L = [("temb_w1", (2 * NF, TH)), ("temb_b1", (TH,)), ("temb_w2", (TH, NTB)), ("temb_b2", (NTB,)),
         ("lift_w", (3, C0)), ("lift_b", (C0,))]

    def blk(n, c):
        return [(f"{n}_w1", (9 * c, c)), (f"{n}_b1", (c,)), (f"{n}_w2", (9 * c, c)), (f"{n}_b2", (c,))]

    L += blk("b0a", C0) + [("down0_w", (C0, C1)), ("down0_b", (C1,))]
    L += blk("b1a", C1) + [("down1_w", (C1, C2)), ("down1_b", (C2,))]
    L += blk("b2", C2) + [("up1_w", (C2, C1)), ("up1_b", (C1,))]
    L += blk("b1b", C1) + [("up0_w", (C1, C0)), ("up0_b", (C0,))]
    L += blk("b0b", C0) + [("head_w", (C0,)), ("head_b", (1,))]
    return L


def param_count() -> int:
    return int(sum(np.prod(s) for _, s in layout()))


def unpack(vec) -> dict:
    vec = np.asarray(vec, np.float64)
    out, o = {}, 0
    for n, s in layout():
        k = int(np.prod(s))
        out[n] = vec[o:o + k].reshape(s)
        o += k
    assert o == vec.size
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[n], np.float64).reshape(-1) for n, _ in layout()])


def init_params(seed: int = 0) -> dict:
    """He-style random initialisation (the training starting point; any values serve the checks)."""
    rng = np.random.default_rng(seed)
    p = {}
    for n, s in layout():
        if n.endswith("_b") or n.endswith("_b1") or n.endswith("_b2"):
            p[n] = np.zeros(s)
        else:
            fan_in = s[0] if len(s) == 2 else C0
            p[n] = rng.standard_normal(s) * np.sqrt(2.0 / fan_in)
    for n, c, _ in BLOCKS:   # residual branches start small
        p[f"{n}_w2"] *= 0.1
    p["head_w"] *= 0.1
    return p


def time_features(t):
    t = np.asarray(t, np.float64).reshape(-1)
    f = np.exp(-np.log(10000.0) * np.arange(NF) / NF)
    a = 1000.0 * t[:, None] * f[None, :]
    return np.concatenate([np.sin(a), np.cos(a)], axis=1)


def im2col(h):
    """h [n, S, S, C] -> [n, S, S, 9 C] (zero padding), column tap * C + c, tap = 3 dy + dx."""
    n, S, _, Cc = h.shape
    hp = np.zeros((n, S + 2, S + 2, Cc))
    hp[:, 1:-1, 1:-1, :] = h
    cols = [hp[:, dy:dy + S, dx:dx + S, :] for dy in range(3) for dx in range(3)]
    return np.concatenate(cols, axis=3)


def col2im(dcol, Cc):
    """Transpose of im2col: [n, S, S, 9 C] -> [n, S, S, C]."""
    n, S = dcol.shape[0], dcol.shape[1]
    dhp = np.zeros((n, S + 2, S + 2, Cc))
    for tap in range(9):
        dy, dx = divmod(tap, 3)
        dhp[:, dy:dy + S, dx:dx + S, :] += dcol[..., tap * Cc:(tap + 1) * Cc]
    return dhp[:, 1:-1, 1:-1, :]


def pool(h):
    return 0.25 * (((h[:, 0::2, 0::2] + h[:, 0::2, 1::2]) + h[:, 1::2, 0::2]) + h[:, 1::2, 1::2])


def up2(y):
    return np.repeat(np.repeat(y, 2, axis=1), 2, axis=2)


def up2_transpose(d):
    return ((d[:, 0::2, 0::2] + d[:, 0::2, 1::2]) + d[:, 1::2, 0::2]) + d[:, 1::2, 1::2]


def forward(params: dict, x, t, skip=None, scale=None, rounding: bool = True):
    """out [B, 70, 70] and the cache for backward.  skip/scale: per-sample output map (default eps)."""
    R = bf if rounding else (lambda a: np.asarray(a, np.float64))
    x = np.asarray(x, np.float64)
    B = x.shape[0]
    skip = np.zeros(B) if skip is None else np.asarray(skip, np.float64).reshape(B)
    scale = np.ones(B) if scale is None else np.asarray(scale, np.float64).reshape(B)
    P = params
    W = {n: (R(P[n]) if n in GEMM_WEIGHTS else np.asarray(P[n], np.float64)) for n in P}
    cache = {"x": x, "skip": skip, "scale": scale, "W": W}
    # time embedding (FP32 on the GPU, no BF16)
    e = time_features(t)
    a1 = e @ P["temb_w1"] + P["temb_b1"]
    h1 = gelu(a1)
    tb = h1 @ P["temb_w2"] + P["temb_b2"]
    cache.update(e=e, a1=a1, th=h1, tb=tb)
    # lift
    feat = np.zeros((B, G, G, 3))
    feat[:, 1:71, 1:71, 0] = x
    ii = (np.arange(G) - 35.5) / 36.0
    feat[:, :, :, 1] = ii[None, :, None]
    feat[:, :, :, 2] = ii[None, None, :]
    h0 = R(feat @ P["lift_w"] + P["lift_b"])
    cache.update(feat=feat, h0=h0)

    def block(name, h):
        col1 = im2col(h)
        off = TB_OFF[name]
        Cc = h.shape[3]
        p = R(col1 @ W[f"{name}_w1"] + P[f"{name}_b1"] + tb[:, None, None, off:off + Cc])
        q = R(gelu(p))
        y2 = im2col(q) @ W[f"{name}_w2"] + P[f"{name}_b2"]
        out = R(h + R(y2))
        cache[name] = dict(h=h, p=p, q=q)
        return out

    hb0a = block("b0a", h0)
    pl0 = R(pool(hb0a))
    d1 = R(pl0 @ W["down0_w"] + P["down0_b"])
    hb1a = block("b1a", d1)
    pl1 = R(pool(hb1a))
    d2 = R(pl1 @ W["down1_w"] + P["down1_b"])
    hb2 = block("b2", d2)
    y1 = R(hb2 @ W["up1_w"] + P["up1_b"])
    u1 = R(up2(y1) + hb1a)
    hb1b = block("b1b", u1)
    y0 = R(hb1b @ W["up0_w"] + P["up0_b"])
    u0 = R(up2(y0) + hb0a)
    hb0b = block("b0b", u0)
    e72 = hb0b @ P["head_w"] + P["head_b"][0]
    eps = e72[:, 1:71, 1:71]
    out = skip[:, None, None] * x + scale[:, None, None] * eps
    cache.update(hb0a=hb0a, pl0=pl0, d1=d1, hb1a=hb1a, pl1=pl1, d2=d2, hb2=hb2, y1=y1, u1=u1, hb1b=hb1b, y0=y0,
                 u0=u0, hb0b=hb0b, eps=eps, rounding=rounding)
    return out, cache


def backward(params: dict, cache: dict, dout):
    """(dx [B, 70, 70], dparams dict) for the output map of forward()."""
    R = bf if cache["rounding"] else (lambda a: np.asarray(a, np.float64))
    P, W = params, cache["W"]
    dout = np.asarray(dout, np.float64)
    B = dout.shape[0]
    g = {}
    dx = cache["skip"][:, None, None] * dout
    de72 = np.zeros((B, G, G))
    de72[:, 1:71, 1:71] = cache["scale"][:, None, None] * dout
    g["head_w"] = np.einsum("bij,bijc->c", de72, cache["hb0b"])
    g["head_b"] = np.array([de72.sum()])
    dtb = np.zeros((B, NTB))

    def block_bwd(name, dh_out):
        c = cache[name]
        h, p, q = c["h"], c["p"], c["q"]
        Cc = h.shape[3]
        d16 = R(dh_out)
        g[f"{name}_b2"] = dh_out.sum(axis=(0, 1, 2))
        colq = im2col(q)
        g[f"{name}_w2"] = np.einsum("bijk,bijc->kc", colq, d16)
        dq = col2im(d16 @ W[f"{name}_w2"].T, Cc)
        dp = dq * gelu_grad(p)
        dp16 = R(dp)
        g[f"{name}_b1"] = dp.sum(axis=(0, 1, 2))
        off = TB_OFF[name]
        dtb[:, off:off + Cc] += dp.sum(axis=(1, 2))
        colh = im2col(h)
        g[f"{name}_w1"] = np.einsum("bijk,bijc->kc", colh, dp16)
        return dh_out + col2im(dp16 @ W[f"{name}_w1"].T, Cc)

    def lin_bwd(name, inp, dy):
        """y = R(inp W + b): gradients of W, b; returns d inp."""
        d16 = R(dy)
        g[f"{name}_b"] = dy.sum(axis=(0, 1, 2))
        g[f"{name}_w"] = np.einsum("bijk,bijc->kc", inp, d16)
        return d16 @ W[f"{name}_w"].T

    dh = de72[..., None] * P["head_w"][None, None, None, :]
    du0 = block_bwd("b0b", dh)
    dhb0a = du0.copy()                                  # skip of the upper U-Net level
    dhb1b = lin_bwd("up0", cache["hb1b"], up2_transpose(du0))
    du1 = block_bwd("b1b", dhb1b)
    dhb1a = du1.copy()
    dhb2 = lin_bwd("up1", cache["hb2"], up2_transpose(du1))
    dd2 = block_bwd("b2", dhb2)
    dpl1 = lin_bwd("down1", cache["pl1"], dd2)
    dhb1a += 0.25 * up2(dpl1)
    dd1 = block_bwd("b1a", dhb1a)
    dpl0 = lin_bwd("down0", cache["pl0"], dd1)
    dhb0a += 0.25 * up2(dpl0)
    dh0 = block_bwd("b0a", dhb0a)
    # lift
    feat = cache["feat"]
    g["lift_w"] = np.einsum("bijf,bijc->fc", feat, dh0)
    g["lift_b"] = dh0.sum(axis=(0, 1, 2))
    dx = dx + (dh0[:, 1:71, 1:71, :] @ P["lift_w"][0])
    # time embedding
    g["temb_w2"] = cache["th"].T @ dtb
    g["temb_b2"] = dtb.sum(axis=0)
    da1 = (dtb @ P["temb_w2"].T) * gelu_grad(cache["a1"])
    g["temb_w1"] = cache["e"].T @ da1
    g["temb_b1"] = da1.sum(axis=0)
    return dx, g


def dsm_loss(params: dict, x0, noise, t_index, abar, rounding: bool = True):
    """Denoising score matching in the noise-prediction form (Sec. 3, Eq. L2_rewrite with the weight
    lambda = 1 - abar): mean over samples and nodes of (eps_theta(x_t, t) - noise)^2 with
    x_t = sqrt(abar_i) x0 + sqrt(1 - abar_i) noise and t = i / N.  Returns (loss, dparams)."""
    x0 = np.asarray(x0, np.float64)
    noise = np.asarray(noise, np.float64)
    i = np.asarray(t_index).reshape(-1)
    ab = np.asarray(abar, np.float64)[i - 1]
    xt = np.sqrt(ab)[:, None, None] * x0 + np.sqrt(1.0 - ab)[:, None, None] * noise
    out, cache = forward(params, xt, i / float(len(abar)), rounding=rounding)
    r = out - noise
    n = r.size
    loss = float(np.sum(r * r) / n)
    _, g = backward(params, cache, 2.0 * r / n)
    return loss, g
