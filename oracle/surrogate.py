"""FP64 reference of the learned trace surrogate (TEST INFRASTRUCTURE ONLY).

Only the tests may import this module.  It is the plain numpy statement of
the network the HIP kernels implement, layer by layer, plus its backward pass
written out by the chain rule.  ``rounding=True`` rounds to BF16 exactly where
the GPU stores BF16 (activations and GEMM weights), so that GPU and reference
see the same numbers; ``rounding=False`` is pure FP64 (used for the
finite-difference pins of the backward pass).

Network (v -> traces for 5 surface shots x 70 receivers x 1000 samples):
  lift      h = W_l^T [ (v - 3000)/1500, z/72, x/72 ] + b_l   on a 72 x 72 grid
            (the 70 x 70 model edge-extended), 64 channels
  encoder   4 x { a = dw3x3(h); h = h + W2^T gelu(W1^T a + b1) + b2 }
  depth->time  y[t] = sum_z T[t, z] h[z]             (256 time rows)
  decoder   4 x { g = g + X g (mixing along x); a = dw3x3(g); g = g + W2^T gelu(W1^T a + b1) + b2 }
  head      o = W_p^T g + b_p (8 channels, 5 used)
  time      out[u] = sum_t U[u, t] o[t] (1000 samples), traces = out_scale * out
"""
from __future__ import annotations

import numpy as np

Z = X = 72
C, CH, T, S = 64, 128, 256, 8
NT, NR, NS = 1000, 70, 5
NZ = NX = 70
NBLK = 4


def bf(x):
    """Round to BFloat16 (nearest even) through FP32, returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def gelu(p):
    from scipy.special import erf

    return 0.5 * p * (1.0 + erf(p / np.sqrt(2.0)))


def gelu_grad(p):
    from scipy.special import erf

    return 0.5 * (1.0 + erf(p / np.sqrt(2.0))) + p * np.exp(-0.5 * p * p) / np.sqrt(2.0 * np.pi)


def dw3x3(h, k, b):
    """Depthwise 3x3 correlation with zero padding; h [n, H, W, C], k [C, 3, 3]."""
    n, H, W, Cc = h.shape
    hp = np.zeros((n, H + 2, W + 2, Cc))
    hp[:, 1:-1, 1:-1, :] = h
    out = np.zeros_like(h) + b[None, None, None, :]
    for dy in range(3):
        for dx in range(3):
            out += hp[:, dy:dy + H, dx:dx + W, :] * k[None, None, None, :, dy, dx]
    return out


def dw3x3_backward(h, k, dout):
    """Gradients of dw3x3 w.r.t. its input, kernel and bias."""
    n, H, W, Cc = h.shape
    hp = np.zeros((n, H + 2, W + 2, Cc))
    hp[:, 1:-1, 1:-1, :] = h
    dhp = np.zeros_like(hp)
    dk = np.zeros_like(k)
    for dy in range(3):
        for dx in range(3):
            dk[:, dy, dx] = np.sum(hp[:, dy:dy + H, dx:dx + W, :] * dout, axis=(0, 1, 2))
            dhp[:, dy:dy + H, dx:dx + W, :] += dout * k[None, None, None, :, dy, dx]
    return dhp[:, 1:-1, 1:-1, :], dk, dout.sum(axis=(0, 1, 2))


def init_params(seed: int = 0) -> dict:
    """Random parameters with the shapes of the network (any values serve the checks)."""
    rng = np.random.default_rng(seed)
    p = {"lift_w": rng.standard_normal((3, C)) * 0.5, "lift_b": rng.standard_normal(C) * 0.1}
    for name in ("enc", "dec"):
        for i in range(NBLK):
            q = f"{name}{i}_"
            p[q + "dw_k"] = rng.standard_normal((C, 3, 3)) * 0.3
            p[q + "dw_b"] = rng.standard_normal(C) * 0.05
            p[q + "w1"] = rng.standard_normal((C, CH)) / np.sqrt(C)
            p[q + "b1"] = rng.standard_normal(CH) * 0.05
            p[q + "w2"] = rng.standard_normal((CH, C)) / np.sqrt(CH) * 0.3
            p[q + "b2"] = rng.standard_normal(C) * 0.02
            if name == "dec":
                p[q + "xm"] = rng.standard_normal((X, X)) / np.sqrt(X) * 0.3
    p["d2t"] = rng.standard_normal((T, Z)) / np.sqrt(Z)
    p["proj_w"] = rng.standard_normal((C, S)) / np.sqrt(C)
    p["proj_b"] = rng.standard_normal(S) * 0.01
    p["up"] = rng.standard_normal((NT, T)) / np.sqrt(T)
    p["out_scale"] = 0.05
    return p


def _pad_input(v):
    """[n, 70, 70] m/s -> [n, 72, 72, 3] (normalised velocity, z/72, x/72)."""
    n = v.shape[0]
    zi = np.minimum(np.arange(Z), NZ - 1)
    xi = np.minimum(np.arange(X), NX - 1)
    vp = v[:, zi][:, :, xi]
    feat = np.zeros((n, Z, X, 3))
    feat[..., 0] = (vp - 3000.0) / 1500.0
    feat[..., 1] = (np.arange(Z) / Z)[None, :, None]
    feat[..., 2] = (np.arange(X) / X)[None, None, :]
    return feat


def forward(params, v, rounding: bool = True):
    """Traces [n, 5, 70, 1000] and the saved activations for backward."""
    R = bf if rounding else (lambda a: np.asarray(a, np.float64))
    W = bf if rounding else (lambda a: np.asarray(a, np.float64))
    v = np.asarray(v, np.float64)
    n = v.shape[0]
    cache = {"v": v}
    feat = _pad_input(v)
    cache["feat"] = feat
    h = R(feat @ params["lift_w"] + params["lift_b"])
    for i in range(NBLK):
        q = f"enc{i}_"
        a = R(dw3x3(h, params[q + "dw_k"], params[q + "dw_b"]))
        pp = R(a @ W(params[q + "w1"]) + params[q + "b1"])
        g = R(gelu(pp))
        r = R(g @ W(params[q + "w2"]) + params[q + "b2"])
        cache[q] = (h, a, pp, g)
        h = R(h + r)
    cache["enc_out"] = h
    y = R(np.einsum("tz,nzxc->ntxc", W(params["d2t"]), h))
    g = y
    for i in range(NBLK):
        q = f"dec{i}_"
        m = R(np.einsum("ab,ntbc->ntac", W(params[q + "xm"]), g))
        g1 = R(g + m)
        a = R(dw3x3(g1, params[q + "dw_k"], params[q + "dw_b"]))
        pp = R(a @ W(params[q + "w1"]) + params[q + "b1"])
        gg = R(gelu(pp))
        r = R(gg @ W(params[q + "w2"]) + params[q + "b2"])
        cache[q] = (g, g1, a, pp, gg)
        g = R(g1 + r)
    cache["dec_out"] = g
    o = R(g @ W(params["proj_w"]) + params["proj_b"])
    cache["o"] = o
    out = np.einsum("ut,ntk->nuk", W(params["up"]), o.reshape(n, T, X * S))  # [n, 1000, 72*8], FP32 on the GPU
    out = out.reshape(n, NT, X, S)
    traces = params["out_scale"] * np.transpose(out[:, :, :NR, :NS], (0, 3, 2, 1))
    return traces, cache


def backward(params, cache, dtraces):
    """Chain rule through forward(): returns (dv, grads dict)."""
    v = cache["v"]
    n = v.shape[0]
    grads = {}
    dout = np.zeros((n, NT, X, S))
    dout[:, :, :NR, :NS] = params["out_scale"] * np.transpose(dtraces, (0, 3, 2, 1))
    dout = dout.reshape(n, NT, X * S)
    o = cache["o"]
    o2 = o.reshape(n, T, X * S)
    grads["up"] = np.einsum("nuk,ntk->ut", dout, o2)
    do = np.einsum("ut,nuk->ntk", params["up"], dout).reshape(n, T, X, S)
    g = cache["dec_out"]
    grads["proj_w"] = np.einsum("ntxc,ntxs->cs", g, do)
    grads["proj_b"] = do.sum(axis=(0, 1, 2))
    dg = do @ params["proj_w"].T
    for i in reversed(range(NBLK)):
        q = f"dec{i}_"
        g0, g1, a, pp, gg = cache[q]
        dr = dg
        grads[q + "w2"] = np.einsum("ntxh,ntxc->hc", gg, dr)
        grads[q + "b2"] = dr.sum(axis=(0, 1, 2))
        dgg = dr @ params[q + "w2"].T
        dpp = dgg * gelu_grad(pp)
        grads[q + "w1"] = np.einsum("ntxc,ntxh->ch", a, dpp)
        grads[q + "b1"] = dpp.sum(axis=(0, 1, 2))
        da = dpp @ params[q + "w1"].T
        dg1_dw, grads[q + "dw_k"], grads[q + "dw_b"] = dw3x3_backward(g1, params[q + "dw_k"], da)
        dg1 = dg + dg1_dw
        grads[q + "xm"] = np.einsum("ntac,ntbc->ab", dg1, g0)
        dg = dg1 + np.einsum("ab,ntac->ntbc", params[q + "xm"], dg1)
    h = cache["enc_out"]
    grads["d2t"] = np.einsum("ntxc,nzxc->tz", dg, h)
    dh = np.einsum("tz,ntxc->nzxc", params["d2t"], dg)
    for i in reversed(range(NBLK)):
        q = f"enc{i}_"
        h0, a, pp, gg = cache[q]
        dr = dh
        grads[q + "w2"] = np.einsum("nzxh,nzxc->hc", gg, dr)
        grads[q + "b2"] = dr.sum(axis=(0, 1, 2))
        dgg = dr @ params[q + "w2"].T
        dpp = dgg * gelu_grad(pp)
        grads[q + "w1"] = np.einsum("nzxc,nzxh->ch", a, dpp)
        grads[q + "b1"] = dpp.sum(axis=(0, 1, 2))
        da = dpp @ params[q + "w1"].T
        dh_dw, grads[q + "dw_k"], grads[q + "dw_b"] = dw3x3_backward(h0, params[q + "dw_k"], da)
        dh = dh + dh_dw
    feat = cache["feat"]
    grads["lift_w"] = np.einsum("nzxf,nzxc->fc", feat, dh)
    grads["lift_b"] = dh.sum(axis=(0, 1, 2))
    dfeat0 = dh @ params["lift_w"][0] / 1500.0  # d(feature 0)/dv = 1/1500
    dv = np.zeros((n, NZ, NX))
    zi = np.minimum(np.arange(Z), NZ - 1)
    xi = np.minimum(np.arange(X), NX - 1)
    for z in range(Z):
        for x in range(X):
            dv[:, zi[z], xi[x]] += dfeat0[:, z, x]
    return dv, grads
