"""Fused pointwise MLP of the surrogate blocks (fwi_nn_mlp_forward /
fwi_nn_mlp_vjp) on the GPU.

Against an FP64 reference of the same block on the same BF16 inputs, rounding
to BF16 at the same points: the GPU accumulates in FP32 on the matrix cores,
so a rounded value can land one BF16 step away where the FP64 sum sits near a
rounding boundary; those isolated one-step differences bound the error at a
few 1e-3 relative L2.  The surrogate's fused path is then compared with its
two-GEMM path, which must give the same bits, and the mixing along x
(fwi_nn_mix_forward / fwi_nn_mix_vjp) with the tiled GEMM plus the same
roundings, also bit for bit.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _bf(x):  # FP64 values rounded to BF16, as FP64
    return torch.from_numpy(np.asarray(x, np.float64)).float().to(torch.bfloat16).double().numpy()


def _gelu(p):
    from scipy.special import erf

    return 0.5 * p * (1.0 + erf(p / np.sqrt(2.0)))


def _gelu_d(p):
    from scipy.special import erf

    return 0.5 * (1.0 + erf(p / np.sqrt(2.0))) + p * np.exp(-0.5 * p * p) / np.sqrt(2.0 * np.pi)


def _inputs(R, seed):
    rng = np.random.default_rng(seed)
    f = lambda *s, sc=1.0: _bf(rng.standard_normal(s) * sc)
    return dict(a=f(R, 64), res=f(R, 64), dg=f(R, 64), W1=f(64, 128, sc=64 ** -0.5), W2=f(128, 64, sc=128 ** -0.5),
                b1=(rng.standard_normal(128) * 0.1).astype(np.float32).astype(np.float64),
                b2=(rng.standard_normal(64) * 0.1).astype(np.float32).astype(np.float64))


def _reference(x):
    p = _bf(x["a"] @ x["W1"] + x["b1"])
    h = _bf(x["res"] + _bf(_bf(_gelu(p)) @ x["W2"] + x["b2"]))
    dp = _bf((x["dg"] @ x["W2"].T) * _gelu_d(p))
    return h, dp @ x["W1"].T


def _dev16(a, dev, extra_rows=0):
    t = torch.from_numpy(np.asarray(a, np.float64)).float().to(torch.bfloat16)
    if extra_rows:
        t = torch.cat([t, torch.zeros((extra_rows,) + tuple(t.shape[1:]), dtype=torch.bfloat16)])
    return t.to(dev).contiguous()


def _run(x, dev, R, pad=16):
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    t = {k: _dev16(x[k], dev) for k in ("a", "res", "dg", "W1", "W2")}
    b1 = torch.tensor(x["b1"], dtype=torch.float32, device=dev)
    b2 = torch.tensor(x["b2"], dtype=torch.float32, device=dev)
    sentinel16 = torch.full((R + pad, 64), 7.0, dtype=torch.bfloat16, device=dev)
    sentinel32 = torch.full((R + pad, 64), 7.0, dtype=torch.float32, device=dev)
    assert L.fwi_nn_mlp_forward(R, _p(t["a"]), _p(t["W1"]), _p(b1), _p(t["W2"]), _p(b2), _p(t["res"]),
                                _p(sentinel16), _stream()) == 0
    assert L.fwi_nn_mlp_vjp(R, _p(t["dg"]), _p(t["a"]), _p(t["W1"]), _p(b1), _p(t["W2"]), _p(sentinel32),
                            _stream()) == 0
    torch.cuda.synchronize()
    h = sentinel16.double().cpu().numpy()
    da = sentinel32.double().cpu().numpy()
    # rows past R untouched
    assert np.all(h[R:] == 7.0) and np.all(da[R:] == 7.0)
    return h[:R], da[:R]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("R", [1, 17, 64, 1007, 4096 + 48])
def test_mlp_forward_and_vjp_match_reference(dev, R):
    x = _inputs(R, 11 + R)
    h, da = _run(x, dev, R)
    h_ref, da_ref = _reference(x)
    eh, ea = _rel(h, h_ref), _rel(da, da_ref)
    print(f"R={R} h rel L2 {eh:.2e}  da rel L2 {ea:.2e}")
    assert eh <= 3e-3 and ea <= 5e-3
    # element-wise: at most a couple of BF16 steps of the block output
    assert np.all(np.abs(h - h_ref) <= 2 * 2.0 ** -7 * np.maximum(np.abs(h_ref), 1.0))


def test_mlp_large_rows_sampled(dev):
    """The decoder's row count at 16 samples (16 x 256 x 72), checked on a
    sample of rows (rows are independent)."""
    R = 16 * 256 * 72
    x = _inputs(R, 5)
    h, da = _run(x, dev, R)
    rows = np.random.default_rng(0).choice(R, 2000, replace=False)
    xs = {k: (v[rows] if k in ("a", "res", "dg") else v) for k, v in x.items()}
    h_ref, da_ref = _reference(xs)
    assert _rel(h[rows], h_ref) <= 3e-3 and _rel(da[rows], da_ref) <= 5e-3


def test_mlp_argument_errors(dev):
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    a = torch.zeros((33, 64), dtype=torch.bfloat16, device=dev)
    W1 = torch.zeros((64, 128), dtype=torch.bfloat16, device=dev)
    W2 = torch.zeros((128, 64), dtype=torch.bfloat16, device=dev)
    b = torch.zeros(128, dtype=torch.float32, device=dev)
    o32 = torch.zeros((33, 64), dtype=torch.float32, device=dev)
    s = _stream()
    assert L.fwi_nn_mlp_forward(-1, _p(a), _p(W1), _p(b), _p(W2), _p(b), _p(a), _p(a), s) == -1
    assert L.fwi_nn_mlp_forward(0, None, None, None, None, None, None, None, s) == 0
    assert L.fwi_nn_mlp_forward(16, _p(a), _p(W1), None, _p(W2), _p(b), _p(a), _p(a), s) == -1
    mis = ctypes.c_void_p(a.data_ptr() + 2)  # one element off: not 16-byte aligned
    assert L.fwi_nn_mlp_forward(16, mis, _p(W1), _p(b), _p(W2), _p(b), _p(a), _p(a), s) == -1
    assert L.fwi_nn_mlp_vjp(16, _p(a), mis, _p(W1), _p(b), _p(W2), _p(o32), s) == -1
    assert L.fwi_nn_mlp_vjp(16, _p(a), _p(a), _p(W1), _p(b), _p(W2), None, s) == -1


@pytest.fixture(scope="module")
def sur_case(dev):
    from oracle import surrogate as S
    import fwi_inputs as fi
    from paper_2603_16393_amd.surrogate import Surrogate

    params = S.init_params(4)
    v = np.stack([fi.faulted_model(70, 70, s) for s in (3, 4, 5)]).astype(np.float32)
    dtr = np.random.default_rng(9).standard_normal((3, S.NS, S.NR, S.NT)).astype(np.float32)
    sur = Surrogate(max_batch=4, device=dev)
    sur.set_params(params)
    yield params, torch.tensor(v, device=dev), torch.tensor(dtr, device=dev), sur
    sur.close()


def test_surrogate_fused_path_is_bitwise_the_gemm_path(dev, sur_case):
    """Forward traces, the input VJP, and the weight gradients (which, after a
    fused forward, recompute the hidden activations) agree bit for bit."""
    params, v, dtr, sur = sur_case
    out = {}
    for fused in (False, True):
        sur.set_fused_mlp(fused)
        tr = sur.forward(v).clone()
        dv = sur.backward(dtr).clone()
        dv_w = sur.backward(dtr, want_weight_grads=True).clone()
        out[fused] = (tr, dv, dv_w, sur.get_grads())
    sur.set_fused_mlp(True)
    for i in range(3):
        assert torch.equal(out[False][i], out[True][i]), i
    assert np.array_equal(out[False][3], out[True][3])
    assert torch.equal(out[True][1], out[True][2])


def test_surrogate_train_step_fused_equals_gemm_path(dev, sur_case):
    from paper_2603_16393_amd.surrogate import Surrogate

    params, v, dtr, _ = sur_case
    target = dtr * 0.01
    got = []
    for fused in (False, True):
        s = Surrogate(max_batch=4, device=dev)
        s.set_params(params)
        s.set_fused_mlp(fused)
        losses = [float(s.train_step(v, target, lr=1e-3)) for _ in range(2)]
        got.append((losses, s.get_params()))
        s.close()
    assert got[0][0] == got[1][0]
    assert np.array_equal(got[0][1], got[1][1])


def test_set_fused_mlp_rejects_other_values(dev, sur_case):
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    sur = sur_case[3]
    assert L.fwi_sur_set_fused_mlp(sur._h, 2) == -1
    assert L.fwi_sur_set_fused_mlp(None, 1) == -1


def _gemm32(L, M, N, K, batch, A, lda, sA, tA, B, ldb, sB, C32, ldc, sC, beta):
    rc = L.fwi_nn_gemm(M, N, K, batch, _p(A), lda, sA, tA, _p(B), ldb, sB, 0, _p(C32), None, ldc, sC, 1.0, beta,
                       None, 0, 1, None, _stream())
    assert rc == 0


@pytest.mark.parametrize("S", [1, 3, 37, 4096])
def test_mix_matches_gemm_path_bitwise(dev, S):
    """Mixing along x (fwi_nn_mix_forward / fwi_nn_mix_vjp) equals the tiled GEMM
    (FP32 output) followed by the same roundings, bit for bit."""
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    gen = torch.Generator(device="cpu").manual_seed(S)
    bf = lambda *s, sc=1.0: (torch.randn(*s, generator=gen) * sc).to(torch.bfloat16).to(dev).contiguous()
    Xm = bf(72, 72, sc=72 ** -0.5)
    g = bf(S, 72, 64)
    d32 = (torch.randn(S, 72, 64, generator=gen)).to(dev)
    # forward: g1 = R(g + R(Xm g))
    g1 = torch.full_like(g, 3.0)
    assert L.fwi_nn_mix_forward(S, _p(Xm), _p(g), _p(g1), _stream()) == 0
    acc = torch.empty(S, 72, 64, device=dev)
    _gemm32(L, 72, 64, 72, S, Xm, 72, 0, 0, g, 64, 72 * 64, acc, 64, 72 * 64, 0.0)
    ref = (g.float() + acc.to(torch.bfloat16).float()).to(torch.bfloat16)
    torch.cuda.synchronize()
    assert torch.equal(g1, ref)
    # VJP: d32 += Xm^T d1, d16 = R(d32)
    ref32 = d32.clone()
    _gemm32(L, 72, 64, 72, S, Xm, 72, 0, 1, g, 64, 72 * 64, ref32, 64, 72 * 64, 1.0)
    d16 = torch.full_like(g, 3.0)
    assert L.fwi_nn_mix_vjp(S, _p(Xm), _p(g), _p(d32), _p(d16), _stream()) == 0
    torch.cuda.synchronize()
    assert torch.equal(d32, ref32)
    assert torch.equal(d16, ref32.to(torch.bfloat16))


def test_mix_argument_errors(dev):
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    x = torch.zeros(2, 72, 64, dtype=torch.bfloat16, device=dev)
    assert L.fwi_nn_mix_forward(-1, _p(x), _p(x), _p(x), _stream()) == -1
    assert L.fwi_nn_mix_forward(0, None, None, None, _stream()) == 0
    assert L.fwi_nn_mix_forward(1, _p(x), ctypes.c_void_p(x.data_ptr() + 2), _p(x), _stream()) == -1
    assert L.fwi_nn_mix_vjp(1, _p(x), _p(x), None, _p(x), _stream()) == -1
