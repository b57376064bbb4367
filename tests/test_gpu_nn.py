"""Surrogate building blocks on the GPU vs FP64 references of the same BF16 values.

GEMM: every product of BF16 inputs is exact in FP64, so the only GPU error is
FP32 accumulation: |C - C_ref| <= 1e-5 * (|A| |B|)_ij element-wise (FP32 output)
or one BF16 rounding of the reference (BF16 output).
"""
import ctypes
import sys

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


def _bf16(x, dev):
    return torch.tensor(x, dtype=torch.float32, device=dev).to(torch.bfloat16).contiguous()


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


def _gemm(M, N, K, batch, A, lda, sA, tA, B, ldb, sB, tB, C32=None, C16=None, ldc=None, sC=0, alpha=1.0, beta=0.0,
          bias=None, reduce_batch=0, splitk=1, work=None):
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    rc = L.fwi_nn_gemm(M, N, K, batch, p(A), lda, sA, tA, p(B), ldb, sB, tB, p(C32), p(C16), ldc or N, sC, alpha,
                       beta, p(bias), reduce_batch, splitk, p(work),
                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()


def _ref(A, B, tA, tB):
    a = A.T if tA else A
    b = B.T if tB else B
    return a @ b, np.abs(a) @ np.abs(b)


@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (77, 50, 45), (128, 192, 96), (5, 3, 7), (300, 72, 256)])
@pytest.mark.parametrize("tA,tB", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_shapes_and_transposes(dev, M, N, K, tA, tB):
    rng = np.random.default_rng(M * 7 + N * 3 + K + 10 * tA + 20 * tB)
    A = _bf16(rng.standard_normal((K, M) if tA else (M, K)), dev)
    B = _bf16(rng.standard_normal((N, K) if tB else (K, N)), dev)
    C = torch.empty((M, N), dtype=torch.float32, device=dev)
    _gemm(M, N, K, 1, A, A.shape[1], 0, tA, B, B.shape[1], 0, tB, C32=C)
    ref, mag = _ref(_np(A), _np(B), tA, tB)
    assert np.all(np.abs(C.cpu().numpy() - ref) <= 1e-5 * mag + 1e-30), (M, N, K, tA, tB)


def test_gemm_batched_bias_beta_bf16_out(dev):
    rng = np.random.default_rng(1)
    M, N, K, nb = 70, 96, 64, 3
    A = _bf16(rng.standard_normal((nb, M, K)), dev)
    B = _bf16(rng.standard_normal((nb, K, N)), dev)
    C0 = rng.standard_normal((nb, M, N)).astype(np.float32)
    C = torch.tensor(C0, device=dev)
    bias = torch.tensor(rng.standard_normal(N).astype(np.float32), device=dev)
    _gemm(M, N, K, nb, A, K, M * K, 0, B, N, K * N, 0, C32=C, sC=M * N, alpha=0.5, beta=2.0, bias=bias)
    a, b = _np(A), _np(B)
    ref = 0.5 * np.einsum("bmk,bkn->bmn", a, b) + 2.0 * C0 + bias.cpu().numpy()[None, None, :]
    mag = 0.5 * np.einsum("bmk,bkn->bmn", np.abs(a), np.abs(b)) + 2 * np.abs(C0) + 1.0
    assert np.all(np.abs(C.cpu().numpy() - ref) <= 1e-5 * mag)
    C16 = torch.empty((nb, M, N), dtype=torch.bfloat16, device=dev)
    _gemm(M, N, K, nb, A, K, M * K, 0, B, N, K * N, 0, C16=C16, sC=M * N)
    ref16 = torch.tensor(np.einsum("bmk,bkn->bmn", a, b), dtype=torch.float32).to(torch.bfloat16).float().numpy()
    got = C16.float().cpu().numpy()
    # one BF16 rounding apart at most (FP32 accumulation order may flip a tie)
    assert np.all(np.abs(got - ref16) <= 2.0 ** -7 * np.abs(ref16) + 1e-30)


@pytest.mark.parametrize("splitk", [1, 4, 13])
def test_gemm_reduce_batch_splitk(dev, splitk):
    """Weight-gradient form: C = sum_b A_b^T B_b with a long reduction."""
    rng = np.random.default_rng(2)
    M, N, K, nb = 72, 40, 100, 9
    A = _bf16(rng.standard_normal((nb, K, M)), dev)   # stored [k][m] -> transA
    B = _bf16(rng.standard_normal((nb, N, K)), dev)   # stored [n][k] -> transB
    C = torch.empty((M, N), dtype=torch.float32, device=dev)
    work = torch.empty((splitk, M, N), dtype=torch.float32, device=dev)
    _gemm(M, N, K, nb, A, M, K * M, 1, B, K, N * K, 1, C32=C, reduce_batch=1, splitk=splitk, work=work)
    a, b = _np(A), _np(B)
    ref = np.einsum("bkm,bnk->mn", a, b)
    mag = np.einsum("bkm,bnk->mn", np.abs(a), np.abs(b))
    assert np.all(np.abs(C.cpu().numpy() - ref) <= 1e-5 * mag)
    C2 = torch.empty_like(C)
    _gemm(M, N, K, nb, A, M, K * M, 1, B, K, N * K, 1, C32=C2, reduce_batch=1, splitk=splitk, work=work)
    assert torch.equal(C, C2)  # deterministic


def test_gemm_long_k_splitk_single(dev):
    rng = np.random.default_rng(3)
    M, N, K = 64, 128, 20000
    A = _bf16(rng.standard_normal((K, M)), dev)
    B = _bf16(rng.standard_normal((K, N)), dev)
    C = torch.empty((M, N), dtype=torch.float32, device=dev)
    work = torch.empty((32, M, N), dtype=torch.float32, device=dev)
    _gemm(M, N, K, 1, A, M, 0, 1, B, N, 0, 0, C32=C, splitk=32, work=work)
    ref, mag = _ref(_np(A), _np(B), 1, 0)
    assert np.all(np.abs(C.cpu().numpy() - ref) <= 1e-5 * mag)
