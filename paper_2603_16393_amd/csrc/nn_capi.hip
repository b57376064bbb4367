// C ABI of the learned surrogate's building blocks and model (see fwi.h).
#include "nn_internal.h"

using namespace fwi;

extern "C" {

int fwi_nn_gemm(int M, int N, int K, int batch, const void* A, long lda, long strideA, int transA, const void* B,
                long ldb, long strideB, int transB, float* C32, void* C16, long ldc, long strideC, float alpha,
                float beta, const float* bias, int reduce_batch, int splitk, float* work, void* stream) {
    if (M < 0 || N < 0 || K < 0 || batch < 1 || splitk < 1) return FWI_EINVAL;
    if (lda < 1 || ldb < 1 || ldc < 1) return FWI_EINVAL;
    if (!transA ? lda < K : lda < M) return FWI_EINVAL;
    if (!transB ? ldb < N : ldb < K) return FWI_EINVAL;
    if (ldc < N) return FWI_EINVAL;
    GemmArgs g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.batch = batch;
    g.A = (const bf16_t*)A;
    g.lda = lda;
    g.strideA = strideA;
    g.transA = transA ? 1 : 0;
    g.B = (const bf16_t*)B;
    g.ldb = ldb;
    g.strideB = strideB;
    g.transB = transB ? 1 : 0;
    g.C32 = C32;
    g.C16 = (bf16_t*)C16;
    g.ldc = ldc;
    g.strideC = strideC;
    g.alpha = alpha;
    g.beta = beta;
    g.bias = bias;
    g.reduce_batch = reduce_batch ? 1 : 0;
    g.splitk = splitk;
    g.work = work;
    return gemm_bf16(g, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
