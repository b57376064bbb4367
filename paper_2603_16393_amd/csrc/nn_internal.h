// Internal declarations of the learned surrogate's building blocks (BF16
// storage, FP32 accumulation) and its model object.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "fwi.h"

namespace fwi {

typedef uint16_t bf16_t;  // bfloat16 bit pattern

__host__ __device__ inline float bf2f(bf16_t h) {
    union {
        uint32_t u;
        float f;
    } v;
    v.u = (uint32_t)h << 16;
    return v.f;
}

// round to nearest even; NaN stays NaN.  On the device this is gfx950's
// v_cvt_pk_bf16_f32, which gives the bits of the integer rounding below for
// every non-NaN FP32 input (checked exhaustively over all 2^32 patterns).
__host__ __device__ inline bf16_t f2bf(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_bit_cast(bf16_t, (__bf16)f);
#else
    union {
        uint32_t u;
        float f;
    } v;
    v.f = f;
    if ((v.u & 0x7f800000u) == 0x7f800000u && (v.u & 0x007fffffu)) return (bf16_t)((v.u >> 16) | 0x40);
    const uint32_t r = v.u + 0x7fffu + ((v.u >> 16) & 1u);
    return (bf16_t)(r >> 16);
#endif
}

// GELU (erf form) and its derivative, shared by the element-wise kernels and
// the GEMM epilogues.
__device__ inline float gelu_f(float p) { return 0.5f * p * (1.f + erff(p * 0.70710678118654752f)); }
__device__ inline float gelu_d(float p) {
    return 0.5f * (1.f + erff(p * 0.70710678118654752f)) + p * expf(-0.5f * p * p) * 0.39894228040143268f;
}

// Epilogues of the GEMM (v = alpha acc + beta C + bias), each rounding exactly
// as the separate passes they replace:
enum GemmEpi {
    kEpiNone = 0,
    kEpiGelu = 1,     // C16 = R(v), aux16 = R(gelu(R(v)))
    kEpiResid = 2,    // C16 = R(res16 + R(v))
    kEpiGeluBwd = 3,  // v *= gelu'(p16); C32 = v, aux16 = R(v)
    kEpiDual = 4      // C32 = v, aux16 = R(v)
};

// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b] (+ bias[n]) for b < batch,
// or, with reduce_batch, C = alpha * sum_b op(A[b]) op(B[b]) + beta * C.
// A, B are BF16; op(A)[m][k] = transA ? A[k * lda + m] : A[m * lda + k],
// op(B)[k][n] = transB ? B[n * ldb + k] : B[k * ldb + n].  C is FP32 (C32) or
// BF16 (C16, exactly one of the two non-null).  Accumulation is FP32 on MFMA.
struct GemmArgs {
    int M = 0, N = 0, K = 0, batch = 1;
    const bf16_t* A = nullptr;
    long lda = 0, strideA = 0;
    int transA = 0;
    const bf16_t* B = nullptr;
    long ldb = 0, strideB = 0;
    int transB = 0;
    float* C32 = nullptr;
    bf16_t* C16 = nullptr;
    long ldc = 0, strideC = 0;
    float alpha = 1.f, beta = 0.f;
    const float* bias = nullptr;  // [N], added after alpha*acc + beta*C
    int reduce_batch = 0;
    // split-K over the (batch, k) reduction (batch == 1 or reduce_batch only):
    // partial sums go to work[splitk][M][N] and are added in split order
    int splitk = 1;
    float* work = nullptr;
    // epilogue (splitk == 1 only); aux16, res16 and p16 share C's ldc / strideC
    int epi = kEpiNone;
    bf16_t* aux16 = nullptr;
    const bf16_t* res16 = nullptr;
    const bf16_t* p16 = nullptr;
};

int gemm_bf16(const GemmArgs& g, hipStream_t st);

}  // namespace fwi
