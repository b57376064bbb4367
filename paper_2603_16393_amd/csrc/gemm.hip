// BF16 x BF16 -> FP32 GEMM on gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Block tile 64 x 64 x 32, 256 threads = 4 waves in a 2 x 2 arrangement, each
// wave accumulating a 32 x 32 sub-tile as 2 x 2 MFMA 16 x 16 blocks in FP32.
// Both operands are staged in LDS K-contiguous (A as [m][k], B as [n][k], row
// stride 40 halves = 80 bytes) so every lane fetches its 8 consecutive K
// values of an MFMA operand with one 16-byte LDS read; transposed operands
// are transposed while staging.  Global loads are 16-byte vectors when the
// leading dimension, batch stride and base allow it, element-wise otherwise
// (tails are zero-filled).  Split-K writes FP32 partials that a second kernel
// adds in a fixed order, so results are deterministic.
//
// MFMA 16x16x32 operand layout (wave64): lane l supplies A[l % 16][8 (l / 16) + i]
// and B[8 (l / 16) + i][l % 16], i = 0..7; it receives D[4 (l / 16) + q][l % 16],
// q = 0..3.
#include "nn_internal.h"

namespace fwi {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int GBM = 64, GBN = 64, GBK = 32, GLD = GBK + 8;

struct GemmDev {
    GemmArgs g;
    int vecA, vecB;
    int vecC;        // ldc, strideC and every output / epilogue operand allow 16-byte accesses
    int ksteps;      // K steps per batch
    int total;       // total (batch, k) steps of one output tile
};

__device__ inline void load8(const bf16_t* __restrict__ base, long ld, int row, int col, int rows, int cols, bool vec,
                             bf16_t out[8]) {
    // 8 consecutive elements base[row][col .. col+7] of a rows x cols matrix
    if (vec && row < rows && col + 8 <= cols) {
        const uint4 v = *reinterpret_cast<const uint4*>(base + (long)row * ld + col);
        out[0] = v.x & 0xffff;
        out[1] = v.x >> 16;
        out[2] = v.y & 0xffff;
        out[3] = v.y >> 16;
        out[4] = v.z & 0xffff;
        out[5] = v.z >> 16;
        out[6] = v.w & 0xffff;
        out[7] = v.w >> 16;
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) out[i] = (row < rows && col + i < cols) ? base[(long)row * ld + col + i] : 0;
    }
}

// 8 consecutive elements, as one 16-byte (BF16) or two 16-byte (FP32) accesses when
// `vec`, element-wise for the first n otherwise
__device__ inline void ld8bf(const bf16_t* p, bool vec, int n, float o[8]) {
    if (vec) {
        const uint4 u = *reinterpret_cast<const uint4*>(p);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            o[2 * e] = bf2f((bf16_t)(w[e] & 0xffff));
            o[2 * e + 1] = bf2f((bf16_t)(w[e] >> 16));
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = e < n ? bf2f(p[e]) : 0.f;
    }
}
__device__ inline void st8bf(bf16_t* p, bool vec, int n, const bf16_t h[8]) {
    if (vec) {
        uint4 u;
        u.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        u.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        u.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
        u.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
        *reinterpret_cast<uint4*>(p) = u;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (e < n) p[e] = h[e];
    }
}
__device__ inline void ld8f(const float* p, bool vec, int n, float o[8]) {
    if (vec) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        const float4 b = *reinterpret_cast<const float4*>(p + 4);
        o[0] = a.x, o[1] = a.y, o[2] = a.z, o[3] = a.w, o[4] = b.x, o[5] = b.y, o[6] = b.z, o[7] = b.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = e < n ? p[e] : 0.f;
    }
}
__device__ inline void st8f(float* p, bool vec, int n, const float v[8]) {
    if (vec) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<float4*>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (e < n) p[e] = v[e];
    }
}

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmDev d) {
    const GemmArgs& g = d.g;
    __shared__ __attribute__((aligned(16))) bf16_t As[GBM * GLD];
    __shared__ __attribute__((aligned(16))) bf16_t Bs[GBN * GLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    int split = 0, bout = 0;
    if (g.splitk > 1 || g.reduce_batch)
        split = blockIdx.z;
    else
        bout = blockIdx.z;
    const int s_lo = (int)((long)d.total * split / g.splitk);
    const int s_hi = (int)((long)d.total * (split + 1) / g.splitk);

    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    for (int step = s_lo; step < s_hi; ++step) {
        const int b = (g.reduce_batch || g.splitk > 1) ? step / d.ksteps : bout;
        const int k0 = (step - (step / d.ksteps) * d.ksteps) * GBK;
        const bf16_t* A = g.A + (long)b * g.strideA;
        const bf16_t* B = g.B + (long)b * g.strideB;
        bf16_t v[8];
        if (!g.transA) {  // A[m][k]
            const int m = tid >> 2, kq = (tid & 3) * 8;
            load8(A, g.lda, m0 + m, k0 + kq, g.M, g.K, d.vecA, v);
#pragma unroll
            for (int i = 0; i < 8; ++i) As[m * GLD + kq + i] = v[i];
        } else {  // stored [k][m]
            const int k = tid >> 3, mq = (tid & 7) * 8;
            load8(A, g.lda, k0 + k, m0 + mq, g.K, g.M, d.vecA, v);
#pragma unroll
            for (int i = 0; i < 8; ++i) As[(mq + i) * GLD + k] = v[i];
        }
        if (!g.transB) {  // B[k][n]
            const int k = tid >> 3, nq = (tid & 7) * 8;
            load8(B, g.ldb, k0 + k, n0 + nq, g.K, g.N, d.vecB, v);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[(nq + i) * GLD + k] = v[i];
        } else {  // stored [n][k]
            const int n = tid >> 2, kq = (tid & 3) * 8;
            load8(B, g.ldb, n0 + n, k0 + kq, g.N, g.K, d.vecB, v);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[n * GLD + kq + i] = v[i];
        }
        __syncthreads();
        const int r = lane & 15, kg = (lane >> 4) * 8;
        bf16x8_t af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = *reinterpret_cast<const bf16x8_t*>(&As[(wm * 32 + i * 16 + r) * GLD + kg]);
#pragma unroll
        for (int j = 0; j < 2; ++j) bfr[j] = *reinterpret_cast<const bf16x8_t*>(&Bs[(wn * 32 + j * 16 + r) * GLD + kg]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }

    const int col_l = lane & 15, row_l = (lane >> 4) * 4;
    if (g.splitk > 1) {  // FP32 partials, added in split order by k_splitk_reduce
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = m0 + wm * 32 + i * 16 + row_l + q;
                    const int col = n0 + wn * 32 + j * 16 + col_l;
                    if (row < g.M && col < g.N) g.work[((long)split * g.M + row) * g.N + col] = acc[i][j][q];
                }
        return;
    }
    // Epilogue: the accumulator tile goes through LDS so that each thread then
    // finishes 8 consecutive columns of one row and moves them with 16-byte
    // loads and stores (an MFMA lane's own outputs span only 16 columns).
    __shared__ float Ct[GBM][GBN + 4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) Ct[wm * 32 + i * 16 + row_l + q][wn * 32 + j * 16 + col_l] = acc[i][j][q];
    __syncthreads();
    const int cg = (tid & 7) * 8;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int r = pass * 32 + (tid >> 3);
        const int row = m0 + r, col0 = n0 + cg;
        if (row >= g.M || col0 >= g.N) continue;
        const int ncol = min(8, g.N - col0);
        const bool vec = d.vecC && ncol == 8;
        const long off = (long)bout * g.strideC + (long)row * g.ldc + col0;
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = g.alpha * Ct[r][cg + e];
        if (g.beta != 0.f) {
            float old[8];
            if (g.C32)
                ld8f(g.C32 + off, vec, ncol, old);
            else
                ld8bf(g.C16 + off, vec, ncol, old);
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] += g.beta * old[e];
        }
        if (g.bias) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (e < ncol) v[e] += g.bias[col0 + e];
        }
        bf16_t h[8];
        switch (g.epi) {
            case kEpiGelu: {
                bf16_t q16[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    h[e] = f2bf(v[e]);
                    q16[e] = f2bf(gelu_f(bf2f(h[e])));
                }
                st8bf(g.C16 + off, vec, ncol, h);
                st8bf(g.aux16 + off, vec, ncol, q16);
                break;
            }
            case kEpiResid: {
                float res[8];
                ld8bf(g.res16 + off, vec, ncol, res);
#pragma unroll
                for (int e = 0; e < 8; ++e) h[e] = f2bf(res[e] + bf2f(f2bf(v[e])));
                st8bf(g.C16 + off, vec, ncol, h);
                break;
            }
            case kEpiGeluBwd: {
                float pp[8];
                ld8bf(g.p16 + off, vec, ncol, pp);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    v[e] *= gelu_d(pp[e]);
                    h[e] = f2bf(v[e]);
                }
                st8f(g.C32 + off, vec, ncol, v);
                st8bf(g.aux16 + off, vec, ncol, h);
                break;
            }
            case kEpiDual:
#pragma unroll
                for (int e = 0; e < 8; ++e) h[e] = f2bf(v[e]);
                st8f(g.C32 + off, vec, ncol, v);
                st8bf(g.aux16 + off, vec, ncol, h);
                break;
            default:
                if (g.C32) {
                    st8f(g.C32 + off, vec, ncol, v);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) h[e] = f2bf(v[e]);
                    st8bf(g.C16 + off, vec, ncol, h);
                }
        }
    }
}

__global__ void k_splitk_reduce(GemmArgs g) {
    const long n = (long)g.M * g.N;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int row = (int)(i / g.N), col = (int)(i - (i / g.N) * g.N);
        float s = 0.f;
        for (int k = 0; k < g.splitk; ++k) s += g.work[(long)k * n + i];
        const long off = (long)row * g.ldc + col;
        float val = g.alpha * s;
        if (g.beta != 0.f) val += g.beta * (g.C32 ? g.C32[off] : bf2f(g.C16[off]));
        if (g.bias) val += g.bias[col];
        if (g.C32)
            g.C32[off] = val;
        else
            g.C16[off] = f2bf(val);
    }
}

int gemm_bf16(const GemmArgs& g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) return FWI_OK;
    if (!g.A || !g.B || (!g.C32 == !g.C16)) return FWI_EINVAL;
    if (g.splitk > 1 && (!g.work || (g.batch > 1 && !g.reduce_batch))) return FWI_EINVAL;
    if (g.epi != kEpiNone) {
        if (g.splitk > 1 || g.reduce_batch) return FWI_EINVAL;
        const bool c16 = g.C16 != nullptr, c32 = g.C32 != nullptr;
        if ((g.epi == kEpiGelu && (!c16 || !g.aux16)) || (g.epi == kEpiResid && (!c16 || !g.res16)) ||
            (g.epi == kEpiGeluBwd && (!c32 || !g.aux16 || !g.p16)) || (g.epi == kEpiDual && (!c32 || !g.aux16)))
            return FWI_EINVAL;
    }
    GemmDev d;
    d.g = g;
    if (d.g.splitk < 1) d.g.splitk = 1;
    d.vecA = (g.lda % 8 == 0) && (g.strideA % 8 == 0) && ((uintptr_t)g.A % 16 == 0);
    d.vecB = (g.ldb % 8 == 0) && (g.strideB % 8 == 0) && ((uintptr_t)g.B % 16 == 0);
    auto al16 = [](const void* p) { return ((uintptr_t)p % 16) == 0; };
    d.vecC = (g.ldc % 8 == 0) && (g.strideC % 8 == 0) && al16(g.C32) && al16(g.C16) && al16(g.aux16) &&
             al16(g.res16) && al16(g.p16);
    d.ksteps = (g.K + GBK - 1) / GBK;
    const int nb = g.reduce_batch ? g.batch : 1;
    d.total = nb * d.ksteps;
    if (d.g.splitk > d.total) d.g.splitk = d.total;
    const int gz = (d.g.splitk > 1 || g.reduce_batch) ? d.g.splitk : g.batch;
    if (d.g.splitk == 1 && g.reduce_batch) {
        // one split covering every batch: the kernel reads batch = step / ksteps
    }
    dim3 grid((g.N + GBN - 1) / GBN, (g.M + GBM - 1) / GBM, gz);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, d);
    if (d.g.splitk > 1) {
        const long n = (long)g.M * g.N;
        const int blocks = (int)std::min<long>((n + 255) / 256, 2048);
        hipLaunchKernelGGL(k_splitk_reduce, dim3(blocks), dim3(256), 0, st, d.g);
    }
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

}  // namespace fwi
