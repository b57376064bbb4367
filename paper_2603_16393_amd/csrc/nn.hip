// Element-wise and reduction kernels of the learned surrogate (the GEMMs are
// in gemm.hip).  Activations are BF16 in NHWC order, gradient streams FP32;
// every reduction runs in a fixed order (per-block partials, then one pass
// over the partials), so training and gradients are bitwise reproducible.
#include <cmath>

#include "nn_internal.h"
#include "nn_ops.h"

namespace fwi {
namespace nn {

constexpr int TPB = 256;

static int blocks_for(long n) { return (int)std::min<long>((n + TPB - 1) / TPB, 8192); }

// ---------------------------------------------------------------------------
// lift: h[n][z][x][c] = W[0][c] (v - 3000)/1500 + W[1][c] z/Z + W[2][c] x/X + b[c]
// on the Z x X grid (the nz x nx model edge-extended).
__global__ void k_lift_fwd(int B, const float* __restrict__ v, const float* __restrict__ W,
                           const float* __restrict__ b, bf16_t* __restrict__ h) {
    const long n = (long)B * kZ * kX * kC;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int c = (int)(i % kC);
        const long px = i / kC;
        const int x = (int)(px % kX), z = (int)((px / kX) % kZ), s = (int)(px / ((long)kX * kZ));
        const int mz = min(z, kNZ - 1), mx = min(x, kNX - 1);
        const float f0 = (v[((long)s * kNZ + mz) * kNX + mx] - 3000.f) / 1500.f;
        const float val = W[c] * f0 + W[kC + c] * ((float)z / kZ) + W[2 * kC + c] * ((float)x / kX) + b[c];
        h[i] = f2bf(val);
    }
}

// dv[n][iz][ix] = sum over padded cells replicating (iz, ix) of sum_c dh W[0][c] / 1500
__global__ void k_lift_bwd_input(int B, const float* __restrict__ dh, const float* __restrict__ W,
                                 float* __restrict__ dv) {
    const long n = (long)B * kNZ * kNX;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int ix = (int)(i % kNX), iz = (int)((i / kNX) % kNZ), s = (int)(i / ((long)kNX * kNZ));
        const int zhi = (iz == kNZ - 1) ? kZ - 1 : iz, xhi = (ix == kNX - 1) ? kX - 1 : ix;
        float acc = 0.f;
        for (int z = iz; z <= zhi; ++z)
            for (int x = ix; x <= xhi; ++x) {
                const float* d = dh + (((long)s * kZ + z) * kX + x) * kC;
                float t = 0.f;
                for (int c = 0; c < kC; ++c) t += d[c] * W[c];
                acc += t;
            }
        dv[i] = acc / 1500.f;
    }
}

// partial sums for dW_lift [3][C] and db_lift [C]: block j sums its pixel range
__global__ void k_lift_bwd_weight_partial(int B, const float* __restrict__ v, const float* __restrict__ dh,
                                          float* __restrict__ part, int nparts) {
    const long npx = (long)B * kZ * kX;
    const int c = threadIdx.x % kC;          // 256 threads = 4 pixel lanes x 64 channels
    const int lanep = threadIdx.x / kC;
    const long lo = npx * blockIdx.x / nparts, hi = npx * (blockIdx.x + 1) / nparts;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, sb = 0.f;
    for (long px = lo + lanep; px < hi; px += 4) {
        const int x = (int)(px % kX), z = (int)((px / kX) % kZ), s = (int)(px / ((long)kX * kZ));
        const int mz = min(z, kNZ - 1), mx = min(x, kNX - 1);
        const float f0 = (v[((long)s * kNZ + mz) * kNX + mx] - 3000.f) / 1500.f;
        const float d = dh[px * kC + c];
        s0 += d * f0;
        s1 += d * ((float)z / kZ);
        s2 += d * ((float)x / kX);
        sb += d;
    }
    __shared__ float sh[4][4][kC];
    sh[lanep][0][c] = s0;
    sh[lanep][1][c] = s1;
    sh[lanep][2][c] = s2;
    sh[lanep][3][c] = sb;
    __syncthreads();
    if (lanep == 0) {
        for (int q = 0; q < 4; ++q) {
            float t = 0.f;
            for (int l = 0; l < 4; ++l) t += sh[l][q][c];
            part[((long)blockIdx.x * 4 + q) * kC + c] = t;
        }
    }
}

// out[j] = sum_p part[p][j] for j < len (fixed order)
__global__ void k_sum_partials(const float* __restrict__ part, int nparts, int len, float* __restrict__ out,
                               float beta) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    float s = 0.f;
    for (int p = 0; p < nparts; ++p) s += part[(long)p * len + j];
    out[j] = (beta != 0.f ? beta * out[j] : 0.f) + s;
}

// ---------------------------------------------------------------------------
// depthwise 3x3 correlation, zero padding, NHWC with C = 64
__global__ void k_dw_fwd(int B, int H, int W, const bf16_t* __restrict__ in, const float* __restrict__ k,
                         const float* __restrict__ b, bf16_t* __restrict__ out) {
    const long n = (long)B * H * W * kC;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int c = (int)(i % kC);
        const long px = i / kC;
        const int x = (int)(px % W), y = (int)((px / W) % H);
        const long base = px - (long)y * W - x;  // pixel index of (s, 0, 0)
        float acc = b[c];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yy = y + dy - 1;
            if (yy < 0 || yy >= H) continue;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xx = x + dx - 1;
                if (xx < 0 || xx >= W) continue;
                acc += k[c * 9 + dy * 3 + dx] * bf2f(in[(base + (long)yy * W + xx) * kC + c]);
            }
        }
        out[i] = f2bf(acc);
    }
}

// din += transpose of the correlation applied to dout (FP32), and its BF16 copy if din16
__global__ void k_dw_bwd_input(int B, int H, int W, const float* __restrict__ dout, const float* __restrict__ k,
                               float* __restrict__ din, bf16_t* __restrict__ din16) {
    const long n = (long)B * H * W * kC;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int c = (int)(i % kC);
        const long px = i / kC;
        const int x = (int)(px % W), y = (int)((px / W) % H);
        const long base = px - (long)y * W - x;
        float acc = 0.f;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yy = y - dy + 1;  // output pixel that read (y, x) through tap dy
            if (yy < 0 || yy >= H) continue;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xx = x - dx + 1;
                if (xx < 0 || xx >= W) continue;
                acc += k[c * 9 + dy * 3 + dx] * dout[(base + (long)yy * W + xx) * kC + c];
            }
        }
        const float v = din[i] + acc;
        din[i] = v;
        if (din16) din16[i] = f2bf(v);
    }
}

// partials of dk [C][9] and db [C]: part[block][10][C]
__global__ void k_dw_bwd_weight_partial(int B, int H, int W, const bf16_t* __restrict__ in,
                                        const float* __restrict__ dout, float* __restrict__ part, int nparts) {
    const long npx = (long)B * H * W;
    const int c = threadIdx.x % kC;
    const int lanep = threadIdx.x / kC;  // 4 pixel lanes
    const long lo = npx * blockIdx.x / nparts, hi = npx * (blockIdx.x + 1) / nparts;
    float acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = 0.f;
    for (long px = lo + lanep; px < hi; px += 4) {
        const int x = (int)(px % W), y = (int)((px / W) % H);
        const long base = px - (long)y * W - x;
        const float d = dout[px * kC + c];
        acc[9] += d;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yy = y + dy - 1;
            if (yy < 0 || yy >= H) continue;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xx = x + dx - 1;
                if (xx < 0 || xx >= W) continue;
                acc[dy * 3 + dx] += d * bf2f(in[(base + (long)yy * W + xx) * kC + c]);
            }
        }
    }
    __shared__ float sh[4][10][kC];
#pragma unroll
    for (int q = 0; q < 10; ++q) sh[lanep][q][c] = acc[q];
    __syncthreads();
    if (lanep == 0) {
        for (int q = 0; q < 10; ++q) {
            float t = 0.f;
            for (int l = 0; l < 4; ++l) t += sh[l][q][c];
            part[((long)blockIdx.x * 10 + q) * kC + c] = t;
        }
    }
}

// part [p][10][C] -> dk [C][9] (+= beta), db [C]
__global__ void k_dw_weight_finish(const float* __restrict__ part, int nparts, float* __restrict__ dk,
                                   float* __restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;  // j = q * C + c
    if (j >= 10 * kC) return;
    const int q = j / kC, c = j % kC;
    float s = 0.f;
    for (int p = 0; p < nparts; ++p) s += part[(long)p * 10 * kC + j];
    if (q < 9)
        dk[c * 9 + q] = s;
    else
        db[c] = s;
}

// ---------------------------------------------------------------------------
__global__ void k_gelu_fwd(long n, const bf16_t* __restrict__ p, bf16_t* __restrict__ q) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        q[i] = f2bf(gelu_f(bf2f(p[i])));
}

// dp = dq * gelu'(p), as FP32 and BF16
__global__ void k_gelu_bwd(long n, const float* __restrict__ dq, const bf16_t* __restrict__ p, float* __restrict__ dp,
                           bf16_t* __restrict__ dp16) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float g = dq[i] * gelu_d(bf2f(p[i]));
        dp[i] = g;
        dp16[i] = f2bf(g);
    }
}

__global__ void k_add_bf16(long n, const bf16_t* __restrict__ a, const bf16_t* __restrict__ b, bf16_t* __restrict__ o) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        o[i] = f2bf(bf2f(a[i]) + bf2f(b[i]));
}

__global__ void k_to_bf16(long n, const float* __restrict__ a, bf16_t* __restrict__ o) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        o[i] = f2bf(a[i]);
}

__global__ void k_copy_f32(long n, const float* __restrict__ a, float* __restrict__ o) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) o[i] = a[i];
}

// column sums of a [rows x cols] FP32 matrix: partials part[p][cols]
__global__ void k_colsum_partial(long rows, int cols, const float* __restrict__ a, float* __restrict__ part,
                                 int nparts) {
    // block = 256 threads; thread handles column c = threadIdx.x % cols for cols <= 256 dividing 256
    const int lanes = TPB / cols;
    const int c = threadIdx.x % cols, l = threadIdx.x / cols;
    const long lo = rows * blockIdx.x / nparts, hi = rows * (blockIdx.x + 1) / nparts;
    float s = 0.f;
    if (l < lanes)
        for (long r = lo + l; r < hi; r += lanes) s += a[r * cols + c];
    __shared__ float sh[TPB];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (l == 0) {
        float t = 0.f;
        for (int q = 0; q < lanes; ++q) t += sh[q * cols + c];
        part[(long)blockIdx.x * cols + c] = t;
    }
}

// ---------------------------------------------------------------------------
// head output [n][NT][X*S] (FP32) -> traces [n][NS][NR][NT] * scale
__global__ void k_out_fwd(int B, const float* __restrict__ out, const float* __restrict__ scale,
                          float* __restrict__ tr) {
    const long n = (long)B * kNS * kNR * kNT;
    const float sc = *scale;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int u = (int)(i % kNT);
        const int r = (int)((i / kNT) % kNR), s = (int)((i / ((long)kNT * kNR)) % kNS);
        const long b = i / ((long)kNT * kNR * kNS);
        tr[i] = sc * out[(b * kNT + u) * (kX * kS) + r * kS + s];
    }
}

// dtraces -> dout [n][NT][X*S] (BF16, zero in the unused columns) and d(scale) partial terms
__global__ void k_out_bwd(int B, const float* __restrict__ dtr, const float* __restrict__ scale,
                          bf16_t* __restrict__ dout) {
    const long n = (long)B * kNT * kX * kS;
    const float sc = *scale;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int k = (int)(i % (kX * kS));
        const int u = (int)((i / (kX * kS)) % kNT);
        const long b = i / ((long)kNT * kX * kS);
        const int r = k / kS, s = k % kS;
        float v = 0.f;
        if (r < kNR && s < kNS) v = sc * dtr[((b * kNS + s) * kNR + r) * kNT + u];
        dout[i] = f2bf(v);
    }
}

// ---------------------------------------------------------------------------
// Weighted trace loss L = sum_b sum (w (pred - tgt))^2 / count, w = 1/(1 + kw |tgt| / max_b |tgt|).
// max |t| per sample: grid (chunks, B); each block folds its maximum into
// mx[b] with an integer atomic max (non-negative floats order like their bit
// patterns), so the result is exact and independent of the order.  mx is
// cleared first by k_zero_f32.
__global__ void k_zero_f32(float* __restrict__ x, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.f;
}

__global__ void k_absmax_per_sample(int B, long per, const float* __restrict__ t, float* __restrict__ mx) {
    __shared__ float sh[TPB];
    const int b = blockIdx.y;
    float m = 0.f;
    for (long i = blockIdx.x * (long)TPB + threadIdx.x; i < per; i += (long)gridDim.x * TPB)
        m = fmaxf(m, fabsf(t[b * per + i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(reinterpret_cast<int*>(mx + b), __float_as_int(sh[0]));
}

__global__ void k_loss(int B, long per, const float* __restrict__ pred, const float* __restrict__ tgt,
                       const float* __restrict__ mx, float kw, float inv_count, float* __restrict__ dpred,
                       float* __restrict__ part, int nparts) {
    const long n = (long)B * per;
    const long lo = n * blockIdx.x / nparts, hi = n * (blockIdx.x + 1) / nparts;
    float s = 0.f;
    for (long i = lo + threadIdx.x; i < hi; i += TPB) {
        const long b = i / per;
        const float m = mx[b] > 0.f ? mx[b] : 1.f;
        const float w = 1.f / (1.f + kw * fabsf(tgt[i]) / m);
        const float r = w * (pred[i] - tgt[i]);
        s += r * r;
        dpred[i] = 2.f * w * r * inv_count;
    }
    __shared__ float sh[TPB];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int q = 0; q < TPB; ++q) t += sh[q];
        part[blockIdx.x] = t * inv_count;
    }
}

// Directional (finite-difference) term for pairs: samples h..2h-1 are
// perturbations of 0..h-1.  Adds lam / count_h * sum (w ((p' - p) - (t' - t)))^2,
// w the amplitude weight of the unperturbed target, to the loss and its
// derivative to dpred (after k_loss has written dpred).
__global__ void k_loss_pairs(long half, long per, const float* __restrict__ pred, const float* __restrict__ tgt,
                             const float* __restrict__ mx, float kw, float lam, float inv_count,
                             float* __restrict__ dpred, float* __restrict__ part, int nparts) {
    const long lo = half * blockIdx.x / nparts, hi = half * (blockIdx.x + 1) / nparts;
    float s = 0.f;
    for (long i = lo + threadIdx.x; i < hi; i += TPB) {
        const long b = i / per;
        const float m = mx[b] > 0.f ? mx[b] : 1.f;
        const float w = 1.f / (1.f + kw * fabsf(tgt[i]) / m);  // weight of the unperturbed sample
        const float r = w * ((pred[i + half] - pred[i]) - (tgt[i + half] - tgt[i]));
        s += r * r;
        const float d = 2.f * lam * w * r * inv_count;
        dpred[i] -= d;
        dpred[i + half] += d;
    }
    __shared__ float sh[TPB];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int q = 0; q < TPB; ++q) t += sh[q];
        part[blockIdx.x] = t * lam * inv_count;
    }
}

// Adam on FP32 master parameters; refreshes the BF16 copies of GEMM operands.
__global__ void k_adam(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2,
                       const int* __restrict__ bf_index, bf16_t* __restrict__ pbf) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        const int j = bf_index[i];
        if (j >= 0) pbf[j] = f2bf(pi);
    }
}

__global__ void k_refresh_bf16(long n, const float* __restrict__ p, const int* __restrict__ bf_index,
                               bf16_t* __restrict__ pbf) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int j = bf_index[i];
        if (j >= 0) pbf[j] = f2bf(p[i]);
    }
}

// ---------------------------------------------------------------------------
// judge: per sample cosine between two gradients and relative misfit difference
__global__ void k_judge(int n, const float* __restrict__ ga, const float* __restrict__ gb,
                        const double* __restrict__ Ja, const double* __restrict__ Jb, float* __restrict__ cosv,
                        float* __restrict__ jerr) {
    __shared__ double sab[TPB], saa[TPB], sbb[TPB];
    const int b = blockIdx.x;
    const float* a = ga + (long)b * n;
    const float* c = gb + (long)b * n;
    double ab = 0, aa = 0, bb = 0;
    const int ch = (n + TPB - 1) / TPB;
    const int lo = threadIdx.x * ch, hi = min(n, lo + ch);
    for (int i = lo; i < hi; ++i) {
        ab += (double)a[i] * c[i];
        aa += (double)a[i] * a[i];
        bb += (double)c[i] * c[i];
    }
    sab[threadIdx.x] = ab;
    saa[threadIdx.x] = aa;
    sbb[threadIdx.x] = bb;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tab = 0, taa = 0, tbb = 0;
        for (int q = 0; q < TPB; ++q) {
            tab += sab[q];
            taa += saa[q];
            tbb += sbb[q];
        }
        cosv[b] = (taa > 0 && tbb > 0) ? (float)(tab / sqrt(taa * tbb)) : 0.f;
        if (jerr) jerr[b] = (Ja && Jb && Jb[b] != 0.0) ? (float)fabs((Ja[b] - Jb[b]) / Jb[b]) : 0.f;
    }
}

// multi-fidelity prediction: out = anchor + now - now_at_anchor (gradients and misfits)
// (no __restrict__: out may alias ga or sn)
__global__ void k_mf_predict(long n, const float* ga, const float* sn, const float* sa, float* out, int B,
                             const double* Ja, const double* Jn, const double* Jsa, double* Jout) {
    const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    for (long i = tid; i < n; i += (long)gridDim.x * blockDim.x) out[i] = ga[i] + (sn[i] - sa[i]);
    if (Jout && tid < B) Jout[tid] = Ja[tid] + (Jn[tid] - Jsa[tid]);
}

// ---------------------------------------------------------------------------
// Channel-vectorised forms (C = 64 channels, NHWC): 8 BF16 or 4 FP32 channels
// per 16-byte access, taps in the same order as the scalar forms above.
__device__ inline void unpack8(const uint4 u, float o[8]) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        o[2 * e] = bf2f((bf16_t)(w[e] & 0xffff));
        o[2 * e + 1] = bf2f((bf16_t)(w[e] >> 16));
    }
}
__device__ inline uint4 pack8(const float v[8]) {
    uint4 u;
    u.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
    u.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
    u.z = (uint32_t)f2bf(v[4]) | ((uint32_t)f2bf(v[5]) << 16);
    u.w = (uint32_t)f2bf(v[6]) | ((uint32_t)f2bf(v[7]) << 16);
    return u;
}

__global__ void k_dw_fwd8(int B, int H, int W, const bf16_t* __restrict__ in, const float* __restrict__ k,
                          const float* __restrict__ b, bf16_t* __restrict__ out) {
    __shared__ float ks[kC * 9], bs[kC];
    for (int i = threadIdx.x; i < kC * 9; i += blockDim.x) ks[i] = k[i];
    for (int i = threadIdx.x; i < kC; i += blockDim.x) bs[i] = b[i];
    __syncthreads();
    const long n = (long)B * H * W * (kC / 8);
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int c0 = (int)(i % (kC / 8)) * 8;
        const long px = i / (kC / 8);
        const int x = (int)(px % W), y = (int)((px / W) % H);
        const long base = px - (long)y * W - x;
        float acc[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[e] = bs[c0 + e];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yy = y + dy - 1;
            if (yy < 0 || yy >= H) continue;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xx = x + dx - 1;
                if (xx < 0 || xx >= W) continue;
                float v[8];
                unpack8(*reinterpret_cast<const uint4*>(in + (base + (long)yy * W + xx) * kC + c0), v);
#pragma unroll
                for (int e = 0; e < 8; ++e) acc[e] += ks[(c0 + e) * 9 + dy * 3 + dx] * v[e];
            }
        }
        *reinterpret_cast<uint4*>(out + px * kC + c0) = pack8(acc);
    }
}

__global__ void k_dw_bwd_input4(int B, int H, int W, const float* __restrict__ dout, const float* __restrict__ k,
                                float* __restrict__ din, bf16_t* __restrict__ din16) {
    __shared__ float ks[kC * 9];
    for (int i = threadIdx.x; i < kC * 9; i += blockDim.x) ks[i] = k[i];
    __syncthreads();
    const long n = (long)B * H * W * (kC / 4);
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int c0 = (int)(i % (kC / 4)) * 4;
        const long px = i / (kC / 4);
        const int x = (int)(px % W), y = (int)((px / W) % H);
        const long base = px - (long)y * W - x;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yy = y - dy + 1;
            if (yy < 0 || yy >= H) continue;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xx = x - dx + 1;
                if (xx < 0 || xx >= W) continue;
                const float4 d = *reinterpret_cast<const float4*>(dout + (base + (long)yy * W + xx) * kC + c0);
                const float dv[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[e] += ks[(c0 + e) * 9 + dy * 3 + dx] * dv[e];
            }
        }
        float4* dp = reinterpret_cast<float4*>(din + px * kC + c0);
        const float4 o = *dp;
        const float4 r = make_float4(o.x + acc[0], o.y + acc[1], o.z + acc[2], o.w + acc[3]);
        *dp = r;
        if (din16) {
            uint2 u;
            u.x = (uint32_t)f2bf(r.x) | ((uint32_t)f2bf(r.y) << 16);
            u.y = (uint32_t)f2bf(r.z) | ((uint32_t)f2bf(r.w) << 16);
            *reinterpret_cast<uint2*>(din16 + px * kC + c0) = u;
        }
    }
}

// partials of dk [C][9] and db [C]: thread = (pixel lane, 8-channel group); 32 pixel
// lanes per block summed by a fixed shuffle tree and a fixed pass over the 4 waves
__global__ __launch_bounds__(256) void k_dw_bwd_weight_partial8(int B, int H, int W, const bf16_t* __restrict__ in,
                                                                const float* __restrict__ dout,
                                                                float* __restrict__ part, int nparts) {
    const long npx = (long)B * H * W;
    const int cgp = threadIdx.x & 7, pl = threadIdx.x >> 3;  // 8 channel groups x 32 pixel lanes
    const int c0 = cgp * 8;
    const long lo = npx * blockIdx.x / nparts, hi = npx * (blockIdx.x + 1) / nparts;
    float acc[10][8];
#pragma unroll
    for (int q = 0; q < 10; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[q][e] = 0.f;
    for (long px = lo + pl; px < hi; px += 32) {
        const int x = (int)(px % W), y = (int)((px / W) % H);
        const long base = px - (long)y * W - x;
        const float4 da = *reinterpret_cast<const float4*>(dout + px * kC + c0);
        const float4 db = *reinterpret_cast<const float4*>(dout + px * kC + c0 + 4);
        const float d[8] = {da.x, da.y, da.z, da.w, db.x, db.y, db.z, db.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[9][e] += d[e];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yy = y + dy - 1;
            if (yy < 0 || yy >= H) continue;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xx = x + dx - 1;
                if (xx < 0 || xx >= W) continue;
                float v[8];
                unpack8(*reinterpret_cast<const uint4*>(in + (base + (long)yy * W + xx) * kC + c0), v);
#pragma unroll
                for (int e = 0; e < 8; ++e) acc[dy * 3 + dx][e] += d[e] * v[e];
            }
        }
    }
    // within a wave: lanes with the same channel group are 8 apart
#pragma unroll
    for (int q = 0; q < 10; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float t = acc[q][e];
            t += __shfl_xor(t, 8);
            t += __shfl_xor(t, 16);
            t += __shfl_xor(t, 32);
            acc[q][e] = t;
        }
    __shared__ float sh[4][10][kC];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < 8) {
#pragma unroll
        for (int q = 0; q < 10; ++q)
#pragma unroll
            for (int e = 0; e < 8; ++e) sh[wave][q][c0 + e] = acc[q][e];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < 10 * kC; j += blockDim.x) {
        const int q = j / kC, c = j % kC;
        part[((long)blockIdx.x * 10 + q) * kC + c] = ((sh[0][q][c] + sh[1][q][c]) + sh[2][q][c]) + sh[3][q][c];
    }
}

// column sums of a [rows x cols] FP32 matrix (cols a multiple of 4 dividing 1024): 4 columns per thread
__global__ void k_colsum_partial4(long rows, int cols, const float* __restrict__ a, float* __restrict__ part,
                                  int nparts) {
    const int g4 = cols / 4;                 // column groups
    const int lanes = TPB / g4;              // row lanes
    const int cg = threadIdx.x % g4, l = threadIdx.x / g4;
    const long lo = rows * blockIdx.x / nparts, hi = rows * (blockIdx.x + 1) / nparts;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    if (l < lanes)
        for (long r = lo + l; r < hi; r += lanes) {
            const float4 v = *reinterpret_cast<const float4*>(a + r * cols + cg * 4);
            s.x += v.x, s.y += v.y, s.z += v.z, s.w += v.w;
        }
    __shared__ float4 sh[TPB];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (l == 0) {
        float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int q = 0; q < lanes; ++q) {
            const float4 v = sh[q * g4 + cg];
            t.x += v.x, t.y += v.y, t.z += v.z, t.w += v.w;
        }
        *reinterpret_cast<float4*>(part + (long)blockIdx.x * cols + cg * 4) = t;
    }
}

// ---------------------------------------------------------------------------
// launchers
void lift_fwd(int B, const float* v, const float* W, const float* b, bf16_t* h, hipStream_t st) {
    hipLaunchKernelGGL(k_lift_fwd, dim3(blocks_for((long)B * kZ * kX * kC)), dim3(TPB), 0, st, B, v, W, b, h);
}
void lift_bwd(int B, const float* v, const float* dh, const float* W, float* dv, float* dW, float* db, float* part,
              hipStream_t st) {
    if (dv) hipLaunchKernelGGL(k_lift_bwd_input, dim3(blocks_for((long)B * kNZ * kNX)), dim3(TPB), 0, st, B, dh, W, dv);
    if (dW) {
        const int np = 256;
        hipLaunchKernelGGL(k_lift_bwd_weight_partial, dim3(np), dim3(TPB), 0, st, B, v, dh, part, np);
        // part[p][4][C]: rows 0..2 -> dW, row 3 -> db
        hipLaunchKernelGGL(k_sum_partials, dim3((4 * kC + TPB - 1) / TPB), dim3(TPB), 0, st, part, np, 4 * kC,
                           part + (long)np * 4 * kC, 0.f);
        hipLaunchKernelGGL(k_copy_f32, dim3(1), dim3(TPB), 0, st, (long)3 * kC, part + (long)np * 4 * kC, dW);
        hipLaunchKernelGGL(k_copy_f32, dim3(1), dim3(TPB), 0, st, (long)kC, part + (long)np * 4 * kC + 3 * kC, db);
    }
}
void dw_fwd(int B, int H, int W, const bf16_t* in, const float* k, const float* b, bf16_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_dw_fwd8, dim3(blocks_for((long)B * H * W * (kC / 8))), dim3(TPB), 0, st, B, H, W, in, k, b,
                       out);
}
void dw_bwd(int B, int H, int W, const bf16_t* in, const float* dout, const float* k, float* din, bf16_t* din16,
            float* dk, float* db, float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_dw_bwd_input4, dim3(blocks_for((long)B * H * W * (kC / 4))), dim3(TPB), 0, st, B, H, W, dout,
                       k, din, din16);
    if (dk) {
        const int np = 512;
        hipLaunchKernelGGL(k_dw_bwd_weight_partial8, dim3(np), dim3(TPB), 0, st, B, H, W, in, dout, part, np);
        hipLaunchKernelGGL(k_dw_weight_finish, dim3((10 * kC + TPB - 1) / TPB), dim3(TPB), 0, st, part, np, dk, db);
    }
}
void gelu_fwd(long n, const bf16_t* p, bf16_t* q, hipStream_t st) {
    hipLaunchKernelGGL(k_gelu_fwd, dim3(blocks_for(n)), dim3(TPB), 0, st, n, p, q);
}
void gelu_bwd(long n, const float* dq, const bf16_t* p, float* dp, bf16_t* dp16, hipStream_t st) {
    hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks_for(n)), dim3(TPB), 0, st, n, dq, p, dp, dp16);
}
void add_bf16(long n, const bf16_t* a, const bf16_t* b, bf16_t* o, hipStream_t st) {
    hipLaunchKernelGGL(k_add_bf16, dim3(blocks_for(n)), dim3(TPB), 0, st, n, a, b, o);
}
void to_bf16(long n, const float* a, bf16_t* o, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(TPB), 0, st, n, a, o);
}
void copy_f32(long n, const float* a, float* o, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_f32, dim3(blocks_for(n)), dim3(TPB), 0, st, n, a, o);
}
void colsum(long rows, int cols, const float* a, float* out, float* part, hipStream_t st) {
    const int np = 256;
    if (cols % 4 == 0 && 1024 % cols == 0)
        hipLaunchKernelGGL(k_colsum_partial4, dim3(np), dim3(TPB), 0, st, rows, cols, a, part, np);
    else
        hipLaunchKernelGGL(k_colsum_partial, dim3(np), dim3(TPB), 0, st, rows, cols, a, part, np);
    hipLaunchKernelGGL(k_sum_partials, dim3((cols + TPB - 1) / TPB), dim3(TPB), 0, st, part, np, cols, out, 0.f);
}
void out_fwd(int B, const float* out, const float* scale, float* tr, hipStream_t st) {
    hipLaunchKernelGGL(k_out_fwd, dim3(blocks_for((long)B * kNS * kNR * kNT)), dim3(TPB), 0, st, B, out, scale, tr);
}
void out_bwd(int B, const float* dtr, const float* scale, bf16_t* dout, hipStream_t st) {
    hipLaunchKernelGGL(k_out_bwd, dim3(blocks_for((long)B * kNT * kX * kS)), dim3(TPB), 0, st, B, dtr, scale, dout);
}
void loss(int B, const float* pred, const float* tgt, float kw, float pair_w, float* dpred, float* loss_out, float* mx,
          float* part, hipStream_t st) {
    const long per = (long)kNS * kNR * kNT;
    hipLaunchKernelGGL(k_zero_f32, dim3((B + TPB - 1) / TPB), dim3(TPB), 0, st, mx, B);
    hipLaunchKernelGGL(k_absmax_per_sample, dim3(32, B), dim3(TPB), 0, st, B, per, tgt, mx);
    const int np = 512;
    hipLaunchKernelGGL(k_loss, dim3(np), dim3(TPB), 0, st, B, per, pred, tgt, mx, kw, 1.f / (float)(B * per), dpred,
                       part, np);
    int nparts = np;
    if (pair_w > 0.f) {
        const long half = (long)(B / 2) * per;
        hipLaunchKernelGGL(k_loss_pairs, dim3(np), dim3(TPB), 0, st, half, per, pred, tgt, mx, kw, pair_w,
                           1.f / (float)half, dpred, part + np, np);
        nparts = 2 * np;
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(TPB), 0, st, part, nparts, 1, loss_out, 0.f);
}
void adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, int step,
          const int* bf_index, bf16_t* pbf, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(TPB), 0, st, n, p, g, m, v, lr, b1, b2, eps, c1, c2, bf_index,
                       pbf);
}
void refresh_bf16(long n, const float* p, const int* bf_index, bf16_t* pbf, hipStream_t st) {
    hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks_for(n)), dim3(TPB), 0, st, n, p, bf_index, pbf);
}
void mf_predict(long n, const float* ga, const float* sn, const float* sa, float* out, int B, const double* Ja,
                const double* Jn, const double* Jsa, double* Jout, hipStream_t st) {
    const int blocks = std::max(blocks_for(n), (B + TPB - 1) / TPB);
    hipLaunchKernelGGL(k_mf_predict, dim3(blocks), dim3(TPB), 0, st, n, ga, sn, sa, out, B, Ja, Jn, Jsa, Jout);
}
void judge(int B, int n, const float* ga, const float* gb, const double* Ja, const double* Jb, float* cosv, float* jerr,
           hipStream_t st) {
    hipLaunchKernelGGL(k_judge, dim3(B), dim3(TPB), 0, st, n, ga, gb, Ja, Jb, cosv, jerr);
}

}  // namespace nn
}  // namespace fwi
