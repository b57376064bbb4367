// Score network of the reverse-diffusion loop (Algorithm 2's score line):
// a noise-prediction network eps_theta(x_t, t) trained by denoising score
// matching (Sec. 3, Eqs. L1 / L2_rewrite in the noise-prediction form, score
// s = -eps / sqrt(1 - abar)), its forward pass, its vector-Jacobian product
// (the chain rule of Eq. chain_rule through the clean estimator of Eq. v0hat)
// and one Adam training step.
//
// Network (x [B][70][70], t in [0, 1]; the layer list is in include/fwi.h):
//   time embedding (FP32): sinusoids of 1000 t -> 128 GELU -> 320 per-channel
//   biases; lift to 32 channels on a 72 x 72 grid (zero ring); five residual
//   blocks {3x3 conv, + bias + time bias, GELU, 3x3 conv, + residual} on a
//   three-level U-Net (72^2 x 32, 36^2 x 64, 18^2 x 128) with 2x2 average
//   pooling + 1x1 channel maps down and 1x1 maps + nearest up-sampling +
//   skip additions up; a 1x1 head to one channel.  The output is the
//   per-sample affine map out = skip_b x + scale_b eps (noise, score or
//   clean estimate).
//
// Every 3x3 convolution is an im2col product on the BF16 matrix-core GEMM of
// gemm.hip (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the im2col tile of
// a level is [B * S * S][9 C] BF16 with column tap * C + c, tap = 3 dy + dx.
// Activations are stored BF16 (NHWC), gradient streams FP32 with a BF16 copy
// where they feed a GEMM; every reduction runs in a fixed order, so forward,
// backward and training are bitwise reproducible.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "nn_internal.h"
#include "nn_ops.h"

namespace fwi {
namespace sc {

constexpr int G = 72, NZ = 70, C0 = 32, C1 = 64, C2 = 128, NF = 16, TH = 128, NTB = 320;
constexpr int kMaxBatch = 256;
constexpr int TPB = 256;
constexpr int NBLK = 5;
constexpr int kNParts = 256;                // partial sums of the reductions
constexpr long kWorkFloats = 8L << 20;      // split-K partials of the weight gradients (32 MiB)

struct BlockDef {
    int C, S, tb_off;
};
// b0a, b1a, b2, b1b, b0b
constexpr BlockDef kBlocks[NBLK] = {{C0, 72, 0}, {C1, 36, 32}, {C2, 18, 96}, {C1, 36, 224}, {C0, 72, 288}};

struct Layout {
    long temb_w1, temb_b1, temb_w2, temb_b2, lift_w, lift_b;
    long w1[NBLK], b1[NBLK], w2[NBLK], b2[NBLK];
    long down0_w, down0_b, down1_w, down1_b, up1_w, up1_b, up0_w, up0_b, head_w, head_b;
    long total;
};

inline Layout layout() {
    Layout L{};
    long o = 0;
    auto take = [&](long n) {
        const long r = o;
        o += n;
        return r;
    };
    auto block = [&](int i) {
        const long C = kBlocks[i].C;
        L.w1[i] = take(9 * C * C);
        L.b1[i] = take(C);
        L.w2[i] = take(9 * C * C);
        L.b2[i] = take(C);
    };
    L.temb_w1 = take(2 * NF * TH);
    L.temb_b1 = take(TH);
    L.temb_w2 = take((long)TH * NTB);
    L.temb_b2 = take(NTB);
    L.lift_w = take(3 * C0);
    L.lift_b = take(C0);
    block(0);
    L.down0_w = take(C0 * C1);
    L.down0_b = take(C1);
    block(1);
    L.down1_w = take(C1 * C2);
    L.down1_b = take(C2);
    block(2);
    L.up1_w = take(C2 * C1);
    L.up1_b = take(C1);
    block(3);
    L.up0_w = take(C1 * C0);
    L.up0_b = take(C0);
    block(4);
    L.head_w = take(C0);
    L.head_b = take(1);
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------
// time embedding: e = [sin(1000 t f_k), cos(1000 t f_k)] (phase and sinusoids in
// FP64), a1 = W1^T e + b1, h1 = gelu(a1), tb = W2^T h1 + b2; one block per sample
__global__ __launch_bounds__(TPB) void k_temb_fwd(const float* __restrict__ tcond, const float* __restrict__ P,
                                                  long o_w1, long o_b1, long o_w2, long o_b2, float* __restrict__ e,
                                                  float* __restrict__ a1, float* __restrict__ h1,
                                                  float* __restrict__ tb) {
    const int b = blockIdx.x;
    __shared__ float se[2 * NF], sh[TH];
    if (threadIdx.x < NF) {
        const double f = exp(-log(10000.0) * threadIdx.x / NF);
        const double ph = 1000.0 * (double)tcond[b] * f;
        se[threadIdx.x] = (float)sin(ph);
        se[NF + threadIdx.x] = (float)cos(ph);
    }
    __syncthreads();
    if (threadIdx.x < 2 * NF) e[b * 2 * NF + threadIdx.x] = se[threadIdx.x];
    if (threadIdx.x < TH) {
        const int k = threadIdx.x;
        float s = 0.f;
        for (int j = 0; j < 2 * NF; ++j) s = fmaf(se[j], P[o_w1 + (long)j * TH + k], s);
        s += P[o_b1 + k];
        a1[b * TH + k] = s;
        const float g = gelu_f(s);
        h1[b * TH + k] = g;
        sh[k] = g;
    }
    __syncthreads();
    for (int n = threadIdx.x; n < NTB; n += TPB) {
        float s = 0.f;
        for (int k = 0; k < TH; ++k) s = fmaf(sh[k], P[o_w2 + (long)k * NTB + n], s);
        tb[b * NTB + n] = s + P[o_b2 + n];
    }
}

// dh1 = W2 dtb, da1 = dh1 gelu'(a1), per sample
__global__ __launch_bounds__(TH) void k_temb_bwd_act(const float* __restrict__ dtb, const float* __restrict__ P,
                                                     long o_w2, const float* __restrict__ a1,
                                                     float* __restrict__ da1) {
    const int b = blockIdx.x, k = threadIdx.x;
    float s = 0.f;
    for (int n = 0; n < NTB; ++n) s = fmaf(dtb[b * NTB + n], P[o_w2 + (long)k * NTB + n], s);
    da1[b * TH + k] = s * gelu_d(a1[b * TH + k]);
}

// parameter gradients of the time MLP: one thread per parameter, samples summed in order
__global__ __launch_bounds__(TPB) void k_temb_bwd_w(int B, const float* __restrict__ e, const float* __restrict__ h1,
                                                    const float* __restrict__ da1, const float* __restrict__ dtb,
                                                    float* __restrict__ G, long o_w1, long o_b1, long o_w2,
                                                    long o_b2) {
    const long n_w2 = (long)TH * NTB, n_w1 = 2L * NF * TH;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    float s = 0.f;
    if (i < n_w2) {
        const int k = (int)(i / NTB), n = (int)(i % NTB);
        for (int b = 0; b < B; ++b) s = fmaf(h1[b * TH + k], dtb[b * NTB + n], s);
        G[o_w2 + i] = s;
    } else if (i < n_w2 + NTB) {
        const int n = (int)(i - n_w2);
        for (int b = 0; b < B; ++b) s += dtb[b * NTB + n];
        G[o_b2 + n] = s;
    } else if (i < n_w2 + NTB + n_w1) {
        const long j = i - n_w2 - NTB;
        const int r = (int)(j / TH), k = (int)(j % TH);
        for (int b = 0; b < B; ++b) s = fmaf(e[b * 2 * NF + r], da1[b * TH + k], s);
        G[o_w1 + j] = s;
    } else if (i < n_w2 + NTB + n_w1 + TH) {
        const int k = (int)(i - n_w2 - NTB - n_w1);
        for (int b = 0; b < B; ++b) s += da1[b * TH + k];
        G[o_b1 + k] = s;
    }
}

// ---------------------------------------------------------------------------
// lift: h0[b][i][j][c] = R(x W[0][c] + zi W[1][c] + xj W[2][c] + b[c]) on the
// 72 x 72 grid; x = 0 on the ring, zi = (i - 35.5)/36, xj = (j - 35.5)/36
__device__ inline float ring_x(const float* x, int b, int i, int j) {
    return (i >= 1 && i <= NZ && j >= 1 && j <= NZ) ? x[((long)b * NZ + (i - 1)) * NZ + (j - 1)] : 0.f;
}

__global__ void k_lift_fwd(int B, const float* __restrict__ x, const float* __restrict__ W,
                           const float* __restrict__ bias, bf16_t* __restrict__ h0) {
    const long n = (long)B * G * G * C0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c = (int)(t % C0);
        const long cell = t / C0;
        const int j = (int)(cell % G), i = (int)((cell / G) % G), b = (int)(cell / (G * G));
        const float zi = (i - 35.5f) / 36.f, xj = (j - 35.5f) / 36.f;
        float s = ring_x(x, b, i, j) * W[c];
        s = fmaf(zi, W[C0 + c], s);
        s = fmaf(xj, W[2 * C0 + c], s);
        h0[t] = f2bf(s + bias[c]);
    }
}

// dx[b][i][j] = skip_b dout + sum_c dh0[b][i+1][j+1][c] W[0][c]
__global__ void k_lift_bwd_input(int B, const float* __restrict__ dh0, const float* __restrict__ W,
                                 const float* __restrict__ dout, const float* __restrict__ skip,
                                 float* __restrict__ dx) {
    const long n = (long)B * NZ * NZ;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int j = (int)(t % NZ), i = (int)((t / NZ) % NZ), b = (int)(t / (NZ * NZ));
        const float* d = dh0 + (((long)b * G + i + 1) * G + j + 1) * C0;
        float s = 0.f;
        for (int c = 0; c < C0; ++c) s = fmaf(d[c], W[c], s);
        dx[t] = (skip ? skip[b] * dout[t] : 0.f) + s;
    }
}

// partial sums over the 72 x 72 cells of feat_f dh0[c] (f = x, zi, xj) and of
// dh0[c]: part[p][4 * C0], rows split evenly over kNParts blocks
__global__ __launch_bounds__(TPB) void k_lift_bwd_weight_partial(int B, const float* __restrict__ x,
                                                                 const float* __restrict__ dh0,
                                                                 float* __restrict__ part) {
    const long rows = (long)B * G * G;
    const int c = threadIdx.x % C0, l = threadIdx.x / C0;  // 8 lanes per channel
    const long lo = rows * blockIdx.x / gridDim.x, hi = rows * (blockIdx.x + 1) / gridDim.x;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (long r = lo + l; r < hi; r += TPB / C0) {
        const int j = (int)(r % G), i = (int)((r / G) % G), b = (int)(r / (G * G));
        const float d = dh0[r * C0 + c];
        s0 = fmaf(ring_x(x, b, i, j), d, s0);
        s1 = fmaf((i - 35.5f) / 36.f, d, s1);
        s2 = fmaf((j - 35.5f) / 36.f, d, s2);
        s3 += d;
    }
    __shared__ float sh[4][TPB];
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    sh[2][threadIdx.x] = s2;
    sh[3][threadIdx.x] = s3;
    __syncthreads();
    if (l == 0)
        for (int f = 0; f < 4; ++f) {
            float t = 0.f;
            for (int q = 0; q < TPB / C0; ++q) t += sh[f][q * C0 + c];
            part[(long)blockIdx.x * 4 * C0 + f * C0 + c] = t;
        }
}

// out[j] = sum_p part[p][j] in order (j < len)
__global__ void k_sum_parts(const float* __restrict__ part, int nparts, int len, float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    float s = 0.f;
    for (int p = 0; p < nparts; ++p) s += part[(long)p * len + j];
    out[j] = s;
}

// ---------------------------------------------------------------------------
// im2col: col[row][tap * C + c] = h[b][i + dy - 1][j + dx - 1][c] (0 outside),
// 8 channels (16 bytes) per thread
__global__ void k_im2col(int B, int S, int C, const bf16_t* __restrict__ h, bf16_t* __restrict__ col) {
    const int C8 = C / 8;
    const long n = (long)B * S * S * 9 * C8;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c8 = (int)(t % C8);
        const int tap = (int)((t / C8) % 9);
        const long row = t / (9L * C8);
        const int j = (int)(row % S), i = (int)((row / S) % S);
        const long b = row / ((long)S * S);
        const int ii = i + tap / 3 - 1, jj = j + tap % 3 - 1;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (ii >= 0 && ii < S && jj >= 0 && jj < S)
            v = *reinterpret_cast<const uint4*>(h + ((b * S + ii) * S + jj) * C + c8 * 8);
        *reinterpret_cast<uint4*>(col + row * 9L * C + tap * C + c8 * 8) = v;
    }
}

// transpose of im2col, added to a base: out = base + col2im(dcol) (out may be base)
__global__ void k_col2im(int B, int S, int C, const float* __restrict__ dcol, const float* base, float* out) {
    const long n = (long)B * S * S * C;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c = (int)(t % C);
        const long cell = t / C;
        const int j = (int)(cell % S), i = (int)((cell / S) % S);
        const long b = cell / ((long)S * S);
        float s = 0.f;
        for (int tap = 0; tap < 9; ++tap) {
            const int oi = i - tap / 3 + 1, oj = j - tap % 3 + 1;  // output row whose tap reads (i, j)
            if (oi >= 0 && oi < S && oj >= 0 && oj < S) s += dcol[((b * S + oi) * S + oj) * 9L * C + tap * C + c];
        }
        out[t] = (base ? base[t] : 0.f) + s;
    }
}

// p = R(y + b1[c] + tb[b][off + c]), q = R(gelu(p))
__global__ void k_bias_gelu(int B, int S, int C, const float* __restrict__ y, const float* __restrict__ b1,
                            const float* __restrict__ tb, int off, bf16_t* __restrict__ p, bf16_t* __restrict__ q) {
    const long n = (long)B * S * S * C;
    const long per = (long)S * S * C;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c = (int)(t % C);
        const int b = (int)(t / per);
        const bf16_t pv = f2bf(y[t] + b1[c] + tb[b * NTB + off + c]);
        p[t] = pv;
        q[t] = f2bf(gelu_f(bf2f(pv)));
    }
}

// per-sample column sums of a [B][rows][C] FP32 stream, out[b * ld + c] (fixed order)
__global__ __launch_bounds__(TPB) void k_sample_colsum(long rows, int C, const float* __restrict__ a,
                                                       float* __restrict__ out, int ld) {
    const int b = blockIdx.x;
    const int lanes = TPB / C;
    const int c = threadIdx.x % C, l = threadIdx.x / C;
    float s = 0.f;
    if (l < lanes)
        for (long r = l; r < rows; r += lanes) s += a[((long)b * rows + r) * C + c];
    __shared__ float sh[TPB];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (l == 0) {
        float t = 0.f;
        for (int q = 0; q < lanes; ++q) t += sh[q * C + c];
        out[b * ld + c] = t;
    }
}

// sum over samples: out[c] = sum_b v[b * ld + c]
__global__ void k_sum_samples(int B, int C, const float* __restrict__ v, int ld, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += v[b * ld + c];
    out[c] = s;
}

// 2 x 2 average pooling: out = R(0.25 (((h00 + h01) + h10) + h11))
__global__ void k_pool(int B, int S, int C, const bf16_t* __restrict__ h, bf16_t* __restrict__ out) {
    const int So = S / 2;
    const long n = (long)B * So * So * C;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c = (int)(t % C);
        const long cell = t / C;
        const int j = (int)(cell % So), i = (int)((cell / So) % So);
        const long b = cell / ((long)So * So);
        const bf16_t* r0 = h + ((b * S + 2 * i) * S + 2 * j) * C + c;
        const bf16_t* r1 = r0 + (long)S * C;
        const float s = ((bf2f(r0[0]) + bf2f(r0[C])) + bf2f(r1[0])) + bf2f(r1[C]);
        out[t] = f2bf(0.25f * s);
    }
}

// pooling transpose, accumulated: dh[b][2i + di][2j + dj][c] += 0.25 dp[b][i][j][c]
__global__ void k_pool_bwd(int B, int S, int C, const float* __restrict__ dp, float* __restrict__ dh) {
    const long n = (long)B * S * S * C;
    const int So = S / 2;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c = (int)(t % C);
        const long cell = t / C;
        const int j = (int)(cell % S), i = (int)((cell / S) % S);
        const long b = cell / ((long)S * S);
        dh[t] += 0.25f * dp[((b * So + i / 2) * So + j / 2) * C + c];
    }
}

// nearest up-sampling plus skip: out[b][I][J][c] = R(y[b][I/2][J/2][c] + skip[b][I][J][c])
__global__ void k_up_add(int B, int S, int C, const bf16_t* __restrict__ y, const bf16_t* __restrict__ skip,
                         bf16_t* __restrict__ out) {
    const long n = (long)B * S * S * C;
    const int Si = S / 2;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c = (int)(t % C);
        const long cell = t / C;
        const int j = (int)(cell % S), i = (int)((cell / S) % S);
        const long b = cell / ((long)S * S);
        out[t] = f2bf(bf2f(y[((b * Si + i / 2) * Si + j / 2) * C + c]) + bf2f(skip[t]));
    }
}

// up-sampling transpose: dy[b][i][j][c] = ((d00 + d01) + d10) + d11 over the four children
__global__ void k_up_bwd(int B, int Si, int C, const float* __restrict__ d, float* __restrict__ dy,
                         bf16_t* __restrict__ dy16) {
    const long n = (long)B * Si * Si * C;
    const int S = 2 * Si;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c = (int)(t % C);
        const long cell = t / C;
        const int j = (int)(cell % Si), i = (int)((cell / Si) % Si);
        const long b = cell / ((long)Si * Si);
        const float* r0 = d + ((b * S + 2 * i) * S + 2 * j) * C + c;
        const float* r1 = r0 + (long)S * C;
        const float s = ((r0[0] + r0[C]) + r1[0]) + r1[C];
        dy[t] = s;
        dy16[t] = f2bf(s);
    }
}

// head and output map: out[b][i][j] = skip_b x + scale_b (sum_c h[b][i+1][j+1][c] w[c] + bias)
__global__ void k_head_fwd(int B, const bf16_t* __restrict__ h, const float* __restrict__ w,
                           const float* __restrict__ bias, const float* __restrict__ x, const float* __restrict__ skip,
                           const float* __restrict__ scale, float* __restrict__ out) {
    const long n = (long)B * NZ * NZ;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int j = (int)(t % NZ), i = (int)((t / NZ) % NZ), b = (int)(t / (NZ * NZ));
        const bf16_t* hp = h + (((long)b * G + i + 1) * G + j + 1) * C0;
        float s = 0.f;
        for (int c = 0; c < C0; ++c) s = fmaf(bf2f(hp[c]), w[c], s);
        s += bias[0];
        const float sc = scale ? scale[b] : 1.f;
        out[t] = (skip ? skip[b] * x[t] : 0.f) + sc * s;
    }
}

// head transpose: dh[b][i][j][c] = de[b][i][j] w[c] with de = scale_b dout inside, 0 on the ring
__global__ void k_head_bwd_input(int B, const float* __restrict__ dout, const float* __restrict__ scale,
                                 const float* __restrict__ w, float* __restrict__ dh) {
    const long n = (long)B * G * G * C0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int c = (int)(t % C0);
        const long cell = t / C0;
        const int j = (int)(cell % G), i = (int)((cell / G) % G), b = (int)(cell / (G * G));
        float de = 0.f;
        if (i >= 1 && i <= NZ && j >= 1 && j <= NZ)
            de = (scale ? scale[b] : 1.f) * dout[((long)b * NZ + i - 1) * NZ + j - 1];
        dh[t] = de * w[c];
    }
}

// partials of sum de h[c] and sum de over the model cells: part[p][C0 + 1]
__global__ __launch_bounds__(TPB) void k_head_bwd_weight_partial(int B, const float* __restrict__ dout,
                                                                 const float* __restrict__ scale,
                                                                 const bf16_t* __restrict__ h,
                                                                 float* __restrict__ part) {
    const long rows = (long)B * NZ * NZ;
    const int c = threadIdx.x % C0, l = threadIdx.x / C0;
    const long lo = rows * blockIdx.x / gridDim.x, hi = rows * (blockIdx.x + 1) / gridDim.x;
    float s = 0.f, sb = 0.f;
    for (long r = lo + l; r < hi; r += TPB / C0) {
        const int j = (int)(r % NZ), i = (int)((r / NZ) % NZ), b = (int)(r / (NZ * NZ));
        const float de = (scale ? scale[b] : 1.f) * dout[r];
        s = fmaf(de, bf2f(h[(((long)b * G + i + 1) * G + j + 1) * C0 + c]), s);
        sb += de;
    }
    __shared__ float sh[2][TPB];
    sh[0][threadIdx.x] = s;
    sh[1][threadIdx.x] = sb;
    __syncthreads();
    if (l == 0) {
        float t = 0.f, tb = 0.f;
        for (int q = 0; q < TPB / C0; ++q) {
            t += sh[0][q * C0 + c];
            tb += sh[1][q * C0 + c];
        }
        part[(long)blockIdx.x * (C0 + 1) + c] = t;
        if (c == 0) part[(long)blockIdx.x * (C0 + 1) + C0] = tb;
    }
}

// ---------------------------------------------------------------------------
// denoising score matching: x_t = a_b x0 + s_b noise (per-sample coefficients)
__global__ void k_noise_state(int B, const float* __restrict__ x0, const float* __restrict__ noise,
                              const float* __restrict__ sa, const float* __restrict__ s1a, float* __restrict__ xt) {
    const long n = (long)B * NZ * NZ;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int b = (int)(t / (NZ * NZ));
        xt[t] = fmaf(sa[b], x0[t], s1a[b] * noise[t]);
    }
}

// r = pred - noise: dpred = 2 r / n, partial sums of r^2 per block
__global__ __launch_bounds__(TPB) void k_dsm_loss(long n, const float* __restrict__ pred,
                                                  const float* __restrict__ noise, float* __restrict__ dpred,
                                                  float* __restrict__ part) {
    const long lo = n * blockIdx.x / gridDim.x, hi = n * (blockIdx.x + 1) / gridDim.x;
    const float k = 2.f / (float)n;
    float s = 0.f;
    for (long t = lo + threadIdx.x; t < hi; t += TPB) {
        const float r = pred[t] - noise[t];
        dpred[t] = k * r;
        s = fmaf(r, r, s);
    }
    __shared__ float sh[TPB];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int q = 0; q < TPB; ++q) t += sh[q];
        part[blockIdx.x] = t;
    }
}

__global__ void k_dsm_loss_final(const float* __restrict__ part, int np, long n, float* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0.f;
    for (int p = 0; p < np; ++p) s += part[p];
    *loss = s / (float)n;
}

int grid_for(long n) { return (int)std::min<long>((n + TPB - 1) / TPB, 16384); }

inline int hip_ok(hipError_t e) { return e == hipSuccess ? FWI_OK : FWI_EHIP; }

}  // namespace sc
}  // namespace fwi

struct fwi_score_net {
    int device = 0, max_batch = 0, step = 0, cachedB = 0;
    fwi::sc::Layout L;
    std::vector<void*> allocs;
    // parameters (FP32 master), gradients, Adam moments, BF16 copies of the GEMM weights
    float *P = nullptr, *G = nullptr, *Am = nullptr, *Av = nullptr;
    int* bf_index = nullptr;
    fwi::bf16_t* W = nullptr;
    long bw1[fwi::sc::NBLK], bw2[fwi::sc::NBLK], bdown0, bdown1, bup1, bup0, bf_total;
    // time embedding
    float *e = nullptr, *a1 = nullptr, *h1 = nullptr, *tb = nullptr, *dtb = nullptr, *da1 = nullptr;
    // activations (BF16, NHWC)
    fwi::bf16_t *h0, *hb[fwi::sc::NBLK], *p[fwi::sc::NBLK], *q[fwi::sc::NBLK], *pl0, *d1, *pl1, *d2, *y1, *u1, *y0,
        *u0;
    fwi::bf16_t *col = nullptr, *g16 = nullptr;
    float *xcache = nullptr, *skipc = nullptr, *scalec = nullptr;
    int have_skip = 0, have_scale = 0;
    // gradient streams (FP32)
    float *dA72, *dB72, *dA36, *dB36, *dA18, *scr, *dcol, *y32;
    float *part = nullptr, *work = nullptr;
    // training
    float *xt = nullptr, *pred = nullptr, *dpred = nullptr, *lval = nullptr;
};

namespace fwi {
namespace sc {
namespace {

template <class T>
bool dalloc(fwi_score_net* s, T** p, long n) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)std::max<long>(n, 1) * sizeof(T)) != hipSuccess) return false;
    s->allocs.push_back(q);
    *p = (T*)q;
    return true;
}

void free_all(fwi_score_net* s) {
    for (void* p : s->allocs) (void)hipFree(p);
    s->allocs.clear();
}

int pick_splitk(int M, int N, long ksteps) {
    const long tiles = (long)((M + 63) / 64) * ((N + 63) / 64);
    long sk = (512 + tiles - 1) / tiles;
    sk = std::min<long>(sk, std::max<long>(1, ksteps / 8));
    sk = std::min<long>(sk, kWorkFloats / ((long)M * N));
    return (int)std::max<long>(1, std::min<long>(sk, 256));
}

struct Ctx {
    fwi_score_net* s;
    hipStream_t st;
    int rc = FWI_OK;

    // C = A (op B) (+ bias) over `rows` rows; out FP32 or BF16 with an epilogue
    void mm(long rows, int N, int K, const bf16_t* A, int lda, const bf16_t* Bm, int ldb, int tB, float* C32,
            bf16_t* C16, const float* bias, int epi = kEpiNone, const bf16_t* res16 = nullptr) {
        if (rc != FWI_OK) return;
        GemmArgs g;
        g.M = (int)rows, g.N = N, g.K = K;
        g.A = A, g.lda = lda;
        g.B = Bm, g.ldb = ldb, g.transB = tB;
        g.C32 = C32, g.C16 = C16, g.ldc = N, g.bias = bias;
        g.epi = epi, g.res16 = res16;
        rc = gemm_bf16(g, st);
    }
    // weight gradient dW[K'][N] = A^T B over `rows` rows (A [rows][M], B [rows][N]), split over rows
    void wgrad(long rows, int M, int N, const bf16_t* A, const bf16_t* Bm, float* dW) {
        if (rc != FWI_OK) return;
        GemmArgs g;
        g.M = M, g.N = N, g.K = (int)rows;
        g.A = A, g.lda = M, g.transA = 1;
        g.B = Bm, g.ldb = N;
        g.C32 = dW, g.ldc = N;
        g.splitk = pick_splitk(M, N, (rows + 31) / 32);
        g.work = s->work;
        rc = gemm_bf16(g, st);
    }
    void check() {
        if (rc == FWI_OK && hipGetLastError() != hipSuccess) rc = FWI_EHIP;
    }
};

bf16_t* bfw(fwi_score_net* s, long off) { return s->W + off; }

// block forward: out = R(h + R(conv3(R(gelu(R(conv3(h) + b1 + tb)))) + b2))
void block_fwd(Ctx& c, int i, int B, const bf16_t* h, bf16_t* out) {
    fwi_score_net* s = c.s;
    const BlockDef d = kBlocks[i];
    const long rows = (long)B * d.S * d.S;
    const long n8 = rows * 9 * (d.C / 8);
    hipLaunchKernelGGL(k_im2col, dim3(grid_for(n8)), dim3(TPB), 0, c.st, B, d.S, d.C, h, s->col);
    c.mm(rows, d.C, 9 * d.C, s->col, 9 * d.C, bfw(s, s->bw1[i]), d.C, 0, s->y32, nullptr, nullptr);
    hipLaunchKernelGGL(k_bias_gelu, dim3(grid_for(rows * d.C)), dim3(TPB), 0, c.st, B, d.S, d.C, s->y32,
                       s->P + s->L.b1[i], s->tb, d.tb_off, s->p[i], s->q[i]);
    hipLaunchKernelGGL(k_im2col, dim3(grid_for(n8)), dim3(TPB), 0, c.st, B, d.S, d.C, s->q[i], s->col);
    c.mm(rows, d.C, 9 * d.C, s->col, 9 * d.C, bfw(s, s->bw2[i]), d.C, 0, nullptr, out, s->P + s->L.b2[i], kEpiResid,
         h);
    c.check();
}

// block backward: dh_in = dout + conv3^T(dp), weight gradients when G != nullptr;
// dout and dh_in may be the same buffer.  h is the block's input.
void block_bwd(Ctx& c, int i, int B, const bf16_t* h, const float* dout, float* dh_in, float* G) {
    fwi_score_net* s = c.s;
    const BlockDef d = kBlocks[i];
    const long rows = (long)B * d.S * d.S;
    const long n = rows * d.C;
    const long n8 = rows * 9 * (d.C / 8);
    nn::to_bf16(n, dout, s->g16, c.st);  // R(dy2)
    if (G) {
        nn::colsum(rows, d.C, dout, G + s->L.b2[i], s->part, c.st);
        hipLaunchKernelGGL(k_im2col, dim3(grid_for(n8)), dim3(TPB), 0, c.st, B, d.S, d.C, s->q[i], s->col);
        c.wgrad(rows, 9 * d.C, d.C, s->col, s->g16, G + s->L.w2[i]);
    }
    // dq = col2im(R(dy2) W2^T)
    c.mm(rows, 9 * d.C, d.C, s->g16, d.C, bfw(s, s->bw2[i]), d.C, 1, s->dcol, nullptr, nullptr);
    hipLaunchKernelGGL(k_col2im, dim3(grid_for(n)), dim3(TPB), 0, c.st, B, d.S, d.C, s->dcol, nullptr, s->scr);
    // dp = dq gelu'(p) (FP32, y32) and R(dp) (g16)
    nn::gelu_bwd(n, s->scr, s->p[i], s->y32, s->g16, c.st);
    hipLaunchKernelGGL(k_sample_colsum, dim3(B), dim3(TPB), 0, c.st, (long)d.S * d.S, d.C, s->y32,
                       s->dtb + d.tb_off, NTB);
    if (G) {
        hipLaunchKernelGGL(k_sum_samples, dim3(1), dim3(TPB), 0, c.st, B, d.C, s->dtb + d.tb_off, NTB,
                           G + s->L.b1[i]);
        hipLaunchKernelGGL(k_im2col, dim3(grid_for(n8)), dim3(TPB), 0, c.st, B, d.S, d.C, h, s->col);
        c.wgrad(rows, 9 * d.C, d.C, s->col, s->g16, G + s->L.w1[i]);
    }
    // dh_in = dout + col2im(R(dp) W1^T)
    c.mm(rows, 9 * d.C, d.C, s->g16, d.C, bfw(s, s->bw1[i]), d.C, 1, s->dcol, nullptr, nullptr);
    hipLaunchKernelGGL(k_col2im, dim3(grid_for(n)), dim3(TPB), 0, c.st, B, d.S, d.C, s->dcol, dout, dh_in);
    c.check();
}

// y = R(x W + b) backward: dy FP32 [rows][N]; dx = R(dy) W^T into dx32 [rows][K]
void lin_bwd(Ctx& c, long rows, int K, int N, const bf16_t* x, const float* dy, const bf16_t* Wb, long o_w, long o_b,
             float* dx32, float* G) {
    fwi_score_net* s = c.s;
    nn::to_bf16(rows * N, dy, s->g16, c.st);
    if (G) {
        nn::colsum(rows, N, dy, G + o_b, s->part, c.st);
        c.wgrad(rows, K, N, x, s->g16, G + o_w);
    }
    c.mm(rows, K, N, s->g16, N, Wb, N, 1, dx32, nullptr, nullptr);
    c.check();
}

int forward_impl(fwi_score_net* s, int B, const float* x, const float* tcond, const float* skip, const float* scale,
                 float* out, hipStream_t st) {
    Ctx c{s, st};
    const Layout& L = s->L;
    hipLaunchKernelGGL(k_temb_fwd, dim3(B), dim3(TPB), 0, st, tcond, s->P, L.temb_w1, L.temb_b1, L.temb_w2,
                       L.temb_b2, s->e, s->a1, s->h1, s->tb);
    const long nx = (long)B * NZ * NZ;
    nn::copy_f32(nx, x, s->xcache, st);
    s->have_skip = skip != nullptr;
    s->have_scale = scale != nullptr;
    if (skip) nn::copy_f32(B, skip, s->skipc, st);
    if (scale) nn::copy_f32(B, scale, s->scalec, st);
    hipLaunchKernelGGL(k_lift_fwd, dim3(grid_for((long)B * G * G * C0)), dim3(TPB), 0, st, B, x, s->P + L.lift_w,
                       s->P + L.lift_b, s->h0);
    block_fwd(c, 0, B, s->h0, s->hb[0]);
    hipLaunchKernelGGL(k_pool, dim3(grid_for((long)B * 36 * 36 * C0)), dim3(TPB), 0, st, B, 72, C0, s->hb[0], s->pl0);
    c.mm((long)B * 36 * 36, C1, C0, s->pl0, C0, bfw(s, s->bdown0), C1, 0, nullptr, s->d1, s->P + L.down0_b);
    block_fwd(c, 1, B, s->d1, s->hb[1]);
    hipLaunchKernelGGL(k_pool, dim3(grid_for((long)B * 18 * 18 * C1)), dim3(TPB), 0, st, B, 36, C1, s->hb[1], s->pl1);
    c.mm((long)B * 18 * 18, C2, C1, s->pl1, C1, bfw(s, s->bdown1), C2, 0, nullptr, s->d2, s->P + L.down1_b);
    block_fwd(c, 2, B, s->d2, s->hb[2]);
    c.mm((long)B * 18 * 18, C1, C2, s->hb[2], C2, bfw(s, s->bup1), C1, 0, nullptr, s->y1, s->P + L.up1_b);
    hipLaunchKernelGGL(k_up_add, dim3(grid_for((long)B * 36 * 36 * C1)), dim3(TPB), 0, st, B, 36, C1, s->y1,
                       s->hb[1], s->u1);
    block_fwd(c, 3, B, s->u1, s->hb[3]);
    c.mm((long)B * 36 * 36, C0, C1, s->hb[3], C1, bfw(s, s->bup0), C0, 0, nullptr, s->y0, s->P + L.up0_b);
    hipLaunchKernelGGL(k_up_add, dim3(grid_for((long)B * 72 * 72 * C0)), dim3(TPB), 0, st, B, 72, C0, s->y0,
                       s->hb[0], s->u0);
    block_fwd(c, 4, B, s->u0, s->hb[4]);
    hipLaunchKernelGGL(k_head_fwd, dim3(grid_for(nx)), dim3(TPB), 0, st, B, s->hb[4], s->P + L.head_w,
                       s->P + L.head_b, x, skip, scale, out);
    c.check();
    if (c.rc == FWI_OK) s->cachedB = B;
    return c.rc;
}

// dx = (d out / d x)^T dout through the last forward (same B); parameter
// gradients into s->G when want_w
int backward_impl(fwi_score_net* s, int B, const float* dout, float* dx, bool want_w, hipStream_t st) {
    Ctx c{s, st};
    const Layout& L = s->L;
    float* G = want_w ? s->G : nullptr;
    const float* scale = s->have_scale ? s->scalec : nullptr;
    const float* skip = s->have_skip ? s->skipc : nullptr;
    const long r72 = (long)B * 72 * 72, r36 = (long)B * 36 * 36, r18 = (long)B * 18 * 18;
    // head
    hipLaunchKernelGGL(k_head_bwd_input, dim3(grid_for(r72 * C0)), dim3(TPB), 0, st, B, dout, scale, s->P + L.head_w,
                       s->dA72);
    if (G) {
        hipLaunchKernelGGL(k_head_bwd_weight_partial, dim3(kNParts), dim3(TPB), 0, st, B, dout, scale, s->hb[4],
                           s->part);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(TPB), 0, st, s->part, kNParts, C0 + 1, G + L.head_w);
    }
    // b0b -> du0 (dB72, which then collects the skip gradient of b0a's output)
    block_bwd(c, 4, B, s->u0, s->dA72, s->dB72, G);
    // up0: dy0 = up^T(du0); dhb1b = R(dy0) Wu0^T -> dA36
    hipLaunchKernelGGL(k_up_bwd, dim3(grid_for(r36 * C0)), dim3(TPB), 0, st, B, 36, C0, s->dB72, s->scr, s->g16);
    if (G) {
        nn::colsum(r36, C0, s->scr, G + L.up0_b, s->part, st);
        c.wgrad(r36, C1, C0, s->hb[3], s->g16, G + L.up0_w);
    }
    c.mm(r36, C1, C0, s->g16, C0, bfw(s, s->bup0), C0, 1, s->dA36, nullptr, nullptr);
    // b1b -> du1 (dB36: skip gradient of b1a's output)
    block_bwd(c, 3, B, s->u1, s->dA36, s->dB36, G);
    // up1 -> dA18
    hipLaunchKernelGGL(k_up_bwd, dim3(grid_for(r18 * C1)), dim3(TPB), 0, st, B, 18, C1, s->dB36, s->scr, s->g16);
    if (G) {
        nn::colsum(r18, C1, s->scr, G + L.up1_b, s->part, st);
        c.wgrad(r18, C2, C1, s->hb[2], s->g16, G + L.up1_w);
    }
    c.mm(r18, C2, C1, s->g16, C1, bfw(s, s->bup1), C1, 1, s->dA18, nullptr, nullptr);
    // b2 (in place) -> dd2
    block_bwd(c, 2, B, s->d2, s->dA18, s->dA18, G);
    // down1: dpl1 = R(dd2) Wd1^T; dhb1a += 0.25 up(dpl1)
    lin_bwd(c, r18, C1, C2, s->pl1, s->dA18, bfw(s, s->bdown1), L.down1_w, L.down1_b, s->y32, G);
    hipLaunchKernelGGL(k_pool_bwd, dim3(grid_for(r36 * C1)), dim3(TPB), 0, st, B, 36, C1, s->y32, s->dB36);
    // b1a -> dd1 (dA36)
    block_bwd(c, 1, B, s->d1, s->dB36, s->dA36, G);
    // down0
    lin_bwd(c, r36, C0, C1, s->pl0, s->dA36, bfw(s, s->bdown0), L.down0_w, L.down0_b, s->y32, G);
    hipLaunchKernelGGL(k_pool_bwd, dim3(grid_for(r72 * C0)), dim3(TPB), 0, st, B, 72, C0, s->y32, s->dB72);
    // b0a -> dh0 (dA72)
    block_bwd(c, 0, B, s->h0, s->dB72, s->dA72, G);
    // lift
    if (dx)
        hipLaunchKernelGGL(k_lift_bwd_input, dim3(grid_for((long)B * NZ * NZ)), dim3(TPB), 0, st, B, s->dA72,
                           s->P + L.lift_w, dout, skip, dx);
    if (G) {
        hipLaunchKernelGGL(k_lift_bwd_weight_partial, dim3(kNParts), dim3(TPB), 0, st, B, s->xcache, s->dA72,
                           s->part);
        // lift_w [3][C0] and lift_b [C0] are contiguous: 4 C0 sums in that order
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(TPB), 0, st, s->part, kNParts, 4 * C0, G + L.lift_w);
        // time embedding
        hipLaunchKernelGGL(k_temb_bwd_act, dim3(B), dim3(TH), 0, st, s->dtb, s->P, L.temb_w2, s->a1, s->da1);
        const long nw = (long)TH * NTB + NTB + 2L * NF * TH + TH;
        hipLaunchKernelGGL(k_temb_bwd_w, dim3((nw + TPB - 1) / TPB), dim3(TPB), 0, st, B, s->e, s->h1, s->da1,
                           s->dtb, G, L.temb_w1, L.temb_b1, L.temb_w2, L.temb_b2);
    }
    c.check();
    return c.rc;
}

}  // namespace
}  // namespace sc
}  // namespace fwi

using namespace fwi;
using namespace fwi::sc;

extern "C" {

long fwi_score_param_count(void) { return sc::layout().total; }

int fwi_score_create(int max_batch, fwi_score_net** out) {
    if (!out || max_batch < 1 || max_batch > kMaxBatch) return FWI_EINVAL;
    *out = nullptr;
    fwi_score_net* s = new (std::nothrow) fwi_score_net();
    if (!s) return FWI_ENOMEM;
    (void)hipGetDevice(&s->device);
    s->max_batch = max_batch;
    s->L = sc::layout();
    const Layout& L = s->L;
    // BF16 copies of the GEMM weights
    long o = 0;
    for (int i = 0; i < NBLK; ++i) {
        const long C = kBlocks[i].C;
        s->bw1[i] = o, o += 9 * C * C;
        s->bw2[i] = o, o += 9 * C * C;
    }
    s->bdown0 = o, o += C0 * C1;
    s->bdown1 = o, o += C1 * C2;
    s->bup1 = o, o += C2 * C1;
    s->bup0 = o, o += C1 * C0;
    s->bf_total = o;
    std::vector<int> bfi(L.total, -1);
    for (int i = 0; i < NBLK; ++i) {
        const long C = kBlocks[i].C;
        for (long k = 0; k < 9 * C * C; ++k) {
            bfi[L.w1[i] + k] = (int)(s->bw1[i] + k);
            bfi[L.w2[i] + k] = (int)(s->bw2[i] + k);
        }
    }
    for (long k = 0; k < C0 * C1; ++k) bfi[L.down0_w + k] = (int)(s->bdown0 + k);
    for (long k = 0; k < C1 * C2; ++k) bfi[L.down1_w + k] = (int)(s->bdown1 + k);
    for (long k = 0; k < C2 * C1; ++k) bfi[L.up1_w + k] = (int)(s->bup1 + k);
    for (long k = 0; k < C1 * C0; ++k) bfi[L.up0_w + k] = (int)(s->bup0 + k);

    const long Bm = max_batch;
    const long r72 = Bm * 72 * 72, r36 = Bm * 36 * 36, r18 = Bm * 18 * 18;
    bool ok = dalloc(s, &s->P, L.total) && dalloc(s, &s->G, L.total) && dalloc(s, &s->Am, L.total) &&
              dalloc(s, &s->Av, L.total) && dalloc(s, &s->bf_index, L.total) && dalloc(s, &s->W, s->bf_total) &&
              dalloc(s, &s->e, Bm * 2 * NF) && dalloc(s, &s->a1, Bm * TH) && dalloc(s, &s->h1, Bm * TH) &&
              dalloc(s, &s->tb, Bm * NTB) && dalloc(s, &s->dtb, Bm * NTB) && dalloc(s, &s->da1, Bm * TH) &&
              dalloc(s, &s->h0, r72 * C0) && dalloc(s, &s->pl0, r36 * C0) && dalloc(s, &s->d1, r36 * C1) &&
              dalloc(s, &s->pl1, r18 * C1) && dalloc(s, &s->d2, r18 * C2) && dalloc(s, &s->y1, r18 * C1) &&
              dalloc(s, &s->u1, r36 * C1) && dalloc(s, &s->y0, r36 * C0) && dalloc(s, &s->u0, r72 * C0) &&
              dalloc(s, &s->col, r72 * 9 * C0) && dalloc(s, &s->g16, r72 * C0) && dalloc(s, &s->xcache, Bm * NZ * NZ) &&
              dalloc(s, &s->skipc, Bm) && dalloc(s, &s->scalec, Bm) && dalloc(s, &s->dA72, r72 * C0) &&
              dalloc(s, &s->dB72, r72 * C0) && dalloc(s, &s->dA36, r36 * C1) && dalloc(s, &s->dB36, r36 * C1) &&
              dalloc(s, &s->dA18, r18 * C2) && dalloc(s, &s->scr, r72 * C0) && dalloc(s, &s->dcol, r72 * 9 * C0) &&
              dalloc(s, &s->y32, r72 * C0) && dalloc(s, &s->part, (long)kNParts * 4 * C0) &&
              dalloc(s, &s->work, kWorkFloats) && dalloc(s, &s->xt, Bm * NZ * NZ) &&
              dalloc(s, &s->pred, Bm * NZ * NZ) && dalloc(s, &s->dpred, Bm * NZ * NZ) && dalloc(s, &s->lval, 1);
    for (int i = 0; ok && i < NBLK; ++i) {
        const long rows = Bm * kBlocks[i].S * kBlocks[i].S * kBlocks[i].C;
        ok = dalloc(s, &s->hb[i], rows) && dalloc(s, &s->p[i], rows) && dalloc(s, &s->q[i], rows);
    }
    if (!ok) {
        (void)hipGetLastError();
        free_all(s);
        delete s;
        return FWI_ENOMEM;
    }
    int rc = hip_ok(hipMemcpy(s->bf_index, bfi.data(), bfi.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!rc) rc = hip_ok(hipMemset(s->P, 0, L.total * sizeof(float)));
    if (!rc) rc = hip_ok(hipMemset(s->G, 0, L.total * sizeof(float)));
    if (!rc) rc = hip_ok(hipMemset(s->Am, 0, L.total * sizeof(float)));
    if (!rc) rc = hip_ok(hipMemset(s->Av, 0, L.total * sizeof(float)));
    if (!rc) rc = hip_ok(hipMemset(s->W, 0, s->bf_total * sizeof(bf16_t)));
    if (!rc) rc = hip_ok(hipDeviceSynchronize());
    if (rc) {
        free_all(s);
        delete s;
        return rc;
    }
    *out = s;
    return FWI_OK;
}

int fwi_score_destroy(fwi_score_net* s) {
    if (!s) return FWI_EINVAL;
    (void)hipSetDevice(s->device);
    const int rc = hip_ok(hipDeviceSynchronize());
    free_all(s);
    delete s;
    return rc;
}

int fwi_score_set_params(fwi_score_net* s, const float* host_params) {
    if (!s || !host_params) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    const long n = s->L.total;
    int rc = hip_ok(hipMemcpy(s->P, host_params, n * sizeof(float), hipMemcpyHostToDevice));
    if (!rc) nn::refresh_bf16(n, s->P, s->bf_index, s->W, nullptr);
    if (!rc) rc = hip_ok(hipMemset(s->Am, 0, n * sizeof(float)));
    if (!rc) rc = hip_ok(hipMemset(s->Av, 0, n * sizeof(float)));
    if (!rc) rc = hip_ok(hipDeviceSynchronize());
    s->step = 0;
    return rc;
}

int fwi_score_get_params(fwi_score_net* s, float* host_params) {
    if (!s || !host_params) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    if (hipDeviceSynchronize() != hipSuccess) return FWI_EHIP;
    return hip_ok(hipMemcpy(host_params, s->P, s->L.total * sizeof(float), hipMemcpyDeviceToHost));
}

int fwi_score_get_grads(fwi_score_net* s, float* host_grads) {
    if (!s || !host_grads) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    if (hipDeviceSynchronize() != hipSuccess) return FWI_EHIP;
    return hip_ok(hipMemcpy(host_grads, s->G, s->L.total * sizeof(float), hipMemcpyDeviceToHost));
}

int fwi_score_get_adam(fwi_score_net* s, float* host_m, float* host_v, int* step) {
    if (!s || !host_m || !host_v || !step) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    if (hipDeviceSynchronize() != hipSuccess) return FWI_EHIP;
    int rc = hip_ok(hipMemcpy(host_m, s->Am, s->L.total * sizeof(float), hipMemcpyDeviceToHost));
    if (!rc) rc = hip_ok(hipMemcpy(host_v, s->Av, s->L.total * sizeof(float), hipMemcpyDeviceToHost));
    *step = s->step;
    return rc;
}

int fwi_score_set_adam(fwi_score_net* s, const float* host_m, const float* host_v, int step) {
    if (!s || !host_m || !host_v || step < 0) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    int rc = hip_ok(hipMemcpy(s->Am, host_m, s->L.total * sizeof(float), hipMemcpyHostToDevice));
    if (!rc) rc = hip_ok(hipMemcpy(s->Av, host_v, s->L.total * sizeof(float), hipMemcpyHostToDevice));
    if (!rc) rc = hip_ok(hipDeviceSynchronize());
    if (!rc) s->step = step;
    return rc;
}

int fwi_score_forward(fwi_score_net* s, int B, const float* x, const float* tcond, const float* skip,
                      const float* scale, float* out, void* stream) {
    if (!s || B < 1 || B > s->max_batch || !x || !tcond || !out) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    return forward_impl(s, B, x, tcond, skip, scale, out, (hipStream_t)stream);
}

int fwi_score_backward(fwi_score_net* s, int B, const float* dout, float* dx, int want_weight_grads, void* stream) {
    if (!s || B < 1 || !dout || (want_weight_grads != 0 && want_weight_grads != 1)) return FWI_EINVAL;
    if (B != s->cachedB) return FWI_ESTATE;
    if (!dx && !want_weight_grads) return FWI_OK;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    return backward_impl(s, B, dout, dx, want_weight_grads != 0, (hipStream_t)stream);
}

int fwi_score_train_step(fwi_score_net* s, int B, const float* x0, const float* noise, const float* tcond,
                         const float* sqrt_abar, const float* sqrt_1m_abar, const fwi_score_train_params* tp,
                         float* loss_out, void* stream) {
    if (!s || B < 1 || B > s->max_batch || !x0 || !noise || !tcond || !sqrt_abar || !sqrt_1m_abar || !tp)
        return FWI_EINVAL;
    if (!(tp->lr > 0.f) || !(tp->beta1 >= 0.f && tp->beta1 < 1.f) || !(tp->beta2 >= 0.f && tp->beta2 < 1.f) ||
        !(tp->eps > 0.f))
        return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    hipStream_t st = (hipStream_t)stream;
    const long n = (long)B * NZ * NZ;
    hipLaunchKernelGGL(k_noise_state, dim3(grid_for(n)), dim3(TPB), 0, st, B, x0, noise, sqrt_abar, sqrt_1m_abar,
                       s->xt);
    int rc = forward_impl(s, B, s->xt, tcond, nullptr, nullptr, s->pred, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_dsm_loss, dim3(kNParts), dim3(TPB), 0, st, n, s->pred, noise, s->dpred, s->part);
    hipLaunchKernelGGL(k_dsm_loss_final, dim3(1), dim3(64), 0, st, s->part, kNParts, n,
                       loss_out ? loss_out : s->lval);
    rc = backward_impl(s, B, s->dpred, nullptr, true, st);
    if (rc) return rc;
    ++s->step;
    nn::adam(s->L.total, s->P, s->G, s->Am, s->Av, tp->lr, tp->beta1, tp->beta2, tp->eps, s->step, s->bf_index, s->W,
             st);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

}  // extern "C"
