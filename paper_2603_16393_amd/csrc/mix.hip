// Mixing along x of the trace surrogate's decoder blocks on gfx950 matrix
// cores: for every (sample, time row) slab g [72 x][64 channels] (BF16),
//   forward  g1 = R(g + R(Xm g))                  Xm [72][72]
//   VJP      d32 <- d32 + Xm^T d1,  d16 = R(d32)  (d1 the BF16 copy of the incoming gradient)
// with R rounding to BF16.  Each is a 72 x 72 by 72 x 64 product per slab,
// thousands of slabs per call; as a tiled GEMM the 72 rows take two 64-row
// tiles (the second with 8 live rows) and every block covers three K steps,
// so block overhead dominates.  Here a wave owns a slab: it transposes the
// slab into its own LDS tile (the product needs 8 consecutive x' per channel
// as an MFMA operand, and channels are contiguous in memory), prefetches the
// next slab, and runs 5 x 4 blocks of v_mfma_f32_16x16x32_bf16 over three
// 32-wide K steps (zero beyond x' = 72), with Xm (or Xm^T) staged once per
// workgroup.  Operand layout, K split and rounding points are those of the
// tiled GEMM with its residual and dual-output epilogues, so results are
// bitwise the same.
//
// MFMA 16x16x32 operands (wave64): lane l supplies A[l % 16][8 (l / 16) + i]
// and B[8 (l / 16) + i][l % 16], i = 0..7, and receives D[4 (l / 16) + q][l % 16].
#include "nn_internal.h"
#include "nn_ops.h"

namespace fwi {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMixWaves = 4;
constexpr int kKP = 104;        // LDS row stride (halves): K padded to 96 plus 8
constexpr int kMR = 80;         // A rows: 72 padded to five 16-row blocks
constexpr int kChunks = kX * kC / 8;  // 16-byte pieces of a slab (576)
constexpr int kPer = kChunks / 64;    // per lane (9)
static_assert(kChunks % 64 == 0, "slab pieces must split evenly over a wave");

__device__ inline bf16x8_t frag(const bf16_t* p) { return *reinterpret_cast<const bf16x8_t*>(p); }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct MixArgs {
    long S;               // slabs
    const bf16_t* Xm;     // [72][72]
    const bf16_t* in;     // [S][72][64]: g (forward) or d1 (VJP)
    bf16_t* out16;        // [S][72][64]: g1 (forward) or R(d32) (VJP)
    float* io32;          // VJP: [S][72][64] FP32 accumulated in place
};

template <bool VJP>
__global__ __launch_bounds__(64 * kMixWaves) void k_mix(MixArgs p) {
    __shared__ __attribute__((aligned(16))) bf16_t Xs[kMR * kKP];               // A: Xm (or Xm^T), zero padded
    __shared__ __attribute__((aligned(16))) bf16_t Ts[kMixWaves * kC * kKP];    // per wave: slab^T [c][x']
    for (int e = threadIdx.x; e < kMR * kKP; e += blockDim.x) {
        const int m = e / kKP, k = e - m * kKP;
        bf16_t v = 0;
        if (m < kX && k < kX) v = VJP ? p.Xm[k * kX + m] : p.Xm[m * kX + k];
        Xs[e] = v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    bf16_t* T = Ts + wave * kC * kKP;
    for (int e = lane; e < kC * (kKP - kX); e += 64) {  // K padding of the slab tile, never overwritten
        const int c = e / (kKP - kX), k = kX + e - c * (kKP - kX);
        T[c * kKP + k] = 0;
    }
    __syncthreads();

    const long stride = (long)gridDim.x * kMixWaves;
    long s = (long)blockIdx.x * kMixWaves + wave;
    uint4 buf[kPer];
    auto fetch = [&](long slab) {
        if (slab < p.S) {
            const uint4* src = reinterpret_cast<const uint4*>(p.in + slab * (kX * kC));
#pragma unroll
            for (int j = 0; j < kPer; ++j) buf[j] = src[lane + 64 * j];
        }
    };
    fetch(s);
    for (; s < p.S; s += stride) {
        wave_sync();  // the previous slab's reads of T are done
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int e = lane + 64 * j, x = e >> 3, c8 = (e & 7) * 8;
            const uint32_t w[4] = {buf[j].x, buf[j].y, buf[j].z, buf[j].w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                T[(c8 + 2 * i) * kKP + x] = (bf16_t)(w[i] & 0xffff);
                T[(c8 + 2 * i + 1) * kKP + x] = (bf16_t)(w[i] >> 16);
            }
        }
        fetch(s + stride);
        wave_sync();

        const long base = s * (kX * kC);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            bf16x8_t b[3];
#pragma unroll
            for (int ks = 0; ks < 3; ++ks) b[ks] = frag(T + (16 * nb + r) * kKP + 32 * ks + 8 * g);
            const int c = 16 * nb + r;
#pragma unroll
            for (int mb = 0; mb < 5; ++mb) {
                f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 3; ++ks)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(Xs + (16 * mb + r) * kKP + 32 * ks + 8 * g),
                                                                  b[ks], acc, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = 16 * mb + 4 * g + q;
                    if (m >= kX) continue;
                    const long o = base + m * kC + c;
                    if (VJP) {
                        const float v = acc[q] + p.io32[o];
                        p.io32[o] = v;
                        p.out16[o] = f2bf(v);
                    } else {
                        p.out16[o] = f2bf(bf2f(T[c * kKP + m]) + bf2f(f2bf(acc[q])));
                    }
                }
            }
        }
    }
}

// Input VJP of a decoder block's depthwise convolution followed by its mixing along x, for B samples of
// kT x kX slabs (the gradient never leaves the chip between the two):
//   d1  = d32 + dw^T(da)   (FP32; the depthwise transpose taps in the order of the separate kernel)
//   d32 = d1 + Xm^T R(d1),  d16 = R(d32)
// The product is formed transposed, D' = R(d1)^T Xm (the slab as the A operand, Xm^T as B), so that a lane
// receives 4 consecutive channels of one row: exactly the positions whose d1 it computed itself and holds in
// registers; only R(d1) goes through the wave's LDS tile.
struct DwMixArgs {
    int B;
    const bf16_t* Xm;   // [72][72]
    const float* dwk;   // depthwise kernel [64][3][3]
    const float* da;    // [B][kT][72][64] gradient at the depthwise output
    float* d32;         // [B][kT][72][64] in: gradient at the block output; out: at the block input
    bf16_t* d16;        // [B][kT][72][64] out: R(d32)
};

__global__ __launch_bounds__(64 * kMixWaves) void k_dwmix_vjp(DwMixArgs p) {
    __shared__ __attribute__((aligned(16))) bf16_t Xs[kMR * kKP];             // Xm^T, zero padded
    __shared__ __attribute__((aligned(16))) bf16_t Ts[kMixWaves * kC * kKP];  // per wave: R(d1)^T [c][x']
    __shared__ float ks[kC * 9];
    for (int e = threadIdx.x; e < kMR * kKP; e += blockDim.x) {
        const int m = e / kKP, k = e - m * kKP;
        Xs[e] = (m < kX && k < kX) ? p.Xm[k * kX + m] : (bf16_t)0;
    }
    for (int e = threadIdx.x; e < kC * 9; e += blockDim.x) ks[e] = p.dwk[e];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    bf16_t* T = Ts + wave * kC * kKP;
    for (int e = lane; e < kC * (kKP - kX); e += 64) {
        const int c = e / (kKP - kX), k = kX + e - c * (kKP - kX);
        T[c * kKP + k] = 0;
    }
    __syncthreads();

    const long S = (long)p.B * kT, stride = (long)gridDim.x * kMixWaves;
    for (long s = (long)blockIdx.x * kMixWaves + wave; s < S; s += stride) {
        const int t = (int)(s % kT);
        const long base = s * (kX * kC);
        float4 d1[5][4];
        wave_sync();  // the previous slab's reads of T are done
#pragma unroll
        for (int mb = 0; mb < 5; ++mb) {
            const int m = 16 * mb + r;
            if (m >= kX) continue;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int c0 = 16 * cb + 4 * g;
                float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const int tt = t - dy + 1;
                    if (tt < 0 || tt >= kT) continue;
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        const int xx = m - dx + 1;
                        if (xx < 0 || xx >= kX) continue;
                        const float4 d = *reinterpret_cast<const float4*>(
                            p.da + base + (long)(tt - t) * (kX * kC) + (long)xx * kC + c0);
                        const float dv[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[e] = fmaf(ks[(c0 + e) * 9 + dy * 3 + dx], dv[e], acc[e]);
                    }
                }
                const float4 o = *reinterpret_cast<const float4*>(p.d32 + base + (long)m * kC + c0);
                const float4 v = make_float4(o.x + acc[0], o.y + acc[1], o.z + acc[2], o.w + acc[3]);
                d1[mb][cb] = v;
                T[(c0 + 0) * kKP + m] = f2bf(v.x);
                T[(c0 + 1) * kKP + m] = f2bf(v.y);
                T[(c0 + 2) * kKP + m] = f2bf(v.z);
                T[(c0 + 3) * kKP + m] = f2bf(v.w);
            }
        }
        wave_sync();
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            bf16x8_t a[3];
#pragma unroll
            for (int ks3 = 0; ks3 < 3; ++ks3) a[ks3] = frag(T + (16 * cb + r) * kKP + 32 * ks3 + 8 * g);
            const int c0 = 16 * cb + 4 * g;
#pragma unroll
            for (int mb = 0; mb < 5; ++mb) {
                f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks3 = 0; ks3 < 3; ++ks3)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks3], frag(Xs + (16 * mb + r) * kKP + 32 * ks3 + 8 * g),
                                                                  acc, 0, 0, 0);
                const int m = 16 * mb + r;
                if (m >= kX) continue;
                const float4 o = d1[mb][cb];
                const float4 v = make_float4(acc[0] + o.x, acc[1] + o.y, acc[2] + o.z, acc[3] + o.w);
                *reinterpret_cast<float4*>(p.d32 + base + (long)m * kC + c0) = v;
                uint2 u;
                u.x = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
                u.y = (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16);
                *reinterpret_cast<uint2*>(p.d16 + base + (long)m * kC + c0) = u;
            }
        }
    }
}

int launch_mix(bool vjp, long S, const bf16_t* Xm, const bf16_t* in, bf16_t* out16, float* io32, hipStream_t st) {
    if (S <= 0) return FWI_OK;
    if (((uintptr_t)in % 16) != 0) return FWI_EINVAL;
    static int cached[2][64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return FWI_EHIP;
    const void* k = vjp ? (const void*)k_mix<true> : (const void*)k_mix<false>;
    if (!cached[vjp][dev]) {
        int cu = 0, per = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, 64 * kMixWaves, 0) != hipSuccess || cu < 1 ||
            per < 1)
            return FWI_EHIP;
        cached[vjp][dev] = cu * per;
    }
    const long need = (S + kMixWaves - 1) / kMixWaves;
    const int grid = (int)std::min<long>(need, cached[vjp][dev]);
    MixArgs a{S, Xm, in, out16, io32};
    if (vjp)
        hipLaunchKernelGGL(k_mix<true>, dim3(grid), dim3(64 * kMixWaves), 0, st, a);
    else
        hipLaunchKernelGGL(k_mix<false>, dim3(grid), dim3(64 * kMixWaves), 0, st, a);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

int launch_dwmix(const DwMixArgs& a, hipStream_t st) {
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return FWI_EHIP;
    if (!cached[dev]) {
        int cu = 0, per = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_dwmix_vjp, 64 * kMixWaves, 0) !=
                hipSuccess ||
            cu < 1 || per < 1)
            return FWI_EHIP;
        cached[dev] = cu * per;
    }
    const long S = (long)a.B * kT;
    const int grid = (int)std::min<long>((S + kMixWaves - 1) / kMixWaves, cached[dev]);
    hipLaunchKernelGGL(k_dwmix_vjp, dim3(grid), dim3(64 * kMixWaves), 0, st, a);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

}  // namespace

namespace nn {

int dwmix_vjp(int B, const bf16_t* Xm, const float* dwk, const float* da, float* d32, bf16_t* d16, hipStream_t st) {
    if (B < 0 || (B > 0 && (!Xm || !dwk || !da || !d32 || !d16))) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (((uintptr_t)da % 16) != 0 || ((uintptr_t)d32 % 16) != 0 || ((uintptr_t)d16 % 8) != 0) return FWI_EINVAL;
    return launch_dwmix(DwMixArgs{B, Xm, dwk, da, d32, d16}, st);
}

int mix_fwd(long S, const bf16_t* Xm, const bf16_t* g, bf16_t* g1, hipStream_t st) {
    if (S < 0 || (S > 0 && (!Xm || !g || !g1))) return FWI_EINVAL;
    return launch_mix(false, S, Xm, g, g1, nullptr, st);
}

int mix_vjp(long S, const bf16_t* Xm, const bf16_t* d1, float* d32, bf16_t* d16, hipStream_t st) {
    if (S < 0 || (S > 0 && (!Xm || !d1 || !d32 || !d16))) return FWI_EINVAL;
    return launch_mix(true, S, Xm, d1, d16, d32, st);
}

}  // namespace nn
}  // namespace fwi

using namespace fwi;

extern "C" {

int fwi_nn_mix_forward(long S, const void* Xm, const void* g, void* g1, void* stream) {
    return nn::mix_fwd(S, (const bf16_t*)Xm, (const bf16_t*)g, (bf16_t*)g1, (hipStream_t)stream);
}

int fwi_nn_mix_vjp(long S, const void* Xm, const void* d1, float* d32, void* d16, void* stream) {
    return nn::mix_vjp(S, (const bf16_t*)Xm, (const bf16_t*)d1, d32, (bf16_t*)d16, (hipStream_t)stream);
}

}  // extern "C"
