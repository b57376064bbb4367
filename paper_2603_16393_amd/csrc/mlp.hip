// Fused pointwise MLP of the trace surrogate's encoder and decoder blocks
// (64 -> 128 GELU -> 64 per pixel) on gfx950 matrix cores.
//
//   forward  h  = R(res + R(R(gelu(p)) W2 + b2)),   p = R(a W1 + b1)
//   VJP      da = R(dq gelu'(p)) W1^T,              dq = dg W2^T
//
// R rounds to BF16.  The two-GEMM form of the same block writes p and
// R(gelu(p)) (128 channels each) to HBM and reads them back; here the 128-wide
// hidden tile of 16 rows lives in LDS only, so a row costs 3 x 128 bytes of
// HBM traffic forward (a, res in; h out) and 2 x 128 + 256 in the VJP (dg, a
// in; FP32 da out), which recomputes p from a instead of storing it.
//
// p is a BF16 value, so R(gelu(p)) and gelu'(p) are functions of 16 bits:
// both come from per-device tables of all 65536 entries, filled by the same
// device functions the GEMM epilogues evaluate (gelu_f, gelu_d).  An epilogue
// then costs one rounding and one gather per hidden value instead of an erf
// evaluation, which would otherwise bound these kernels by vector ALU work.
//
// Work split: a workgroup (16 waves forward, 12 in the VJP, one per CU)
// stages the weights and tables in LDS once; its waves then take 16-row slabs
// in a grid-stride loop, each on its own part of the LDS hidden tile and
// without workgroup barriers, loading the next slab's activations before
// computing the current one.
//
// Every product is formed transposed, D = W^T x^T, on v_mfma_f32_16x16x32_bf16
// with the weights as the A operand and the 16 activation rows as B: lane l
// supplies A[l % 16][8 (l / 16) + i] (8 consecutive K entries of one output
// channel) and B[8 (l / 16) + i][l % 16] (8 consecutive K entries of row
// l % 16) and receives D[4 (l / 16) + q][l % 16].  The output channel of MFMA
// row i in 16 x 16 block nb is chan(nb, i), chosen so that the 16 values a
// lane receives from four consecutive blocks are 16 consecutive channels of
// one row, which then move as 16-byte loads and stores.  K is summed in
// 32-wide steps in increasing order with the same lane split as the tiled
// GEMM, and the epilogues round at the same points, so both entry points give
// exactly the results of the two-GEMM path.
#include <mutex>

#include "nn_internal.h"
#include "nn_ops.h"

namespace fwi {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// indexed by the BF16 bit pattern of p: R(gelu(p)) and gelu'(p)
__device__ bf16_t gelu_q_tab[65536];
__device__ float gelu_d_tab[65536];

__global__ void k_gelu_tables() {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 65536) {
        const float p = bf2f((bf16_t)i);
        gelu_q_tab[i] = f2bf(gelu_f(p));
        gelu_d_tab[i] = gelu_d(p);
    }
}

// two FP32 values rounded to BF16 (round to nearest even), packed low | high << 16
__device__ inline uint32_t cvt2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t));
}
__device__ inline float lo_f(uint32_t w) { return bf2f((bf16_t)(w & 0xffff)); }
__device__ inline float hi_f(uint32_t w) { return bf2f((bf16_t)(w >> 16)); }

constexpr int kS64 = kC + 8;    // LDS row stride (halves) of an operand 64 deep
constexpr int kS128 = kCH + 8;  // of an operand 128 deep
constexpr int kSlab = 16;       // rows a wave owns per iteration
constexpr int kWavesFwd = 16;   // waves per workgroup: 114 KB of LDS, one workgroup per CU
constexpr int kWavesVjp = 12;   // 125 KB of LDS

// LDS copy of the tables for |p| in [2^-16, 16) (20 binades of 128 BF16 values
// per sign): almost every hidden value hits it, and an LDS gather costs a few
// cycles where a scattered global gather occupies the CU's address unit for
// about one cycle per lane.  Other p read the global table.
constexpr int kTabLo = 127 - 16, kTabHalf = 20 * 128, kTabN = 2 * kTabHalf;

// BF16 pattern held by LDS slot `slot`
__device__ inline uint32_t tab_pattern(int slot) {
    const int sgn = slot >= kTabHalf;
    return ((uint32_t)sgn << 15) | (uint32_t)(slot - sgn * kTabHalf + (kTabLo << 7));
}
// LDS slot of the BF16 pattern b; outside the range slot 0, and `out` is set
__device__ inline uint32_t tab_slot(uint32_t b, bool& out) {
    const uint32_t off = (b & 0x7fffu) - (uint32_t)(kTabLo << 7);
    const bool in = off < (uint32_t)kTabHalf;
    out |= !in;
    return in ? off + (b >> 15) * kTabHalf : 0u;
}
__device__ inline bool tab_in(uint32_t b) { return (b & 0x7fffu) - (uint32_t)(kTabLo << 7) < (uint32_t)kTabHalf; }

struct MlpArgs {
    long R;                    // rows
    const bf16_t* a;           // [R][64] block input of the pointwise layers
    const bf16_t *W1, *W2;     // W1 [64][128], W2 [128][64], row-major
    const float *b1, *b2;      // [128], [64]
    const bf16_t* res;         // forward: residual [R][64]
    bf16_t* h;                 // forward: output [R][64]
    const bf16_t* dg;          // VJP: gradient at the block output [R][64]
    float* da;                 // VJP: gradient at a [R][64]
};

__device__ inline int chan(int nb, int i) { return 64 * (nb >> 2) + 16 * (i >> 2) + 4 * (nb & 3) + (i & 3); }

__device__ inline bf16x8_t frag(const bf16_t* p) { return *reinterpret_cast<const bf16x8_t*>(p); }

__device__ inline f32x4_t mma(bf16x8_t w, bf16x8_t x, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x, c, 0, 0, 0);
}

// W [K][N] row-major -> Wt[n][k] (LDS row stride `ld`): 16-byte loads of 8
// consecutive n, scattered 2-byte LDS stores
__device__ inline void stage_transposed(const bf16_t* __restrict__ W, int K, int N, bf16_t* Wt, int ld) {
    const int per = N / 8;
    for (int e = threadIdx.x; e < K * per; e += blockDim.x) {
        const int k = e / per, n8 = (e - k * per) * 8;
        const uint4 u = *reinterpret_cast<const uint4*>(W + (long)k * N + n8);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Wt[(n8 + 2 * i) * ld + k] = (bf16_t)(w[i] & 0xffff);
            Wt[(n8 + 2 * i + 1) * ld + k] = (bf16_t)(w[i] >> 16);
        }
    }
}

// W [N][K] row-major -> Ws[n][k] (LDS row stride `ld`), 16-byte pieces
__device__ inline void stage_rows(const bf16_t* __restrict__ W, int N, int K, bf16_t* Ws, int ld) {
    const int per = K / 8;
    for (int e = threadIdx.x; e < N * per; e += blockDim.x) {
        const int n = e / per, k8 = (e - n * per) * 8;
        *reinterpret_cast<uint4*>(Ws + n * ld + k8) = *reinterpret_cast<const uint4*>(W + (long)n * K + k8);
    }
}

// the lane's two K = 64 fragments of row `row` of a [R][64] matrix (zero past R)
__device__ inline void load_row(const bf16_t* __restrict__ base, long row, long R, int g, bf16x8_t (&x)[2]) {
    if (row < R) {
        x[0] = frag(base + row * kC + 8 * g);
        x[1] = frag(base + row * kC + 32 + 8 * g);
    } else {
        x[0] = bf16x8_t{};
        x[1] = bf16x8_t{};
    }
}

// Orders one wave's LDS accesses to its own hidden tile: lanes read what other
// lanes of the same wave wrote, and a wave's LDS operations execute in order,
// so a wavefront-scope release/acquire (which keeps the compiler from moving
// memory accesses across it) is all that is needed; the waves of the
// workgroup stay independent.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void unpack16(const uint4 (&u)[2], float (&o)[16]) {
    const uint32_t w[8] = {u[0].x, u[0].y, u[0].z, u[0].w, u[1].x, u[1].y, u[1].z, u[1].w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        o[2 * e] = bf2f((bf16_t)(w[e] & 0xffff));
        o[2 * e + 1] = bf2f((bf16_t)(w[e] >> 16));
    }
}

__global__ __launch_bounds__(64 * kWavesFwd) void k_mlp_fwd(MlpArgs p) {
    constexpr int kWaves = kWavesFwd;
    __shared__ __attribute__((aligned(16))) bf16_t W1t[kCH * kS64];        // [n][k] = W1[k][n]
    __shared__ __attribute__((aligned(16))) bf16_t W2t[kC * kS128];        // [n][k] = W2[k][n]
    __shared__ __attribute__((aligned(16))) bf16_t Q[kWaves * kSlab * kS128];  // R(gelu(p)) per wave
    __shared__ bf16_t tq[kTabN];
    __shared__ __attribute__((aligned(16))) float bs[kCH + kC];  // b1, b2
    // a lane's output channels are 16 g + j (and 64 + 16 g + j of the hidden layer)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, m = lane & 15, g = lane >> 4;
    const long nslab = (p.R + kSlab - 1) / kSlab, stride = (long)gridDim.x * kWaves;
    long s = (long)blockIdx.x * kWaves + wave;
    bf16x8_t x[2];
    uint4 r[2] = {};
    auto fetch = [&](long slab) {
        const long row = slab * kSlab + m;
        load_row(p.a, row, p.R, g, x);
        if (row < p.R) {
            r[0] = *reinterpret_cast<const uint4*>(p.res + row * kC + 16 * g);
            r[1] = *reinterpret_cast<const uint4*>(p.res + row * kC + 16 * g + 8);
        }
    };
    fetch(s);  // the first slab's loads overlap the staging
    stage_transposed(p.W1, kC, kCH, W1t, kS64);
    stage_transposed(p.W2, kCH, kC, W2t, kS128);
    for (int i = threadIdx.x; i < kTabN; i += blockDim.x) tq[i] = gelu_q_tab[tab_pattern(i)];
    for (int i = threadIdx.x; i < kCH + kC; i += blockDim.x) bs[i] = i < kCH ? p.b1[i] : p.b2[i - kCH];
    __syncthreads();
    bf16_t* q = Q + (wave * kSlab + m) * kS128;  // the hidden row this lane reads and writes
    for (; s < nslab; s += stride) {
        const long row = s * kSlab + m;
        const bf16x8_t xc[2] = {x[0], x[1]};
        const uint4 rc[2] = {r[0], r[1]};
        fetch(s + stride);

        // hidden channels in two halves of 64 (blocks 4 hh .. 4 hh + 3)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            f32x4_t acc[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[b] = mma(frag(&W1t[chan(4 * hh + b, m) * kS64 + 32 * ks + 8 * g]), xc[ks], acc[b]);
            float bb[16];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                *reinterpret_cast<float4*>(bb + 4 * i) = *reinterpret_cast<const float4*>(bs + 64 * hh + 16 * g + 4 * i);
            uint32_t pv[8], w[8];
            bool out = false;
#pragma unroll
            for (int j = 0; j < 16; j += 2) {
                const f32x4_t& c = acc[j / 4];
                pv[j / 2] = cvt2(c[j % 4] + bb[j], c[j % 4 + 1] + bb[j + 1]);
                w[j / 2] = (uint32_t)tq[tab_slot(pv[j / 2] & 0xffff, out)] |
                           ((uint32_t)tq[tab_slot(pv[j / 2] >> 16, out)] << 16);
            }
            if (out) {  // rare: a pre-activation outside the LDS table's range
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t lo = pv[i] & 0xffff, hi = pv[i] >> 16;
                    if (!tab_in(lo)) w[i] = (w[i] & 0xffff0000u) | gelu_q_tab[lo];
                    if (!tab_in(hi)) w[i] = (w[i] & 0xffffu) | ((uint32_t)gelu_q_tab[hi] << 16);
                }
            }
            *reinterpret_cast<uint4*>(q + 64 * hh + 16 * g) = make_uint4(w[0], w[1], w[2], w[3]);
            *reinterpret_cast<uint4*>(q + 64 * hh + 16 * g + 8) = make_uint4(w[4], w[5], w[6], w[7]);
        }
        wave_sync();

        f32x4_t acc2[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc2[nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8_t xq = frag(q + 32 * ks + 8 * g);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc2[nb] = mma(frag(&W2t[chan(nb, m) * kS128 + 32 * ks + 8 * g]), xq, acc2[nb]);
        }
        if (row < p.R) {
            float res[16], bb[16];
            unpack16(rc, res);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                *reinterpret_cast<float4*>(bb + 4 * i) = *reinterpret_cast<const float4*>(bs + kCH + 16 * g + 4 * i);
            uint32_t w[8];
#pragma unroll
            for (int j = 0; j < 16; j += 2) {
                const f32x4_t& c = acc2[j / 4];
                const uint32_t y = cvt2(c[j % 4] + bb[j], c[j % 4 + 1] + bb[j + 1]);
                w[j / 2] = cvt2(res[j] + lo_f(y), res[j + 1] + hi_f(y));
            }
            *reinterpret_cast<uint4*>(p.h + row * kC + 16 * g) = make_uint4(w[0], w[1], w[2], w[3]);
            *reinterpret_cast<uint4*>(p.h + row * kC + 16 * g + 8) = make_uint4(w[4], w[5], w[6], w[7]);
        }
        wave_sync();  // the tile is rewritten in the next iteration
    }
}

__global__ __launch_bounds__(64 * kWavesVjp) void k_mlp_vjp(MlpArgs p) {
    constexpr int kWaves = kWavesVjp;
    __shared__ __attribute__((aligned(16))) bf16_t W2s[kCH * kS64];   // [n][k] = W2[n][k], n < 128, k < 64
    __shared__ __attribute__((aligned(16))) bf16_t W1t[kCH * kS64];   // [n][k] = W1[k][n]
    __shared__ __attribute__((aligned(16))) bf16_t W1s[kC * kS128];   // [n][k] = W1[n][k], n < 64, k < 128
    __shared__ __attribute__((aligned(16))) bf16_t Q[kWaves * kSlab * kS128];  // R(dq gelu'(p)) per wave
    __shared__ float td[kTabN];
    __shared__ __attribute__((aligned(16))) float bs[kCH];  // b1
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, m = lane & 15, g = lane >> 4;
    const long nslab = (p.R + kSlab - 1) / kSlab, stride = (long)gridDim.x * kWaves;
    long s = (long)blockIdx.x * kWaves + wave;
    bf16x8_t y[2], x[2];
    auto fetch = [&](long slab) {
        const long row = slab * kSlab + m;
        load_row(p.dg, row, p.R, g, y);
        load_row(p.a, row, p.R, g, x);
    };
    fetch(s);  // the first slab's loads overlap the staging
    stage_rows(p.W2, kCH, kC, W2s, kS64);
    stage_transposed(p.W1, kC, kCH, W1t, kS64);
    stage_rows(p.W1, kC, kCH, W1s, kS128);
    for (int i = threadIdx.x; i < kTabN; i += blockDim.x) td[i] = gelu_d_tab[tab_pattern(i)];
    for (int i = threadIdx.x; i < kCH; i += blockDim.x) bs[i] = p.b1[i];
    __syncthreads();
    bf16_t* q = Q + (wave * kSlab + m) * kS128;
    for (; s < nslab; s += stride) {
        const long row = s * kSlab + m;
        const bf16x8_t yc[2] = {y[0], y[1]}, xc[2] = {x[0], x[1]};
        fetch(s + stride);

        // hidden channels in two halves of 64 (blocks 4 hh .. 4 hh + 3)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            f32x4_t dq[4], pp[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) dq[b] = pp[b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int off = chan(4 * hh + b, m) * kS64 + 32 * ks + 8 * g;
                    dq[b] = mma(frag(&W2s[off]), yc[ks], dq[b]);
                    pp[b] = mma(frag(&W1t[off]), xc[ks], pp[b]);
                }
            float bb[16];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                *reinterpret_cast<float4*>(bb + 4 * i) = *reinterpret_cast<const float4*>(bs + 64 * hh + 16 * g + 4 * i);
            uint32_t w[8];
            float d[16];
            bool out = false;
#pragma unroll
            for (int j = 0; j < 16; j += 2) {
                const f32x4_t& cp = pp[j / 4];
                const uint32_t pv = cvt2(cp[j % 4] + bb[j], cp[j % 4 + 1] + bb[j + 1]);
                w[j / 2] = pv;
                d[j] = td[tab_slot(pv & 0xffff, out)];
                d[j + 1] = td[tab_slot(pv >> 16, out)];
            }
            if (out) {  // rare: a pre-activation outside the LDS table's range
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const uint32_t b = j % 2 ? w[j / 2] >> 16 : w[j / 2] & 0xffff;
                    if (!tab_in(b)) d[j] = gelu_d_tab[b];
                }
            }
#pragma unroll
            for (int j = 0; j < 16; j += 2) {
                const f32x4_t& cq = dq[j / 4];
                w[j / 2] = cvt2(cq[j % 4] * d[j], cq[j % 4 + 1] * d[j + 1]);
            }
            *reinterpret_cast<uint4*>(q + 64 * hh + 16 * g) = make_uint4(w[0], w[1], w[2], w[3]);
            *reinterpret_cast<uint4*>(q + 64 * hh + 16 * g + 8) = make_uint4(w[4], w[5], w[6], w[7]);
        }
        wave_sync();

        f32x4_t acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8_t xq = frag(q + 32 * ks + 8 * g);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[nb] = mma(frag(&W1s[chan(nb, m) * kS128 + 32 * ks + 8 * g]), xq, acc[nb]);
        }
        if (row < p.R) {
            float* o = p.da + row * kC + 16 * g;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                *reinterpret_cast<float4*>(o + 4 * nb) = make_float4(acc[nb][0], acc[nb][1], acc[nb][2], acc[nb][3]);
        }
        wave_sync();  // the tile is rewritten in the next iteration
    }
}

// workgroups that fit on the device at once (at most one per `waves` slabs)
int mlp_grid(const void* kernel, int waves, long R) {
    static int cached[2][64] = {};
    const int which = kernel == (const void*)k_mlp_fwd ? 0 : 1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
    if (!cached[which][dev]) {
        int cu = 0, per = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 64 * waves, 0) != hipSuccess || cu < 1 ||
            per < 1)
            return -1;
        cached[which][dev] = cu * per;
    }
    const long need = (R + (long)kSlab * waves - 1) / ((long)kSlab * waves);
    return (int)std::min<long>(need, cached[which][dev]);
}

bool al16(const void* p) { return ((uintptr_t)p % 16) == 0; }

std::mutex g_tab_mu;
bool g_tab_built[64] = {};

}  // namespace

namespace nn {

int mlp_prepare(hipStream_t st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return FWI_EHIP;
    std::lock_guard<std::mutex> lock(g_tab_mu);
    if (g_tab_built[dev]) return FWI_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return FWI_EHIP;
    if (cs != hipStreamCaptureStatusNone) return FWI_ESTATE;
    hipLaunchKernelGGL(k_gelu_tables, dim3(256), dim3(256), 0, st);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return FWI_EHIP;
    g_tab_built[dev] = true;
    return FWI_OK;
}

int mlp_fwd(long R, const bf16_t* a, const bf16_t* W1, const float* b1, const bf16_t* W2, const float* b2,
            const bf16_t* res, bf16_t* h, hipStream_t st) {
    if (R < 0) return FWI_EINVAL;
    if (R == 0) return FWI_OK;
    if (!a || !W1 || !b1 || !W2 || !b2 || !res || !h) return FWI_EINVAL;
    if (!al16(a) || !al16(W1) || !al16(W2) || !al16(res) || !al16(h)) return FWI_EINVAL;
    const int rc = mlp_prepare(st);
    if (rc != FWI_OK) return rc;
    const int grid = mlp_grid((const void*)k_mlp_fwd, kWavesFwd, R);
    if (grid < 1) return FWI_EHIP;
    MlpArgs p{};
    p.R = R, p.a = a, p.W1 = W1, p.W2 = W2, p.b1 = b1, p.b2 = b2, p.res = res, p.h = h;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(grid), dim3(64 * kWavesFwd), 0, st, p);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

int mlp_vjp(long R, const bf16_t* dg, const bf16_t* a, const bf16_t* W1, const float* b1, const bf16_t* W2, float* da,
            hipStream_t st) {
    if (R < 0) return FWI_EINVAL;
    if (R == 0) return FWI_OK;
    if (!dg || !a || !W1 || !b1 || !W2 || !da) return FWI_EINVAL;
    if (!al16(dg) || !al16(a) || !al16(W1) || !al16(W2) || !al16(da)) return FWI_EINVAL;
    const int rc = mlp_prepare(st);
    if (rc != FWI_OK) return rc;
    const int grid = mlp_grid((const void*)k_mlp_vjp, kWavesVjp, R);
    if (grid < 1) return FWI_EHIP;
    MlpArgs p{};
    p.R = R, p.a = a, p.W1 = W1, p.W2 = W2, p.b1 = b1, p.dg = dg, p.da = da;
    hipLaunchKernelGGL(k_mlp_vjp, dim3(grid), dim3(64 * kWavesVjp), 0, st, p);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

}  // namespace nn
}  // namespace fwi

using namespace fwi;

extern "C" {

int fwi_nn_mlp_forward(long R, const void* a, const void* W1, const float* b1, const void* W2, const float* b2,
                       const void* res, void* h, void* stream) {
    return nn::mlp_fwd(R, (const bf16_t*)a, (const bf16_t*)W1, b1, (const bf16_t*)W2, b2, (const bf16_t*)res,
                       (bf16_t*)h, (hipStream_t)stream);
}

int fwi_nn_mlp_vjp(long R, const void* dg, const void* a, const void* W1, const float* b1, const void* W2, float* da,
                   void* stream) {
    return nn::mlp_vjp(R, (const bf16_t*)dg, (const bf16_t*)a, (const bf16_t*)W1, b1, (const bf16_t*)W2, da,
                       (hipStream_t)stream);
}

}  // extern "C"
