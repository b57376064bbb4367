// Shapes of the trace surrogate and launchers of its non-GEMM kernels.
//
// Network (v -> traces of 5 surface shots x 70 receivers x 1000 samples):
//   lift      h = W_l^T [(v - 3000)/1500, z/72, x/72] + b_l on a 72 x 72 grid (the
//             70 x 70 model edge-extended), 64 channels
//   encoder   4 x { a = dw3x3(h); h = h + W2^T gelu(W1^T a + b1) + b2 }
//   depth->time  y[t] = sum_z T[t, z] h[z]  (256 time rows)
//   decoder   4 x { g = g + Xm g (mixing along x); a = dw3x3(g); g = g + W2^T gelu(W1^T a + b1) + b2 }
//   head      o = W_p^T g + b_p (8 channels, 5 used)
//   time      out[u] = sum_t U[u, t] o[t] (1000 samples); traces = out_scale * out
#pragma once

#include "nn_internal.h"

namespace fwi {

constexpr int kZ = 72, kX = 72, kC = 64, kCH = 128, kT = 256, kS = 8;
constexpr int kNT = 1000, kNR = 70, kNS = 5, kNZ = 70, kNX = 70, kNBLK = 4;

// FP32 parameter vector layout (the order the C ABI documents).
struct SurLayout {
    long lift_w, lift_b;
    long enc_dw_k[kNBLK], enc_dw_b[kNBLK], enc_w1[kNBLK], enc_b1[kNBLK], enc_w2[kNBLK], enc_b2[kNBLK];
    long d2t;
    long dec_xm[kNBLK], dec_dw_k[kNBLK], dec_dw_b[kNBLK], dec_w1[kNBLK], dec_b1[kNBLK], dec_w2[kNBLK],
        dec_b2[kNBLK];
    long proj_w, proj_b, up, out_scale;
    long total;
};

inline SurLayout sur_layout() {
    SurLayout L{};
    long o = 0;
    auto take = [&](long n) {
        const long r = o;
        o += n;
        return r;
    };
    L.lift_w = take(3 * kC);
    L.lift_b = take(kC);
    for (int i = 0; i < kNBLK; ++i) {
        L.enc_dw_k[i] = take(kC * 9);
        L.enc_dw_b[i] = take(kC);
        L.enc_w1[i] = take(kC * kCH);
        L.enc_b1[i] = take(kCH);
        L.enc_w2[i] = take(kCH * kC);
        L.enc_b2[i] = take(kC);
    }
    L.d2t = take(kT * kZ);
    for (int i = 0; i < kNBLK; ++i) {
        L.dec_xm[i] = take(kX * kX);
        L.dec_dw_k[i] = take(kC * 9);
        L.dec_dw_b[i] = take(kC);
        L.dec_w1[i] = take(kC * kCH);
        L.dec_b1[i] = take(kCH);
        L.dec_w2[i] = take(kCH * kC);
        L.dec_b2[i] = take(kC);
    }
    L.proj_w = take(kC * kS);
    L.proj_b = take(kS);
    L.up = take(kNT * kT);
    L.out_scale = take(1);
    L.total = o;
    return L;
}

namespace nn {
void lift_fwd(int B, const float* v, const float* W, const float* b, bf16_t* h, hipStream_t st);
void lift_bwd(int B, const float* v, const float* dh, const float* W, float* dv, float* dW, float* db, float* part,
              hipStream_t st);
void dw_fwd(int B, int H, int W, const bf16_t* in, const float* k, const float* b, bf16_t* out, hipStream_t st);
void dw_bwd(int B, int H, int W, const bf16_t* in, const float* dout, const float* k, float* din, bf16_t* din16,
            float* dk, float* db, float* part, hipStream_t st);
void gelu_fwd(long n, const bf16_t* p, bf16_t* q, hipStream_t st);
void gelu_bwd(long n, const float* dq, const bf16_t* p, float* dp, bf16_t* dp16, hipStream_t st);
void add_bf16(long n, const bf16_t* a, const bf16_t* b, bf16_t* o, hipStream_t st);
void to_bf16(long n, const float* a, bf16_t* o, hipStream_t st);
void copy_f32(long n, const float* a, float* o, hipStream_t st);
void colsum(long rows, int cols, const float* a, float* out, float* part, hipStream_t st);
void out_fwd(int B, const float* out, const float* scale, float* tr, hipStream_t st);
// fused pointwise MLP (64 -> 128 GELU -> 64) over R rows: forward with residual,
// and the input VJP recomputing the pre-activation (FWI_EINVAL on NULL or
// misaligned operands).  mlp_prepare fills the device's GELU tables once
// (synchronous on st; FWI_ESTATE if st is capturing a graph at that point);
// both entry points call it.
// mixing along x, per slab s < S of [72][64]: g1 = R(g + R(Xm g)); VJP d32 += Xm^T d1, d16 = R(d32)
int mix_fwd(long S, const bf16_t* Xm, const bf16_t* g, bf16_t* g1, hipStream_t st);
int mix_vjp(long S, const bf16_t* Xm, const bf16_t* d1, float* d32, bf16_t* d16, hipStream_t st);
// decoder block input VJP of the depthwise convolution and the mixing along x in one pass, B samples of
// [kT][72][64]: d1 = d32 + dw^T(da); d32 = d1 + Xm^T R(d1); d16 = R(d32)
int dwmix_vjp(int B, const bf16_t* Xm, const float* dwk, const float* da, float* d32, bf16_t* d16, hipStream_t st);
int mlp_prepare(hipStream_t st);
int mlp_fwd(long R, const bf16_t* a, const bf16_t* W1, const float* b1, const bf16_t* W2, const float* b2,
            const bf16_t* res, bf16_t* h, hipStream_t st);
int mlp_vjp(long R, const bf16_t* dg, const bf16_t* a, const bf16_t* W1, const float* b1, const bf16_t* W2, float* da,
            hipStream_t st);
void out_bwd(int B, const float* dtr, const float* scale, bf16_t* dout, hipStream_t st);
void loss(int B, const float* pred, const float* tgt, float kw, float pair_w, float* dpred, float* loss_out, float* mx,
          float* part, hipStream_t st);
void adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, int step,
          const int* bf_index, bf16_t* pbf, hipStream_t st);
void refresh_bf16(long n, const float* p, const int* bf_index, bf16_t* pbf, hipStream_t st);
void mf_predict(long n, const float* ga, const float* sn, const float* sa, float* out, int B, const double* Ja,
                const double* Jn, const double* Jsa, double* Jout, hipStream_t st);
void judge(int B, int n, const float* ga, const float* gb, const double* Ja, const double* Jb, float* cosv, float* jerr,
           hipStream_t st);
}  // namespace nn

}  // namespace fwi
