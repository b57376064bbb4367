// The learned trace surrogate: model object, forward (inference), backward
// (input gradient and weight gradients), and one Adam training step, all on
// the BF16 matrix-core GEMM of gemm.hip and the kernels of nn.hip.
//
// Storage: FP32 master parameters in one vector (layout of SurLayout), a BF16
// copy of every GEMM weight (W1, W2, Xm, T, W_p, U), BF16 NHWC activations
// kept for the backward pass, FP32 gradient streams with a BF16 copy wherever
// a gradient is a GEMM operand.  The order of the layers is that of the
// network description in nn_ops.h.
#include <cmath>
#include <cstring>
#include <new>
#include <utility>

#include "nn_internal.h"
#include "nn_ops.h"

namespace fwi {
namespace {

constexpr int kMaxSurBatch = 128;
constexpr long kWorkFloats = 4L << 20;   // split-K partials (16 MiB)
constexpr long kPartFloats = 512L * 10 * kC + 1024;

struct BfMap {  // offsets of the BF16 copies
    long enc_w1[kNBLK], enc_w2[kNBLK], dec_w1[kNBLK], dec_w2[kNBLK], dec_xm[kNBLK], d2t, proj_w, up, total;
};

}  // namespace
}  // namespace fwi

struct fwi_surrogate {
    int device = 0, max_batch = 0, step = 0;
    // fused: each pointwise MLP runs as one kernel (forward and input VJP), and
    // an input VJP also takes a decoder block's depthwise convolution and mixing
    // along x in one pass; the forward then keeps no hidden activations
    // (pq_valid false) and a weight gradient recomputes them
    bool fused = true, pq_valid = false;
    fwi::SurLayout L;
    fwi::BfMap M;
    std::vector<void*> allocs;
    float *P = nullptr, *G = nullptr, *Am = nullptr, *Av = nullptr;
    int* bf_index = nullptr;
    fwi::bf16_t* W = nullptr;
    // activations (BF16)
    fwi::bf16_t *hin[fwi::kNBLK + 1], *ae[fwi::kNBLK], *pe[fwi::kNBLK], *qe[fwi::kNBLK];
    fwi::bf16_t *gin[fwi::kNBLK + 1], *g1[fwi::kNBLK], *ad[fwi::kNBLK], *pd[fwi::kNBLK], *qd[fwi::kNBLK];
    fwi::bf16_t* o = nullptr;
    float *out32 = nullptr, *vcache = nullptr;
    int cachedB = 0;
    // gradient streams
    fwi::bf16_t *dout16 = nullptr, *do16 = nullptr, *dg16 = nullptr, *dg16b = nullptr, *dp16 = nullptr;
    float *do32 = nullptr, *dg32 = nullptr, *dp32 = nullptr, *da32 = nullptr;
    float *part = nullptr, *work = nullptr;
    // training
    float *pred = nullptr, *dtr = nullptr, *mx = nullptr, *lpart = nullptr, *lval = nullptr;
};

namespace fwi {
namespace {

BfMap bf_map() {
    BfMap m{};
    long o = 0;
    for (int i = 0; i < kNBLK; ++i) {
        m.enc_w1[i] = o, o += kC * kCH;
        m.enc_w2[i] = o, o += kCH * kC;
    }
    m.d2t = o, o += kT * kZ;
    for (int i = 0; i < kNBLK; ++i) {
        m.dec_xm[i] = o, o += kX * kX;
        m.dec_w1[i] = o, o += kC * kCH;
        m.dec_w2[i] = o, o += kCH * kC;
    }
    m.proj_w = o, o += kC * kS;
    m.up = o, o += kNT * kT;
    m.total = o;
    return m;
}

template <class T>
bool dalloc(fwi_surrogate* s, T** p, long n) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)std::max<long>(n, 1) * sizeof(T)) != hipSuccess) return false;
    s->allocs.push_back(q);
    *p = (T*)q;
    return true;
}

void free_all(fwi_surrogate* s) {
    for (void* p : s->allocs) hipFree(p);
    s->allocs.clear();
}

// split count for a reduction of `steps` K-steps onto `tiles` output tiles
int pick_splitk(int M, int N, long steps) {
    const long tiles = (long)((M + 63) / 64) * ((N + 63) / 64);
    long sk = (512 + tiles - 1) / tiles;
    sk = std::min<long>(sk, std::max<long>(1, steps / 8));
    sk = std::min<long>(sk, kWorkFloats / ((long)M * N));
    return (int)std::max<long>(1, std::min<long>(sk, 256));
}

struct Ctx {
    fwi_surrogate* s;
    hipStream_t st;
    int rc = FWI_OK;

    // C = op(A) op(B) (+ bias) per batch
    void mm(int M, int N, int K, int batch, const bf16_t* A, long lda, long sA, int tA, const bf16_t* B, long ldb,
            long sB, int tB, float* C32, bf16_t* C16, long ldc, long sC, const float* bias, float beta = 0.f,
            int epi = kEpiNone, bf16_t* aux16 = nullptr, const bf16_t* res16 = nullptr, const bf16_t* p16 = nullptr) {
        if (rc != FWI_OK) return;
        GemmArgs g;
        g.M = M, g.N = N, g.K = K, g.batch = batch;
        g.A = A, g.lda = lda, g.strideA = sA, g.transA = tA;
        g.B = B, g.ldb = ldb, g.strideB = sB, g.transB = tB;
        g.C32 = C32, g.C16 = C16, g.ldc = ldc, g.strideC = sC, g.beta = beta, g.bias = bias;
        g.epi = epi, g.aux16 = aux16, g.res16 = res16, g.p16 = p16;
        rc = gemm_bf16(g, st);
    }
    // weight gradient C = sum over batch (and rows) of op(A) op(B), split-K
    void wgrad(int M, int N, int K, int batch, const bf16_t* A, long lda, long sA, int tA, const bf16_t* B, long ldb,
               long sB, int tB, float* C32, long ldc) {
        if (rc != FWI_OK) return;
        GemmArgs g;
        g.M = M, g.N = N, g.K = K, g.batch = batch;
        g.A = A, g.lda = lda, g.strideA = sA, g.transA = tA;
        g.B = B, g.ldb = ldb, g.strideB = sB, g.transB = tB;
        g.C32 = C32, g.ldc = ldc;
        g.reduce_batch = batch > 1;
        g.splitk = pick_splitk(M, N, (long)batch * ((K + 31) / 32));
        g.work = s->work;
        rc = gemm_bf16(g, st);
    }
};

// pre-activation p = R(a W1 + b1) and q = R(gelu(p)) of one pointwise MLP
void mlp_hidden(Ctx& c, int rows, const bf16_t* a, const bf16_t* W1, const float* b1, bf16_t* p, bf16_t* q) {
    c.mm(rows, kCH, kC, 1, a, kC, 0, 0, W1, kCH, 0, 0, nullptr, p, kCH, 0, b1, 0.f, kEpiGelu, q);
}

// h = R(res + R(q W2 + b2)) for one pointwise MLP of the forward, fused or as two GEMMs
void mlp_forward(Ctx& c, bool fused, int rows, const bf16_t* a, const bf16_t* W1, const float* b1, const bf16_t* W2,
                 const float* b2, const bf16_t* res, bf16_t* h, bf16_t* p, bf16_t* q) {
    if (c.rc != FWI_OK) return;
    if (fused) {
        c.rc = nn::mlp_fwd(rows, a, W1, b1, W2, b2, res, h, c.st);
        return;
    }
    mlp_hidden(c, rows, a, W1, b1, p, q);
    c.mm(rows, kC, kCH, 1, q, kCH, 0, 0, W2, kC, 0, 0, nullptr, h, kC, 0, b2, 0.f, kEpiResid, nullptr, res);
}

// ---------------------------------------------------------------------------
int forward_impl(fwi_surrogate* s, int B, const float* v, float* traces, hipStream_t st) {
    Ctx c{s, st};
    const SurLayout& L = s->L;
    const BfMap& M = s->M;
    const float* P = s->P;
    const bf16_t* W = s->W;
    const int re = B * kZ * kX, rd = B * kT * kX;
    nn::copy_f32((long)B * kNZ * kNX, v, s->vcache, st);
    nn::lift_fwd(B, v, P + L.lift_w, P + L.lift_b, s->hin[0], st);
    const bool fused = s->fused;
    for (int i = 0; i < kNBLK; ++i) {
        nn::dw_fwd(B, kZ, kX, s->hin[i], P + L.enc_dw_k[i], P + L.enc_dw_b[i], s->ae[i], st);
        // h_next = R(h + R(R(gelu(R(a W1 + b1))) W2 + b2))
        mlp_forward(c, fused, re, s->ae[i], W + M.enc_w1[i], P + L.enc_b1[i], W + M.enc_w2[i], P + L.enc_b2[i],
                    s->hin[i], s->hin[i + 1], s->pe[i], s->qe[i]);
    }
    // depth -> time: per sample [T][X C] = T[T][Z] h[Z][X C]
    const long xc = (long)kX * kC;
    c.mm(kT, (int)xc, kZ, B, W + M.d2t, kZ, 0, 0, s->hin[kNBLK], xc, kZ * xc, 0, nullptr, s->gin[0], xc, kT * xc,
         nullptr);
    for (int i = 0; i < kNBLK; ++i) {
        // mixing along x: per (sample, t) [X][C] = Xm[X][X] g[X][C]
        // g1 = R(g + R(Xm g))
        if (c.rc == FWI_OK) c.rc = nn::mix_fwd((long)B * kT, W + M.dec_xm[i], s->gin[i], s->g1[i], st);
        nn::dw_fwd(B, kT, kX, s->g1[i], P + L.dec_dw_k[i], P + L.dec_dw_b[i], s->ad[i], st);
        mlp_forward(c, fused, rd, s->ad[i], W + M.dec_w1[i], P + L.dec_b1[i], W + M.dec_w2[i], P + L.dec_b2[i],
                    s->g1[i], s->gin[i + 1], s->pd[i], s->qd[i]);
    }
    c.mm(rd, kS, kC, 1, s->gin[kNBLK], kC, 0, 0, W + M.proj_w, kS, 0, 0, nullptr, s->o, kS, 0, P + L.proj_b);
    // time up-sampling: per sample [NT][X S] = U[NT][T] o[T][X S] (FP32 out)
    const long xs = (long)kX * kS;
    c.mm(kNT, (int)xs, kT, B, W + M.up, kT, 0, 0, s->o, xs, kT * xs, 0, s->out32, nullptr, xs, kNT * xs, nullptr);
    if (c.rc != FWI_OK) return c.rc;
    nn::out_fwd(B, s->out32, P + L.out_scale, traces, st);
    s->cachedB = B;
    s->pq_valid = !fused;
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

// Through one pointwise MLP: s->da32 = dL/da from dL/dh (s->dg16, BF16, and
// dg32, FP32, the latter read only for the bias gradient), and with want_w
// the gradients of W1, b1, W2, b2.  The input VJP alone runs fused; the
// weight gradients take the GEMM path and need p and q, which are recomputed
// when the forward did not keep them.
void mlp_backward(Ctx& c, int want_w, int rows, const bf16_t* a, bf16_t* p, bf16_t* q, const bf16_t* W1,
                  const float* b1, const bf16_t* W2, float* gW1, float* gb1, float* gW2, float* gb2,
                  const float* dg32) {
    fwi_surrogate* s = c.s;
    if (c.rc != FWI_OK) return;
    if (!want_w && (s->fused || !s->pq_valid)) {
        c.rc = nn::mlp_vjp(rows, s->dg16, a, W1, b1, W2, s->da32, c.st);
        return;
    }
    if (!s->pq_valid) mlp_hidden(c, rows, a, W1, b1, p, q);
    if (want_w) {
        c.wgrad(kCH, kC, rows, 1, q, kCH, 0, 1, s->dg16, kC, 0, 0, gW2, kC);
        nn::colsum(rows, kC, dg32, gb2, s->part, c.st);
    }
    // dp = (dg W2^T) gelu'(p), FP32 and BF16, from one GEMM epilogue
    c.mm(rows, kCH, kC, 1, s->dg16, kC, 0, 0, W2, kC, 0, 1, s->dp32, nullptr, kCH, 0, nullptr, 0.f, kEpiGeluBwd,
         s->dp16, nullptr, p);
    if (want_w) {
        c.wgrad(kC, kCH, rows, 1, a, kC, 0, 1, s->dp16, kCH, 0, 0, gW1, kCH);
        nn::colsum(rows, kCH, s->dp32, gb1, s->part, c.st);
    }
    c.mm(rows, kC, kCH, 1, s->dp16, kCH, 0, 0, W1, kCH, 0, 1, s->da32, nullptr, kC, 0, nullptr);
}

// Chain rule through the last forward_impl (same B).  dv may be NULL; with
// want_w the weight gradients are written to s->G (every entry but out_scale).
int backward_impl(fwi_surrogate* s, int B, const float* dtr, float* dv, int want_w, hipStream_t st) {
    Ctx c{s, st};
    const SurLayout& L = s->L;
    const BfMap& M = s->M;
    const float* P = s->P;
    float* G = s->G;
    const bf16_t* W = s->W;
    const int re = B * kZ * kX, rd = B * kT * kX;
    const long xc = (long)kX * kC, xs = (long)kX * kS;

    nn::out_bwd(B, dtr, P + L.out_scale, s->dout16, st);
    if (want_w)  // dU = sum_n dout_n o_n^T
        c.wgrad(kNT, kT, (int)xs, B, s->dout16, xs, kNT * xs, 0, s->o, xs, kT * xs, 1, G + L.up, kT);
    // do_n = U^T dout_n
    c.mm(kT, (int)xs, kNT, B, W + M.up, kT, 0, 1, s->dout16, xs, kNT * xs, 0, s->do32, nullptr, xs, kT * xs, nullptr,
         0.f, kEpiDual, s->do16);
    if (want_w) {
        c.wgrad(kC, kS, rd, 1, s->gin[kNBLK], kC, 0, 1, s->do16, kS, 0, 0, G + L.proj_w, kS);
        nn::colsum(rd, kS, s->do32, G + L.proj_b, s->part, st);
    }
    c.mm(rd, kC, kS, 1, s->do16, kS, 0, 0, W + M.proj_w, kS, 0, 1, s->dg32, nullptr, kC, 0, nullptr, 0.f, kEpiDual,
         s->dg16);

    // every producer of dg32 also writes its BF16 copy dg16
    for (int i = kNBLK - 1; i >= 0; --i) {
        mlp_backward(c, want_w, rd, s->ad[i], s->pd[i], s->qd[i], W + M.dec_w1[i], P + L.dec_b1[i], W + M.dec_w2[i],
                     G + L.dec_w1[i], G + L.dec_b1[i], G + L.dec_w2[i], G + L.dec_b2[i], s->dg32);
        if (c.rc != FWI_OK) return c.rc;
        if (!want_w && s->fused) {
            // dg1 = dg + dw^T(da) and dg = dg1 + Xm^T R(dg1) in one pass (dg1 stays on the chip)
            c.rc = nn::dwmix_vjp(B, W + M.dec_xm[i], P + L.dec_dw_k[i], s->da32, s->dg32, s->dg16b, st);
            std::swap(s->dg16, s->dg16b);
            continue;
        }
        // dg1 = dg + dw^T(da)   (in place in dg32)
        nn::dw_bwd(B, kT, kX, s->g1[i], s->da32, P + L.dec_dw_k[i], s->dg32, s->dg16,
                   want_w ? G + L.dec_dw_k[i] : nullptr, G + L.dec_dw_b[i], s->part, st);
        if (want_w)  // dXm = sum_{n,t} dg1_{nt} g_{nt}^T
            c.wgrad(kX, kX, kC, B * kT, s->dg16, kC, xc, 0, s->gin[i], kC, xc, 1, G + L.dec_xm[i], kX);
        // dg = dg1 + Xm^T dg1
        // the x-mixing's transpose accumulates into dg32; it reads dg16 (dg1) as its B operand,
        // so its BF16 copy goes to the second buffer, which then becomes dg16
        if (c.rc == FWI_OK) c.rc = nn::mix_vjp((long)B * kT, W + M.dec_xm[i], s->dg16, s->dg32, s->dg16b, st);
        std::swap(s->dg16, s->dg16b);
    }
    if (want_w)  // dT = sum_n dy_n h_n^T
        c.wgrad(kT, kZ, (int)xc, B, s->dg16, xc, kT * xc, 0, s->hin[kNBLK], xc, kZ * xc, 1, G + L.d2t, kZ);
    // dh_n = T^T dy_n  (into dg32, whose FP32 contents are no longer needed)
    float* dh = s->dg32;
    c.mm(kZ, (int)xc, kT, B, W + M.d2t, kZ, 0, 1, s->dg16, xc, kT * xc, 0, dh, nullptr, xc, kZ * xc, nullptr, 0.f,
         kEpiDual, s->dg16b);
    std::swap(s->dg16, s->dg16b);

    for (int i = kNBLK - 1; i >= 0; --i) {
        mlp_backward(c, want_w, re, s->ae[i], s->pe[i], s->qe[i], W + M.enc_w1[i], P + L.enc_b1[i], W + M.enc_w2[i],
                     G + L.enc_w1[i], G + L.enc_b1[i], G + L.enc_w2[i], G + L.enc_b2[i], dh);
        if (c.rc != FWI_OK) return c.rc;
        nn::dw_bwd(B, kZ, kX, s->hin[i], s->da32, P + L.enc_dw_k[i], dh, s->dg16,
                   want_w ? G + L.enc_dw_k[i] : nullptr, G + L.enc_dw_b[i], s->part, st);
    }
    nn::lift_bwd(B, s->vcache, dh, P + L.lift_w, dv, want_w ? G + L.lift_w : nullptr, G + L.lift_b, s->part, st);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

int build_bf_index(fwi_surrogate* s) {
    const SurLayout& L = s->L;
    const BfMap& M = s->M;
    std::vector<int> idx((size_t)L.total, -1);
    auto map = [&](long p, long b, long n) {
        for (long i = 0; i < n; ++i) idx[(size_t)(p + i)] = (int)(b + i);
    };
    for (int i = 0; i < kNBLK; ++i) {
        map(L.enc_w1[i], M.enc_w1[i], kC * kCH);
        map(L.enc_w2[i], M.enc_w2[i], kCH * kC);
        map(L.dec_w1[i], M.dec_w1[i], kC * kCH);
        map(L.dec_w2[i], M.dec_w2[i], kCH * kC);
        map(L.dec_xm[i], M.dec_xm[i], kX * kX);
    }
    map(L.d2t, M.d2t, kT * kZ);
    map(L.proj_w, M.proj_w, kC * kS);
    map(L.up, M.up, kNT * kT);
    return hipMemcpy(s->bf_index, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess
               ? FWI_OK
               : FWI_EHIP;
}

bool create_buffers(fwi_surrogate* s) {
    const long Bm = s->max_batch;
    const long pe = Bm * kZ * kX, pd = Bm * kT * kX;
    const long T = s->L.total;
    bool ok = dalloc(s, &s->P, T) && dalloc(s, &s->G, T) && dalloc(s, &s->Am, T) && dalloc(s, &s->Av, T) &&
              dalloc(s, &s->bf_index, T) && dalloc(s, &s->W, s->M.total);
    for (int i = 0; i <= kNBLK && ok; ++i) ok = dalloc(s, &s->hin[i], pe * kC) && dalloc(s, &s->gin[i], pd * kC);
    for (int i = 0; i < kNBLK && ok; ++i)
        ok = dalloc(s, &s->ae[i], pe * kC) && dalloc(s, &s->pe[i], pe * kCH) && dalloc(s, &s->qe[i], pe * kCH) &&
             dalloc(s, &s->g1[i], pd * kC) && dalloc(s, &s->ad[i], pd * kC) && dalloc(s, &s->pd[i], pd * kCH) &&
             dalloc(s, &s->qd[i], pd * kCH);
    const long ntr = Bm * kNS * kNR * kNT;
    ok = ok && dalloc(s, &s->o, pd * kS) && dalloc(s, &s->out32, Bm * kNT * kX * kS) &&
         dalloc(s, &s->vcache, Bm * kNZ * kNX) && dalloc(s, &s->dout16, Bm * kNT * kX * kS) &&
         dalloc(s, &s->do16, pd * kS) && dalloc(s, &s->do32, pd * kS) && dalloc(s, &s->dg16, pd * kC) &&
         dalloc(s, &s->dg32, pd * kC) && dalloc(s, &s->dg16b, pd * kC) && dalloc(s, &s->dp32, pd * kCH) &&
         dalloc(s, &s->dp16, pd * kCH) && dalloc(s, &s->da32, pd * kC) && dalloc(s, &s->part, kPartFloats) &&
         dalloc(s, &s->work, kWorkFloats) && dalloc(s, &s->pred, ntr) && dalloc(s, &s->dtr, ntr) &&
         dalloc(s, &s->mx, Bm) && dalloc(s, &s->lpart, 2048) && dalloc(s, &s->lval, 1);
    return ok;
}

}  // namespace
}  // namespace fwi

using namespace fwi;

extern "C" {

int fwi_sur_shape(int* dims) {
    if (!dims) return FWI_EINVAL;
    dims[0] = kNZ, dims[1] = kNX, dims[2] = kNS, dims[3] = kNR, dims[4] = kNT;
    return FWI_OK;
}

long fwi_sur_param_count(void) { return sur_layout().total; }

int fwi_sur_create(int max_batch, fwi_surrogate** out) {
    if (!out || max_batch < 1 || max_batch > kMaxSurBatch) return FWI_EINVAL;
    *out = nullptr;
    fwi_surrogate* s = new (std::nothrow) fwi_surrogate();
    if (!s) return FWI_ENOMEM;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return FWI_EHIP;
    }
    s->max_batch = max_batch;
    s->L = sur_layout();
    s->M = bf_map();
    if (!create_buffers(s)) {
        free_all(s);
        delete s;
        return FWI_ENOMEM;
    }
    int rc = build_bf_index(s);
    const size_t pb = (size_t)s->L.total * sizeof(float);
    if (rc == FWI_OK &&
        (hipMemset(s->P, 0, pb) != hipSuccess || hipMemset(s->G, 0, pb) != hipSuccess ||
         hipMemset(s->Am, 0, pb) != hipSuccess || hipMemset(s->Av, 0, pb) != hipSuccess ||
         hipMemset(s->W, 0, (size_t)s->M.total * sizeof(bf16_t)) != hipSuccess || hipDeviceSynchronize() != hipSuccess))
        rc = FWI_EHIP;
    if (rc == FWI_OK) rc = nn::mlp_prepare(nullptr);  // the fused MLP's GELU tables, once per device
    if (rc != FWI_OK) {
        free_all(s);
        delete s;
        return rc;
    }
    *out = s;
    return FWI_OK;
}

int fwi_sur_destroy(fwi_surrogate* s) {
    if (!s) return FWI_OK;
    hipSetDevice(s->device);
    hipDeviceSynchronize();
    free_all(s);
    delete s;
    return FWI_OK;
}

int fwi_sur_set_params(fwi_surrogate* s, const float* host) {
    if (!s || !host) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    const size_t pb = (size_t)s->L.total * sizeof(float);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(s->P, host, pb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->Am, 0, pb) != hipSuccess || hipMemset(s->Av, 0, pb) != hipSuccess)
        return FWI_EHIP;
    s->step = 0;
    nn::refresh_bf16(s->L.total, s->P, s->bf_index, s->W, nullptr);
    return hipDeviceSynchronize() == hipSuccess ? FWI_OK : FWI_EHIP;
}

static int copy_out(fwi_surrogate* s, const float* src, float* host) {
    if (!s || !host) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return FWI_EHIP;
    return hipMemcpy(host, src, (size_t)s->L.total * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess ? FWI_OK
                                                                                                         : FWI_EHIP;
}

int fwi_sur_get_params(fwi_surrogate* s, float* host) { return copy_out(s, s ? s->P : nullptr, host); }
int fwi_sur_get_grads(fwi_surrogate* s, float* host) { return copy_out(s, s ? s->G : nullptr, host); }

int fwi_sur_get_adam(fwi_surrogate* s, float* host_m, float* host_v, int* step) {
    if (!s || !host_m || !host_v || !step) return FWI_EINVAL;
    int rc = copy_out(s, s->Am, host_m);
    if (rc == FWI_OK) rc = copy_out(s, s->Av, host_v);
    *step = s->step;
    return rc;
}

int fwi_sur_set_adam(fwi_surrogate* s, const float* host_m, const float* host_v, int step) {
    if (!s || !host_m || !host_v || step < 0) return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    const size_t pb = (size_t)s->L.total * sizeof(float);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(s->Am, host_m, pb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->Av, host_v, pb, hipMemcpyHostToDevice) != hipSuccess)
        return FWI_EHIP;
    s->step = step;
    return hipDeviceSynchronize() == hipSuccess ? FWI_OK : FWI_EHIP;
}

int fwi_sur_set_fused_mlp(fwi_surrogate* s, int fused) {
    if (!s || (fused != 0 && fused != 1)) return FWI_EINVAL;
    s->fused = fused == 1;
    return FWI_OK;
}

int fwi_sur_forward(fwi_surrogate* s, int B, const float* v, float* traces, void* stream) {
    if (!s || !v || !traces || B < 0 || B > s->max_batch) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    return forward_impl(s, B, v, traces, (hipStream_t)stream);
}

int fwi_sur_backward(fwi_surrogate* s, int B, const float* dtraces, float* dv, int want_weight_grads, void* stream) {
    if (!s || !dtraces || B < 0 || B > s->max_batch) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (B != s->cachedB) return FWI_ESTATE;
    if (!dv && !want_weight_grads) return FWI_OK;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    return backward_impl(s, B, dtraces, dv, want_weight_grads, (hipStream_t)stream);
}

int fwi_sur_train_step(fwi_surrogate* s, int B, const float* v, const float* target,
                       const fwi_sur_train_params* tp, float* loss_out, void* stream) {
    if (!s || !v || !target || !tp || B < 1 || B > s->max_batch) return FWI_EINVAL;
    if (!(tp->lr > 0.f) || !(tp->beta1 >= 0.f && tp->beta1 < 1.f) || !(tp->beta2 >= 0.f && tp->beta2 < 1.f) ||
        !(tp->eps > 0.f) || !(tp->loss_k >= 0.f) || !(tp->pair_weight >= 0.f) ||
        (tp->pair_weight > 0.f && B % 2 != 0))
        return FWI_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return FWI_EHIP;
    hipStream_t st = (hipStream_t)stream;
    int rc = forward_impl(s, B, v, s->pred, st);
    if (rc != FWI_OK) return rc;
    nn::loss(B, s->pred, target, tp->loss_k, tp->pair_weight, s->dtr, loss_out ? loss_out : s->lval, s->mx, s->lpart, st);
    rc = backward_impl(s, B, s->dtr, nullptr, 1, st);
    if (rc != FWI_OK) return rc;
    ++s->step;
    nn::adam(s->L.total, s->P, s->G, s->Am, s->Av, tp->lr, tp->beta1, tp->beta2, tp->eps, s->step, s->bf_index, s->W,
             st);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

int fwi_judge(int B, int n, const float* g_a, const float* g_b, const double* J_a, const double* J_b, float* cos_out,
              float* jerr_out, void* stream) {
    if (B < 0 || n < 1 || !g_a || !g_b || !cos_out || (jerr_out && (!J_a || !J_b))) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    nn::judge(B, n, g_a, g_b, J_a, J_b, cos_out, jerr_out, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

int fwi_mf_predict(int B, int n, const float* g_anchor, const float* s_now, const float* s_anchor, float* g_out,
                   const double* J_anchor, const double* Js_now, const double* Js_anchor, double* J_out,
                   void* stream) {
    if (B < 0 || n < 1 || !g_anchor || !s_now || !s_anchor || !g_out) return FWI_EINVAL;
    if (J_out && (!J_anchor || !Js_now || !Js_anchor)) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    nn::mf_predict((long)B * n, g_anchor, s_now, s_anchor, g_out, B, J_anchor, Js_now, Js_anchor, J_out,
                   (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? FWI_OK : FWI_EHIP;
}

}  // extern "C"
