// Wasserstein-2 trace misfit on gfx950 (Sec. 5.1 (I)-(III), numerics of Sec. 6.2).
//
// One 256-thread workgroup per trace.  Per trace, in FP64 with the trace held
// in LDS:
//   h_k   = omega_k d_k + c'                          shifted, weighted trace
//   Z     = dt sum_k (h_k + h_{k+1}) / 2              trapezoid mass
//   F_0   = 0,  F_k = F_{k-1} + dt (h_{k-1} + h_k) / (2 (Z + eps'))   (block prefix scan)
//   Q_j   = inf{t : F(t) >= x_j},  x_j = min(j/(n_xi-1), max F)       (binary search on the
//           running maximum of F, linear interpolation on the bracketing segment)
//   W2^2  = sum_j w_j (Q_j - Q_obs,j)^2               trapezoid weights in xi
// and the adjoint source by the chain rule with the brackets k*_j fixed:
//   dQ_j/dF_{k*-1} = dt (alpha - 1)/Delta, dQ_j/dF_{k*} = -dt alpha/Delta
//   Fbar_k collects, in ascending j, the terms of the xi nodes whose bracket
//   touches k (k*_j is non-decreasing in j, so each range is found by binary search),
//   rhobar_m = dt/2 (S_{m+1} + [m >= 1] S_m) with S the suffix sums of Fbar,
//   hbar_m = rhobar_m/(Z+eps') - dt tau_m sum_k rhobar_k h_k/(Z+eps')^2,
//   a_m = omega_m hbar_m.
// Every reduction and scan has a fixed order, so results are bitwise
// reproducible run to run.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "fwi_internal.h"

namespace fwi {

constexpr int W2T = 256;
constexpr int W2W = W2T / 64;

struct OpSum {
    __device__ static double apply(double a, double b) { return a + b; }
    __device__ static double ident() { return 0.0; }
};
struct OpMax {
    __device__ static double apply(double a, double b) { return a > b ? a : b; }
    __device__ static double ident() { return -INFINITY; }
};
struct OpMin {
    __device__ static double apply(double a, double b) { return a < b ? a : b; }
    __device__ static double ident() { return INFINITY; }
};

// Block-wide reduction; every thread receives the same value.
template <class Op>
__device__ double block_reduce(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = Op::apply(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = sh[0];
    for (int i = 1; i < W2W; ++i) t = Op::apply(t, sh[i]);
    return t;
}

// In-place inclusive scan of X[0..n) (REV: suffix scan), contiguous chunk per thread.
template <class Op, bool REV>
__device__ void block_scan(double* X, int n, double* sh) {
    const int T = W2T;
    const int ch = (n + T - 1) / T;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int lo = threadIdx.x * ch, hi = min(lo + ch, n);
    __syncthreads();
    double s = Op::ident();
    for (int c = lo; c < hi; ++c) s = Op::apply(s, X[REV ? n - 1 - c : c]);
    double incl = s;
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(incl, o);
        if (lane >= o) incl = Op::apply(t, incl);
    }
    double ex = __shfl_up(incl, 1);
    if (lane == 0) ex = Op::ident();
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    double woff = Op::ident();
    for (int i = 0; i < wid; ++i) woff = Op::apply(woff, sh[i]);
    double run = Op::apply(woff, ex);
    for (int c = lo; c < hi; ++c) {
        const int i = REV ? n - 1 - c : c;
        run = Op::apply(run, X[i]);
        X[i] = run;
    }
    __syncthreads();
}

// First index k in [0, n) with A[k] >= x (A non-decreasing); n if none.
__device__ int lower_bound_d(const double* A, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Q searches of one non-decreasing array in lockstep (the same steps for all, so
// their reads overlap instead of waiting one by one): out[q] = first index k in
// [0, n) with A[k] >= x[q], n if none.  Each step halves the candidate range
// [base, base + len] of every query.
template <int Q, class T>
__device__ void lower_bound_n(const T* A, int n, const T (&x)[Q], int (&out)[Q]) {
    int base[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) base[q] = 0;
    int len = n;
    while (len > 1) {
        const int half = len >> 1;
#pragma unroll
        for (int q = 0; q < Q; ++q) base[q] = (A[base[q] + half] < x[q]) ? base[q] + half : base[q];
        len -= half;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) out[q] = (n > 0 && A[base[q]] < x[q]) ? base[q] + 1 : base[q];
}

__device__ inline double xi_weight(int j, int nxi) {
    const double w = 1.0 / (double)(nxi - 1);
    return (j == 0 || j == nxi - 1) ? 0.5 * w : w;
}

// From the shifted trace H builds F (trapezoid CDF) and Fh (its running max);
// returns Z.
__device__ double build_cdf(const double* H, double* F, double* Fh, int nt, double dt, double epsp, double* sh) {
    double part = 0.0;
    const int ch = (nt - 1 + W2T - 1) / W2T;
    const int lo = threadIdx.x * ch, hi = min(lo + ch, nt - 1);
    for (int k = lo; k < hi; ++k) part += dt * (H[k] + H[k + 1]) / 2.0;
    const double Z = block_reduce<OpSum>(part, sh);
    const double inv = 1.0 / (Z + epsp);
    for (int k = threadIdx.x; k < nt; k += W2T) F[k] = (k == 0) ? 0.0 : dt * (H[k - 1] * inv + H[k] * inv) / 2.0;
    block_scan<OpSum, false>(F, nt, sh);
    for (int k = threadIdx.x; k < nt; k += W2T) Fh[k] = F[k];
    block_scan<OpMax, false>(Fh, nt, sh);
    return Z;
}

// Quantile at xi_j (see the file comment); k is the bracket index.
__device__ inline double quantile(const double* F, const double* Fh, int nt, double dt, double xi, double Fmax,
                                  int* kout) {
    const double x = xi > Fmax ? Fmax : xi;
    // x <= Fh[nt-1] keeps k <= nt-1; the min only matters for non-finite traces
    const int k = min(lower_bound_d(Fh, nt, x), nt - 1);
    *kout = k;
    if (k == 0) return 0.0;
    return dt * ((double)(k - 1) + (x - F[k - 1]) / (F[k] - F[k - 1]));
}

// ---------------------------------------------------------------------------
// Observation side.
// max |d| over n values: per-block maxima (grid-stride), then one block
// reduces them (max is exact in any order).
__global__ __launch_bounds__(256) void k_absmax_partial(const float* __restrict__ d, long n, double* __restrict__ part) {
    __shared__ float sh[4];
    float m = 0.f;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float a = fabsf(d[i]);
        m = a > m ? a : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const float t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = sh[i] > t ? sh[i] : t;
        part[blockIdx.x] = (double)t;
    }
}

__global__ __launch_bounds__(256) void k_absmax_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double sh[4];
    double m = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) m = part[i] > m ? part[i] : m;
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = sh[i] > t ? sh[i] : t;
        *out = t;
    }
}

__global__ __launch_bounds__(W2T) void k_w2_obs(int nt, int nxi, double dt, const float* __restrict__ dobs,
                                                const double* __restrict__ gmax, double kw, double epsp, double cfac,
                                                int squared, double* __restrict__ omega, double* __restrict__ cprime,
                                                double* __restrict__ qobs, double* __restrict__ qnorm) {
    extern __shared__ double smem[];
    __shared__ double sh[W2W + 1];
    double* H = smem;
    double* F = H + nt;
    double* Fh = F + nt;
    const int t = blockIdx.x;
    const double M = *gmax;
    double mn = INFINITY;
    for (int k = threadIdx.x; k < nt; k += W2T) {
        const double o = (double)dobs[(size_t)t * nt + k];
        const double a = (M > 0.0) ? fabs(o) / M : 0.0;
        const double om = 1.0 / (1.0 + kw * a);
        omega[(size_t)t * nt + k] = om;
        H[k] = om * o;
        mn = H[k] < mn ? H[k] : mn;
    }
    mn = block_reduce<OpMin>(mn, sh);
    const double cp = cfac * fabs(mn);
    if (threadIdx.x == 0) cprime[t] = cp;
    for (int k = threadIdx.x; k < nt; k += W2T) H[k] += cp;
    __syncthreads();
    build_cdf(H, F, Fh, nt, dt, epsp, sh);
    const double Fmax = Fh[nt - 1];
    double m2 = 0.0;
    for (int j = threadIdx.x; j < nxi; j += W2T) {
        int k;
        const double Q = quantile(F, Fh, nt, dt, (double)j / (double)(nxi - 1), Fmax, &k);
        qobs[(size_t)t * nxi + j] = Q;
        m2 += xi_weight(j, nxi) * Q * Q;
    }
    m2 = block_reduce<OpSum>(m2, sh);
    if (threadIdx.x == 0) qnorm[t] = squared ? m2 : sqrt(m2);
}

// Fixed-order sum of n values by one block.
__global__ __launch_bounds__(W2T) void k_sum_fixed(const double* __restrict__ x, int n, double* __restrict__ out) {
    __shared__ double sh[W2W + 1];
    double s = 0.0;
    const int ch = (n + W2T - 1) / W2T;
    const int lo = threadIdx.x * ch, hi = min(lo + ch, n);
    for (int i = lo; i < hi; ++i) s += x[i];
    s = block_reduce<OpSum>(s, sh);
    if (threadIdx.x == 0) *out = s;
}

static size_t w2_lds_bytes(int nt, int nxi) { return (size_t)3 * nt * sizeof(double) + (size_t)nxi * (sizeof(double) + sizeof(int)); }

int launch_w2_obs(Plan& p, const float* d_obs, hipStream_t st) {
    const int ntr = p.g.ns * p.g.nr;
    const int nt = p.g.nt;
    const int nxi = p.w2p.n_xi;
    double* gmax = p.sobs + 1;  // scratch slot next to S_obs
    // per-block maxima in the misfit's pair buffer (max_batch * ns * nr >= ntr slots; the misfit overwrites it)
    const int nb = std::min(ntr, 2048);
    hipLaunchKernelGGL(k_absmax_partial, dim3(nb), dim3(256), 0, st, d_obs, (long)ntr * nt, p.w2pair);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, st, p.w2pair, nb, gmax);
    const size_t bytes = (size_t)3 * nt * sizeof(double);
    hipFuncSetAttribute((const void*)k_w2_obs, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL(k_w2_obs, dim3(ntr), dim3(W2T), bytes, st, nt, nxi, p.g.dt, d_obs, gmax, p.w2p.k,
                       p.w2p.eps_prime, p.w2p.c_factor, p.w2p.squared, p.omega, p.cprime, p.qobs, p.qnorm);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(W2T), 0, st, p.qnorm, ntr, p.sobs);
    return hip_ok(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Synthetic side: per-pair J contribution and the adjoint source.
__global__ __launch_bounds__(W2T) void k_w2_misfit(int ntr, int nt, int nxi, double dt, const float* __restrict__ dsyn,
                                                   const double* __restrict__ omega, const double* __restrict__ cprime,
                                                   const double* __restrict__ qobs, const double* __restrict__ sobs,
                                                   double epsp, int squared, int reduction, double* __restrict__ jpair,
                                                   float* __restrict__ adj) {
    extern __shared__ double smem[];
    __shared__ double sh[W2W + 1];
    double* H = smem;
    double* F = H + nt;
    double* Fh = F + nt;
    double* dl = Fh + nt;                 // [nxi] Q_syn - Q_obs
    int* kst = (int*)(dl + nxi);          // [nxi] bracket index
    const long u = blockIdx.x;
    const int t = (int)(u % ntr);
    const double* om = omega + (size_t)t * nt;
    const double* qo = qobs + (size_t)t * nxi;
    const float* y = dsyn + (size_t)u * nt;
    const double cp = cprime[t];
    const double norm = reduction ? (double)ntr : *sobs;
    // loops over a thread's elements e = threadIdx.x + i W2T take G of them at a time, so that their global
    // loads and LDS searches overlap
    constexpr int G = 4;
    for (int k0 = threadIdx.x; k0 < nt; k0 += G * W2T) {
        double ov[G];
        float yv[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int k = min(k0 + g * W2T, nt - 1);
            ov[g] = om[k];
            yv[g] = y[k];
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (k0 + g * W2T < nt) H[k0 + g * W2T] = ov[g] * (double)yv[g] + cp;
    }
    __syncthreads();
    const double Z = build_cdf(H, F, Fh, nt, dt, epsp, sh);
    const double inv = 1.0 / (Z + epsp);
    const double Fmax = Fh[nt - 1];
    double m2 = 0.0;
    // quantiles (as quantile() forms them), G xi nodes per thread at a time
    for (int j0 = threadIdx.x; j0 < nxi; j0 += G * W2T) {
        double x[G], qv[G];
        int kk[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int j = min(j0 + g * W2T, nxi - 1);
            const double xi = (double)j / (double)(nxi - 1);
            x[g] = xi > Fmax ? Fmax : xi;
            qv[g] = qo[j];
        }
        lower_bound_n<G>(Fh, nt, x, kk);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int j = j0 + g * W2T;
            if (j >= nxi) break;
            // x <= Fh[nt-1] keeps k <= nt-1; the min only matters for non-finite traces
            const int k = min(kk[g], nt - 1);
            const double Q = k == 0 ? 0.0 : dt * ((double)(k - 1) + (x[g] - F[k - 1]) / (F[k] - F[k - 1]));
            const double d = Q - qv[g];
            dl[j] = d;
            kst[j] = k;
            m2 += xi_weight(j, nxi) * d * d;
        }
    }
    m2 = block_reduce<OpSum>(m2, sh);
    const double W2 = sqrt(m2);
    if (threadIdx.x == 0) jpair[u] = (squared ? m2 : W2) / norm;
    if (!adj) return;
    const double dm = squared ? 1.0 / norm : (W2 > 0.0 ? 1.0 / (2.0 * W2 * norm) : 0.0);
    // Fbar_k into Fh (the running max is no longer needed after the barrier in block_reduce)
    for (int k0 = threadIdx.x; k0 < nt; k0 += G * W2T) {
        int kx[3 * G], jr[3 * G];  // first xi nodes bracketed at k, k + 1, k + 2 of the G elements
#pragma unroll
        for (int g = 0; g < G; ++g) {
            kx[3 * g] = k0 + g * W2T;
            kx[3 * g + 1] = k0 + g * W2T + 1;
            kx[3 * g + 2] = k0 + g * W2T + 2;
        }
        lower_bound_n<3 * G>(kst, nxi, kx, jr);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int k = k0 + g * W2T;
            if (k >= nt) break;
            const int j0 = jr[3 * g], j1 = jr[3 * g + 1], j2 = jr[3 * g + 2];
            double fb = 0.0;
            // xi nodes bracketed by [k-1, k]: term dQ/dF_k
            for (int j = j0; j < j1; ++j) {
                const double xi = (double)j / (double)(nxi - 1);
                if (k == 0 || xi > Fmax) continue;
                const double den = F[k] - F[k - 1];
                const double al = (xi - F[k - 1]) / den;
                const double qb = dm * 2.0 * xi_weight(j, nxi) * dl[j];
                fb += qb * (-dt * al / den);
            }
            // xi nodes bracketed by [k, k+1]: term dQ/dF_k as the left end
            for (int j = j1; j < j2; ++j) {
                const double xi = (double)j / (double)(nxi - 1);
                if (xi > Fmax) continue;
                const double den = F[k + 1] - F[k];
                const double al = (xi - F[k]) / den;
                const double qb = dm * 2.0 * xi_weight(j, nxi) * dl[j];
                fb += qb * (dt * (al - 1.0) / den);
            }
            Fh[k] = fb;
        }
    }
    block_scan<OpSum, true>(Fh, nt, sh);  // Fh[m] = S_m = sum_{k >= m} Fbar_k
    double part = 0.0;
    for (int m = threadIdx.x; m < nt; m += W2T) {
        const double S1 = (m + 1 < nt) ? Fh[m + 1] : 0.0;
        const double S0 = (m >= 1) ? Fh[m] : 0.0;
        const double rb = 0.5 * dt * (S1 + S0);
        F[m] = rb;  // F is no longer needed: rhobar
        part += rb * H[m];
    }
    const double T = block_reduce<OpSum>(part, sh);
    const double Zb = -T * inv * inv;
    float* a = adj + (size_t)u * nt;
    for (int m0 = threadIdx.x; m0 < nt; m0 += G * W2T) {
        double ov[G];
#pragma unroll
        for (int g = 0; g < G; ++g) ov[g] = om[min(m0 + g * W2T, nt - 1)];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int m = m0 + g * W2T;
            if (m >= nt) break;
            const double tau = (m == 0 || m == nt - 1) ? 0.5 : 1.0;
            const double hb = F[m] * inv + Zb * dt * tau;
            a[m] = (float)(ov[g] * hb);
        }
    }
}

// J[b] = sum over the sample's pairs, in a fixed order.
__global__ __launch_bounds__(W2T) void k_sum_pairs(const double* __restrict__ jpair, int ntr, double* __restrict__ J) {
    __shared__ double sh[W2W + 1];
    const int b = blockIdx.x;
    const double* x = jpair + (size_t)b * ntr;
    double s = 0.0;
    const int ch = (ntr + W2T - 1) / W2T;
    const int lo = threadIdx.x * ch, hi = min(lo + ch, ntr);
    for (int i = lo; i < hi; ++i) s += x[i];
    s = block_reduce<OpSum>(s, sh);
    if (threadIdx.x == 0) J[b] = s;
}

static int launch_w2_misfit_into(const Plan& p, int B, const float* d_syn, double* J, float* adj, double* pairs,
                                 hipStream_t st) {
    const int ntr = p.g.ns * p.g.nr;
    const int nt = p.g.nt;
    const int nxi = p.w2p.n_xi;
    const size_t bytes = w2_lds_bytes(nt, nxi);
    hipFuncSetAttribute((const void*)k_w2_misfit, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL(k_w2_misfit, dim3(B * ntr), dim3(W2T), bytes, st, ntr, nt, nxi, p.g.dt, d_syn, p.omega,
                       p.cprime, p.qobs, p.sobs, p.w2p.eps_prime, p.w2p.squared, p.w2p.reduction, pairs, adj);
    hipLaunchKernelGGL(k_sum_pairs, dim3(B), dim3(W2T), 0, st, pairs, ntr, J);
    return hip_ok(hipGetLastError());
}

int launch_w2_misfit(const Plan& p, int B, const float* d_syn, double* J, float* adj, hipStream_t st) {
    return launch_w2_misfit_into(p, B, d_syn, J, adj, p.w2pair, st);
}

// Per-pair terms of the allocation-free entry point (fwi_w2_misfit_noalloc):
// a fixed array in device memory instead of the plan's workspace.  Every GPU
// the library runs on holds its own copy until the process ends, and every
// call on that GPU reuses it.  k_w2_misfit writes each pair's term before
// k_sum_pairs reads it, so nothing has to be cleared between calls; two calls
// that overlap on one GPU (different streams) race on it.
static __device__ __align__(256) double w2_scratch[FWI_W2_SCRATCH_PAIRS];

// Device address of w2_scratch on each device, looked up once per device with
// that device current (the array's host-side name is not a device address).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch[kMaxDevices] = {};

static int scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return FWI_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return FWI_EHIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return FWI_EHIP;
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(w2_scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return FWI_EHIP;
        }
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch[dev];
    return FWI_OK;
}

int launch_w2_misfit_noalloc(const Plan& p, int B, const float* d_syn, double* J, float* adj, hipStream_t st) {
    if ((long long)B * p.g.ns * p.g.nr > FWI_W2_SCRATCH_PAIRS) return FWI_ENOMEM;
    double* pairs = nullptr;
    const int rc = scratch_address(p.device, &pairs);
    if (rc) return rc;
    return launch_w2_misfit_into(p, B, d_syn, J, adj, pairs, st);
}

size_t w2_lds_requirement(int nt, int nxi) { return w2_lds_bytes(nt, nxi); }

}  // namespace fwi
