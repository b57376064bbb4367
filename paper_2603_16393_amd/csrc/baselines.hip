// The comparison and ablation variants of the guidance on gfx950: the
// least-squares potential of baseline DPS (Sec. 4, Phi_l2 with Sigma = sigma^2 I,
// Algorithm 1) with the ablation's optional amplitude weighting and
// misfit-scale normalisation (Sec. 6, after Sec. 5.1 (I)), and the total-
// variation subgradient the TV-regularised descent baselines add to the
// misfit gradient (Sec. 6, TV of Eq. tv).  Both reuse the forward and adjoint
// sweeps and the update kernel unchanged.
//
// Least squares, for observations d_obs [ntr][nt] shared by the B samples:
//   w = 1/(1 + k |d_obs| / max|d_obs|)      (1 when k = 0 or d_obs = 0)
//   S = sigma^2, or sum (w d_obs)^2 (1 if that is 0) when normalising
//   J_b = (1/2) sum (w (d_syn_b - d_obs))^2 / S,  adj_b = w^2 (d_syn_b - d_obs) / S
// One workgroup per trace for the observation statistics, one per (trace,
// sample) for the terms; every sum is FP64 in a fixed order and the maximum
// is exact, so results are bitwise reproducible.
//
// TV subgradient: per cell, the signs of the forward differences (right and
// lower neighbour) the cell is the head (+) or tail (-) of, times alpha / (nz nx),
// added to g; sign(0) = 0.  The differences are taken in FP64 from FP32
// values (exact), so every sign is exact.
#include <cmath>

#include "fwi_internal.h"

namespace fwi {
namespace {

constexpr int LT = 256;

__device__ double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
    for (int i = 1; i < LT / 64; ++i) t += sh[i];
    return t;
}

__device__ double block_max(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
    for (int i = 1; i < LT / 64; ++i) t = sh[i] > t ? sh[i] : t;
    return t;
}

// fixed-order sum of x[0..n) by one workgroup (contiguous chunk per thread)
__device__ double block_sum_array(const double* x, int n, double* sh) {
    const int ch = (n + LT - 1) / LT;
    const int lo = threadIdx.x * ch, hi = min(lo + ch, n);
    double s = 0.0;
    for (int i = lo; i < hi; ++i) s += x[i];
    return block_sum(s, sh);
}

__device__ double array_max(const double* x, int n, double* sh) {
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += LT) m = x[i] > m ? x[i] : m;
    return block_max(m, sh);
}

__device__ inline double weight(float o, double k, double amax) {
    return (k > 0.0 && amax > 0.0) ? 1.0 / (1.0 + k * fabs((double)o) / amax) : 1.0;
}

// stat[tr] = max_t |d_obs[tr][t]|
__global__ __launch_bounds__(LT) void k_l2_trmax(int nt, const float* __restrict__ dobs, double* __restrict__ stat) {
    __shared__ double sh[LT / 64];
    const float* o = dobs + (size_t)blockIdx.x * nt;
    double m = 0.0;
    for (int t = threadIdx.x; t < nt; t += LT) m = fabs((double)o[t]) > m ? fabs((double)o[t]) : m;
    m = block_max(m, sh);
    if (threadIdx.x == 0) stat[blockIdx.x] = m;
}

// stat[ntr + tr] = sum_t (w d_obs)^2, with the global maximum of stat[0..ntr)
__global__ __launch_bounds__(LT) void k_l2_trenergy(int ntr, int nt, const float* __restrict__ dobs, double k,
                                                    double* __restrict__ stat) {
    __shared__ double sh[LT / 64];
    const double amax = array_max(stat, ntr, sh);
    const float* o = dobs + (size_t)blockIdx.x * nt;
    const int ch = (nt + LT - 1) / LT;
    const int lo = threadIdx.x * ch, hi = min(lo + ch, nt);
    double s = 0.0;
    for (int t = lo; t < hi; ++t) {
        const double wd = weight(o[t], k, amax) * (double)o[t];
        s += wd * wd;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) stat[ntr + blockIdx.x] = s;
}

// stat[2 ntr] = max |d_obs|, stat[2 ntr + 1] = S
__global__ __launch_bounds__(LT) void k_l2_scale(int ntr, int normalize, double sigma, double* __restrict__ stat) {
    __shared__ double sh[LT / 64];
    const double amax = array_max(stat, ntr, sh);
    double S = sigma * sigma;
    if (normalize) {
        S = block_sum_array(stat + ntr, ntr, sh);
        if (S == 0.0) S = 1.0;
    }
    if (threadIdx.x == 0) {
        stat[2 * ntr] = amax;
        stat[2 * ntr + 1] = S;
    }
}

// part[b][tr] = sum_t (w r)^2 and adj = w^2 r / S for trace tr = blockIdx.x of sample b = blockIdx.y
__global__ __launch_bounds__(LT) void k_l2_terms(int ntr, int nt, const float* __restrict__ dsyn,
                                                 const float* __restrict__ dobs, double k,
                                                 const double* __restrict__ stat, double* __restrict__ part,
                                                 float* __restrict__ adj) {
    __shared__ double sh[LT / 64];
    const int tr = blockIdx.x, b = blockIdx.y;
    const double amax = stat[2 * ntr], S = stat[2 * ntr + 1];
    const float* o = dobs + (size_t)tr * nt;
    const size_t base = ((size_t)b * ntr + tr) * nt;
    const int ch = (nt + LT - 1) / LT;
    const int lo = threadIdx.x * ch, hi = min(lo + ch, nt);
    double s = 0.0;
    for (int t = lo; t < hi; ++t) {
        const double w = weight(o[t], k, amax);
        const double r = (double)dsyn[base + t] - (double)o[t];
        s += (w * r) * (w * r);
        if (adj) adj[base + t] = (float)(w * w * r / S);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[(size_t)b * ntr + tr] = s;
}

__global__ __launch_bounds__(LT) void k_l2_final(int ntr, const double* __restrict__ part,
                                                 const double* __restrict__ stat, double* __restrict__ J) {
    __shared__ double sh[LT / 64];
    const double s = block_sum_array(part + (size_t)blockIdx.x * ntr, ntr, sh);
    if (threadIdx.x == 0) J[blockIdx.x] = 0.5 * s / stat[2 * ntr + 1];
}

__device__ inline double sgn(double d) { return (double)((d > 0.0) - (d < 0.0)); }

__global__ __launch_bounds__(LT) void k_tv_subgradient(int B, int nz, int nx, const float* __restrict__ x,
                                                       const float* g, double alpha, float* out) {
    const long n = (long)nz * nx, total = (long)B * n;
    const double f = alpha / (double)n;
    for (long i = blockIdx.x * (long)LT + threadIdx.x; i < total; i += (long)gridDim.x * LT) {
        const long b = i / n, l = i - b * n;
        const int iz = (int)(l / nx), ix = (int)(l - (long)iz * nx);
        const float* xb = x + b * n;
        const double xv = (double)xb[l];
        double c = 0.0;
        if (ix > 0) c += sgn(xv - (double)xb[l - 1]);
        if (ix + 1 < nx) c -= sgn((double)xb[l + 1] - xv);
        if (iz > 0) c += sgn(xv - (double)xb[l - nx]);
        if (iz + 1 < nz) c -= sgn((double)xb[l + nx] - xv);
        out[i] = (float)((g ? (double)g[i] : 0.0) + f * c);
    }
}

}  // namespace

int launch_l2_misfit(const Plan& p, int B, const float* d_syn, const float* d_obs, const fwi_l2_params& lp, double* J,
                     float* adj, hipStream_t st) {
    const int ntr = p.g.ns * p.g.nr, nt = p.g.nt;
    hipLaunchKernelGGL(k_l2_trmax, dim3(ntr), dim3(LT), 0, st, nt, d_obs, p.l2stat);
    if (lp.normalize) hipLaunchKernelGGL(k_l2_trenergy, dim3(ntr), dim3(LT), 0, st, ntr, nt, d_obs, lp.k, p.l2stat);
    hipLaunchKernelGGL(k_l2_scale, dim3(1), dim3(LT), 0, st, ntr, lp.normalize, lp.sigma, p.l2stat);
    hipLaunchKernelGGL(k_l2_terms, dim3(ntr, B), dim3(LT), 0, st, ntr, nt, d_syn, d_obs, lp.k, p.l2stat, p.w2pair,
                       adj);
    hipLaunchKernelGGL(k_l2_final, dim3(B), dim3(LT), 0, st, ntr, p.w2pair, p.l2stat, J);
    return hip_ok(hipGetLastError());
}

int launch_tv_subgradient(int B, int nz, int nx, const float* v, const float* g, double alpha, float* out,
                          hipStream_t st) {
    const long total = (long)B * nz * nx;
    const int grid = (int)std::min<long>((total + LT - 1) / LT, 4096);
    hipLaunchKernelGGL(k_tv_subgradient, dim3(grid), dim3(LT), 0, st, B, nz, nx, v, g, alpha, out);
    return hip_ok(hipGetLastError());
}

}  // namespace fwi
