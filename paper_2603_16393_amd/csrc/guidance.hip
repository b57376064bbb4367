// Preconditioned guidance update on gfx950 (Sec. 5.2: Eqs. tv, rho, kappa,
// precond_step; the gradient, preconditioner and update lines of Algorithm 2).
//
// kGP 256-thread workgroups per sample: each forms the sample's fixed-order
// FP64 reduction (the total variation of the clean estimate) and exact max
// (||s g||_inf) in the same order, so all hold the same values, and then
// updates its share of the cells (the FP64 power per cell dominates).
#include <cmath>

#include "fwi_internal.h"

namespace fwi {

constexpr int GT = 256;
constexpr int kGP = 8;  // workgroups per sample

__global__ __launch_bounds__(GT) void k_guidance(int nz, int nx, const float* __restrict__ vprop,
                                                 const float* __restrict__ h, const float* __restrict__ g,
                                                 const float* __restrict__ v0hat, double rho0, double c, double tau,
                                                 double gamma, double eps, double kappa_max, double s,
                                                 float* __restrict__ vnext, float* __restrict__ rho_out) {
    __shared__ double shs[GT / 64];
    __shared__ double shm[GT / 64];
    const int b = blockIdx.x;
    const size_t n = (size_t)nz * nx;
    const float* x = v0hat + b * n;
    const float* gb = g + b * n;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;

    const int ch = (int)((n + GT - 1) / GT);
    const int lo = threadIdx.x * ch, hi = min((int)n, lo + ch);
    double tv = 0.0;
    double gm = 0.0;
    for (int i = lo; i < hi; ++i) {
        const int iz = i / nx, ix = i - (i / nx) * nx;
        const double xv = (double)x[i];
        if (ix + 1 < nx) tv += fabs((double)x[i + 1] - xv);
        if (iz + 1 < nz) tv += fabs((double)x[i + nx] - xv);
        const double a = fabs(s * (double)gb[i]);
        gm = a > gm ? a : gm;
    }
    for (int o = 32; o > 0; o >>= 1) {
        tv += __shfl_xor(tv, o);
        const double t = __shfl_xor(gm, o);
        gm = t > gm ? t : gm;
    }
    if (lane == 0) {
        shs[wid] = tv;
        shm[wid] = gm;
    }
    __syncthreads();
    tv = shs[0];
    gm = shm[0];
    for (int i = 1; i < GT / 64; ++i) {
        tv += shs[i];
        gm = shm[i] > gm ? shm[i] : gm;
    }
    tv /= (double)n;
    const double ex = tv - tau > 0.0 ? tv - tau : 0.0;
    const double rho = rho0 * exp(-ex / c);
    if (blockIdx.y == 0 && threadIdx.x == 0 && rho_out) rho_out[b] = (float)rho;
    const double num = gm + eps;
    for (size_t i = blockIdx.y * GT + threadIdx.x; i < n; i += (size_t)GT * gridDim.y) {
        const double gi = fabs(s * (double)gb[i]);
        double kap = pow(num / (gi + eps), gamma);
        if (kappa_max > 0.0 && kap > kappa_max) kap = kappa_max;
        vnext[b * n + i] = (float)((double)vprop[b * n + i] - rho * kap * s * (double)h[b * n + i]);
    }
}

int launch_guidance(int B, int nz, int nx, const float* v_prop, const float* h, const float* g, const float* v0hat,
                    const fwi_guidance_params& gp, float* v_next, float* rho_out, hipStream_t st) {
    if (B == 0) return FWI_OK;
    hipLaunchKernelGGL(k_guidance, dim3(B, kGP), dim3(GT), 0, st, nz, nx, v_prop, h, g, v0hat, gp.rho0, gp.c, gp.tau,
                       gp.gamma, gp.eps, gp.kappa_max, gp.unit_scale, v_next, rho_out);
    return hip_ok(hipGetLastError());
}

}  // namespace fwi
