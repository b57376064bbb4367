// Reverse DDPM step of Algorithm 2 without its guidance term: the clean
// estimator (Eq. v0hat) from the score network's output and the posterior
// mean plus noise,
//   v0hat = (v + (1 - abar_i) s) / sqrt(abar_i)
//   v'    = sqrt(alpha_i) (1 - abar_{i-1}) / (1 - abar_i) v + sqrt(abar_{i-1}) beta_i / (1 - abar_i) v0hat
//           + sigma z,       alpha_i = 1 - beta_i,
// one element per thread, float4 where the pointers allow.  The guidance
// update that follows is fwi_guidance_step with v_prop = v'.
#include <cmath>

#include "fwi_internal.h"

namespace fwi {
namespace {

struct DdpmCoef {
    float inv_sqrt_abar, one_minus_abar, ca, cb, sigma;
};

__device__ __forceinline__ void ddpm_one(const DdpmCoef& c, float v, float s_or_x0, float z, bool have_score,
                                         bool have_z, float& x0, float& vp) {
    x0 = have_score ? c.inv_sqrt_abar * fmaf(c.one_minus_abar, s_or_x0, v) : s_or_x0;
    vp = fmaf(c.ca, v, c.cb * x0);
    if (have_z) vp = fmaf(c.sigma, z, vp);
}

__global__ void k_ddpm_step(long n, const float* __restrict__ v, const float* __restrict__ score,
                            const float* __restrict__ z, DdpmCoef c, float* __restrict__ v0hat,
                            float* __restrict__ vprop) {
    const bool hs = score != nullptr, hz = z != nullptr;
    const float* sx = hs ? score : v0hat;  // input of the estimator line: s, or the caller's v0hat
    const long n4 = n / 4;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 a = reinterpret_cast<const float4*>(v)[i];
        const float4 b = reinterpret_cast<const float4*>(sx)[i];
        const float4 w = hz ? reinterpret_cast<const float4*>(z)[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        float4 x, p;
        ddpm_one(c, a.x, b.x, w.x, hs, hz, x.x, p.x);
        ddpm_one(c, a.y, b.y, w.y, hs, hz, x.y, p.y);
        ddpm_one(c, a.z, b.z, w.z, hs, hz, x.z, p.z);
        ddpm_one(c, a.w, b.w, w.w, hs, hz, x.w, p.w);
        if (hs) reinterpret_cast<float4*>(v0hat)[i] = x;
        reinterpret_cast<float4*>(vprop)[i] = p;
    }
    for (long i = 4 * n4 + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float x, p;
        ddpm_one(c, v[i], sx[i], hz ? z[i] : 0.f, hs, hz, x, p);
        if (hs) v0hat[i] = x;
        vprop[i] = p;
    }
}

bool aligned16(const void* p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace
}  // namespace fwi

using namespace fwi;

extern "C" int fwi_ddpm_step(long n, const float* v, const float* score, const float* z, double beta, double abar,
                             double abar_prev, double sigma, float* v0hat, float* v_prop, void* stream) {
    if (n < 0 || !(beta > 0 && beta < 1) || !(abar > 0 && abar < 1) || !(abar_prev > 0 && abar_prev <= 1) ||
        !(abar < abar_prev) || !std::isfinite(sigma) || sigma < 0)
        return FWI_EINVAL;
    if (n == 0) return FWI_OK;
    if (!v || !v0hat || !v_prop) return FWI_EINVAL;
    if (!aligned16(v) || !aligned16(score) || !aligned16(z) || !aligned16(v0hat) || !aligned16(v_prop))
        return FWI_EINVAL;
    const double alpha = 1.0 - beta;
    DdpmCoef c;
    c.inv_sqrt_abar = (float)(1.0 / std::sqrt(abar));
    c.one_minus_abar = (float)(1.0 - abar);
    c.ca = (float)(std::sqrt(alpha) * (1.0 - abar_prev) / (1.0 - abar));
    c.cb = (float)(std::sqrt(abar_prev) * beta / (1.0 - abar));
    c.sigma = (float)sigma;
    const long work = (n + 3) / 4;
    const int blocks = (int)std::min<long>((work + 255) / 256, 4096);
    hipLaunchKernelGGL(k_ddpm_step, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), n, v, score, z,
                       c, v0hat, v_prop);
    return hip_ok(hipGetLastError());
}
