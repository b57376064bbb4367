// Forward and adjoint sweeps with a perfectly matched layer as the absorbing
// boundary (Sec. 2.1: absorbing conditions on the non-reflecting sides,
// realised by a PML; Sec. 6.1: a PML of 6 grid points on the left, right and
// bottom, reflecting top).  The paper does not state its PML equations; this
// is the unsplit second-order form that a complex coordinate stretch
// s = 1 + zeta/(i w) per axis gives (Grote and Sim, 2010), with v^2 outside
// the divergence (exact here: the padded velocity is constant along each
// layer's normal):
//
//   u_tt + (zx + zz) u_t + zx zz u = v^2 (Lap u + d_x psi_x + d_z psi_z + s)
//   psi_x,t = -zx psi_x + (zz - zx) d_x u,   psi_z,t = -zz psi_z + (zx - zz) d_z u
//
// Discretisation, with tx = zx dt/2, tz = zz dt/2 per column and row, 8th-order
// central first derivatives Dx, Dz and psi at half steps (trapezoid rule):
//
//   Q_x = c_x (psi_x + (tz - tx) Dx u^n),  Q_z = c_z (psi_z + (tx - tz) Dz u^n),  c = 1/(1 + t)
//   psi <- 2 Q - psi
//   D   = L u^n + Dx Q_x + Dz Q_z + s^n
//   w^{n+1} = q w^n - b u^n + r D,  u^{n+1} = u^n + w^{n+1}     (w^n = u^n - u^{n-1})
//   E = 1/(1 + tx + tz),  q = (1 - tx - tz) E,  b = 4 tx tz E,  r = (v dt)^2 E.
//
// On a reflecting top u is even and Q_z odd across row 0.  In the model
// region t = 0, so q = 1, b = 0, r = (v dt)^2 and Q = 0: the leapfrog of the
// sponge sweeps.
//
// Adjoint.  With mu = W^{-1} dJ/du (W = 1/2 on a reflecting top row, 1
// elsewhere; the same scaling as the sponge sweeps' adjoint), y = r mu and
// (phx, phz) = W^{-1} dJ/dpsi, the exact transpose of one step is
//
//   Qh_x = 2 phx - Dx y,  Qh_z = 2 phz - Dz y            (y even across row 0)
//   ph <- c Qh - ph,      G_x = c_x (tz - tx) Qh_x,  G_z = c_z (tx - tz) Qh_z  (G_z odd)
//   nu^n = q nu^{n+1} - b mu^{n+1} + L y - Dx G_x - Dz G_z + a^n / w,  mu^n = mu^{n+1} + nu^n
//
// (the transposes of the mirrored first derivatives are the opposite
// mirror's gathers once scaled by W; Dx is antisymmetric on the zero-extended
// grid), and dJ/d(v dt)^2 = (W / (v dt)^2) sum_n y^{n+1} D^n: the imaging sum
// has the form of the sponge sweeps', so the same gradient fold applies.
//
// One workgroup of kPmlThreads threads holds a whole (sample, shot) field in
// LDS: three gather planes (u or y, Q_x or G_x, Q_z or G_z) of (nzp + 8) x
// (nxp + 8) floats with 4-cell zero halos (mirror rows above a reflecting
// top), and r and E per cell.  Thread t owns the slots t + k kPmlThreads of
// the order PmlOrder defines (model cells away from the layer, the model ring
// next to it, the layer), so a wavefront of the first group skips the
// divergence of Q and one of the first two skips the auxiliary fields.  The
// history of D is kept in slot order (coalesced); the imaging sum leaves in
// padded order.  Two barriers per step separate the gradient phase (writes
// Q) from the divergence phase (writes u^{n+1}).

#include "fwi_internal.h"

namespace fwi {

namespace {

constexpr float kD1 = 4.0f / 5.0f;
constexpr float kD2 = -1.0f / 5.0f;
constexpr float kD3 = 4.0f / 105.0f;
constexpr float kD4 = -1.0f / 280.0f;

// Central first difference sum_k d_k (f(+k s) - f(-k s)) at c (unscaled).
__device__ __forceinline__ float dfirst(const float* c, int s) {
    return fmaf(kD1, c[s] - c[-s], fmaf(kD2, c[2 * s] - c[-2 * s], fmaf(kD3, c[3 * s] - c[-3 * s], kD4 * (c[4 * s] - c[-4 * s]))));
}

// Returns x unchanged, opaque to the optimiser: per-slot addresses derived
// from it are recomputed in every step instead of being held in registers
// across the time loop (7 slots of them would spill).
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

struct PmlArgs {
    int nzp, nxp, npts;
    int nz, nx, nb, ztop;  // model grid inside the padded one
    int S;                 // LDS row stride nxp + 8
    int fs;                // reflecting top
    int nt, ns, nr;
    float idz, idx, idz2, idx2, src_scale;
    const float* K;          // [B][npts] (v dt)^2, padded row-major
    const float* tx;         // [nxp] zeta_x dt / 2
    const float* tz;         // [nzp] zeta_z dt / 2
    const float* wavelet;
    const int* src_pt;       // [ns] padded index
    const int* rec_slot;     // [npts] receiver index of each slot, or -1
    const float* rec_invw;   // [nr]
    float* traces;           // forward out [B][ns][nr][nt]
    const float* adj;        // adjoint in [B][ns][nr][nt]
    float* Dstore;           // [B*ns][nt-1][npts], slot order
    float* gpad;             // adjoint out [B*ns][npts], padded order
    int store;
};

template <int KC, bool ADJ>
__global__ void __launch_bounds__(kPmlThreads) k_wave_pml(const PmlArgs a) {
    extern __shared__ float lds[];
    const int S = a.S, nxp = a.nxp, nzp = a.nzp, npts = a.npts;
    const int plane = (nzp + 8) * S;
    float* F = lds;               // u^n (forward) or y = r mu (adjoint)
    float* GX = lds + plane;      // Q_x or G_x
    float* GZ = lds + 2 * plane;  // Q_z or G_z
    float* rs = lds + 3 * plane;  // [npts] r per slot
    float* Es = rs + npts;        // [npts] E per slot
    float* tcx = Es + npts;
    float* ttx = tcx + nxp;
    float* tcz = ttx + nxp;
    float* ttz = tcz + nzp;
    const int field = blockIdx.x;
    const int b = field / a.ns, s = field - (field / a.ns) * a.ns;
    const int tid = threadIdx.x;
    const int nsteps = a.nt - 1;
    const PmlOrder ord(a.nz, a.nx, a.nb, a.fs);
    const int nint = ord.nint, ndeep = ord.ndeep;

    for (int i = tid; i < 3 * plane; i += kPmlThreads) lds[i] = 0.f;
    for (int i = tid; i < nxp; i += kPmlThreads) {
        ttx[i] = a.tx[i];
        tcx[i] = 1.f / (1.f + a.tx[i]);
    }
    for (int i = tid; i < nzp; i += kPmlThreads) {
        ttz[i] = a.tz[i];
        tcz[i] = 1.f / (1.f + a.tz[i]);
    }
    int pos[KC];  // iz << 16 | ix of each slot, -1 past the grid
    int rec[KC];  // receiver of each slot, or -1
    const float* Kb = a.K + (size_t)b * npts;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int j = tid + k * kPmlThreads;
        pos[k] = -1;
        rec[k] = -1;
        if (j < npts) {
            rec[k] = a.rec_slot[j];
            int iz, ix;
            ord.cell(j, iz, ix);
            pos[k] = (iz << 16) | ix;
            const float E = 1.f / (1.f + a.tx[ix] + a.tz[iz]);
            rs[j] = Kb[iz * nxp + ix] * E;
            Es[j] = E;
        }
    }
    // source slot (a model cell) and this thread's receiver
    const int sp = a.src_pt[s];
    const int sj = ord.model_slot(sp / nxp - a.ztop, sp % nxp - a.nb);
    const bool own_src = (sj % kPmlThreads) == tid;
    const int ksrc = sj / kPmlThreads;
    const size_t trfield = (size_t)field * a.nr * a.nt;
    float* Dfield = a.Dstore + (size_t)field * nsteps * npts;

    float w[KC], px[KC], pz[KC], acc[KC], mu[KC], dnext[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        w[k] = 0.f;
        px[k] = 0.f;
        pz[k] = 0.f;
        acc[k] = 0.f;
        mu[k] = 0.f;
        dnext[k] = 0.f;
    }
    __syncthreads();

    if (!ADJ) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (rec[k] >= 0) a.traces[trfield + (size_t)rec[k] * a.nt] = 0.f;
    } else {
        // mu^{N-1} = a^{N-1} / w at the receivers, mu^N = 0, nu^{N-1} = mu^{N-1}
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (rec[k] >= 0) {
                mu[k] = a.adj[trfield + (size_t)rec[k] * a.nt + nsteps] * a.rec_invw[rec[k]];
                w[k] = mu[k];
                const float y = rs[tid + k * kPmlThreads] * mu[k];
                const int iz = pos[k] >> 16, ix = pos[k] & 0xffff;
                const int o = (iz + 4) * S + ix + 4;
                F[o] = y;
                if (a.fs && iz >= 1 && iz <= 4) F[o - 2 * iz * S] = y;
            }
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (pos[k] >= 0) dnext[k] = Dfield[(size_t)(nsteps - 1) * npts + tid + k * kPmlThreads];
    }
    __syncthreads();

    for (int m = 0; m < nsteps; ++m) {
        const int n = ADJ ? nsteps - 1 - m : m;  // forward step index
        // phase 1: Laplacian of the gathered field; in the layer the auxiliary
        // update and the Q (G) planes (zero in the model: psi stays 0 there, and
        // its adjoint never reaches u)
        float lap[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            // one slot at a time: overlapping the slots' neighbour loads costs
            // registers (spills at 7 slots) and buys little with 16 waves per CU
            __builtin_amdgcn_sched_barrier(0);
            lap[k] = 0.f;
            if (pos[k] < 0) continue;
            const int pk = opaque(pos[k]);
            const int iz = pk >> 16, ix = pk & 0xffff;
            const int o = (iz + 4) * S + ix + 4;
            const float* c = F + o;
            const float c0 = c[0];
            const float lz = FWI_LAPD(c0, c[-4 * S], c[-3 * S], c[-2 * S], c[-S], c[S], c[2 * S], c[3 * S], c[4 * S]);
            const float lx = FWI_LAPD(c0, c[-4], c[-3], c[-2], c[-1], c[1], c[2], c[3], c[4]);
            lap[k] = fmaf(a.idx2, lx, a.idz2 * lz);
            if (ADJ) acc[k] = fmaf(c0, dnext[k], acc[k]);  // imaging: y^{n+1} D^n
            if (opaque(tid + k * kPmlThreads) >= nint) {
                const float gx = a.idx * dfirst(c, 1);
                const float gz = a.idz * dfirst(c, S);
                const float cxv = tcx[ix], txv = ttx[ix], czv = tcz[iz], tzv = ttz[iz];
                float ox, oz;
                if (!ADJ) {
                    const float Qx = cxv * fmaf(tzv - txv, gx, px[k]);
                    const float Qz = czv * fmaf(txv - tzv, gz, pz[k]);
                    px[k] = 2.f * Qx - px[k];
                    pz[k] = 2.f * Qz - pz[k];
                    ox = Qx;
                    oz = Qz;
                } else {
                    const float Qx = 2.f * px[k] - gx;
                    const float Qz = 2.f * pz[k] - gz;
                    px[k] = cxv * Qx - px[k];
                    pz[k] = czv * Qz - pz[k];
                    ox = cxv * (tzv - txv) * Qx;
                    oz = czv * (txv - tzv) * Qz;
                }
                GX[o] = ox;
                GZ[o] = oz;
                if (a.fs && iz >= 1 && iz <= 4) GZ[o - 2 * iz * S] = -oz;
            }
        }
        float sv = 0.f, av[KC];
        if (!ADJ) {
            if (own_src) sv = a.wavelet[n] * a.src_scale;
        } else {
#pragma unroll
            for (int k = 0; k < KC; ++k)
                av[k] = rec[k] >= 0 ? a.adj[trfield + (size_t)rec[k] * a.nt + n] * a.rec_invw[rec[k]] : 0.f;
            if (n >= 1) {
#pragma unroll
                for (int k = 0; k < KC; ++k)
                    if (pos[k] >= 0) dnext[k] = Dfield[(size_t)(n - 1) * npts + opaque(tid + k * kPmlThreads)];
            }
        }
        __syncthreads();
        // phase 2: divergence of the Q (G) planes and the time update
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            __builtin_amdgcn_sched_barrier(0);
            if (pos[k] < 0) continue;
            const int j = opaque(tid + k * kPmlThreads);
            const int pk = opaque(pos[k]);
            const int iz = pk >> 16, ix = pk & 0xffff;
            const int o = (iz + 4) * S + ix + 4;
            // Q is zero within 4 cells of a deep cell
            const float div = j < ndeep ? 0.f : fmaf(a.idx, dfirst(GX + o, 1), a.idz * dfirst(GZ + o, S));
            const float r = rs[j];
            float q = 1.f, bq = 0.f;
            if (j >= nint) {
                const float E = Es[j], txv = ttx[ix], tzv = ttz[iz];
                q = (1.f - txv - tzv) * E;
                bq = 4.f * txv * tzv * E;
            }
            float out;
            if (!ADJ) {
                float D = lap[k] + div;
                if (own_src && k == ksrc) D += sv;
                const float u0 = F[o];
                w[k] = fmaf(r, D, fmaf(q, w[k], -bq * u0));
                out = u0 + w[k];
                if (a.store) Dfield[(size_t)n * npts + j] = D;
                if (rec[k] >= 0) a.traces[trfield + (size_t)rec[k] * a.nt + n + 1] = out;
            } else {
                const float Fv = (lap[k] - div) + av[k];
                w[k] = fmaf(q, w[k], fmaf(-bq, mu[k], Fv));
                mu[k] += w[k];
                out = r * mu[k];
            }
            F[o] = out;
            if (a.fs && iz >= 1 && iz <= 4) F[o - 2 * iz * S] = out;
        }
        __syncthreads();
    }
    if (ADJ) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (pos[k] >= 0) a.gpad[(size_t)field * npts + (pos[k] >> 16) * nxp + (pos[k] & 0xffff)] = acc[k];
    }
}

PmlArgs make_pml_args(const Plan& p) {
    PmlArgs a{};
    a.nzp = p.nzp;
    a.nxp = p.nxp;
    a.npts = p.npts;
    a.S = p.nxp + 8;
    a.fs = p.g.free_surface;
    a.nt = p.g.nt;
    a.ns = p.g.ns;
    a.nr = p.g.nr;
    a.idz = (float)(1.0 / p.g.dz);
    a.idx = (float)(1.0 / p.g.dx);
    a.idz2 = (float)(1.0 / (p.g.dz * p.g.dz));
    a.idx2 = (float)(1.0 / (p.g.dx * p.g.dx));
    a.src_scale = (float)(1.0 / (p.g.dx * p.g.dz));
    a.K = p.K;
    a.tx = p.pml_tx;
    a.tz = p.pml_tz;
    a.src_pt = p.src_pt;
    a.nz = p.g.nz;
    a.nx = p.g.nx;
    a.nb = p.g.nb;
    a.ztop = p.ztop;
    a.rec_slot = p.pml_rec;
    a.rec_invw = p.rec_invw;
    a.Dstore = p.Dstore;
    a.gpad = p.gpad;
    return a;
}

template <bool ADJ>
int pml_dispatch(const PmlArgs& a, int nf, hipStream_t st) {
    const size_t bytes = pml_lds_bytes(a.nzp, a.nxp);
    const int kc = (a.npts + kPmlThreads - 1) / kPmlThreads;
#define FWI_PML_CASE(KC)                                                                                         \
    if (kc <= KC) {                                                                                              \
        if (hipFuncSetAttribute((const void*)k_wave_pml<KC, ADJ>, hipFuncAttributeMaxDynamicSharedMemorySize,    \
                                (int)bytes) != hipSuccess)                                                       \
            return hip_ok(hipGetLastError());                                                                    \
        hipLaunchKernelGGL((k_wave_pml<KC, ADJ>), dim3(nf), dim3(kPmlThreads), bytes, st, a);                     \
        return hip_ok(hipGetLastError());                                                                        \
    }
    FWI_PML_CASE(2)
    FWI_PML_CASE(4)
    FWI_PML_CASE(kPmlMaxCells)
#undef FWI_PML_CASE
    return FWI_EINVAL;
}

}  // namespace

size_t pml_lds_bytes(int nzp, int nxp) {
    return ((size_t)3 * (nzp + 8) * (nxp + 8) + 2 * (size_t)nzp * nxp + 2 * (size_t)nxp + 2 * (size_t)nzp) *
           sizeof(float);
}

bool pml_fits(int nzp, int nxp) {
    return (long long)nzp * nxp <= (long long)kPmlMaxCells * kPmlThreads && nxp < (1 << 15) &&
           pml_lds_bytes(nzp, nxp) <= (size_t)kLdsBytes;
}

int launch_pml_forward(const Plan& p, int B, float* traces, const float* wavelet, int store, hipStream_t st) {
    PmlArgs a = make_pml_args(p);
    a.traces = traces;
    a.wavelet = wavelet;
    a.store = store;
    return pml_dispatch<false>(a, B * p.g.ns, st);
}

int launch_pml_adjoint(const Plan& p, int B, const float* adj, hipStream_t st) {
    PmlArgs a = make_pml_args(p);
    a.adj = adj;
    return pml_dispatch<true>(a, B * p.g.ns, st);
}

}  // namespace fwi
