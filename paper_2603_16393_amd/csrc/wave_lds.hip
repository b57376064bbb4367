// LDS-resident time loop of the forward and adjoint sweeps (the scheme is
// described at the top of wave.hip).
//
// One 512-thread workgroup per (sample, shot) field keeps u^n and u^{n+1} of
// the whole padded field in LDS for all nt-1 steps, so HBM sees only the
// history of D = L u + s (written by the forward sweep, read by the adjoint)
// and the traces.  Thread (cg, strip) owns an X-column by P-row register tile
// (columns cg*X.., rows strip*P..): it keeps w, K and, in the adjoint, the
// imaging sum of its points in registers, loads its (P+8)-row column window
// once per step and only the 4 + 4 outer x-neighbours of each row, so a step
// costs (P+8)/P + 8/X LDS reads and one LDS write per point.
//
// LDS layout: two planes of R = nstrip*P + 8 rows x S = ncg*X + 8 columns with
// a 4-cell zero apron (padded cell (z, x) lives at LDS (z + 4, x + 4)), then
// the per-row sponge term ez[nstrip*P].  Rows and columns beyond the padded
// grid that round the tiles up are never written and stay zero.  All
// receivers sit on one padded row, so the owner of a receiver node records
// it (forward) or injects its adjoint source (adjoint) itself.
#include <algorithm>

#include "fwi_internal.h"

namespace fwi {

template <int X, int P, bool ADJ>
__global__ __launch_bounds__(kLdsThreads) void k_wave_lds(LdsArgs a, const float* __restrict__ ex_g,
                                                          const float* __restrict__ ez_g) {
    extern __shared__ float lds[];
    const int S = a.S;
    const int R = a.nstrip * P + 8;
    const int plane = R * S;
    float* ez_s = lds + 2 * plane;
    const int field = blockIdx.x;
    const int b = field / a.ns;
    const int s = field - b * a.ns;
    const int tid = threadIdx.x;
    const int npts = a.npts;
    const int nxp = a.nxp, nzp = a.nzp;
    const int nsteps = a.nt - 1;

    for (int i = tid; i < 2 * plane; i += blockDim.x) lds[i] = 0.f;
    for (int i = tid; i < a.nstrip * P; i += blockDim.x) ez_s[i] = (i < nzp) ? ez_g[i] : 0.f;

    const int cg = tid % a.ncg;
    const int strip = tid / a.ncg;
    const bool active = strip < a.nstrip;
    const int x0 = cg * X;
    const int z0 = strip * P;

    float Kr[P][X];
    float wr[P][X];
    float acc[P][X];
    float exv[X];
    int rr[X];
    int src_jc = -1;  // j * X + c of this field's source, if this thread owns it
    int rec_j = -1;   // tile row of the receiver row, if it crosses this tile
    const float* Kb = a.K + (size_t)b * npts;
#pragma unroll
    for (int c = 0; c < X; ++c) {
        const int x = x0 + c;
        exv[c] = (active && x < nxp) ? ex_g[x] : 0.f;
        rr[c] = -1;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int z = z0 + j;
            Kr[j][c] = (active && z < nzp && x < nxp) ? Kb[z * nxp + x] : 0.f;
            wr[j][c] = 0.f;
            acc[j][c] = 0.f;
        }
    }
    if (active) {
        if (!ADJ) {
            const int sp = a.src_pt[s];
            const int sz = sp / nxp, sx = sp - (sp / nxp) * nxp;
            if (sx >= x0 && sx < x0 + X && sz >= z0 && sz < z0 + P) src_jc = (sz - z0) * X + (sx - x0);
        }
        if (a.rec_row >= z0 && a.rec_row < z0 + P) {
            rec_j = a.rec_row - z0;
#pragma unroll
            for (int c = 0; c < X; ++c) rr[c] = (x0 + c < nxp) ? a.rec_of_col[x0 + c] : -1;
        }
    }
    const size_t trfield = (size_t)field * a.nr * a.nt;
    if (!ADJ) {
#pragma unroll
        for (int c = 0; c < X; ++c)
            if (rr[c] >= 0) a.traces[trfield + (size_t)rr[c] * a.nt] = 0.f;
    }
    const float* Dfield = a.Dstore + (size_t)field * nsteps * npts;
    __syncthreads();

    float* cur = lds;          // u^n
    float* nxt = lds + plane;  // receives u^{n+1}
    for (int m = 0; m < nsteps; ++m) {
        if (active) {
            float win[P + 8][X];
#pragma unroll
            for (int q = 0; q < P + 8; ++q) {
                int row = z0 - 4 + q;
                if (a.fs) row = row < 0 ? -row : row;  // even mirror above a reflecting top
                const float* rp = cur + (row + 4) * S + x0 + 4;
#pragma unroll
                for (int c = 0; c < X; ++c) win[q][c] = rp[c];
            }
            float inj[X];
#pragma unroll
            for (int c = 0; c < X; ++c) {
                inj[c] = 0.f;
                if (ADJ && rr[c] >= 0) inj[c] = a.adj[trfield + (size_t)rr[c] * a.nt + (nsteps - m)] * a.rec_invw;
            }
            const float srcv = (!ADJ && src_jc >= 0) ? a.wavelet[m] * a.src_scale : 0.f;
            float* Dw = (!ADJ && a.store) ? const_cast<float*>(Dfield) + (size_t)m * npts : nullptr;
            const float* Dr = ADJ ? Dfield + (size_t)(nsteps - 1 - m) * npts : nullptr;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int z = z0 + j;
                const float* rp = cur + (z + 4) * S + x0 + 4;
                float xr[X + 8];  // row z, columns x0-4 .. x0+X+3
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    xr[c] = rp[c - 4];
                    xr[X + 4 + c] = rp[X + c];
                }
#pragma unroll
                for (int c = 0; c < X; ++c) xr[c + 4] = win[j + 4][c];
                const float e_z = ez_s[z];
#pragma unroll
                for (int c = 0; c < X; ++c) {
                    const float u0 = win[j + 4][c];
                    const float lz = FWI_LAPD(u0, win[j][c], win[j + 1][c], win[j + 2][c], win[j + 3][c],
                                              win[j + 5][c], win[j + 6][c], win[j + 7][c], win[j + 8][c]);
                    const float lx = FWI_LAPD(u0, xr[c], xr[c + 1], xr[c + 2], xr[c + 3], xr[c + 5], xr[c + 6],
                                              xr[c + 7], xr[c + 8]);
                    float D = lz * a.idz2 + lx * a.idx2;
                    if (!ADJ && j * X + c == src_jc) D += srcv;
                    if (ADJ && j == rec_j) D += inj[c];
                    const float e = exv[c] + e_z;
                    const float wn = ((1.f - e) * wr[j][c] + Kr[j][c] * D) / (1.f + e);
                    const float un = u0 + wn;
                    wr[j][c] = wn;
                    const int x = x0 + c;
                    if (z < nzp && x < nxp) {
                        nxt[(z + 4) * S + x + 4] = un;
                        const int p = z * nxp + x;
                        if (Dw) Dw[p] = D;
                        if (ADJ) acc[j][c] += un * Dr[p];  // psi^{N-1-m} D^{N-2-m}
                        if (!ADJ && j == rec_j && rr[c] >= 0) a.traces[trfield + (size_t)rr[c] * a.nt + m + 1] = un;
                    }
                }
            }
        }
        __syncthreads();
        float* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (ADJ && active) {
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int c = 0; c < X; ++c) {
                const int z = z0 + j, x = x0 + c;
                if (z < nzp && x < nxp) a.gpad[(size_t)field * npts + z * nxp + x] = acc[j][c];
            }
    }
}

// Instantiated tiles (X columns, P rows): those whose forward and adjoint
// kernels fit the 256 VGPRs a 512-thread workgroup allows without (or, for
// (3, 12), with a small) spill.
#define FWI_LDS_TILES(M) \
    M(1, 8) M(1, 12) M(1, 16) M(1, 20) M(1, 24) \
    M(2, 8) M(2, 12)                            \
    M(3, 8) M(3, 12)                            \
    M(4, 8)

size_t lds_bytes(int X, int P, int ncg, int nstrip) {
    const size_t S = (size_t)ncg * X + 8;
    const size_t R = (size_t)nstrip * P + 8;
    return (2 * R * S + (size_t)nstrip * P) * sizeof(float);
}

// Chooses the instantiated tile with the fewest LDS operations per step
// (reads (P+8)/P + 8/X and one write per point, counting the rounding-up
// waste) among those that fit 512 threads and the LDS.
bool lds_choose_layout(int nzp, int nxp, int* Xo, int* Po, int* ncgo, int* nstripo) {
    double best = 1e300;
    bool found = false;
#define FWI_TRY(XX, PP)                                                                                   \
    {                                                                                                     \
        const int ncg = (nxp + XX - 1) / XX;                                                              \
        const int nstrip = (nzp + PP - 1) / PP;                                                           \
        if (ncg * nstrip <= kLdsThreads && lds_bytes(XX, PP, ncg, nstrip) <= (size_t)kLdsBytes) {         \
            const double pts = (double)ncg * XX * nstrip * PP;                                           \
            const double cost = pts * ((PP + 8.0) / PP + 8.0 / XX + 1.0);                                 \
            if (cost < best) {                                                                            \
                best = cost;                                                                              \
                *Xo = XX;                                                                                 \
                *Po = PP;                                                                                 \
                *ncgo = ncg;                                                                              \
                *nstripo = nstrip;                                                                        \
                found = true;                                                                             \
            }                                                                                             \
        }                                                                                                 \
    }
    FWI_LDS_TILES(FWI_TRY)
#undef FWI_TRY
    return found;
}

template <bool ADJ>
static int lds_dispatch(const LdsArgs& a, int nfields, hipStream_t st, const float* ex, const float* ez) {
    const size_t bytes = lds_bytes(a.X, a.P, a.ncg, a.nstrip);
#define FWI_CASE(XX, PP)                                                                                  \
    if (a.X == XX && a.P == PP) {                                                                         \
        auto kern = k_wave_lds<XX, PP, ADJ>;                                                              \
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);   \
        hipLaunchKernelGGL(kern, dim3(nfields), dim3(kLdsThreads), bytes, st, a, ex, ez);                 \
        return hip_ok(hipGetLastError());                                                                 \
    }
    FWI_LDS_TILES(FWI_CASE)
#undef FWI_CASE
    return FWI_EINVAL;
}

static LdsArgs make_lds_args(const Plan& p) {
    LdsArgs a{};
    a.nzp = p.nzp;
    a.nxp = p.nxp;
    a.npts = p.npts;
    a.X = p.lds_X;
    a.P = p.lds_P;
    a.ncg = p.lds_ncg;
    a.nstrip = p.lds_nstrip;
    a.S = a.ncg * a.X + 8;
    a.fs = p.g.free_surface ? 1 : 0;
    a.nt = p.g.nt;
    a.ns = p.g.ns;
    a.nr = p.g.nr;
    a.rec_row = p.rec_row;
    a.rec_invw = (p.g.free_surface && p.rec_row == 0) ? 2.f : 1.f;
    a.idz2 = (float)(1.0 / (p.g.dz * p.g.dz));
    a.idx2 = (float)(1.0 / (p.g.dx * p.g.dx));
    a.src_scale = (float)(1.0 / (p.g.dx * p.g.dz));
    a.K = p.K;
    a.src_pt = p.src_pt;
    a.rec_of_col = p.rec_of_col;
    a.Dstore = p.Dstore;
    a.gpad = p.gpad;
    return a;
}

int launch_lds_forward(const Plan& p, int B, float* traces, const float* wavelet, int store, hipStream_t st) {
    LdsArgs a = make_lds_args(p);
    a.traces = traces;
    a.wavelet = wavelet;
    a.store = store;
    return lds_dispatch<false>(a, B * p.g.ns, st, p.ex, p.ez);
}

int launch_lds_adjoint(const Plan& p, int B, const float* adj, const float* wavelet, hipStream_t st) {
    LdsArgs a = make_lds_args(p);
    a.adj = adj;
    a.wavelet = wavelet;
    return lds_dispatch<true>(a, B * p.g.ns, st, p.ex, p.ez);
}

}  // namespace fwi
