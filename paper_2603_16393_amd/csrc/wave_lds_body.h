// Body of the LDS-resident time loop of one (sample, shot) field, shared by
// the per-batch kernel (wave_lds.hip) and the persistent uneven-batch kernel
// (batch.hip).  The whole workgroup (kLdsThreads threads) must call it; it
// uses `lds` (lds_bytes(X, P, ncg, nstrip) bytes) and synchronises the
// workgroup internally.  See wave_lds.hip for the layout and the scheme.
#pragma once

#include "fwi_internal.h"

namespace fwi {

// L u at one point (without the source term) from the column values
// zc = u(z-4 .. z+4) and the row values xr = u(x-4 .. x+4), the weights with
// 1/h^2 folded in; zc[4] = xr[4] = u.  The forward sweep writes each pair as
// (u(+k) - u) - (u - u(-k)): equal bit for bit to (u(-k) - u) + (u(+k) - u),
// and its second difference is the first difference of the point k rows
// (columns) before, which the compiler then computes once for both points
// (10 % fewer VALU operations; in the adjoint sweep the longer live ranges
// cost more in scheduling than they save, so it keeps the plain form).  Every
// LDS-resident sweep evaluates exactly this, so their results agree bitwise.
template <bool ADJ>
__device__ __forceinline__ float lds_lap(const float (&zc)[9], const float (&xr)[9], float wz1, float wz2, float wz3,
                                         float wz4, float wx1, float wx2, float wx3, float wx4) {
    const float u0 = zc[4];
    float D;
    if (!ADJ) {
        D = wz1 * ((zc[5] - u0) - (u0 - zc[3]));
        D = fmaf(wz2, (zc[6] - u0) - (u0 - zc[2]), D);
        D = fmaf(wz3, (zc[7] - u0) - (u0 - zc[1]), D);
        D = fmaf(wz4, (zc[8] - u0) - (u0 - zc[0]), D);
        D = fmaf(wx1, (xr[5] - u0) - (u0 - xr[3]), D);
        D = fmaf(wx2, (xr[6] - u0) - (u0 - xr[2]), D);
        D = fmaf(wx3, (xr[7] - u0) - (u0 - xr[1]), D);
        D = fmaf(wx4, (xr[8] - u0) - (u0 - xr[0]), D);
    } else {
        D = wz1 * ((zc[3] - u0) + (zc[5] - u0));
        D = fmaf(wz2, (zc[2] - u0) + (zc[6] - u0), D);
        D = fmaf(wz3, (zc[1] - u0) + (zc[7] - u0), D);
        D = fmaf(wz4, (zc[0] - u0) + (zc[8] - u0), D);
        D = fmaf(wx1, (xr[3] - u0) + (xr[5] - u0), D);
        D = fmaf(wx2, (xr[2] - u0) + (xr[6] - u0), D);
        D = fmaf(wx3, (xr[1] - u0) + (xr[7] - u0), D);
        D = fmaf(wx4, (xr[0] - u0) + (xr[8] - u0), D);
    }
    return D;
}

template <int X, int P, bool ADJ, bool EXACT, bool STORE>
__device__ __forceinline__ void lds_field(const LdsArgs a, const int field, const float* __restrict__ ax_g,
                                          const float* __restrict__ az_g, float* lds) {
    const int S = a.S;
    const int R = a.nstrip * P + 8;
    const int plane = R * S;
    float* az_s = lds + 2 * plane;
    const int b = field / a.ns;
    const int s = field - b * a.ns;
    const int tid = threadIdx.x;
    const int npts = a.npts;
    const int nxp = a.nxp, nzp = a.nzp;
    const int nsteps = a.nt - 1;

    for (int i = tid; i < 2 * plane; i += blockDim.x) lds[i] = 0.f;
    for (int i = tid; i < a.nstrip * P; i += blockDim.x) az_s[i] = (i < nzp) ? gmem(az_g)[i] : 1.f;

    const int cg = tid % a.ncg;
    const int strip = tid / a.ncg;
    const bool active = strip < a.nstrip;
    const int x0 = cg * X;
    const int z0 = strip * P;
    const bool mirror_top = a.fs && z0 == 0;

    // weights of the Laplacian with the grid spacings folded in
    const float wz1 = FWI_W1 * a.idz2, wz2 = FWI_W2 * a.idz2, wz3 = FWI_W3 * a.idz2, wz4 = FWI_W4 * a.idz2;
    const float wx1 = FWI_W1 * a.idx2, wx2 = FWI_W2 * a.idx2, wx3 = FWI_W3 * a.idx2, wx4 = FWI_W4 * a.idx2;

    float Kr[P][X];
    float wr[P][X];
    float acc[P][X];
    float axv[X];
    int rr[X];
    int src_j = -1, src_c = -1;  // tile position of this field's source, if this thread owns it
    int rec_j = -1;              // tile row of the receiver row, if it crosses this tile
    const FWI_AS_GLOBAL float* Kb = gmem(a.K) + (size_t)b * npts;
#pragma unroll
    for (int c = 0; c < X; ++c) {
        const int x = x0 + c;
        axv[c] = (active && x < nxp) ? gmem(ax_g)[x] : 1.f;
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
        const int sp = gmem(a.src_pt)[s];
        const int sz = sp / nxp, sx = sp - (sp / nxp) * nxp;
        if (sx >= x0 && sx < x0 + X && sz >= z0 && sz < z0 + P) {
            src_j = sz - z0;
            src_c = sx - x0;
        }
        if (a.rec_row >= z0 && a.rec_row < z0 + P) {
            rec_j = a.rec_row - z0;
#pragma unroll
            for (int c = 0; c < X; ++c) rr[c] = (x0 + c < nxp) ? gmem(a.rec_of_col)[x0 + c] : -1;
        }
    }
    const size_t trfield = (size_t)field * a.nr * a.nt;
    if (!ADJ && rec_j >= 0) {
#pragma unroll
        for (int c = 0; c < X; ++c)
            if (rr[c] >= 0) gmem(a.traces)[trfield + (size_t)rr[c] * a.nt] = 0.f;
    }
    FWI_AS_GLOBAL float* Dfield = gmem(a.Dstore) + (size_t)field * nsteps * npts;
    FWI_AS_GLOBAL float* Drow0 = Dfield + z0 * nxp + x0;  // this thread's tile corner in one D slice
    __syncthreads();

    float* cur = lds;          // u^n
    float* nxt = lds + plane;  // receives u^{n+1}
    // Adjoint: dc holds the tile's slice of D for the current step.  As soon as
    // row j has been imaged its registers receive row j of the next step's
    // slice, so every load has a whole step to arrive and no extra registers are
    // needed.  The adjoint-source values of this thread's receivers (adjv) are
    // likewise requested a step ahead.
    float dc[P][X];
    float adjv[X];
    if (ADJ && active) {
        const FWI_AS_GLOBAL float* Dr = Drow0 + (size_t)(nsteps - 1) * npts;
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int c = 0; c < X; ++c) dc[j][c] = (EXACT || (z0 + j < nzp && x0 + c < nxp)) ? Dr[j * nxp + c] : 0.f;
#pragma unroll
        for (int c = 0; c < X; ++c)
            adjv[c] = (rec_j >= 0 && rr[c] >= 0) ? gmem(a.adj)[trfield + (size_t)rr[c] * a.nt + nsteps] : 0.f;
    }
    for (int m = 0; m < nsteps; ++m) {
        if (active) {
            const bool more = ADJ && m + 1 < nsteps;
            // next step's slice (the last step re-reads slice 0: harmless, and the
            // reload stays unconditional so old and new values never coexist)
            const FWI_AS_GLOBAL float* Dn = ADJ ? Drow0 + (size_t)max(nsteps - 2 - m, 0) * npts : nullptr;
            float drec[X];  // D at this thread's receivers for the current step
            if (ADJ && rec_j >= 0) {
#pragma unroll
                for (int c = 0; c < X; ++c) drec[c] = 0.f;
#pragma unroll
                for (int j = 0; j < P; ++j)
                    if (j == rec_j) {
#pragma unroll
                        for (int c = 0; c < X; ++c) drec[c] = dc[j][c];
                    }
            }
            float win[P + 8][X];
            const float* cb = cur + (z0 + 4) * S + x0 + 4;  // LDS cell of the tile corner
#pragma unroll
            for (int q = 0; q < P + 8; ++q) {
                const float* rp = cb + (q - 4) * S;
                if (q < 4 && mirror_top) rp = cb + (4 - q) * S;  // even mirror above a reflecting top
#pragma unroll
                for (int c = 0; c < X; ++c) win[q][c] = rp[c];
            }
            FWI_AS_GLOBAL float* Dw = (!ADJ && STORE) ? Drow0 + (size_t)m * npts : nullptr;
            float* nb_ = nxt + (z0 + 4) * S + x0 + 4;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const float* rp = cb + j * S;
                float xl[4], xh[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    xl[c] = rp[c - 4];
                    xh[c] = rp[X + c];
                }
                const float azr = az_s[z0 + j];
#pragma unroll
                for (int c = 0; c < X; ++c) {
                    // row neighbours x-4 .. x+4 of column c
                    float xr[9];
#pragma unroll
                    for (int k = 0; k < 9; ++k) {
                        const int cc = c + k - 4;
                        xr[k] = cc < 0 ? xl[cc + 4] : (cc >= X ? xh[cc - X] : win[j + 4][cc]);
                    }
                    const float u0 = win[j + 4][c];
                    float zc[9];
#pragma unroll
                    for (int k = 0; k < 9; ++k) zc[k] = win[j + k][c];
                    const float D = lds_lap<ADJ>(zc, xr, wz1, wz2, wz3, wz4, wx1, wx2, wx3, wx4);
                    const float wn = fmaf(Kr[j][c], D, (axv[c] * azr) * wr[j][c]);
                    const float un = u0 + wn;
                    wr[j][c] = wn;
                    nb_[j * S + c] = un;
                    if (ADJ) acc[j][c] = fmaf(un, dc[j][c], acc[j][c]);  // imaging: psi^{N-1-m} D^{N-2-m}
                    if (STORE && !ADJ) {
                        if (EXACT || (z0 + j < nzp && x0 + c < nxp)) Dw[j * nxp + c] = D;
                    }
                }
                if (ADJ) {
                    // keep the reload after the row that frees its registers
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int c = 0; c < X; ++c)
                        dc[j][c] = (EXACT || (z0 + j < nzp && x0 + c < nxp)) ? Dn[j * nxp + c] : 0.f;
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // point corrections of the owning threads
            if (ADJ && rec_j >= 0) {
                // adjoint sources a^{N-1-m}/w enter like the forward source: w += K inj
#pragma unroll
                for (int j = 0; j < P; ++j)
                    if (j == rec_j) {
#pragma unroll
                        for (int c = 0; c < X; ++c)
                            if (rr[c] >= 0) {
                                const float dv = Kr[j][c] * adjv[c] * a.rec_invw;
                                wr[j][c] += dv;
                                nb_[j * S + c] += dv;
                                acc[j][c] = fmaf(dv, drec[c], acc[j][c]);  // the injection's share of the imaging
                            }
                    }
                if (more) {
#pragma unroll
                    for (int c = 0; c < X; ++c)
                        adjv[c] = rr[c] >= 0 ? gmem(a.adj)[trfield + (size_t)rr[c] * a.nt + (nsteps - m - 1)] : 0.f;
                }
            }
            if (src_j >= 0) {
                if (!ADJ) {
                    const float sv = gmem(a.wavelet)[m] * a.src_scale;
#pragma unroll
                    for (int j = 0; j < P; ++j)
#pragma unroll
                        for (int c = 0; c < X; ++c)
                            if (j == src_j && c == src_c) {
                                const float dv = Kr[j][c] * sv;
                                wr[j][c] += dv;
                                nb_[j * S + c] += dv;
                            }
                } else {
                    // the source's share of D^{N-2-m}: acc += psi^{N-1-m} s^{N-2-m}
                    const float sv = gmem(a.wavelet)[nsteps - 1 - m] * a.src_scale;
#pragma unroll
                    for (int j = 0; j < P; ++j)
#pragma unroll
                        for (int c = 0; c < X; ++c)
                            if (j == src_j && c == src_c) acc[j][c] = fmaf(nb_[j * S + c], sv, acc[j][c]);
                }
            }
            if (!ADJ && rec_j >= 0) {
#pragma unroll
                for (int c = 0; c < X; ++c)
                    if (rr[c] >= 0) gmem(a.traces)[trfield + (size_t)rr[c] * a.nt + m + 1] = nb_[rec_j * S + c];
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
                if (z < nzp && x < nxp) gmem(a.gpad)[(size_t)field * npts + z * nxp + x] = acc[j][c];
            }
    }
}

}  // namespace fwi
