// LDS-resident time loop of the forward and adjoint sweeps (the scheme is
// described at the top of wave.hip).
//
// One 512-thread workgroup per (sample, shot) field keeps u^n and u^{n+1} of
// the whole padded field in LDS for all nt-1 steps, so HBM sees only the
// history of D = L u (written by the forward sweep, read by the adjoint) and
// the traces.  Thread (cg, strip) owns an X-column by P-row register tile
// (columns cg*X.., rows strip*P..): it keeps w, K and, in the adjoint, the
// imaging sum of its points in registers, loads its (P+8)-row column window
// once per step and only the 4 + 4 outer x-neighbours of each row, so a step
// costs (P+8)/P + 8/X LDS reads and one LDS write per point.
//
// The per-point loop is branch-free: the few points with a source, a receiver
// or an adjoint injection are corrected afterwards by their owning thread.
// The source term is left out of the stored D; the adjoint adds its
// correlation psi s at the source node itself.
//
// LDS layout: two planes of R = nstrip*P + 8 rows x S = ncg*X + 8 columns with
// a 4-cell zero apron (padded cell (z, x) lives at LDS (z + 4, x + 4)), then
// the per-row sponge factor az[nstrip*P].  Cells beyond the padded grid that
// round the tiles up have K = 0 and start at zero, so they remain zero even
// though they are written every step.
#include <algorithm>

#include "fwi_internal.h"

namespace fwi {

template <int X, int P, bool ADJ, bool EXACT, bool STORE>
__global__ __launch_bounds__(kLdsThreads) void k_wave_lds(LdsArgs a, const float* __restrict__ ax_g,
                                                          const float* __restrict__ az_g) {
    extern __shared__ float lds[];
    const int S = a.S;
    const int R = a.nstrip * P + 8;
    const int plane = R * S;
    float* az_s = lds + 2 * plane;
    const int field = blockIdx.x;
    const int b = field / a.ns;
    const int s = field - b * a.ns;
    const int tid = threadIdx.x;
    const int npts = a.npts;
    const int nxp = a.nxp, nzp = a.nzp;
    const int nsteps = a.nt - 1;

    for (int i = tid; i < 2 * plane; i += blockDim.x) lds[i] = 0.f;
    for (int i = tid; i < a.nstrip * P; i += blockDim.x) az_s[i] = (i < nzp) ? az_g[i] : 1.f;

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
    const float* Kb = a.K + (size_t)b * npts;
#pragma unroll
    for (int c = 0; c < X; ++c) {
        const int x = x0 + c;
        axv[c] = (active && x < nxp) ? ax_g[x] : 1.f;
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
        const int sp = a.src_pt[s];
        const int sz = sp / nxp, sx = sp - (sp / nxp) * nxp;
        if (sx >= x0 && sx < x0 + X && sz >= z0 && sz < z0 + P) {
            src_j = sz - z0;
            src_c = sx - x0;
        }
        if (a.rec_row >= z0 && a.rec_row < z0 + P) {
            rec_j = a.rec_row - z0;
#pragma unroll
            for (int c = 0; c < X; ++c) rr[c] = (x0 + c < nxp) ? a.rec_of_col[x0 + c] : -1;
        }
    }
    const size_t trfield = (size_t)field * a.nr * a.nt;
    if (!ADJ && rec_j >= 0) {
#pragma unroll
        for (int c = 0; c < X; ++c)
            if (rr[c] >= 0) a.traces[trfield + (size_t)rr[c] * a.nt] = 0.f;
    }
    float* Dfield = a.Dstore + (size_t)field * nsteps * npts;
    float* Drow0 = Dfield + z0 * nxp + x0;  // this thread's tile corner in one D slice
    __syncthreads();

    float* cur = lds;          // u^n
    float* nxt = lds + plane;  // receives u^{n+1}
    for (int m = 0; m < nsteps; ++m) {
        if (active) {
            // D^{N-2-m} of the tile is requested first so its latency overlaps the LDS work
            float dr[P][X];
            if (ADJ) {
                const float* Dr = Drow0 + (size_t)(nsteps - 1 - m) * npts;
#pragma unroll
                for (int j = 0; j < P; ++j)
#pragma unroll
                    for (int c = 0; c < X; ++c)
                        dr[j][c] = (EXACT || (z0 + j < nzp && x0 + c < nxp)) ? Dr[j * nxp + c] : 0.f;
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
            float* Dw = (!ADJ && STORE) ? Drow0 + (size_t)m * npts : nullptr;
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
                    float D = wz1 * ((win[j + 3][c] - u0) + (win[j + 5][c] - u0));
                    D = fmaf(wz2, (win[j + 2][c] - u0) + (win[j + 6][c] - u0), D);
                    D = fmaf(wz3, (win[j + 1][c] - u0) + (win[j + 7][c] - u0), D);
                    D = fmaf(wz4, (win[j][c] - u0) + (win[j + 8][c] - u0), D);
                    D = fmaf(wx1, (xr[3] - u0) + (xr[5] - u0), D);
                    D = fmaf(wx2, (xr[2] - u0) + (xr[6] - u0), D);
                    D = fmaf(wx3, (xr[1] - u0) + (xr[7] - u0), D);
                    D = fmaf(wx4, (xr[0] - u0) + (xr[8] - u0), D);
                    const float wn = fmaf(Kr[j][c], D, (axv[c] * azr) * wr[j][c]);
                    const float un = u0 + wn;
                    wr[j][c] = wn;
                    nb_[j * S + c] = un;
                    if (STORE && !ADJ) {
                        if (EXACT || (z0 + j < nzp && x0 + c < nxp)) Dw[j * nxp + c] = D;
                    }
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
                                const float dv = Kr[j][c] * a.adj[trfield + (size_t)rr[c] * a.nt + (nsteps - m)] *
                                                 a.rec_invw;
                                wr[j][c] += dv;
                                nb_[j * S + c] += dv;
                            }
                    }
            }
            if (ADJ) {
                // imaging: psi^{N-1-m} (read back from this thread's own LDS writes) times
                // D^{N-2-m}, whose loads were issued at the top of the step
#pragma unroll
                for (int j = 0; j < P; ++j)
#pragma unroll
                    for (int c = 0; c < X; ++c) acc[j][c] = fmaf(nb_[j * S + c], dr[j][c], acc[j][c]);
            }
            if (src_j >= 0) {
                if (!ADJ) {
                    const float sv = a.wavelet[m] * a.src_scale;
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
                    const float sv = a.wavelet[nsteps - 1 - m] * a.src_scale;
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
                    if (rr[c] >= 0) a.traces[trfield + (size_t)rr[c] * a.nt + m + 1] = nb_[rec_j * S + c];
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

// Instantiated tiles (X columns, P rows).  (3, 11) tiles the 110 x 150 padded
// field of a 70 x 70 model with a 40-cell sponge exactly.
#define FWI_LDS_TILES(M) \
    M(1, 8) M(1, 12) M(1, 16) M(1, 20) \
    M(2, 8) M(2, 12)                   \
    M(3, 8) M(3, 11) M(3, 12)          \
    M(4, 8)

size_t lds_bytes(int X, int P, int ncg, int nstrip) {
    const size_t S = (size_t)ncg * X + 8;
    const size_t R = (size_t)nstrip * P + 8;
    return (2 * R * S + (size_t)nstrip * P) * sizeof(float);
}

// Chooses the instantiated tile with the fewest LDS operations per step
// (reads (P+8)/P + 8/X and one write per point, counting the rounding-up
// waste) among those that fit 512 threads and the LDS.
bool lds_choose_layout(int nzp, int nxp, int req_X, int req_P, int* Xo, int* Po, int* ncgo, int* nstripo) {
    double best = 1e300;
    bool found = false;
#define FWI_TRY(XX, PP)                                                                                   \
    if ((req_X <= 0 || req_X == XX) && (req_P <= 0 || req_P == PP)) {                                     \
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

template <bool ADJ, bool STORE>
static int lds_dispatch(const LdsArgs& a, int nfields, hipStream_t st, const float* ax, const float* az) {
    const size_t bytes = lds_bytes(a.X, a.P, a.ncg, a.nstrip);
    const bool exact = a.ncg * a.X == a.nxp && a.nstrip * a.P == a.nzp;
#define FWI_CASE(XX, PP)                                                                                  \
    if (a.X == XX && a.P == PP) {                                                                         \
        auto kern = exact ? k_wave_lds<XX, PP, ADJ, true, STORE> : k_wave_lds<XX, PP, ADJ, false, STORE>; \
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);   \
        hipLaunchKernelGGL(kern, dim3(nfields), dim3(kLdsThreads), bytes, st, a, ax, az);                 \
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
    if (store) return lds_dispatch<false, true>(a, B * p.g.ns, st, p.ax, p.az);
    return lds_dispatch<false, false>(a, B * p.g.ns, st, p.ax, p.az);
}

int launch_lds_adjoint(const Plan& p, int B, const float* adj, const float* wavelet, hipStream_t st) {
    LdsArgs a = make_lds_args(p);
    a.adj = adj;
    a.wavelet = wavelet;
    return lds_dispatch<true, false>(a, B * p.g.ns, st, p.ax, p.az);
}

}  // namespace fwi
