// Body of the split LDS-resident time loop: G workgroups share one
// (sample, shot) field, workgroup g holding the band of padded rows
// [g H, g H + H) with 4-row halos above and below in LDS.
//
// Within a band the rows are cut in two kinds of register tiles that every
// thread (cg, .) owns side by side in column group cg (columns cg*X ..):
//   * a boundary tile: one of the 8 rows that neighbours need (band rows 0..3
//     and H-4..H-1), computed first in every step and published at once;
//   * an interior tile: PI consecutive rows of band rows 4 .. H-5.
// The neighbours' boundary rows are requested while the interior rows are
// computed and land in the halos of the next step's plane, so the exchange
// latency overlaps the larger part of the step.  Each published value carries
// its time level (SplitArgs), so a reader checks every value itself.
//
// Per point the arithmetic is the whole-field body's (lds_lap, the same
// leapfrog update, corrections and imaging), so results agree bit for bit.
#pragma once

#include "wave_lds_body.h"

namespace fwi {

__device__ __forceinline__ void split_put(unsigned long long* p, float v, unsigned level) {
    __hip_atomic_store(gmem(p), ((unsigned long long)level << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long split_get(const unsigned long long* p) {
    return __hip_atomic_load(gmem(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One register tile of R rows x X columns: per-point K, w, imaging sum and
// D slice, plus the source and receivers it holds.
template <int R, int X>
struct SplitTile {
    float K[R][X], w[R][X], acc[R][X], dc[R][X];
    float ax[X];
    float adjv[X];  // adjoint-source values of its receivers, a step ahead
    int rr[X];      // receiver index of each column on the receiver row, or -1
    int lz;         // first row, counted in the band
    int z;          // first row, padded field
    int src_j, src_c, rec_j;
    bool on;        // this thread owns the tile
};

template <int R, int X, bool ADJ>
__device__ __forceinline__ void split_tile_init(SplitTile<R, X>& t, const LdsArgs& a, bool on, int lz, int zs, int x0,
                                                int s, const float* __restrict__ Kb, const float* __restrict__ ax_g,
                                                const float* __restrict__ Dr, size_t trfield) {
    const int nxp = a.nxp, nzp = a.nzp;
    t.on = on;
    t.lz = lz;
    t.z = zs + lz;
    t.src_j = t.src_c = t.rec_j = -1;
#pragma unroll
    for (int c = 0; c < X; ++c) {
        const int x = x0 + c;
        t.ax[c] = (on && x < nxp) ? gmem(ax_g)[x] : 1.f;
        t.rr[c] = -1;
        t.adjv[c] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int z = t.z + j;
            const bool in = on && z < nzp && x < nxp;
            t.K[j][c] = in ? gmem(Kb)[z * nxp + x] : 0.f;
            t.w[j][c] = 0.f;
            t.acc[j][c] = 0.f;
            t.dc[j][c] = (ADJ && in) ? gmem(Dr)[j * nxp + c] : 0.f;  // the adjoint's first slice
        }
    }
    if (on) {
        const int sp = gmem(a.src_pt)[s];
        const int sz = sp / nxp, sx = sp - (sp / nxp) * nxp;
        if (sx >= x0 && sx < x0 + X && sz >= t.z && sz < t.z + R) {
            t.src_j = sz - t.z;
            t.src_c = sx - x0;
        }
        if (a.rec_row >= t.z && a.rec_row < t.z + R) {
            t.rec_j = a.rec_row - t.z;
#pragma unroll
            for (int c = 0; c < X; ++c) t.rr[c] = (x0 + c < nxp) ? gmem(a.rec_of_col)[x0 + c] : -1;
            if (!ADJ) {
#pragma unroll
                for (int c = 0; c < X; ++c)
                    if (t.rr[c] >= 0) gmem(a.traces)[trfield + (size_t)t.rr[c] * a.nt] = 0.f;
            } else {
                const int nsteps = a.nt - 1;
#pragma unroll
                for (int c = 0; c < X; ++c)
                    if (t.rr[c] >= 0) t.adjv[c] = gmem(a.adj)[trfield + (size_t)t.rr[c] * a.nt + nsteps];
            }
        }
    }
}

// Step m of one tile: its R rows of u^{n+1} into nxt, then the corrections
// of the points it owns (as the whole-field body orders them).  `Dt` is the
// tile corner in D slice 0 (Df: the field's slice 0); `mirror`: rows above
// padded row 0 reflect.  After
// row `issue_after` (if `fetch`) the X halo values at `src` (column c at
// src + c * ncg) are requested
// into hv, so that their latency overlaps the remaining rows.
template <int R, int X, bool ADJ, bool XEXACT, bool STORE>
__device__ __forceinline__ void split_tile_step(SplitTile<R, X>& t, const LdsArgs& a, const float* cur, float* nxt,
                                                const float* az_s, int x0, bool mirror, int m, float* Dt, float* Df,
                                                size_t trfield, const float (&wz)[4], const float (&wx)[4],
                                                int issue_after = -1, bool fetch = false,
                                                const unsigned long long* src = nullptr,
                                                unsigned long long* hv = nullptr) {
    const int S = a.S, nxp = a.nxp, nzp = a.nzp, npts = a.npts;
    const int nsteps = a.nt - 1;
    const float* cb = cur + (t.lz + 4) * S + x0 + 4;
    float* nb = nxt + (t.lz + 4) * S + x0 + 4;
    const FWI_AS_GLOBAL float* Dn = ADJ ? gmem(Dt) + (size_t)max(nsteps - 2 - m, 0) * npts : nullptr;
    FWI_AS_GLOBAL float* Dw = (!ADJ && STORE) ? gmem(Dt) + (size_t)m * npts : nullptr;
    // with exact columns, D goes through buffer accesses bounded by the field's
    // slice: rows past the field (last band) are dropped on store and read as 0,
    // so no per-point guard is needed
    float* sliceD = Df + (size_t)(ADJ ? max(nsteps - 2 - m, 0) : m) * npts;
    const __amdgpu_buffer_rsrc_t rsD =
        __builtin_amdgcn_make_buffer_rsrc(sliceD, (short)0, npts * (int)sizeof(float), kBufferRsrcWord3);
    const int offD = (t.z * nxp + x0) * (int)sizeof(float);
    float drec[X];
    if (ADJ && t.rec_j >= 0) {
#pragma unroll
        for (int c = 0; c < X; ++c) drec[c] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (j == t.rec_j) {
#pragma unroll
                for (int c = 0; c < X; ++c) drec[c] = t.dc[j][c];
            }
    }
    float win[R + 8][X];
#pragma unroll
    for (int q = 0; q < R + 8; ++q) {
        const float* rp = cb + (q - 4) * S;
        // even mirror above a reflecting top: padded row t.z + q - 4 < 0 reads row 4 - q - t.z
        if (q < 4 && mirror && t.z + q < 4) rp = cb + (4 - q - 2 * t.z) * S;
#pragma unroll
        for (int c = 0; c < X; ++c) win[q][c] = rp[c];
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const float* rp = cb + j * S;
        float xl[4], xh[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            xl[c] = rp[c - 4];
            xh[c] = rp[X + c];
        }
        const float azr = az_s[t.lz + j];
#pragma unroll
        for (int c = 0; c < X; ++c) {
            float xr[9], zc[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int cc = c + k - 4;
                xr[k] = cc < 0 ? xl[cc + 4] : (cc >= X ? xh[cc - X] : win[j + 4][cc]);
                zc[k] = win[j + k][c];
            }
            const float u0 = zc[4];
            const float D = lds_lap<ADJ>(zc, xr, wz[0], wz[1], wz[2], wz[3], wx[0], wx[1], wx[2], wx[3]);
            const float wn = fmaf(t.K[j][c], D, (t.ax[c] * azr) * t.w[j][c]);
            const float un = u0 + wn;
            t.w[j][c] = wn;
            nb[j * S + c] = un;
            if (ADJ) t.acc[j][c] = fmaf(un, t.dc[j][c], t.acc[j][c]);
            if (STORE && !ADJ) {
                if constexpr (XEXACT)
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(D), rsD,
                                                          offD + (j * nxp + c) * (int)sizeof(float), 0, 0);
                else if (t.z + j < nzp && x0 + c < nxp)
                    Dw[j * nxp + c] = D;
            }
        }
        if (ADJ) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < X; ++c)
                if constexpr (XEXACT)
                    t.dc[j][c] = __uint_as_float(
                        __builtin_amdgcn_raw_buffer_load_b32(rsD, offD + (j * nxp + c) * (int)sizeof(float), 0, 0));
                else
                    t.dc[j][c] = (t.z + j < nzp && x0 + c < nxp) ? Dn[j * nxp + c] : 0.f;
            __builtin_amdgcn_sched_barrier(0);
        }
        if (j == issue_after && fetch) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < X; ++c) hv[c] = split_get(src + c * a.ncg);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (ADJ && t.rec_j >= 0) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (j == t.rec_j) {
#pragma unroll
                for (int c = 0; c < X; ++c)
                    if (t.rr[c] >= 0) {
                        const float dv = t.K[j][c] * t.adjv[c] * a.rec_invw;
                        t.w[j][c] += dv;
                        nb[j * S + c] += dv;
                        t.acc[j][c] = fmaf(dv, drec[c], t.acc[j][c]);
                    }
            }
        if (m + 1 < nsteps) {
#pragma unroll
            for (int c = 0; c < X; ++c)
                t.adjv[c] = t.rr[c] >= 0 ? gmem(a.adj)[trfield + (size_t)t.rr[c] * a.nt + (nsteps - m - 1)] : 0.f;
        }
    }
    if (t.src_j >= 0) {
        if (!ADJ) {
            const float sv = gmem(a.wavelet)[m] * a.src_scale;
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int c = 0; c < X; ++c)
                    if (j == t.src_j && c == t.src_c) {
                        const float dv = t.K[j][c] * sv;
                        t.w[j][c] += dv;
                        nb[j * S + c] += dv;
                    }
        } else {
            const float sv = gmem(a.wavelet)[nsteps - 1 - m] * a.src_scale;
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int c = 0; c < X; ++c)
                    if (j == t.src_j && c == t.src_c) t.acc[j][c] = fmaf(nb[j * S + c], sv, t.acc[j][c]);
        }
    }
    if (!ADJ && t.rec_j >= 0) {
#pragma unroll
        for (int c = 0; c < X; ++c)
            if (t.rr[c] >= 0) gmem(a.traces)[trfield + (size_t)t.rr[c] * a.nt + m + 1] = nb[t.rec_j * S + c];
    }
}

template <int R, int X>
__device__ __forceinline__ void split_tile_gpad(const SplitTile<R, X>& t, const LdsArgs& a, int field, int x0) {
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
        for (int c = 0; c < X; ++c) {
            const int z = t.z + j, x = x0 + c;
            if (t.on && z < a.nzp && x < a.nxp) gmem(a.gpad)[(size_t)field * a.npts + z * a.nxp + x] = t.acc[j][c];
        }
}

// The whole workgroup calls this for band g of `field` (k_wave_split: 768
// threads with 2-row interior tiles, 512 otherwise; the batch kernel: 512);
// a.nstrip is the number of interior strips of PI rows, so the band has
// H = 8 + a.nstrip * PI rows and uses (2 (H + 8) S + H) floats of LDS.
// XEXACT: the column groups tile the padded width exactly (no column guards;
// rows past the field, in the last band, are always guarded).
template <int X, int PI, bool ADJ, bool XEXACT, bool STORE>
__device__ __forceinline__ void split_field(const LdsArgs a, const SplitArgs sp, const int field, const int g,
                                            const float* __restrict__ ax_g, const float* __restrict__ az_g,
                                            float* lds) {
    const int S = a.S, ncg = a.ncg;
    const int H = 8 + a.nstrip * PI;
    const int plane = (H + 8) * S;
    const int zs = g * H;
    float* az_s = lds + 2 * plane;
    const int b = field / a.ns;
    const int s = field - b * a.ns;
    const int tid = threadIdx.x;
    const int nxp = a.nxp, nzp = a.nzp, npts = a.npts;
    const int nsteps = a.nt - 1;

    for (int i = tid; i < 2 * plane; i += blockDim.x) lds[i] = 0.f;
    for (int i = tid; i < H; i += blockDim.x) az_s[i] = (zs + i < nzp) ? gmem(az_g)[zs + i] : 1.f;

    const int cg = tid % ncg;
    const int row = tid / ncg;  // boundary row 0..7 / interior strip / halo row
    const int x0 = cg * X;
    const bool has_b = row < 8;
    const bool has_i = row < a.nstrip;
    const int lb = row < 4 ? row : H - 8 + row;  // band row of the boundary tile
    const bool mirror = a.fs && g == 0;

    const float wz[4] = {FWI_W1 * a.idz2, FWI_W2 * a.idz2, FWI_W3 * a.idz2, FWI_W4 * a.idz2};
    const float wx[4] = {FWI_W1 * a.idx2, FWI_W2 * a.idx2, FWI_W3 * a.idx2, FWI_W4 * a.idx2};
    const size_t trfield = (size_t)field * a.nr * a.nt;
    const float* Kb = a.K + (size_t)b * npts;
    float* Dfield = a.Dstore + (size_t)field * nsteps * npts;
    // tile corners in D slice 0 (rows past the field are never dereferenced)
    float* Db = Dfield + (size_t)min(zs + lb, nzp - 1) * nxp + x0;
    float* Di = Dfield + (size_t)min(zs + 4 + row * PI, nzp - 1) * nxp + x0;
    const size_t last = (size_t)(nsteps - 1) * npts;

    SplitTile<1, X> tb;
    SplitTile<PI, X> ti;
    split_tile_init<1, X, ADJ>(tb, a, has_b, lb, zs, x0, s, Kb, ax_g, Db + last, trfield);
    split_tile_init<PI, X, ADJ>(ti, a, has_i, 4 + row * PI, zs, x0, s, Kb, ax_g, Di + last, trfield);

    // halo row this thread receives: row < 4 -> top halo row `row` from band g - 1's
    // last rows, 4..7 -> bottom halo row `row - 4` from band g + 1's first rows
    const bool recv = has_b && (row < 4 ? g > 0 : g < sp.G - 1);
    const size_t fb = (size_t)(field - sp.field0) * sp.G;
    const unsigned long long* src0 = sp.xchg;
    if (recv) {
        const size_t nbr = row < 4 ? ((fb + g - 1) * 2 + 1) : ((fb + g + 1) * 2 + 0);
        src0 = sp.xchg + nbr * 2 * 4 * sp.W + (size_t)(row & 3) * sp.W + cg;
    }
    const int halo_row = row < 4 ? row : H + row;  // LDS row of the received values
    // where this thread's boundary row goes, if a neighbour reads it
    const bool pub = has_b && (row < 4 ? g > 0 : g < sp.G - 1);
    unsigned long long* dst0 =
        sp.xchg + ((fb + g) * 2 + (row < 4 ? 0 : 1)) * 2 * 4 * sp.W + (size_t)(row & 3) * sp.W + cg;
    bool gave_up = false;
    __syncthreads();

    float* cur = lds;
    float* nxt = lds + plane;
    for (int m = 0; m < nsteps; ++m) {
        const unsigned level = (unsigned)m + 1;
        const size_t slot = (size_t)(level & 1) * 4 * sp.W;
        if (has_b) {
            split_tile_step<1, X, ADJ, XEXACT, STORE>(tb, a, cur, nxt, az_s, x0, mirror, m, Db, Dfield, trfield, wz,
                                                      wx);
            if (pub) {
                const float* nb = nxt + (lb + 4) * S + x0 + 4;
#pragma unroll
                for (int c = 0; c < X; ++c) split_put(dst0 + slot + c * ncg, nb[c], level);
            }
        }
        // the neighbours' rows are requested after the first interior row: by then
        // they have published theirs (boundary rows come first everywhere)
        unsigned long long hv[X];
        if (has_i) {
            split_tile_step<PI, X, ADJ, XEXACT, STORE>(ti, a, cur, nxt, az_s, x0, false, m, Di, Dfield, trfield, wz, wx, 0,
                                                      recv, src0 + slot, hv);
        } else if (recv) {
#pragma unroll
            for (int c = 0; c < X; ++c) hv[c] = split_get(src0 + slot + c * ncg);
        }
        if (recv) {
            // values that were not yet there are requested again together, so each
            // round costs one round trip whatever the number of stale values
            int spins = 0;
            for (;;) {
                bool stale = false;
#pragma unroll
                for (int c = 0; c < X; ++c) stale |= (unsigned)(hv[c] >> 32) != level;
                if (!stale || gave_up) break;
                if (++spins > kSplitSpinMax) {  // a neighbour is not running: flag it, never wait again
                    atomicOr(sp.err, 2);
                    gave_up = true;
                    break;
                }
#pragma unroll
                for (int c = 0; c < X; ++c)
                    if ((unsigned)(hv[c] >> 32) != level) hv[c] = split_get(src0 + slot + c * ncg);
            }
#pragma unroll
            for (int c = 0; c < X; ++c) nxt[halo_row * S + x0 + 4 + c] = __uint_as_float((unsigned)hv[c]);
        }
        __syncthreads();
        float* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (ADJ) {
        split_tile_gpad<1, X>(tb, a, field, x0);
        split_tile_gpad<PI, X>(ti, a, field, x0);
    }
}

}  // namespace fwi
