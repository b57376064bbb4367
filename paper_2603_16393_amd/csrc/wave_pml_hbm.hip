// Sweeps of the PML (Sec. 2.1 absorbing boundary realised by a PML; Sec. 6.1:
// 6 grid points on the left, right and bottom, reflecting top) over fields
// kept in device memory: plan path 3, for grids too large for the
// LDS-resident PML sweeps of wave_pml.hip, histories that do not fit, and
// checkpointed gradients.  The scheme and its exact adjoint are those stated
// in wave_pml.hip (unsplit second-order form of a complex coordinate stretch,
// Grote and Sim 2010).

#include "fwi_internal.h"
#include "pml_stencil.h"

#include <algorithm>
#include <utility>

// No implicit fusing of a multiply and an add: this sweep must round every
// operation as the LDS-resident sweeps do.
#pragma clang fp contract(off)

namespace fwi {
namespace {

// HBM sweep (path 3): the fields stay in device memory, for grids too large
// for the LDS-resident sweeps and for checkpointed gradients.  The gathered
// field (u or y) is stored with the 4-cell border of the LDS planes,
// (nzp + 8) x (nxp + 8) per field, so a stencil never leaves its plane: the
// border holds zeros, or the even mirror rows above a reflecting top, written
// by the producer of each row.  The auxiliary fields of the layer cells are
// kept compact.  One launch per step: each tile evaluates Q (G) of the layer
// cells in it and in its 4-cell ring in LDS, then the time update of its
// cells.  Each cell undergoes the operations of the LDS-resident sweep in the
// same order, so the two give the same bits.
struct PmlHbmArgs {
    int nzp, nxp, npts;
    int S, plane;                 // bordered row stride nxp + 8 and plane size (nzp + 8) S
    int nz, nx, nb, ztop, fs;
    int zlo, zhi, dw;             // deep model cells (no Q within 4 cells): rows [zlo, zhi), columns [4, 4 + dw)
    int nt, ns, nr, nl;           // nl: layer cells
    float idz, idx, idz2, idx2, src_scale;
    const float* K;               // [B][npts] (v dt)^2
    const float* tx;              // [nxp]
    const float* tz;              // [nzp]
    const float* wavelet;         // [nt]
    const int* src_pt;            // [ns] padded index
    const int* rec_map;           // [npts] receiver of each padded cell, or -1
    int rec_z0, rec_z1;           // padded rows holding receivers (inclusive): rec_map is read only there
    const int* rec_pt;            // [nr]
    const float* rec_invw;        // [nr]
    float* traces;                // forward: [nf][nr][nt], or null (recomputation)
    const float* adj;             // adjoint: [nf][nr][nt]
    float* gpad;                  // adjoint: [nf][npts] imaging sums, padded order
};

// Index of layer cell (iz, ix) in the compact order of the auxiliary fields:
// row-major over the padded cells outside the model.
__device__ __forceinline__ int pml_layer_index(const PmlHbmArgs& a, int iz, int ix) {
    const int top = a.ztop * a.nxp, side = 2 * a.nb;
    if (iz < a.ztop) return iz * a.nxp + ix;
    if (iz < a.ztop + a.nz) return top + (iz - a.ztop) * side + (ix < a.nb ? ix : ix - a.nx);
    return top + a.nz * side + (iz - a.ztop - a.nz) * a.nxp + ix;
}

// Per-cell pieces, each written with the LDS-resident sweep's expressions in
// its order.  Global values come in as arguments: a kernel first issues all
// loads of a phase, then computes (a load inside the compute loop would be
// waited for in every iteration).

// Q (forward) or G (adjoint) of a layer cell from the gathered field around it
// (gp at the cell, row stride gs), its damping (txv, tzv) and its auxiliary
// values before the step (pxv, pzv); px1, pz1 receive them after the step.
template <bool ADJ>
__device__ __forceinline__ void pml_aux(const PmlHbmArgs& a, const float* gp, int gs, float txv, float tzv, float pxv,
                                        float pzv, float& ox, float& oz, float& px1, float& pz1) {
    const float gx = a.idx * dfirst(gp, 1);
    const float gz = a.idz * dfirst(gp, gs);
    const float cxv = 1.f / (1.f + txv), czv = 1.f / (1.f + tzv);
    if (!ADJ) {
        const float Qx = cxv * fmaf(tzv - txv, gx, pxv);
        const float Qz = czv * fmaf(txv - tzv, gz, pzv);
        px1 = 2.f * Qx - pxv;
        pz1 = 2.f * Qz - pzv;
        ox = Qx;
        oz = Qz;
    } else {
        const float Qx = 2.f * pxv - gx;
        const float Qz = 2.f * pzv - gz;
        px1 = cxv * Qx - pxv;
        pz1 = czv * Qz - pzv;
        ox = cxv * (tzv - txv) * Qx;
        oz = czv * (txv - tzv) * Qz;
    }
}

// Coefficients of cell (iz, ix) with (v dt)^2 = kv: r = kv E, and q, bq of the
// layer's update (1 and 0 in the model).
struct PmlCoef {
    float r, q, bq;
    bool deep;
};
__device__ __forceinline__ PmlCoef pml_coef(const PmlHbmArgs& a, float kv, float txv, float tzv, int iz, int ix) {
    PmlCoef c;
    const int zm = iz - a.ztop, xm = ix - a.nb;
    const bool model = zm >= 0 && zm < a.nz && xm >= 0 && xm < a.nx;
    c.deep = zm >= a.zlo && zm < a.zhi && xm >= 4 && xm < 4 + a.dw;
    const float E = 1.f / (1.f + txv + tzv);
    c.r = kv * E;
    c.q = 1.f;
    c.bq = 0.f;
    if (!model) {
        c.q = (1.f - txv - tzv) * E;
        c.bq = 4.f * txv * tzv * E;
    }
    return c;
}

__device__ __forceinline__ float pml_lap(const PmlHbmArgs& a, const float* c, int s) {
    const float c0 = c[0];
    const float lz = FWI_LAPD(c0, c[-4 * s], c[-3 * s], c[-2 * s], c[-s], c[s], c[2 * s], c[3 * s], c[4 * s]);
    const float lx = FWI_LAPD(c0, c[-4], c[-3], c[-2], c[-1], c[1], c[2], c[3], c[4]);
    return fmaf(a.idx2, lx, a.idz2 * lz);
}

__device__ __forceinline__ float pml_div(const PmlHbmArgs& a, const float* gx, const float* gz, int s) {
    return fmaf(a.idx, dfirst(gx, 1), a.idz * dfirst(gz, s));
}

__device__ __forceinline__ bool pml_in_layer(const PmlHbmArgs& a, int iz, int ix) {
    const int zm = iz - a.ztop, xm = ix - a.nb;
    return iz >= 0 && iz < a.nzp && ix >= 0 && ix < a.nxp && !(zm >= 0 && zm < a.nz && xm >= 0 && xm < a.nx);
}

__device__ __forceinline__ int pml_rec_of(const PmlHbmArgs& a, int iz, int p) {
    return (iz >= a.rec_z0 && iz <= a.rec_z1) ? a.rec_map[p] : -1;
}

constexpr int kPtX = 64, kPtZ = 16;                  // tile
constexpr int kPqX = kPtX + 8, kPqZ = kPtZ + 8;      // Q region: the tile and a 4-cell ring

// Position of the n-th (from 0) set bit of m, for n < popcount(m).
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int n) {
    int pos = 0;
    unsigned int w = (unsigned int)m;
    int c = __popc(w);
    if (n >= c) {
        n -= c;
        pos = 32;
        w = (unsigned int)(m >> 32);
    }
#pragma unroll
    for (int h = 16; h >= 1; h >>= 1) {
        c = __popc(w & ((1u << h) - 1u));
        if (n >= c) {
            n -= c;
            pos += h;
            w >>= h;
        }
    }
    return pos;
}

// Damping of the staged columns and rows (thread t holds column t and row t;
// a staged window is at most 80 columns and 32 rows), loaded with the
// staging loads from clamped addresses and stored to txs, tzs after them:
// zero past the grid.
template <int HW>
__device__ __forceinline__ void pml_stage_damping_load(const PmlHbmArgs& a, int zt, int x0, float& dxv, float& dzv) {
    const int t = threadIdx.x;
    dxv = a.tx[min(max(x0 - HW + t, 0), a.nxp - 1)];
    dzv = a.tz[min(max(zt - HW + t, 0), a.nzp - 1)];
}
template <int HW>
__device__ __forceinline__ void pml_stage_damping_store(const PmlHbmArgs& a, int zt, int x0, float dxv, float dzv,
                                                        float* txs, float* tzs) {
    constexpr int GX = kPtX + 2 * HW, GZ = kPtZ + 2 * HW;
    static_assert(GX <= 256 && GZ <= 256, "one damping value per thread");
    const int t = threadIdx.x, ix = x0 - HW + t, iz = zt - HW + t;
    if (t < GX) txs[t] = ix >= 0 && ix < a.nxp ? dxv : 0.f;
    if (t < GZ) tzs[t] = iz >= 0 && iz < a.nzp ? dzv : 0.f;
}

// Stages the gathered field of the tile and an HW-cell ring into fw (row
// stride WX, offset off rows and columns), from the bordered plane (zero past
// its border), and the damping of those columns and rows into txs, tzs (zero
// past the grid).
template <int HW, int WX, bool DAMP>
__device__ __forceinline__ void pml_stage(const PmlHbmArgs& a, const float* __restrict__ Ff, float* fw, float* txs,
                                          float* tzs, int zt, int x0, int off) {
    constexpr int GX = kPtX + 2 * HW, GZ = kPtZ + 2 * HW, N = (GZ * GX + 255) / 256;
    float v[N];  // all loads of a thread first (clamped addresses), then the stores
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int i = threadIdx.x + k * 256;
        const int r = i / GX, c = i - (i / GX) * GX;
        const int iz = zt - HW + r, ix = x0 - HW + c;
        const bool in = i < GZ * GX && iz >= -4 && iz < a.nzp + 4 && ix >= -4 && ix < a.nxp + 4;
        const float t = Ff[in ? (size_t)(iz + 4) * a.S + ix + 4 : 0];
        v[k] = in ? t : 0.f;
    }
    float dxv = 0.f, dzv = 0.f;
    if (DAMP) pml_stage_damping_load<HW>(a, zt, x0, dxv, dzv);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int i = threadIdx.x + k * 256;
        const int r = i / GX, c = i - (i / GX) * GX;
        if (i < GZ * GX) fw[(r + off) * WX + c + off] = v[k];
    }
    if (DAMP) pml_stage_damping_store<HW>(a, zt, x0, dxv, dzv, txs, tzs);
}

// Without DAMP (plain tiles: the staged cells are model cells, or outside the
// grid), the damping is not staged; in the adjoint's gathered field E = 1 /
// (1 + 0 + 0) = 1 there, so y = K mu has the bits of (K E) mu.

// The adjoint's gathered field y = r mu of the tile and an HW-cell ring, from
// mu and K (r = (v dt)^2 E, the product every sweep forms), into fw; rows
// above a reflecting top are the even mirror images, cells past the grid (and
// more than 4 rows above a reflecting top) zero.  Also the damping of the
// staged columns and rows into txs, tzs.
template <int HW, int WX, bool DAMP>
__device__ __forceinline__ void pml_stage_y(const PmlHbmArgs& a, const float* __restrict__ Mf,
                                            const float* __restrict__ Kb, float* fw, float* txs, float* tzs, int zt,
                                            int x0) {
    constexpr int GX = kPtX + 2 * HW, GZ = kPtZ + 2 * HW, N = (GZ * GX + 255) / 256;
    float kv[N], mv[N], tv[N], zv[N];  // all loads of a thread first (clamped addresses), then the products
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int i = threadIdx.x + k * 256;
        const int r = i / GX, c = i - (i / GX) * GX;
        const int iz = zt - HW + r, ix = x0 - HW + c;
        const int cz = a.fs && iz < 0 ? -iz : iz;
        const bool in = i < GZ * GX && iz >= -4 && cz >= 0 && cz < a.nzp && ix >= 0 && ix < a.nxp;
        const int zz = in ? cz : 0, xx = in ? ix : 0;
        const int p = zz * a.nxp + xx;
        kv[k] = Kb[p];
        mv[k] = Mf[p];
        if (DAMP) {
            tv[k] = a.tx[xx];
            zv[k] = a.tz[zz];
        }
        if (!in) mv[k] = 0.f;
    }
    float dxv = 0.f, dzv = 0.f;
    if (DAMP) pml_stage_damping_load<HW>(a, zt, x0, dxv, dzv);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int i = threadIdx.x + k * 256;
        // formed for every k (clamped loads), stored where the window has the cell: a conditional product
        // lets the compiler move its loads into the condition, where they would be waited for one by one
        float y;
        if (DAMP) {
            const float E = 1.f / (1.f + tv[k] + zv[k]);
            y = (kv[k] * E) * mv[k];
        } else {
            y = kv[k] * mv[k];  // (K E) mu with E = 1
        }
        if (i < GZ * GX) fw[i] = y;
    }
    if (DAMP) pml_stage_damping_store<HW>(a, zt, x0, dxv, dzv, txs, tzs);
}

// One time step on a 64 x 16 tile of one field (block: 64 columns x 4 strips
// of 4 rows; grid: the tiles of one class from a host list x fields, XCD-aware
// order).
// Forward: F = u^n and Fn = u^{n+1} (bordered planes), W = w, Dst = D^n slice
// (or null).  Adjoint: F = mu^{n+1} and Fn = mu^n ([nf][npts]; the gathered
// field y = r mu is formed while staging), W = nu, Dst = D^n.
// Pin / Pout: auxiliary fields before / after the step, [nf][2][nl] each
// (psi or phi, x then z); two buffers, because a tile also evaluates the Q
// (G) values of the layer cells in its 4-cell ring, from their values before
// the step, while the owning tile replaces them.  Plain tiles (LAYER false:
// no layer cell within 4 cells, rows past a reflecting top being mirror
// images of model rows) stage u with a 4-cell ring and run the leapfrog (their
// cells and rings are model cells: no damping is staged, E = 1); layer
// tiles stage an 8-cell ring and keep Q (G) of the tile and its ring in LDS,
// zero outside the layer and the grid, odd across a reflecting top.  The two
// classes are separate launches so that the plain tiles, most of the grid,
// hold only their 7 KB of LDS.
template <bool ADJ, bool LAYER>
__global__ void __launch_bounds__(256) k_pml_hbm_tile(const PmlHbmArgs a, const int* __restrict__ tiles, int n,
                                                      const float* __restrict__ F, float* __restrict__ Fn,
                                                      const float* __restrict__ Pin, float* __restrict__ Pout,
                                                      float* __restrict__ W, float* __restrict__ Dst, size_t dstride) {
    constexpr int HW = LAYER ? 8 : 4;  // staged ring
    constexpr int FX = kPtX + 2 * HW, FZ = kPtZ + 2 * HW;
    __shared__ float fw[FZ * FX];
    __shared__ float gxs[LAYER ? kPqZ * kPqX : 1];
    __shared__ float gzs[LAYER ? kPqZ * kPqX : 1];
    __shared__ float txs[FX], tzs[FZ];
    const TileIdx ti = tile_of_block();
    const int code = tiles[ti.tx];
    const int f = ti.field, x0 = (code & 0xffff) * kPtX, zt = (code >> 16) * kPtZ;
    const int b = f / a.ns, s = f - (f / a.ns) * a.ns;
    // the thread's 4 cells of the update (column tx, rows 4 ts .. 4 ts + 3 of the tile): their loads go out
    // before the staging, since no block writes what another block reads of them (column clamped, so that
    // the threads past the grid's last column load too); the adjoint's layer tiles issue them after the Q
    // phase instead, since their staging holds 40 values per thread and both would cost occupancy
    constexpr bool EARLY = !(ADJ && LAYER);
    const int tx = threadIdx.x & 63, ts = threadIdx.x >> 6;
    const int ix = x0 + tx;
    float kv[4], wv[4], mv[4], gv[4], dv[4];
    int rv[4];  // receiver of each cell, or -1
    auto load_update = [&]() {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int iz = min(zt + ts * 4 + j, a.nzp - 1);
            const int p = iz * a.nxp + min(ix, a.nxp - 1);
            const size_t fp = (size_t)f * a.npts + p;
            kv[j] = a.K[(size_t)b * a.npts + p];
            wv[j] = W[fp];
            rv[j] = pml_rec_of(a, iz, p);
            if (ADJ) {
                mv[j] = F[fp];
                gv[j] = a.gpad[fp];
                dv[j] = Dst[(size_t)f * dstride + p];
            }
        }
    };
    if (EARLY) load_update();
    // Layer tiles: the layer cells of the Q region are a small part of it (a frame nb cells wide), so each wave
    // lists those among its candidates (chunk k: region cells wave base + k * 256 + lane) by ballots and
    // evaluates Q (G) of the listed cells only, two per lane at a time; the other cells of gxs, gzs hold zero.
    constexpr int NQ = (kPqZ * kPqX + 255) / 256;
    const int lane = threadIdx.x & 63, wbase = threadIdx.x & ~63;
    unsigned long long qm[NQ];  // layer cells among the wave's candidates of chunk k
    int qc[NQ + 1];             // listed cells in the chunks before k
    if (LAYER) {
        qc[0] = 0;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int i = threadIdx.x + k * 256;
            const int r = i / kPqX, c = i - (i / kPqX) * kPqX;
            const int iz = zt - 4 + r, ix = x0 - 4 + c;
            const int cz = a.fs && iz < 0 ? -iz : iz;
            qm[k] = __ballot(i < kPqZ * kPqX && pml_in_layer(a, cz, ix));
            qc[k + 1] = qc[k] + __popcll(qm[k]);
        }
        for (int i = threadIdx.x; i < kPqZ * kPqX; i += 256) {
            gxs[i] = 0.f;
            gzs[i] = 0.f;
        }
    }
    if (ADJ)
        pml_stage_y<HW, FX, LAYER>(a, F + (size_t)f * a.npts, a.K + (size_t)b * a.npts, fw, txs, tzs, zt, x0);
    else
        pml_stage<HW, FX, LAYER>(a, F + (size_t)f * a.plane, fw, txs, tzs, zt, x0, 0);
    __syncthreads();
    if (LAYER) {
        const size_t pf = (size_t)f * 2 * a.nl;
        const int total = qc[NQ];
        for (int t0 = 0; t0 < total; t0 += 128) {
            int iv[2];
            float pxv[2], pzv[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = t0 + u * 64 + lane;  // entry t of the wave's list
                int k = 0;
#pragma unroll
                for (int kk = 1; kk < NQ; ++kk) k += t >= qc[kk];
                unsigned long long m = qm[0];
                int base = 0;
#pragma unroll
                for (int kk = 1; kk < NQ; ++kk)
                    if (k == kk) {
                        m = qm[kk];
                        base = qc[kk];
                    }
                const int i = wbase + k * 256 + nth_set_bit(m, t - base);
                iv[u] = t < total ? i : -1;
                const int r = i / kPqX, c = i - (i / kPqX) * kPqX;
                const int iz = zt - 4 + r, ix = x0 - 4 + c;
                const int cz = a.fs && iz < 0 ? -iz : iz;
                // a listed cell exists, so the field has layer cells; past the list, the field's first one
                const int l = t < total ? pml_layer_index(a, cz, ix) : 0;
                pxv[u] = Pin[pf + l];
                pzv[u] = Pin[pf + a.nl + l];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int i = iv[u];
                if (i < 0) continue;
                const int r = i / kPqX, c = i - (i / kPqX) * kPqX;
                const int iz = zt - 4 + r, ix = x0 - 4 + c;
                // rows above a reflecting top hold the odd mirror of Q_z (G_z) of the layer cells below
                const bool mirror = a.fs && iz < 0;
                const int cz = mirror ? -iz : iz;
                float ox, oz, px1, pz1;
                pml_aux<ADJ>(a, fw + (cz - zt + HW) * FX + (ix - x0 + HW), FX, txs[ix - x0 + HW], tzs[cz - zt + HW],
                             pxv[u], pzv[u], ox, oz, px1, pz1);
                if (!mirror && r >= 4 && r < 4 + kPtZ && c >= 4 && c < 4 + kPtX) {
                    const int l = pml_layer_index(a, cz, ix);
                    Pout[pf + l] = px1;
                    Pout[pf + a.nl + l] = pz1;
                }
                if (mirror) {
                    ox = 0.f;
                    oz = -oz;
                }
                gxs[i] = ox;
                gzs[i] = oz;
            }
        }
        __syncthreads();
    }
    if (!EARLY) load_update();
    if (ix >= a.nxp) return;
    const int sp = a.src_pt[s];
    const float srcv = ADJ ? 0.f : a.wavelet[n] * a.src_scale;
    float av[4];  // adjoint: sources of the receiver cells, loaded before the update's first store
    if (ADJ) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            av[j] = rv[j] >= 0 ? a.adj[((size_t)f * a.nr + rv[j]) * a.nt + n] * a.rec_invw[rv[j]] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int lz = ts * 4 + j;
        const int iz = zt + lz;
        if (iz >= a.nzp) break;
        const int p = iz * a.nxp + ix;
        const float* c = fw + (lz + HW) * FX + tx + HW;
        const float c0 = c[0];
        const float lap = pml_lap(a, c, FX);
        PmlCoef pc;
        if (LAYER) {
            pc = pml_coef(a, kv[j], txs[tx + HW], tzs[lz + HW], iz, ix);
        } else {  // a model cell with both damping values 0: E = 1, so r = K, q = 1, bq = 0
            pc.r = kv[j];
            pc.q = 1.f;
            pc.bq = 0.f;
            pc.deep = true;
        }
        float div = 0.f;  // Q (G) is zero within 4 cells of a deep cell, and in a tile whose ring has no layer
        if (LAYER && !pc.deep) {
            const int q = (lz + 4) * kPqX + tx + 4;
            div = pml_div(a, gxs + q, gzs + q, kPqX);
        }
        const size_t fp = (size_t)f * a.npts + p;
        const int rec = rv[j];
        const size_t tr = ((size_t)f * a.nr + (rec >= 0 ? rec : 0)) * a.nt;
        float out = 0.f;
        if (!ADJ) {
            float D = lap + div;
            if (p == sp) D += srcv;
            const float w = fmaf(pc.r, D, fmaf(pc.q, wv[j], -pc.bq * c0));
            W[fp] = w;
            out = c0 + w;
            if (Dst) Dst[(size_t)f * dstride + p] = D;
            if (rec >= 0 && a.traces) a.traces[tr + n + 1] = out;
        } else {
            a.gpad[fp] = fmaf(c0, dv[j], gv[j]);  // imaging: y^{n+1} D^n
            const float Fv = (lap - div) + av[j];
            const float w = fmaf(pc.q, wv[j], fmaf(-pc.bq, mv[j], Fv));
            W[fp] = w;
            Fn[fp] = mv[j] + w;
        }
        if (!ADJ) {
            const size_t o = (size_t)f * a.plane + (size_t)(iz + 4) * a.S + ix + 4;
            Fn[o] = out;
            if (a.fs && iz >= 1 && iz <= 4) Fn[o - 2 * iz * a.S] = out;
        }
    }
}

// Receivers at the start of a sweep (grid: receivers x fields).  Forward:
// sample 0 of every trace is u^0 = 0.  Adjoint: mu^{N-1} = a^{N-1} / w at the
// receivers and nu^{N-1} = mu^{N-1} (the other cells are zero).
template <bool ADJ>
__global__ void k_pml_hbm_start(const PmlHbmArgs a, float* __restrict__ W, float* __restrict__ MU) {
    const int rcv = blockIdx.x * 256 + threadIdx.x;
    if (rcv >= a.nr) return;
    const int f = blockIdx.y;
    const size_t tr = ((size_t)f * a.nr + rcv) * a.nt;
    if (!ADJ) {
        a.traces[tr] = 0.f;
        return;
    }
    const size_t fp = (size_t)f * a.npts + a.rec_pt[rcv];
    const float mu = a.adj[tr + a.nt - 1] * a.rec_invw[rcv];
    W[fp] = mu;
    MU[fp] = mu;
}

// Saves (SAVE) or restores the forward state of every field at checkpoint
// `seg`: the bordered u plane, w, and the layer's psi.
// ckpt = [max fields][nseg][plane + npts + 2 nl].
template <bool SAVE>
__global__ void k_pml_hbm_ckpt(float* __restrict__ ckpt, float* __restrict__ F, float* __restrict__ W,
                               float* __restrict__ PS, int nf, int nseg, int seg, int plane, int npts, int nl) {
    const size_t per = (size_t)plane + npts + 2 * (size_t)nl;
    const size_t total = (size_t)nf * per;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t f = i / per, e = i - (i / per) * per;
        float* x = e < (size_t)plane ? F + f * plane + e
                   : e < (size_t)plane + npts ? W + f * npts + (e - plane)
                                              : PS + f * 2 * nl + (e - plane - npts);
        float* c = ckpt + (f * nseg + seg) * per + e;
        if (SAVE)
            *c = *x;
        else
            *x = *c;
    }
}

PmlHbmArgs make_pml_hbm_args(const Plan& p) {
    PmlHbmArgs a{};
    a.nzp = p.nzp;
    a.nxp = p.nxp;
    a.npts = p.npts;
    a.S = p.nxp + 8;
    a.plane = (p.nzp + 8) * a.S;
    a.nz = p.g.nz;
    a.nx = p.g.nx;
    a.nb = p.g.nb;
    a.ztop = p.ztop;
    a.fs = p.g.free_surface;
    const PmlOrder ord(p.g.nz, p.g.nx, p.g.nb, p.g.free_surface);
    a.zlo = ord.zlo;
    a.zhi = ord.zhi;
    a.dw = ord.dw;
    a.nt = p.g.nt;
    a.ns = p.g.ns;
    a.nr = p.g.nr;
    a.nl = p.pml_nl;
    a.idz = (float)(1.0 / p.g.dz);
    a.idx = (float)(1.0 / p.g.dx);
    a.idz2 = (float)(1.0 / (p.g.dz * p.g.dz));
    a.idx2 = (float)(1.0 / (p.g.dx * p.g.dx));
    a.src_scale = (float)(1.0 / (p.g.dx * p.g.dz));
    a.K = p.K;
    a.tx = p.pml_tx;
    a.tz = p.pml_tz;
    a.wavelet = p.wav;
    a.src_pt = p.src_pt;
    a.rec_map = p.rec_map;
    a.rec_z0 = p.rec_z0;
    a.rec_z1 = p.rec_z1;
    a.rec_pt = p.rec_pt;
    a.rec_invw = p.rec_invw;
    a.gpad = p.gpad;
    return a;
}

// State buffers of the HBM sweep, offsets fixed by max_batch.
struct PmlHbmState {
    float *F0, *F1, *W, *P0, *P1;      // forward: u planes (ping-pong), w, psi (ping-pong)
    float *M0, *M1, *NU, *H0, *H1;     // adjoint: mu (ping-pong), nu, phi (ping-pong)
};

PmlHbmState pml_hbm_state(const Plan& p) {
    const size_t mf = (size_t)p.max_batch * p.g.ns;
    const size_t plane = (size_t)(p.nzp + 8) * (p.nxp + 8), npts = (size_t)p.npts, nl2 = 2 * (size_t)p.pml_nl;
    PmlHbmState s{};
    s.F0 = p.state;
    s.F1 = s.F0 + mf * plane;
    s.W = s.F1 + mf * plane;
    s.P0 = s.W + mf * npts;
    s.P1 = s.P0 + mf * nl2;
    s.M0 = p.astate;
    s.M1 = s.M0 + mf * npts;
    s.NU = s.M1 + mf * npts;
    s.H0 = s.NU + mf * npts;
    s.H1 = s.H0 + mf * nl2;
    return s;
}

int hbm_grid(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

// One step over all tiles: the plain tiles, then the layer tiles (independent launches within a step).
template <bool ADJ>
void pml_hbm_step(const Plan& p, const PmlHbmArgs& a, int nf, int n, const float* F, float* Fn, const float* Pin,
                  float* Pout, float* W, float* D, size_t dstride, hipStream_t st) {
    if (p.pml_ntp > 0)
        hipLaunchKernelGGL((k_pml_hbm_tile<ADJ, false>), dim3(p.pml_ntp, 1, nf), dim3(256), 0, st, a, p.pml_tiles, n,
                           F, Fn, Pin, Pout, W, D, dstride);
    if (p.pml_ntl > 0)
        hipLaunchKernelGGL((k_pml_hbm_tile<ADJ, true>), dim3(p.pml_ntl, 1, nf), dim3(256), 0, st, a,
                           p.pml_tiles + p.pml_ntp, n, F, Fn, Pin, Pout, W, D, dstride);
}

// Enqueues the whole forward sweep of B samples on st (reads p.wav, writes p.trace_buf; keeps the history of D
// or the checkpoints when keep is set).
void pml_hbm_enqueue_forward(Plan& p, int B, int keep, hipStream_t st) {
    const int nf = B * p.g.ns;
    PmlHbmArgs a = make_pml_hbm_args(p);
    a.traces = p.trace_buf;
    PmlHbmState s = pml_hbm_state(p);
    const size_t plane = (size_t)a.plane, npts = (size_t)p.npts, nl2 = 2 * (size_t)p.pml_nl;
    launch_fill(s.F0, nf * plane, 0.f, st);
    launch_fill(s.F1, nf * plane, 0.f, st);
    launch_fill(s.W, nf * npts, 0.f, st);
    launch_fill(s.P0, nf * nl2, 0.f, st);
    launch_fill(s.P1, nf * nl2, 0.f, st);
    hipLaunchKernelGGL(k_pml_hbm_start<false>, dim3((p.g.nr + 255) / 256, nf), dim3(256), 0, st, a, nullptr,
                       nullptr);
    const int nsteps = p.g.nt - 1;
    const bool full = keep && p.store_mode == 0, ck = keep && p.store_mode == 1;
    const size_t dstride = (size_t)nsteps * npts;
    float *F0 = s.F0, *F1 = s.F1, *P0 = s.P0, *P1 = s.P1;
    for (int n = 0; n < nsteps; ++n) {
        if (ck && n % p.ckpt_every == 0)
            hipLaunchKernelGGL(k_pml_hbm_ckpt<true>, dim3(hbm_grid(nf * (plane + npts + nl2))), dim3(256), 0, st,
                               p.ckpt, F0, s.W, P0, nf, p.nseg, n / p.ckpt_every, (int)plane, (int)npts, p.pml_nl);
        pml_hbm_step<false>(p, a, nf, n, F0, F1, P0, P1, s.W, full ? p.Dstore + (size_t)n * npts : nullptr, dstride,
                            st);
        std::swap(F0, F1);
        std::swap(P0, P1);
    }
}

// Enqueues the whole adjoint sweep (reads p.adj_buf, p.wav; writes p.gpad).
void pml_hbm_enqueue_adjoint(Plan& p, int B, hipStream_t st) {
    const int nf = B * p.g.ns;
    PmlHbmArgs a = make_pml_hbm_args(p);
    a.adj = p.adj_buf;
    PmlHbmState s = pml_hbm_state(p);
    const size_t plane = (size_t)a.plane, npts = (size_t)p.npts, nl2 = 2 * (size_t)p.pml_nl;
    const int nsteps = p.g.nt - 1;
    launch_fill(s.M0, nf * npts, 0.f, st);
    launch_fill(s.M1, nf * npts, 0.f, st);
    launch_fill(s.NU, nf * npts, 0.f, st);
    launch_fill(s.H0, nf * nl2, 0.f, st);
    launch_fill(s.H1, nf * nl2, 0.f, st);
    launch_fill(p.gpad, nf * npts, 0.f, st);
    hipLaunchKernelGGL(k_pml_hbm_start<true>, dim3((p.g.nr + 255) / 256, nf), dim3(256), 0, st, a, s.NU, s.M0);
    float *M0 = s.M0, *M1 = s.M1, *H0 = s.H0, *H1 = s.H1;
    auto adjoint_step = [&](int n, float* Dn, size_t dstride) {
        pml_hbm_step<true>(p, a, nf, n, M0, M1, H0, H1, s.NU, Dn, dstride, st);
        std::swap(M0, M1);
        std::swap(H0, H1);
    };
    if (p.store_mode == 0) {
        for (int n = nsteps - 1; n >= 0; --n) adjoint_step(n, p.Dstore + (size_t)n * npts, (size_t)nsteps * npts);
        return;
    }
    // checkpointed: recompute each segment's D from its checkpoint, then step the adjoint through it
    PmlHbmArgs fa = make_pml_hbm_args(p);
    fa.traces = nullptr;
    const int K = p.ckpt_every;
    const size_t dstride = (size_t)K * npts;
    for (int c = p.nseg - 1; c >= 0; --c) {
        const int n0 = c * K, n1 = std::min(n0 + K, nsteps);
        float *F0 = s.F0, *F1 = s.F1, *P0 = s.P0, *P1 = s.P1;
        hipLaunchKernelGGL(k_pml_hbm_ckpt<false>, dim3(hbm_grid(nf * (plane + npts + nl2))), dim3(256), 0, st,
                           p.ckpt, F0, s.W, P0, nf, p.nseg, c, (int)plane, (int)npts, p.pml_nl);
        for (int n = n0; n < n1; ++n) {
            pml_hbm_step<false>(p, fa, nf, n, F0, F1, P0, P1, s.W, p.Dstore + (size_t)(n - n0) * npts, dstride, st);
            std::swap(F0, F1);
            std::swap(P0, P1);
        }
        for (int n = n1 - 1; n >= n0; --n) adjoint_step(n, p.Dstore + (size_t)(n - n0) * npts, dstride);
    }
}

}  // namespace

void pml_tile_classes(const fwi_geometry& g, int nzp, int nxp, int ztop, std::vector<int>& plain,
                      std::vector<int>& layer) {
    plain.clear();
    layer.clear();
    for (int tz = 0; tz * kPtZ < nzp; ++tz)
        for (int tx = 0; tx * kPtX < nxp; ++tx) {
            const int x0 = tx * kPtX, zt = tz * kPtZ;
            // no layer cell, nor a cell past the grid, within 4 cells (above a reflecting top: model mirror rows)
            const bool ok = x0 - 4 >= g.nb && x0 + kPtX + 4 <= g.nb + g.nx && zt + kPtZ + 4 <= ztop + g.nz &&
                            (g.free_surface || zt - 4 >= ztop);
            (ok ? plain : layer).push_back((tz << 16) | tx);
        }
}

// The sweeps are captured as graphs on the plan's private stream and replayed on the caller's, as the tiled
// sponge sweeps are.
int pml_hbm_forward(Plan& p, int B, float* traces, const float* wavelet, int keep, hipStream_t st) {
    int rc = launch_copy(p.wav, wavelet, (size_t)p.g.nt, st);
    if (rc) return rc;
    const int k = keep ? 1 : 0;
    if (!p.g_fwd[k] || p.g_fwd_B[k] != B) {
        rc = capture_graph(p, &p.g_fwd[k], [&](hipStream_t cs) { pml_hbm_enqueue_forward(p, B, keep, cs); });
        if (rc) return rc;
        p.g_fwd_B[k] = B;
    }
    if (hipGraphLaunch(p.g_fwd[k], st) != hipSuccess) return FWI_EHIP;
    return launch_copy(traces, p.trace_buf, (size_t)B * p.g.ns * p.g.nr * p.g.nt, st);
}

int pml_hbm_adjoint(Plan& p, int B, const float* adj, hipStream_t st) {
    int rc = launch_copy(p.adj_buf, adj, (size_t)B * p.g.ns * p.g.nr * p.g.nt, st);
    if (rc) return rc;
    if (!p.g_adj || p.g_adj_B != B) {
        rc = capture_graph(p, &p.g_adj, [&](hipStream_t cs) { pml_hbm_enqueue_adjoint(p, B, cs); });
        if (rc) return rc;
        p.g_adj_B = B;
    }
    if (hipGraphLaunch(p.g_adj, st) != hipSuccess) return FWI_EHIP;
    return hip_ok(hipGetLastError());
}

}  // namespace fwi
