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
//
// Row bands.  When a batch leaves CUs idle, G workgroups share a field, band
// g holding padded rows [g H, g H + H) (k_wave_pml_band, launched
// cooperatively so that all bands are resident).  A band keeps its rows plus
// 8 halo rows above and below in LDS (u or y twice, for u^n and u^{n+1}, and
// the Q planes).  The auxiliary fields reach 4 rows past a cell (their
// divergence) and depend on the field 4 rows further (their gradient), so in
// the columns of the side layers a band also steps psi_z of the 4 rows past
// each of its edges itself (ghost rows: the same operations on the same
// values as the owning band, hence the same bits) and receives 8 halo rows
// there, 4 elsewhere.  Band edges keep 8 rows from the top and bottom layers,
// so no other column needs them.  Every step a band publishes the rows its
// neighbours read (computed first), as tagged 64-bit words as the split
// sponge sweep does, and fetches its halos while it computes its interior.
// Each cell undergoes the operations of the whole-field sweep above, and the
// history of D keeps its cell order, so the two sweeps give the same bits
// and either may run the adjoint of the other's forward pass.

#include "fwi_internal.h"
#include "pml_stencil.h"
#include "wave_split_body.h"

#include <algorithm>
#include <utility>

// No implicit fusing of a multiply and an add: the whole-field and the band
// sweeps must round every operation alike (the compiler otherwise fuses,
// say, the source term's product into the following sum in one kernel and
// not in the other).  Fused multiply-adds are written out with fmaf.
#pragma clang fp contract(off)

namespace fwi {

namespace {

// Returns x unchanged, opaque to the optimiser: per-slot addresses derived
// from it are recomputed in every step instead of being held in registers
// across the time loop (7 slots of them would spill).
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Cells per thread of the compiled band kernels.
#define FWI_PML_BAND_CASES(X) X(1) X(2) X(3) X(4)

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
    const int* rec_pt;       // [nr] padded index of each receiver
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


// Row bands of the PML sweep (see the file comment).
struct PmlBandArgs {
    int G, H;                    // bands per field, rows per band
    int NW;                      // words per exchanged edge: 4 nxp + 4 ndc
    int ndc;                     // columns of the side layers (2 nb)
    const int* cells;            // [G][KC * T] own cells iz << 16 | ix, published ones first; -1 = none
    const int* qcells;           // [G][KQ * T] layer cells and ghost cells of the auxiliary update; -1 = none
    const int* npub;             // [G] published cells at the head of each list
    unsigned long long* xchg;    // [fields][G][2 edges][2 parity][NW]
    int* err;                    // |= 2 when a wait gave up
};

// Word of a published cell in its band's exchange area: edge 0 carries band
// rows 0..3 (all columns) and 4..7 (side-layer columns) for band g - 1, edge
// 1 rows H - 4..H - 1 and H - 8..H - 5 for band g + 1.
__device__ __forceinline__ int pml_pub_word(int r, int ix, int H, int nxp, int nb, int nx, int ndc, int NW) {
    const int dc = ix < nb ? ix : ix - nx;
    if (r < 4) return r * nxp + ix;
    if (r < 8) return 4 * nxp + (r - 4) * ndc + dc;
    if (r >= H - 4) return 2 * NW + (r - (H - 4)) * nxp + ix;
    return 2 * NW + 4 * nxp + (r - (H - 8)) * ndc + dc;
}

template <int KC, bool ADJ>
__global__ void __launch_bounds__(kPmlBandThreads) k_wave_pml_band(const PmlArgs a, const PmlBandArgs bd) {
    constexpr int T = kPmlBandThreads, KQ = kPmlBandKQ, KH = kPmlBandKH;
    extern __shared__ float lds[];
    const int S = a.S, nxp = a.nxp, npts = a.npts, H = bd.H, G = bd.G;
    const int NW = bd.NW, ndc = bd.ndc;
    const int plane = (H + 16) * S;
    float* cur = lds;             // u^n (y^{n+1}): band rows and 8 halo rows on each side
    float* nxt = lds + plane;
    float* GX = lds + 2 * plane;  // Q_x or G_x
    float* GZ = lds + 3 * plane;  // Q_z or G_z (with the ghost rows)
    const int field = blockIdx.x / G, g = blockIdx.x - (blockIdx.x / G) * G;
    const int b = field / a.ns, s = field - (field / a.ns) * a.ns;
    const int tid = threadIdx.x;
    const int z0 = g * H;
    const int nsteps = a.nt - 1;
    const PmlOrder ord(a.nz, a.nx, a.nb, a.fs);
    const int nint = ord.nint, ndeep = ord.ndeep;
    const float* Kb = a.K + (size_t)b * npts;
    const size_t trfield = (size_t)field * a.nr * a.nt;
    float* Dfield = a.Dstore + (size_t)field * nsteps * npts;
    unsigned long long* xself = bd.xchg + ((size_t)field * G + g) * 4 * NW;

    for (int i = tid; i < 4 * plane; i += T) lds[i] = 0.f;

    // own cells: LDS offset, slot of the whole-field order (D history, receivers), mirror offset, published word
    const int* cl = bd.cells + (size_t)g * KC * T;
    const int npub = bd.npub[g];
    const int sp = a.src_pt[s];
    int off[KC], slot[KC], rec[KC], mir[KC], pubw[KC];
    float w[KC], r[KC], q[KC], bq[KC], acc[KC], mu[KC], dnext[KC], rinv[KC];
    int ksrc = -1;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int j = tid + k * T;
        const int c = cl[j];
        off[k] = -1;
        slot[k] = 0;
        rec[k] = -1;
        mir[k] = 0;
        pubw[k] = -1;
        w[k] = r[k] = bq[k] = acc[k] = mu[k] = dnext[k] = rinv[k] = 0.f;
        q[k] = 1.f;
        if (c >= 0) {
            const int iz = c >> 16, ix = c & 0xffff;
            off[k] = (iz - z0 + 8) * S + ix + 4;
            slot[k] = ord.slot_of(iz, ix);
            rec[k] = a.rec_slot[slot[k]];
            if (rec[k] >= 0) rinv[k] = a.rec_invw[rec[k]];
            mir[k] = (a.fs && iz >= 1 && iz <= 4) ? 2 * iz * S : 0;
            const float txv = a.tx[ix], tzv = a.tz[iz];
            const float E = 1.f / (1.f + a.tx[ix] + a.tz[iz]);
            r[k] = Kb[iz * nxp + ix] * E;
            if (slot[k] >= nint) {
                q[k] = (1.f - txv - tzv) * E;
                bq[k] = 4.f * txv * tzv * E;
            }
            if (iz * nxp + ix == sp) ksrc = k;
            if (j < npub) pubw[k] = pml_pub_word(iz - z0, ix, H, nxp, a.nb, a.nx, ndc, NW);
        }
    }
    // cells of the auxiliary update: own layer cells (Q_x and Q_z) and ghost cells (Q_z only)
    const int* ql = bd.qcells + (size_t)g * KQ * T;
    int qoff[KQ], qmir[KQ];
    bool qown[KQ];
    float qcx[KQ], qtx[KQ], qcz[KQ], qtz[KQ], px[KQ], pz[KQ];
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
        const int c = ql[tid + k * T];
        qoff[k] = -1;
        qmir[k] = 0;
        qown[k] = false;
        qcx[k] = qtx[k] = qcz[k] = qtz[k] = px[k] = pz[k] = 0.f;
        if (c >= 0) {
            const int iz = c >> 16, ix = c & 0xffff;
            qoff[k] = (iz - z0 + 8) * S + ix + 4;
            qown[k] = iz >= z0 && iz < z0 + H;
            qmir[k] = (a.fs && iz >= 1 && iz <= 4) ? 2 * iz * S : 0;
            qtx[k] = a.tx[ix];
            qtz[k] = a.tz[iz];
            qcx[k] = 1.f / (1.f + a.tx[ix]);
            qcz[k] = 1.f / (1.f + a.tz[iz]);
        }
    }
    // halo words received: [0, NW) from band g - 1's bottom edge into the rows above,
    // [NW, 2 NW) from band g + 1's top edge into the rows below
    int hsrc[KH], hdst[KH];  // inactive words read word 0 of the buffer and are ignored
    bool hon[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
        const int i = tid + k * T;
        hsrc[k] = 0;
        hdst[k] = 0;
        hon[k] = false;
        const bool top = i < NW && g > 0, bot = i >= NW && i < 2 * NW && g < G - 1;
        if (top || bot) {
            const int wd = top ? i : i - NW;
            int lr, ix;
            if (wd < 4 * nxp) {
                ix = wd % nxp;
                lr = top ? 4 + wd / nxp : 8 + H + wd / nxp;
            } else {
                const int e = wd - 4 * nxp, dc = e % ndc;
                ix = dc < a.nb ? dc : dc + a.nx;
                lr = top ? e / ndc : 8 + H + 4 + e / ndc;
            }
            hdst[k] = lr * S + ix + 4;
            hsrc[k] = (int)((((size_t)field * G + (top ? g - 1 : g + 1)) * 2 + (top ? 1 : 0)) * 2 * NW + wd);
            hon[k] = true;
        }
    }
    __syncthreads();

    if (!ADJ) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (rec[k] >= 0) a.traces[trfield + (size_t)rec[k] * a.nt] = 0.f;
    } else {
        // mu^{N-1} = a^{N-1} / w at the receivers (own cells and halo rows), nu^{N-1} = mu^{N-1}
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            if (rec[k] >= 0) {
                mu[k] = a.adj[trfield + (size_t)rec[k] * a.nt + nsteps] * a.rec_invw[rec[k]];
                w[k] = mu[k];
                const float y = r[k] * mu[k];
                cur[off[k]] = y;
                if (mir[k]) cur[off[k] - mir[k]] = y;
            }
            if (off[k] >= 0) dnext[k] = Dfield[(size_t)(nsteps - 1) * npts + slot[k]];
        }
        for (int i = tid; i < a.nr; i += T) {
            const int pt = a.rec_pt[i];
            const int iz = pt / nxp, ix = pt - (pt / nxp) * nxp;
            if ((iz >= z0 - 8 && iz < z0) || (iz >= z0 + H && iz < z0 + H + 8)) {
                const float E = 1.f / (1.f + a.tx[ix] + a.tz[iz]);
                const float rv = Kb[pt] * E;
                cur[(iz - z0 + 8) * S + ix + 4] = rv * (a.adj[trfield + (size_t)i * a.nt + nsteps] * a.rec_invw[i]);
            }
        }
    }
    // the published cells fill the first ceil(npub / T) slots: the halo is requested after them
    const int kreq = (npub + T - 1) / T;
    bool gave_up = false;
    __syncthreads();

    for (int m = 0; m < nsteps; ++m) {
        const int n = ADJ ? nsteps - 1 - m : m;  // forward step index
        const unsigned level = (unsigned)m + 1;
        const int par = (int)(level & 1) * NW;
        // phase 1: the auxiliary update of the layer and ghost cells, from the gathered field
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            if (qoff[k] < 0) continue;
            const int o = opaque(qoff[k]);
            const float* c = cur + o;
            const float gz = a.idz * dfirst(c, S);
            const float txv = qtx[k], tzv = qtz[k], cxv = qcx[k], czv = qcz[k];
            float oz;
            if (!ADJ) {
                if (qown[k]) {
                    const float gx = a.idx * dfirst(c, 1);
                    const float Qx = cxv * fmaf(tzv - txv, gx, px[k]);
                    px[k] = 2.f * Qx - px[k];
                    GX[o] = Qx;
                }
                const float Qz = czv * fmaf(txv - tzv, gz, pz[k]);
                pz[k] = 2.f * Qz - pz[k];
                oz = Qz;
            } else {
                if (qown[k]) {
                    const float gx = a.idx * dfirst(c, 1);
                    const float Qx = 2.f * px[k] - gx;
                    px[k] = cxv * Qx - px[k];
                    GX[o] = cxv * (tzv - txv) * Qx;
                }
                const float Qz = 2.f * pz[k] - gz;
                pz[k] = czv * Qz - pz[k];
                oz = czv * (txv - tzv) * Qz;
            }
            GZ[o] = oz;
            if (qmir[k]) GZ[o - qmir[k]] = -oz;
        }
        // loads made by every lane (no load in a divergent branch, so no wait where branches join)
        const float sv = ADJ ? 0.f : a.wavelet[n] * a.src_scale;
        float av[KC];
        if (ADJ) {
#pragma unroll
            for (int k = 0; k < KC; ++k)
                av[k] = a.adj[trfield + (size_t)(rec[k] >= 0 ? rec[k] : 0) * a.nt + n] * rinv[k];
        }
        __syncthreads();
        // phase 2: Laplacian, divergence of Q and the time update; published cells first.
        // The halo words and the next step's D values are loaded by every lane (inactive
        // ones from a valid dummy address), so no load sits in a divergent branch and
        // the compiler need not wait for one where the branches join.
        unsigned long long hv[KH];
        const int nm1 = n >= 1 ? n - 1 : 0;
#pragma unroll
        for (int k = 0; k <= KC; ++k) {
            if (k == kreq) {
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int h = 0; h < KH; ++h) hv[h] = split_get(bd.xchg + hsrc[h] + par);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (k == KC) break;
            __builtin_amdgcn_sched_barrier(0);
            if (ADJ) {
                // imaging y^{n+1} D^n, every lane (a slot past the band reads a zero halo cell)
                acc[k] = fmaf(cur[off[k] >= 0 ? off[k] : 0], dnext[k], acc[k]);
                dnext[k] = Dfield[(size_t)nm1 * npts + slot[k]];  // D^{n-1}: a step ahead
            }
            if (off[k] >= 0) {
                const int o = opaque(off[k]);
                const int j = opaque(slot[k]);
                const float* c = cur + o;
                const float c0 = c[0];
                const float lz =
                    FWI_LAPD(c0, c[-4 * S], c[-3 * S], c[-2 * S], c[-S], c[S], c[2 * S], c[3 * S], c[4 * S]);
                const float lx = FWI_LAPD(c0, c[-4], c[-3], c[-2], c[-1], c[1], c[2], c[3], c[4]);
                const float lap = fmaf(a.idx2, lx, a.idz2 * lz);
                // Q is zero within 4 cells of a deep cell
                const float div = j < ndeep ? 0.f : fmaf(a.idx, dfirst(GX + o, 1), a.idz * dfirst(GZ + o, S));
                float out;
                if (!ADJ) {
                    float D = lap + div;
                    if (k == ksrc) D += sv;
                    w[k] = fmaf(r[k], D, fmaf(q[k], w[k], -bq[k] * c0));
                    out = c0 + w[k];
                    if (a.store) Dfield[(size_t)n * npts + j] = D;
                    if (rec[k] >= 0) a.traces[trfield + (size_t)rec[k] * a.nt + n + 1] = out;
                } else {
                    const float Fv = (lap - div) + av[k];
                    w[k] = fmaf(q[k], w[k], fmaf(-bq[k], mu[k], Fv));
                    mu[k] += w[k];
                    out = r[k] * mu[k];
                }
                nxt[o] = out;
                if (mir[k]) nxt[o - mir[k]] = out;
                if (pubw[k] >= 0) split_put(xself + pubw[k] + par, out, level);
            }
        }
        // the neighbours' rows of this step into the halo rows of u^{n+1}; words not yet
        // there are requested again together, so each round costs one round trip
        {
            int spins = 0;
            for (;;) {
                bool stale = false;
#pragma unroll
                for (int h = 0; h < KH; ++h) stale |= hon[h] && (unsigned)(hv[h] >> 32) != level;
                if (!stale || gave_up) break;
                if (++spins > kSplitSpinMax) {  // a neighbour is not running: flag it, never wait again
                    atomicOr(bd.err, 2);
                    gave_up = true;
                    break;
                }
#pragma unroll
                for (int h = 0; h < KH; ++h)
                    if (hon[h] && (unsigned)(hv[h] >> 32) != level) hv[h] = split_get(bd.xchg + hsrc[h] + par);
            }
#pragma unroll
            for (int h = 0; h < KH; ++h)
                if (hon[h]) nxt[hdst[h]] = __uint_as_float((unsigned)hv[h]);
        }
        __syncthreads();
        float* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (ADJ) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (off[k] >= 0) {
                const int c = cl[tid + k * T];
                a.gpad[(size_t)field * npts + (c >> 16) * nxp + (c & 0xffff)] = acc[k];
            }
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
    a.rec_pt = p.rec_pt;
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

template <bool ADJ>
int pml_band_dispatch(const PmlArgs& a, const PmlBandArgs& bd, int KC, int nf, hipStream_t st) {
    const size_t bytes = (size_t)4 * (bd.H + 16) * a.S * sizeof(float);
    void* args[] = {(void*)&a, (void*)&bd};
#define FWI_PML_BAND_CASE(KCC)                                                                                     \
    if (KC == KCC) {                                                                                               \
        const void* kern = (const void*)k_wave_pml_band<KCC, ADJ>;                                                 \
        if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)       \
            return hip_ok(hipGetLastError());                                                                      \
        return hip_ok(hipLaunchCooperativeKernel(kern, dim3(nf * bd.G), dim3(kPmlBandThreads), args,              \
                                                 (unsigned)bytes, st));                                            \
    }
    FWI_PML_BAND_CASES(FWI_PML_BAND_CASE)
#undef FWI_PML_BAND_CASE
    return FWI_EINVAL;
}

// Band arguments of a launch over nf fields; the exchange buffer is cleared to level 0 first.
int pml_band_args(const Plan& p, int nf, PmlBandArgs& bd, hipStream_t st) {
    bd.G = p.pml_G;
    bd.H = p.pml_H;
    bd.NW = p.pml_NW;
    bd.ndc = 2 * p.g.nb;
    bd.cells = p.pml_cells;
    bd.qcells = p.pml_qcells;
    bd.npub = p.pml_npub;
    bd.xchg = p.pml_xchg;
    bd.err = p.flags;
    return launch_fill(reinterpret_cast<float*>(p.pml_xchg), (size_t)nf * bd.G * 4 * bd.NW * 2, 0.f, st);
}

}  // namespace

bool pml_choose_bands(const fwi_geometry& g, int nzp, int nxp, int ztop, int nfields, int ncu, int force, int* Go,
                      int* Ho, int* KCo, int* NWo) {
    if (force < 0 || nfields <= 0 || ncu <= 0) return false;
    const int T = kPmlBandThreads, ndc = 2 * g.nb, NW = 4 * nxp + 4 * ndc;
    const int Gmax = std::min(ncu / nfields, 16);
    const PmlOrder ord(g.nz, g.nx, g.nb, g.free_surface);
    for (int G = Gmax; G >= 2; --G) {
        const int H = (nzp + G - 1) / G;
        if (H < 16 || (G - 1) * H >= nzp) continue;
        bool ok = true;
        // band edges stay 8 rows away from the layers above and below the model
        for (int e = 1; e < G && ok; ++e) ok = e * H - 8 >= ztop && e * H + 8 <= ztop + g.nz;
        if (!ok) continue;
        int KC = 0;
        const int need = (H * nxp + T - 1) / T;
        for (int c : {1, 2, 3, 4})
            if (c >= need) {
                KC = c;
                break;
            }
        if (KC == 0) continue;
        // most auxiliary-update cells of a band: its layer cells and 8 ghost rows of side columns
        int nq_max = 0;
        for (int b = 0; b < G; ++b) {
            int c = 0;
            for (int iz = b * H; iz < std::min(b * H + H, nzp); ++iz)
                for (int ix = 0; ix < nxp; ++ix) c += ord.slot_of(iz, ix) >= ord.nint;
            nq_max = std::max(nq_max, c + 8 * ndc);
        }
        if (nq_max > kPmlBandKQ * T || 2 * NW > kPmlBandKH * T) continue;
        if ((size_t)4 * (H + 16) * (nxp + 8) * sizeof(float) > (size_t)kLdsBytes) continue;
        *Go = G;
        *Ho = H;
        *KCo = KC;
        *NWo = NW;
        return true;
    }
    return false;
}

void pml_band_tables(const fwi_geometry& g, int nzp, int nxp, int ztop, int G, int H, int KC, std::vector<int>& cells,
                     std::vector<int>& qcells, std::vector<int>& npub) {
    const int T = kPmlBandThreads, nb = g.nb, nx = g.nx;
    const PmlOrder ord(g.nz, g.nx, g.nb, g.free_surface);
    (void)ztop;
    cells.assign((size_t)G * KC * T, -1);
    qcells.assign((size_t)G * kPmlBandKQ * T, -1);
    npub.assign(G, 0);
    for (int b = 0; b < G; ++b) {
        const int z0 = b * H, z1 = std::min(z0 + H, nzp);
        std::vector<std::pair<int, int>> P, I, Q, Qg;
        auto side = [&](int ix) { return ix < nb || ix >= nb + nx; };
        for (int iz = z0; iz < z1; ++iz)
            for (int ix = 0; ix < nxp; ++ix) {
                const int r = iz - z0, sl = ord.slot_of(iz, ix), c = (iz << 16) | ix;
                const bool pub = (b > 0 && (r < 4 || (r < 8 && side(ix)))) ||
                                 (b < G - 1 && (r >= H - 4 || (r >= H - 8 && side(ix))));
                (pub ? P : I).push_back({sl, c});
                if (sl >= ord.nint) Q.push_back({sl, c});
            }
        // ghost rows: the 4 rows past each inner edge, in the side-layer columns
        for (int iz = z0 - 4; iz < z1 + 4; ++iz) {
            const bool ghost = (b > 0 && iz < z0 && iz >= z0 - 4) || (b < G - 1 && iz >= z1 && iz < nzp);
            if (!ghost) continue;
            for (int ix = 0; ix < nxp; ++ix)
                if (side(ix)) Qg.push_back({ord.slot_of(iz, ix), (iz << 16) | ix});
        }
        std::sort(P.begin(), P.end());
        std::sort(I.begin(), I.end());
        std::sort(Q.begin(), Q.end());
        std::sort(Qg.begin(), Qg.end());
        int j = 0;
        for (auto& e : P) cells[(size_t)b * KC * T + j++] = e.second;
        for (auto& e : I) cells[(size_t)b * KC * T + j++] = e.second;
        npub[b] = (int)P.size();
        j = 0;
        for (auto& e : Q) qcells[(size_t)b * kPmlBandKQ * T + j++] = e.second;
        for (auto& e : Qg) qcells[(size_t)b * kPmlBandKQ * T + j++] = e.second;
    }
}

size_t pml_lds_bytes(int nzp, int nxp) {
    return ((size_t)3 * (nzp + 8) * (nxp + 8) + 2 * (size_t)nzp * nxp + 2 * (size_t)nxp + 2 * (size_t)nzp) *
           sizeof(float);
}

bool pml_fits(int nzp, int nxp) {
    return (long long)nzp * nxp <= (long long)kPmlMaxCells * kPmlThreads && nxp < (1 << 15) &&
           pml_lds_bytes(nzp, nxp) <= (size_t)kLdsBytes;
}

// Row bands unless the stream is capturing a graph (a cooperative launch cannot be
// captured): then the whole-field sweep, with the same results, if the field fits.
int launch_pml_forward(const Plan& p, int B, float* traces, const float* wavelet, int store, hipStream_t st) {
    PmlArgs a = make_pml_args(p);
    a.traces = traces;
    a.wavelet = wavelet;
    a.store = store;
    const int nf = B * p.g.ns;
    if (p.pml_G > 1 && !stream_capturing(st)) {
        PmlBandArgs bd{};
        const int rc = pml_band_args(p, nf, bd, st);
        return rc ? rc : pml_band_dispatch<false>(a, bd, p.pml_KC, nf, st);
    }
    if (!pml_fits(p.nzp, p.nxp)) return FWI_EINVAL;
    return pml_dispatch<false>(a, nf, st);
}

int launch_pml_adjoint(const Plan& p, int B, const float* adj, hipStream_t st) {
    PmlArgs a = make_pml_args(p);
    a.adj = adj;
    const int nf = B * p.g.ns;
    if (p.pml_G > 1 && !stream_capturing(st)) {
        PmlBandArgs bd{};
        const int rc = pml_band_args(p, nf, bd, st);
        return rc ? rc : pml_band_dispatch<true>(a, bd, p.pml_KC, nf, st);
    }
    if (!pml_fits(p.nzp, p.nxp)) return FWI_EINVAL;
    return pml_dispatch<true>(a, nf, st);
}

}  // namespace fwi
