// Uneven batches: many requests with their own grid sizes, trace lengths and
// shot counts swept by ONE persistent launch.
//
// Work unit = one (request, shot) field for its whole time loop.  The launch
// holds one 512-thread workgroup per compute unit; each workgroup takes the
// next unit from a device counter (units are queued longest first, so the
// long fields start early and the short ones fill the tail) and runs it to the
// end, so no workgroup ever waits on another.  Two kinds of unit:
//  * fields whose padded grid fits the LDS run the register-tiled LDS-resident
//    time loop (wave_lds_body.h) with this request's tile;
//  * larger fields keep (u^n, u^{n+1}, w) in HBM (the unit's own arrays, hot in
//    L2 / MALL) and stream them column panel by column panel each step
//    (glb_field_forward);
//  * in a forward-only batch, larger fields whose receivers share a row are
//    instead cut into G row bands that stay in LDS for the whole time loop,
//    one unit per band, exchanging 4-row halos every step through tagged
//    64-bit words (the split sweep body of wave_split_body.h, bitwise equal to
//    the other sweeps).  The bands of a field are queued next to each other
//    and the launch is cooperative, so they all become resident; a band that
//    starts early waits, with a bounded spin, for its neighbours' first rows.
// The tile of each size class (LDS register tile or HBM prefetch depth) comes from
// the autotuner below, which times the candidates on a short sweep of the
// class's first unit replicated over every compute unit.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "fwi_internal.h"
#include "wave_lds_body.h"
#include "wave_split_body.h"

namespace fwi {

// A value every lane of the workgroup holds alike (a unit's descriptor
// fields), moved into scalar registers word by word.  The unit bodies are
// separate functions whose descriptor pointer arrives in vector registers;
// without this their loop bounds, strides and base pointers would occupy
// vector registers and vector instructions, where the plan's kernels keep
// them in scalar ones.
template <class T>
__device__ __forceinline__ T uniform(const T& v) {
    static_assert(sizeof(T) % 4 == 0, "word-sized");
    T r;
    const unsigned* src = reinterpret_cast<const unsigned*>(&v);
    unsigned* dst = reinterpret_cast<unsigned*>(&r);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return r;
}

// Variants compiled into the persistent kernel.
//   LDS-resident register tiles (X, P, exact cover of the padded grid)
#define FWI_BATCH_LDS(M) M(0, 3, 11, true) M(1, 3, 11, false) M(2, 3, 12, false) M(3, 2, 12, false) M(4, 4, 8, false) M(5, 1, 16, false)
constexpr int kBatchLdsVariants = 6;
//   HBM sweeps (RB rows loaded ahead per block, SMUL x the minimal row segments per column group)
#define FWI_BATCH_GLB(M) M(0, 2, 1) M(1, 4, 1) M(2, 8, 1) M(3, 4, 2) M(4, 8, 2)
constexpr int kBatchGlbVariants = 5;
//   LDS-resident row bands (X columns, PI interior rows per tile, exact column cover); wider tiles
//   than the plan's split sweep, since 8 boundary rows of ncg = nxp / X column groups must fit 512 threads
#define FWI_BATCH_SPLIT(M) \
    M(0, 4, 3, true) M(1, 4, 3, false) M(2, 4, 4, true) M(3, 4, 4, false) M(4, 6, 3, true) M(5, 6, 3, false)

struct BatchUnit {
    int kind;       // 0: LDS-resident, 1: HBM sweep, 2: LDS-resident row band of a split field
    int variant;    // index into the list of its kind
    int nsteps;     // time steps to take (nt - 1, or fewer when tuning)
    long long tr_off, w_off;  // offsets of this unit's traces and wavelet in the call's packed buffers
    LdsArgs la;     // kinds 0 and 2: pointers already offset to this unit (field index 0)
    SplitArgs sp;   // kind 2: bands of the field, its exchange rows (field0 = 0); the band is `part`
    unsigned long long* xchg_adj;  // kind 2 in gradient batches: exchange rows of the adjoint sweep
    // kind 1
    int nzp, nxp, fs, nt, nr, src_pt, rec_z0, rec_z1;
    float idz2, idx2, src_scale;
    const float* K;
    const float* wavelet;
    const int* rec_map;
    float* ua;
    float* ub;
    float* w;
    float* traces;  // [nr][nt] of this unit
    const float* ax;
    const float* az;
    // gradients (fwi_batch_gradient): adjoint sources [nr][nt] (bound per call), imaging sum [npts]
    const float* adj;
    float* gpad;
    const float* rec_invw;  // kind 1: [nr] 1/w per receiver
    // kind 1: adjoint state (psi ping-pong, w_psi), checkpoints [nseg][2][npts], D of one segment [C][npts]
    float *pa, *pb, *pw, *ckpt, *dseg;
    int ckpt_every;
    // kind 1 split into parts: this unit sweeps rows [z_lo, z_hi) of the field;
    // the nparts units of one field meet at a barrier (counter *bar, cleared
    // before each launch) after every step.  nparts = 1: the whole field.
    int z_lo, z_hi, part, nparts;
    int* bar;
    int* flags;     // the batch's device flag (a barrier that gave up sets kFlagPartTimeout)
};

// Barrier of the nparts units of one field (all resident: the launch holds
// at most one workgroup per compute unit, and the parts of a field are
// queued next to each other, so a part waits at most until the next
// workgroup frees up).  Release / acquire at device scope around a counter;
// a wait that exceeds the spin limit raises the batch flag and the part stops
// waiting from then on (its results are then invalid, never a hang).
constexpr int kPartSpinMax = 1 << 22;
constexpr int kFlagPartTimeout = 4;

struct PartSync {
    int nparts;
    int* bar;
    int* flags;
    int k;          // barriers passed
    bool gave_up;   // thread 0 only
};

__device__ inline void part_barrier(PartSync& ps) {
    // every wave's stores complete (reach L2) before the barrier, so that the
    // L2 write-back of thread 0's release fence covers the whole part's writes
    if (ps.nparts > 1) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (ps.nparts > 1) {
        ++ps.k;
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(ps.bar, 1);
            int spins = 0;
            while (!ps.gave_up &&
                   __hip_atomic_load(ps.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < ps.nparts * ps.k) {
                if (++spins > kPartSpinMax) {
                    atomicOr(ps.flags, kFlagPartTimeout);
                    ps.gave_up = true;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __threadfence();
        }
        __syncthreads();
    }
}

// HBM-swept field: wave w of the workgroup owns 64-column panels (column
// group, row segment) and walks down each panel's rows.  Each lane keeps the
// 9-row window of u^n of its column in registers (rolled as it walks), takes
// its 8 x-neighbours from the wave's own row buffer in LDS (the panel's 64
// columns plus 4 halo columns on each side), and issues the loads of the next
// RB rows (u, K, w, halo) before computing the current ones, so the latency
// of HBM / MALL overlaps the arithmetic.  One workgroup barrier per time step
// separates u^n (read) from u^{n+1} (written).
template <int RB, int SMUL>
__device__ void glb_field_forward(const BatchUnit& Ug, float* lds) {
    constexpr int NW = kLdsThreads / 64;
    // descriptor fields in registers: stores to the field arrays may not be
    // assumed to leave a descriptor in global memory unchanged
    const int nzp = Ug.nzp, nxp = Ug.nxp, nsteps = Ug.nsteps, nt = Ug.nt, nr = Ug.nr, fs = Ug.fs;
    const int src_pt = Ug.src_pt, rec_z0 = Ug.rec_z0, rec_z1 = Ug.rec_z1;
    const float idz2 = Ug.idz2, idx2 = Ug.idx2, src_scale = Ug.src_scale;
    const float* __restrict__ K = Ug.K;
    const float* __restrict__ wavelet = Ug.wavelet;
    const int* __restrict__ rec_map = Ug.rec_map;
    const float* __restrict__ ax = Ug.ax;
    const float* __restrict__ az = Ug.az;
    float* ua = Ug.ua;
    float* ub = Ug.ub;
    float* __restrict__ wst = Ug.w;
    float* __restrict__ traces = Ug.traces;
    const int tid = threadIdx.x, lane = tid & 63;
    // the wave index is uniform across the wave: made explicit so that panel
    // rows, bounds and clamps derived from it are scalar (SALU) arithmetic
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int z_lo = Ug.z_lo, z_hi = Ug.z_hi;
    PartSync ps{Ug.nparts, Ug.bar, Ug.flags, 0, false};
    for (int i = z_lo * nxp + tid; i < z_hi * nxp; i += kLdsThreads) {
        ua[i] = 0.f;
        wst[i] = 0.f;
    }
    for (int r = tid; r < nr; r += kLdsThreads) traces[(size_t)r * nt] = 0.f;
    part_barrier(ps);
    const int G = (nxp + 63) / 64;
    int S = 1;
    while ((G * S) % NW != 0) ++S;  // panels a multiple of the wave count (S <= NW)
    S *= SMUL;
    const int seg = (z_hi - z_lo + S - 1) / S;
    float* rb = lds + wave * 72;
    const float* cur = ua;
    float* nxt = ub;
    for (int m = 0; m < nsteps; ++m) {
        for (int pan = wave; pan < G * S; pan += NW) {
            const int g = pan % G, sg = pan / G;
            const int x0 = g * 64, x = x0 + lane;
            const int za = z_lo + sg * seg, zb = min(z_hi, za + seg);
            if (za >= zb) continue;
            const bool xin = x < nxp;
            const float axv = xin ? ax[x] : 0.f;
            const int hx = lane < 4 ? x0 - 4 + lane : x0 + 64 + (lane - 4);  // halo column of lanes 0..7
            const bool hin = lane < 8 && hx >= 0 && hx < nxp;
            auto ld_u = [&](int z) {
                const int zz = (fs && z < 0) ? -z : z;  // even mirror above a reflecting top
                return (xin && zz >= 0 && zz < nzp) ? cur[zz * nxp + x] : 0.f;
            };
            auto ld_h = [&](int z) { return (hin && z >= 0 && z < nzp) ? cur[z * nxp + hx] : 0.f; };
            float col[RB + 8];
#pragma unroll
            for (int k = 0; k < 8; ++k) col[k] = ld_u(za - 4 + k);
            float cu[RB], ck[RB], cw[RB], chl[RB];
#pragma unroll
            for (int jj = 0; jj < RB; ++jj) {
                const int z = za + jj;
                const bool ok = xin && z < zb;
                cu[jj] = ld_u(z + 4);
                ck[jj] = ok ? K[z * nxp + x] : 0.f;
                cw[jj] = ok ? wst[z * nxp + x] : 0.f;
                chl[jj] = (z < zb) ? ld_h(z) : 0.f;
            }
            for (int z0 = za; z0 < zb; z0 += RB) {
                float nu[RB], nk[RB], nw[RB], nh[RB];
                const int z1 = z0 + RB;
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {  // the next block's loads go out first
                    const int z = z1 + jj;
                    const bool ok = xin && z < zb;
                    nu[jj] = (z1 < zb) ? ld_u(z + 4) : 0.f;
                    nk[jj] = ok ? K[z * nxp + x] : 0.f;
                    nw[jj] = ok ? wst[z * nxp + x] : 0.f;
                    nh[jj] = (z < zb) ? ld_h(z) : 0.f;
                }
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) col[8 + jj] = cu[jj];
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {
                    const int z = z0 + jj;
                    if (z >= zb) break;
                    const float c = col[jj + 4];
                    rb[lane + 4] = c;
                    if (lane < 8) rb[lane < 4 ? lane : 64 + lane] = chl[jj];
                    __builtin_amdgcn_wave_barrier();
                    float xr[9];
#pragma unroll
                    for (int k = 0; k < 9; ++k) xr[k] = rb[lane + k];
                    __builtin_amdgcn_wave_barrier();
                    const float lzs = FWI_LAPD(c, col[jj], col[jj + 1], col[jj + 2], col[jj + 3], col[jj + 5],
                                               col[jj + 6], col[jj + 7], col[jj + 8]);
                    const float lxs = FWI_LAPD(c, xr[0], xr[1], xr[2], xr[3], xr[5], xr[6], xr[7], xr[8]);
                    float D = fmaf(lzs, idz2, lxs * idx2);
                    const int p = z * nxp + x;
                    if (xin) {
                        if (p == src_pt) D = fmaf(wavelet[m], src_scale, D);
                        const float wn = fmaf(ck[jj], D, (axv * az[z]) * cw[jj]);
                        const float un = c + wn;
                        wst[p] = wn;
                        nxt[p] = un;
                        if (z >= rec_z0 && z <= rec_z1) {
                            const int r = rec_map[p];
                            if (r >= 0) traces[(size_t)r * nt + m + 1] = un;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) col[k] = col[RB + k];
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {
                    cu[jj] = nu[jj];
                    ck[jj] = nk[jj];
                    cw[jj] = nw[jj];
                    chl[jj] = nh[jj];
                }
            }
        }
        part_barrier(ps);
        float* t = const_cast<float*>(cur);
        cur = nxt;
        nxt = t;
    }
}

// ---------------------------------------------------------------------------
// Gradients of HBM-swept fields.  glb_steps runs steps n0 .. n1-1 of the
// forward recursion (optionally saving (u^n, w^n) before every step n that is
// a multiple of C, and D^n = L u^n + s^n into dseg[n - n0]) or, with ADJ, the
// adjoint steps for n = n1-1 down to n0 (adjoint source a^{n+1}/w injected at
// the receivers, imaging acc += psi^{n+1} D^n with D^n from dseg).  The field
// is streamed column panel by column panel as in glb_field_forward; cur/nxt
// are swapped after every step so that on return *cur holds the newest state.
struct GlbCtx {
    int nzp, nxp, nt, nr, fs, src_pt, rec_z0, rec_z1;
    int z_lo, z_hi;     // rows of this part
    float idz2, idx2, src_scale;
    const float* K;
    const float* wavelet;
    const int* rec_map;
    const float* rec_invw;
    const float* ax;
    const float* az;
    float* traces;      // forward: [nr][nt] or null
    const float* adj;   // adjoint: [nr][nt]
};

template <int RB, int SMUL, bool ADJ>
__device__ void glb_steps(const GlbCtx& c, float*& cur, float*& nxt, float* __restrict__ wst, int n0, int n1,
                          float* __restrict__ ckpt, int C, float* __restrict__ dseg, float* __restrict__ acc,
                          float* lds, PartSync& ps) {
    constexpr int NW = kLdsThreads / 64;
    const int nzp = c.nzp, nxp = c.nxp, npts = nzp * nxp;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = (nxp + 63) / 64;
    int S = 1;
    while ((G * S) % NW != 0) ++S;
    S *= SMUL;
    const int seg = (c.z_hi - c.z_lo + S - 1) / S;
    float* rb = lds + wave * 72;
    for (int it = 0; it < n1 - n0; ++it) {
        const int n = ADJ ? n1 - 1 - it : n0 + it;
        if (!ADJ && ckpt && n % C == 0) {  // state before step n (this part's rows)
            float* ck = ckpt + (size_t)(n / C) * 2 * npts;
            for (int i = c.z_lo * nxp + tid; i < c.z_hi * nxp; i += kLdsThreads) {
                ck[i] = cur[i];
                ck[npts + i] = wst[i];
            }
        }
        float* dn = dseg ? dseg + (size_t)(n - n0) * npts : nullptr;
        const float wm = ADJ ? 0.f : c.wavelet[n];
        for (int pan = wave; pan < G * S; pan += NW) {
            const int g = pan % G, sg = pan / G;
            const int x0 = g * 64, x = x0 + lane;
            const int za = c.z_lo + sg * seg, zb = min(c.z_hi, za + seg);
            if (za >= zb) continue;
            const bool xin = x < nxp;
            const float axv = xin ? c.ax[x] : 0.f;
            const int hx = lane < 4 ? x0 - 4 + lane : x0 + 64 + (lane - 4);
            const bool hin = lane < 8 && hx >= 0 && hx < nxp;
            auto ld_u = [&](int z) {
                const int zz = (c.fs && z < 0) ? -z : z;
                return (xin && zz >= 0 && zz < nzp) ? cur[zz * nxp + x] : 0.f;
            };
            auto ld_h = [&](int z) { return (hin && z >= 0 && z < nzp) ? cur[z * nxp + hx] : 0.f; };
            float col[RB + 8];
#pragma unroll
            for (int k = 0; k < 8; ++k) col[k] = ld_u(za - 4 + k);
            float cu[RB], ck[RB], cw[RB], chl[RB];
#pragma unroll
            for (int jj = 0; jj < RB; ++jj) {
                const int z = za + jj;
                const bool ok = xin && z < zb;
                cu[jj] = ld_u(z + 4);
                ck[jj] = ok ? c.K[z * nxp + x] : 0.f;
                cw[jj] = ok ? wst[z * nxp + x] : 0.f;
                chl[jj] = (z < zb) ? ld_h(z) : 0.f;
            }
            for (int z0 = za; z0 < zb; z0 += RB) {
                float nu[RB], nk[RB], nw[RB], nh[RB];
                const int z1 = z0 + RB;
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {
                    const int z = z1 + jj;
                    const bool ok = xin && z < zb;
                    nu[jj] = (z1 < zb) ? ld_u(z + 4) : 0.f;
                    nk[jj] = ok ? c.K[z * nxp + x] : 0.f;
                    nw[jj] = ok ? wst[z * nxp + x] : 0.f;
                    nh[jj] = (z < zb) ? ld_h(z) : 0.f;
                }
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) col[8 + jj] = cu[jj];
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {
                    const int z = z0 + jj;
                    if (z >= zb) break;
                    const float cc = col[jj + 4];
                    rb[lane + 4] = cc;
                    if (lane < 8) rb[lane < 4 ? lane : 64 + lane] = chl[jj];
                    __builtin_amdgcn_wave_barrier();
                    float xr[9];
#pragma unroll
                    for (int k = 0; k < 9; ++k) xr[k] = rb[lane + k];
                    __builtin_amdgcn_wave_barrier();
                    const float lzs = FWI_LAPD(cc, col[jj], col[jj + 1], col[jj + 2], col[jj + 3], col[jj + 5],
                                               col[jj + 6], col[jj + 7], col[jj + 8]);
                    const float lxs = FWI_LAPD(cc, xr[0], xr[1], xr[2], xr[3], xr[5], xr[6], xr[7], xr[8]);
                    float D = fmaf(lzs, c.idz2, lxs * c.idx2);
                    const int p = z * nxp + x;
                    if (xin) {
                        const bool recrow = z >= c.rec_z0 && z <= c.rec_z1;
                        const int r = recrow ? c.rec_map[p] : -1;
                        if (ADJ) {
                            if (r >= 0) D = fmaf(c.rec_invw[r], c.adj[(size_t)r * c.nt + n + 1], D);
                        } else if (p == c.src_pt) {
                            D = fmaf(wm, c.src_scale, D);
                        }
                        const float wn = fmaf(ck[jj], D, (axv * c.az[z]) * cw[jj]);
                        const float un = cc + wn;
                        wst[p] = wn;
                        nxt[p] = un;
                        if (ADJ) {
                            acc[p] = fmaf(un, dn[p], acc[p]);
                        } else {
                            if (dn) dn[p] = D;
                            if (r >= 0 && c.traces) c.traces[(size_t)r * c.nt + n + 1] = un;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) col[k] = col[RB + k];
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {
                    cu[jj] = nu[jj];
                    ck[jj] = nk[jj];
                    cw[jj] = nw[jj];
                    chl[jj] = nh[jj];
                }
            }
        }
        part_barrier(ps);
        float* t = cur;
        cur = nxt;
        nxt = t;
    }
}

__device__ inline GlbCtx glb_ctx(const BatchUnit* U) {
    GlbCtx c;
    c.nzp = U->nzp, c.nxp = U->nxp, c.nt = U->nt, c.nr = U->nr, c.fs = U->fs, c.src_pt = U->src_pt;
    c.rec_z0 = U->rec_z0, c.rec_z1 = U->rec_z1;
    c.z_lo = U->z_lo, c.z_hi = U->z_hi;
    c.idz2 = U->idz2, c.idx2 = U->idx2, c.src_scale = U->src_scale;
    c.K = U->K, c.wavelet = U->wavelet, c.rec_map = U->rec_map, c.rec_invw = U->rec_invw;
    c.ax = U->ax, c.az = U->az, c.traces = nullptr, c.adj = U->adj;
    return c;
}

// dJ/dv_pad (before the 2 w / v factor) of one HBM-swept field: forward with
// checkpoints every C steps, then per segment (last first) recomputation of
// D from its checkpoint and the adjoint steps through it.
template <int RB, int SM>
__device__ __noinline__ void unit_glb_gradient(const BatchUnit* __restrict__ U, float* lds) {
    const GlbCtx c = glb_ctx(U);
    const int npts = c.nzp * c.nxp, nsteps = U->nsteps, C = U->ckpt_every;
    const int nseg = (nsteps + C - 1) / C;
    float* u0 = U->ua;
    float* u1 = U->ub;
    float* w = U->w;
    float* p0 = U->pa;
    float* p1 = U->pb;
    float* pw = U->pw;
    float* acc = U->gpad;
    PartSync ps{U->nparts, U->bar, U->flags, 0, false};
    const int i0 = c.z_lo * c.nxp, i1 = c.z_hi * c.nxp;  // this part's points
    for (int i = i0 + threadIdx.x; i < i1; i += kLdsThreads) {
        u0[i] = 0.f;
        w[i] = 0.f;
        p0[i] = 0.f;
        pw[i] = 0.f;
        acc[i] = 0.f;
    }
    part_barrier(ps);
    glb_steps<RB, SM, false>(c, u0, u1, w, 0, nsteps, U->ckpt, C, nullptr, nullptr, lds, ps);
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
        const int n0 = sgi * C, n1 = min(n0 + C, nsteps);
        const float* ck = U->ckpt + (size_t)sgi * 2 * npts;
        for (int i = i0 + threadIdx.x; i < i1; i += kLdsThreads) {
            u0[i] = ck[i];
            w[i] = ck[npts + i];
        }
        part_barrier(ps);
        glb_steps<RB, SM, false>(c, u0, u1, w, n0, n1, nullptr, C, U->dseg, nullptr, lds, ps);
        glb_steps<RB, SM, true>(c, p0, p1, pw, n0, n1, nullptr, C, U->dseg, acc, lds, ps);
    }
}

// LDS-resident field: forward sweep keeping the full history of D, then the
// adjoint sweep (separate non-inlined entries: each gets its own registers).
template <int X, int P, bool EX>
__device__ __noinline__ void unit_lds_forward_store(const BatchUnit* __restrict__ U, float* lds) {
    const LdsArgs a = uniform(U->la);
    lds_field<X, P, false, EX, true>(a, 0, uniform(U->ax), uniform(U->az), lds);
}

template <int X, int P, bool EX>
__device__ __noinline__ void unit_lds_adjoint(const BatchUnit* __restrict__ U, float* lds) {
    LdsArgs a = uniform(U->la);
    a.adj = uniform(U->adj);
    a.gpad = uniform(U->gpad);
    lds_field<X, P, true, EX, false>(a, 0, uniform(U->ax), uniform(U->az), lds);
}

template <int X, int P, bool EX>
__device__ void unit_lds_gradient(const BatchUnit* __restrict__ U, float* lds) {
    unit_lds_forward_store<X, P, EX>(U, lds);
    __syncthreads();
    unit_lds_adjoint<X, P, EX>(U, lds);
}

// Row band of a split field: its forward sweep keeping the history of D of
// its rows, then its adjoint sweep with the imaging sum of its rows.  The
// bands of the field exchange halos in both sweeps (separate exchange rows,
// so a band that starts its adjoint early never meets forward words).
template <int X, int PI, bool EX>
__device__ __noinline__ void unit_split_forward_store(const BatchUnit* __restrict__ U, float* lds) {
    const LdsArgs a = uniform(U->la);
    split_field<X, PI, false, EX, true>(a, uniform(U->sp), 0, uniform(U->part), uniform(U->ax), uniform(U->az), lds);
}

template <int X, int PI, bool EX>
__device__ __noinline__ void unit_split_adjoint(const BatchUnit* __restrict__ U, float* lds) {
    LdsArgs a = uniform(U->la);
    a.adj = uniform(U->adj);
    a.gpad = uniform(U->gpad);
    SplitArgs sp = uniform(U->sp);
    sp.xchg = uniform(U->xchg_adj);
    split_field<X, PI, true, EX, false>(a, sp, 0, uniform(U->part), uniform(U->ax), uniform(U->az), lds);
}

template <int X, int PI, bool EX>
__device__ void unit_split_gradient(const BatchUnit* __restrict__ U, float* lds) {
    unit_split_forward_store<X, PI, EX>(U, lds);
    __syncthreads();
    unit_split_adjoint<X, PI, EX>(U, lds);
}

__device__ void run_unit_gradient(const BatchUnit* U, float* lds) {
    const int kind = U->kind, variant = U->variant;
    if (kind == 2) {
#define FWI_SPLIT_CASE(ID, XX, PP, EX)               \
    if (variant == ID) {                             \
        unit_split_gradient<XX, PP, EX>(U, lds);     \
        return;                                      \
    }
        FWI_BATCH_SPLIT(FWI_SPLIT_CASE)
#undef FWI_SPLIT_CASE
        return;
    }
    if (kind == 0) {
#define FWI_LDS_CASE(ID, XX, PP, EX)              \
    if (variant == ID) {                          \
        unit_lds_gradient<XX, PP, EX>(U, lds);    \
        return;                                   \
    }
        FWI_BATCH_LDS(FWI_LDS_CASE)
#undef FWI_LDS_CASE
    } else {
#define FWI_GLB_CASE(ID, RBB, SM)                 \
    if (variant == ID) {                          \
        unit_glb_gradient<RBB, SM>(U, lds);       \
        return;                                   \
    }
        FWI_BATCH_GLB(FWI_GLB_CASE)
#undef FWI_GLB_CASE
    }
}

__global__ __launch_bounds__(kLdsThreads) void k_batch_gradient(const BatchUnit* __restrict__ units, int nunits,
                                                                int* __restrict__ counter) {
    extern __shared__ float lds[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int u = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (u >= nunits) break;
        run_unit_gradient(units + u, lds);
        __syncthreads();
    }
}

// grad_r[iz][ix] = sum over the padded cells replicating (iz, ix) (rows outer,
// columns inner, as the plan's two-pass fold) of sum_s gpad * 2 w dt / sqrt(K)
struct FoldReq {
    long long v_off, pt_off, g_off;
    int nz, nx, nzp, nxp, nb, ztop, ns;
    float dt, w0;  // w0: row weight of padded row 0 (1/2 on a reflecting top)
};

__global__ void k_batch_fold(const FoldReq* __restrict__ req, int nreq, long long total, const float* __restrict__ K,
                             const float* __restrict__ gpad, float* __restrict__ grad) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        int lo = 0, hi = nreq - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (req[mid].v_off <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        const FoldReq& q = req[lo];
        const int cell = (int)(i - q.v_off);
        const int iz = cell / q.nx, ix = cell - (cell / q.nx) * q.nx;
        const int zlo = (iz == 0) ? 0 : iz + q.ztop, zhi = (iz == q.nz - 1) ? q.nzp - 1 : iz + q.ztop;
        const int xlo = (ix == 0) ? 0 : ix + q.nb, xhi = (ix == q.nx - 1) ? q.nxp - 1 : ix + q.nb;
        const int npts = q.nzp * q.nxp;
        float sum = 0.f;
        for (int z = zlo; z <= zhi; ++z) {
            const float wz = 2.f * (z == 0 ? q.w0 : 1.f) * q.dt;
            float row = 0.f;
            for (int x = xlo; x <= xhi; ++x) {
                float gs = 0.f;
                for (int s = 0; s < q.ns; ++s) gs += gpad[q.g_off + (long long)s * npts + z * q.nxp + x];
                row += gs * (wz / sqrtf(K[q.pt_off + z * q.nxp + x]));
            }
            sum += row;
        }
        grad[i] = sum;
    }
}

// One non-inlined entry per compiled variant: each gets its own register
// allocation (the persistent kernel needs only the largest, not their sum);
// the call happens once per unit.
template <int X, int P, bool EX>
__device__ __noinline__ void unit_lds_forward(const BatchUnit* __restrict__ U, float* lds) {
    const LdsArgs a = uniform(U->la);
    lds_field<X, P, false, EX, false>(a, 0, uniform(U->ax), uniform(U->az), lds);
}

template <int RB, int SM>
__device__ __noinline__ void unit_glb_forward(const BatchUnit* __restrict__ U, float* lds) {
    glb_field_forward<RB, SM>(*U, lds);
}

template <int X, int PI, bool EX>
__device__ __noinline__ void unit_split_forward(const BatchUnit* __restrict__ U, float* lds) {
    const LdsArgs a = uniform(U->la);
    split_field<X, PI, false, EX, false>(a, uniform(U->sp), 0, uniform(U->part), uniform(U->ax), uniform(U->az), lds);
}

__device__ void run_unit_forward(const BatchUnit* U, float* lds) {
    const int kind = U->kind, variant = U->variant;
    if (kind == 2) {
#define FWI_SPLIT_CASE(ID, XX, PP, EX)               \
    if (variant == ID) {                             \
        unit_split_forward<XX, PP, EX>(U, lds);      \
        return;                                      \
    }
        FWI_BATCH_SPLIT(FWI_SPLIT_CASE)
#undef FWI_SPLIT_CASE
        return;
    }
    if (kind == 0) {
#define FWI_LDS_CASE(ID, XX, PP, EX)                 \
    if (variant == ID) {                             \
        unit_lds_forward<XX, PP, EX>(U, lds);        \
        return;                                      \
    }
        FWI_BATCH_LDS(FWI_LDS_CASE)
#undef FWI_LDS_CASE
    } else {
#define FWI_GLB_CASE(ID, RBB, SM)                    \
    if (variant == ID) {                             \
        unit_glb_forward<RBB, SM>(U, lds);           \
        return;                                      \
    }
        FWI_BATCH_GLB(FWI_GLB_CASE)
#undef FWI_GLB_CASE
    }
}

__global__ __launch_bounds__(kLdsThreads) void k_batch_forward(const BatchUnit* __restrict__ units, int nunits,
                                                               int* __restrict__ counter) {
    extern __shared__ float lds[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int u = __builtin_amdgcn_readfirstlane(next);  // uniform: descriptor fields load as scalars
        __syncthreads();
        if (u >= nunits) break;  // every workgroup leaves once the queue is drained
        run_unit_forward(units + u, lds);
        __syncthreads();
    }
}

// Points the queued units at this call's packed traces, wavelets and (for
// gradients) adjoint sources.
__global__ void k_batch_bind(BatchUnit* __restrict__ units, int nunits, float* __restrict__ traces,
                             const float* __restrict__ wavelets, const float* __restrict__ adj) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nunits) return;
    BatchUnit& U = units[u];
    U.adj = adj ? adj + U.tr_off : nullptr;
    if (U.kind == 1 && U.nparts > 1 && U.part == 0) *U.bar = 0;
    if (U.kind == 0 || U.kind == 2) {
        U.la.traces = traces + U.tr_off;
        U.la.wavelet = wavelets + U.w_off;
        U.la.adj = U.adj;
    } else {
        U.traces = traces + U.tr_off;
        U.wavelet = wavelets + U.w_off;
    }
}

__global__ void k_reset_counter(int* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

// K = (v dt)^2 on every request's padded grid (edge-replicated velocity) in
// one launch; thread i finds its request by bisection over the point offsets.
struct PrepReq {
    long long pt_off;   // first padded point of the request in the packed K
    long long v_off;    // first model cell in the packed velocity
    int nz, nx, nzp, nxp, ztop, nb;
    float dt, vmax;
};

__global__ void k_batch_prep(const PrepReq* __restrict__ req, int nreq, long long total, const float* __restrict__ v,
                             float* __restrict__ K, int* __restrict__ flags) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        int lo = 0, hi = nreq - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (req[mid].pt_off <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        const PrepReq& q = req[lo];
        const int p = (int)(i - q.pt_off);
        const int iz = p / q.nxp, ix = p - (p / q.nxp) * q.nxp;
        const int mz = min(max(iz - q.ztop, 0), q.nz - 1);
        const int mx = min(max(ix - q.nb, 0), q.nx - 1);
        const float vv = v[q.v_off + (long long)mz * q.nx + mx];
        if (!(vv > 0.f) || !(vv <= q.vmax)) atomicOr(flags, kFlagBadVelocity);
        const float c = vv * q.dt;
        K[i] = c * c;
    }
}

}  // namespace fwi

// ---------------------------------------------------------------------------
// Host side
using namespace fwi;

struct fwi_batch {
    int device = 0, nreq = 0, n_cu = 0;
    std::vector<fwi_geometry> g;
    std::vector<std::vector<int>> idx;           // host copies of the index arrays
    std::vector<int> nzp, nxp, ztop, kind, variant, tuned;
    std::vector<long long> v_off, w_off, tr_off, pt_off;
    long long v_total = 0, w_total = 0, tr_total = 0, pt_total = 0;
    std::vector<BatchUnit> units;                // queue order
    std::vector<int> unit_req;                   // request of each queued unit
    std::vector<int> unit_shot;                  // shot of each queued unit
    int* bars = nullptr;                         // barrier counters of the fields cut into parts
    // kind 2 (row bands in LDS): per request the split layout, and the bands' exchange rows
    std::vector<int> sp_X, sp_P, sp_ncg, sp_nstrip, sp_G;
    unsigned long long* xchg = nullptr;
    size_t xchg_words = 0;
    BatchUnit* d_units = nullptr;
    PrepReq* d_prep = nullptr;
    int* counter = nullptr;
    int* flags = nullptr;
    float* K = nullptr;
    size_t lds_bytes = 0;
    std::vector<void*> allocs;
    std::vector<std::pair<int, int>> shape;      // (nzp, nxp) of each request
    // gradients
    int gradients = 0;
    float* gpad = nullptr;         // per request [ns][npts] at g_off
    float* tr_scratch = nullptr;   // traces of the gradient's forward sweeps
    FoldReq* d_fold = nullptr;
    std::vector<long long> g_off;
    size_t grad_bytes = 0;
};

namespace {

struct TuneKey {
    int nzp, nxp, kind, exact;
    bool operator<(const TuneKey& o) const {
        return std::tie(nzp, nxp, kind, exact) < std::tie(o.nzp, o.nxp, o.kind, o.exact);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;  // process-wide autotuner results

struct LdsVar {
    int X, P;
    bool exact;
};
const LdsVar kLdsVar[kBatchLdsVariants] = {
#define FWI_V(ID, XX, PP, EX) {XX, PP, EX},
    FWI_BATCH_LDS(FWI_V)
#undef FWI_V
};
struct GlbVar {
    int RB, SMUL;
};
const GlbVar kGlbVar[kBatchGlbVariants] = {
#define FWI_V(ID, RBB, SM) {RBB, SM},
    FWI_BATCH_GLB(FWI_V)
#undef FWI_V
};

constexpr int kMaxParts = 4;     // row parts of one HBM-swept field
constexpr int kMinPartRows = 16;

// dynamic LDS of the persistent kernels: all of it but a little for their
// static variables (the work-queue slot)
constexpr int kBatchDynLds = kLdsBytes - 256;

// one 72-float row buffer per wave
size_t glb_lds(int, int) { return (size_t)(kLdsThreads / 64) * 72 * sizeof(float); }

bool lds_var_fits(int v, int nzp, int nxp, int* ncg, int* nstrip) {
    const LdsVar& L = kLdsVar[v];
    *ncg = (nxp + L.X - 1) / L.X;
    *nstrip = (nzp + L.P - 1) / L.P;
    const bool exact = *ncg * L.X == nxp && *nstrip * L.P == nzp;
    if (L.exact != exact) return false;
    return *ncg * *nstrip <= kLdsThreads && lds_bytes(L.X, L.P, *ncg, *nstrip) <= (size_t)kBatchDynLds;
}

// Row-band layout of a field held in LDS by G workgroups (kind 2): X columns
// per thread (4 or 6) so that the 8 boundary rows of ncg column groups fit
// 512 threads, PI interior rows per tile, as many strips as threads allow.
// Among the layouts whose band fits the LDS, the one with the fewest cycles
// per step summed over its bands (VALU and LDS work per point as the split
// sweep's cost model, plus the exchange latency per band).
bool batch_split_layout(int nzp, int nxp, int* Xo, int* Po, int* ncgo, int* nstripo, int* Go, int* vo) {
    double best = 1e300;
    bool found = false;
#define FWI_TRY_SPLIT(ID, XX, PP, EX)                                                                  \
    {                                                                                                \
        const int ncg = (nxp + XX - 1) / XX;                                                         \
        const int smax = kLdsThreads / ncg;                                                          \
        if (smax >= 8 && (ncg * XX == nxp) == EX) {                                                  \
            const int G = (nzp + 8 + smax * PP - 1) / (8 + smax * PP);                               \
            const int nstrip = std::max(1, ((nzp + G - 1) / G - 8 + PP - 1) / PP);                   \
            const int H = 8 + nstrip * PP;                                                           \
            if (G >= 2 && nstrip <= smax && (long long)G * H >= nzp &&                               \
                split_lds_bytes(XX, PP, ncg, nstrip) <= (size_t)kBatchDynLds) {                      \
                const double pts = (double)ncg * XX * H;                                             \
                const double c = G * (pts * (33.0 / 64.0 + ((PP + 8.0) / PP + 8.0 / XX + 1.0) / 32.0) + 1500.0); \
                if (c < best) {                                                                      \
                    best = c;                                                                        \
                    *Xo = XX;                                                                        \
                    *Po = PP;                                                                        \
                    *ncgo = ncg;                                                                     \
                    *nstripo = nstrip;                                                               \
                    *Go = G;                                                                         \
                    *vo = ID;                                                                        \
                    found = true;                                                                    \
                }                                                                                    \
            }                                                                                        \
        }                                                                                            \
    }
    FWI_BATCH_SPLIT(FWI_TRY_SPLIT)
#undef FWI_TRY_SPLIT
    return found;
}

template <class T>
int balloc(fwi_batch* b, T** p, size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return FWI_ENOMEM;
    b->allocs.push_back(q);
    *p = (T*)q;
    return FWI_OK;
}

void bfree(fwi_batch* b) {
    for (void* q : b->allocs) (void)hipFree(q);
    b->allocs.clear();
}

// The persistent kernels run one workgroup per CU at most (grid <= CUs, and
// their LDS allows one per CU).  Row parts of a field wait for each other at
// a per-step barrier, which needs every workgroup resident: outside graph
// capture the launch is cooperative, which guarantees that; a cooperative
// launch cannot be captured, so under capture it is a plain launch, and a
// wait that outlasts its bounded spin raises the batch flag instead of hanging.
int launch_units(BatchUnit* d_units, int nunits, int* counter, int grid, size_t lds, float* traces,
                 const float* wavelets, hipStream_t st, const float* adj = nullptr, bool gradient = false) {
    hipLaunchKernelGGL(k_batch_bind, dim3((nunits + 255) / 256), dim3(256), 0, st, d_units, nunits, traces, wavelets,
                       adj);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
    const void* kern = gradient ? (const void*)k_batch_gradient : (const void*)k_batch_forward;
    if (!stream_capturing(st)) {
        void* args[] = {(void*)&d_units, (void*)&nunits, (void*)&counter};
        return hip_ok(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kLdsThreads), args, (unsigned)lds, st));
    }
    if (gradient)
        hipLaunchKernelGGL(k_batch_gradient, dim3(grid), dim3(kLdsThreads), lds, st, d_units, nunits, counter);
    else
        hipLaunchKernelGGL(k_batch_forward, dim3(grid), dim3(kLdsThreads), lds, st, d_units, nunits, counter);
    return hip_ok(hipGetLastError());
}

// Fills the unit descriptor of (request r, shot s) for a given kind/variant.
// Per-unit device arrays (state, traces) are passed in.
struct ReqDev {
    float* ax;
    float* az;
    int* src_pt;
    int* rec_map;
    int* rec_of_col;
    float* rec_invw;
    HostTables ht;
};

BatchUnit make_unit(const fwi_batch* b, int r, int s, int kind, int variant, const ReqDev& rd, const float* K,
                    long long w_off, long long tr_off, float* state, int nsteps) {
    const fwi_geometry& g = b->g[r];
    BatchUnit U{};
    U.kind = kind;
    U.variant = variant;
    U.nsteps = nsteps;
    U.tr_off = tr_off;
    U.w_off = w_off;
    U.ax = rd.ax;
    U.az = rd.az;
    const int nzp = b->nzp[r], nxp = b->nxp[r];
    if (kind == 0 || kind == 2) {
        LdsArgs& a = U.la;
        a.nzp = nzp;
        a.nxp = nxp;
        a.npts = nzp * nxp;
        if (kind == 0) {
            const LdsVar& V = kLdsVar[variant];
            a.X = V.X;
            a.P = V.P;
            a.ncg = (nxp + V.X - 1) / V.X;
            a.nstrip = (nzp + V.P - 1) / V.P;
        } else {
            a.X = b->sp_X[r];
            a.P = b->sp_P[r];
            a.ncg = b->sp_ncg[r];
            a.nstrip = b->sp_nstrip[r];
        }
        a.S = a.ncg * a.X + 8;
        a.fs = g.free_surface ? 1 : 0;
        a.nt = nsteps + 1;
        a.ns = 1;
        a.nr = g.nr;
        a.rec_row = rd.ht.rec_row;
        a.rec_invw = (g.free_surface && rd.ht.rec_row == 0) ? 2.f : 1.f;
        a.idz2 = (float)(1.0 / (g.dz * g.dz));
        a.idx2 = (float)(1.0 / (g.dx * g.dx));
        a.src_scale = (float)(1.0 / (g.dx * g.dz));
        a.K = K;
        a.src_pt = rd.src_pt + s;
        a.rec_of_col = rd.rec_of_col;
        a.store = 0;
    } else {
        U.nzp = nzp;
        U.nxp = nxp;
        U.fs = g.free_surface ? 1 : 0;
        U.nt = nsteps + 1;
        U.nr = g.nr;
        U.src_pt = rd.ht.src_pt[s];
        U.rec_z0 = rd.ht.rec_z0;
        U.rec_z1 = rd.ht.rec_z1;
        U.idz2 = (float)(1.0 / (g.dz * g.dz));
        U.idx2 = (float)(1.0 / (g.dx * g.dx));
        U.src_scale = (float)(1.0 / (g.dx * g.dz));
        U.K = K;
        U.rec_map = rd.rec_map;
        U.rec_invw = rd.rec_invw;
        const size_t npts = (size_t)nzp * nxp;
        U.ua = state;
        U.ub = state + npts;
        U.w = state + 2 * npts;
        U.z_lo = 0;
        U.z_hi = nzp;
        U.part = 0;
        U.nparts = 1;
        U.bar = nullptr;
        U.flags = b->flags;
    }
    return U;
}

}  // namespace

extern "C" {

int fwi_batch_create(int nreq, const fwi_geometry* geoms, const fwi_batch_options* opt, fwi_batch** out) {
    if (!out || nreq < 1 || !geoms) return FWI_EINVAL;
    *out = nullptr;
    fwi_batch_options o{1, 0, 0};
    if (opt) o = *opt;
    if (o.autotune < 0 || o.autotune > 1 || o.gradients < 0 || o.gradients > 1 || o.bands < -1 || o.bands > 0)
        return FWI_EINVAL;
    for (int r = 0; r < nreq; ++r) {
        const int st = validate_geometry(&geoms[r], 1);
        if (st) return st;
        if (geoms[r].pml) return FWI_EINVAL;  // the persistent kernels implement the sponge only
    }
    // the persistent kernels may use all of the LDS their static variables
    // leave; set here so that the launches make no other runtime calls
    for (const void* kern : {(const void*)k_batch_forward, (const void*)k_batch_gradient}) {
        hipFuncAttributes fa{};
        if (hipFuncGetAttributes(&fa, kern) != hipSuccess || (int)fa.sharedSizeBytes > kLdsBytes - kBatchDynLds ||
            hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, kBatchDynLds) != hipSuccess) {
            (void)hipGetLastError();
            return FWI_EHIP;
        }
    }
    fwi_batch* b = new (std::nothrow) fwi_batch();
    if (!b) return FWI_ENOMEM;
    (void)hipGetDevice(&b->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
        delete b;
        return FWI_EHIP;
    }
    b->n_cu = prop.multiProcessorCount;
    b->nreq = nreq;
    b->g.assign(geoms, geoms + nreq);
    b->idx.resize(4 * (size_t)nreq);
    std::vector<ReqDev> rd(nreq);
    int st = FWI_OK;
    for (int r = 0; r < nreq; ++r) {
        fwi_geometry& g = b->g[r];
        b->idx[4 * r + 0].assign(g.src_iz, g.src_iz + g.ns);
        b->idx[4 * r + 1].assign(g.src_ix, g.src_ix + g.ns);
        b->idx[4 * r + 2].assign(g.rec_iz, g.rec_iz + g.nr);
        b->idx[4 * r + 3].assign(g.rec_ix, g.rec_ix + g.nr);
        g.src_iz = b->idx[4 * r + 0].data();
        g.src_ix = b->idx[4 * r + 1].data();
        g.rec_iz = b->idx[4 * r + 2].data();
        g.rec_ix = b->idx[4 * r + 3].data();
        g.free_surface = g.free_surface ? 1 : 0;
        const int ztop = g.free_surface ? 0 : g.nb;
        const int nzp = g.nz + g.nb + ztop, nxp = g.nx + 2 * g.nb;
        b->ztop.push_back(ztop);
        b->nzp.push_back(nzp);
        b->nxp.push_back(nxp);
        b->v_off.push_back(b->v_total);
        b->w_off.push_back(b->w_total);
        b->tr_off.push_back(b->tr_total);
        b->pt_off.push_back(b->pt_total);
        b->v_total += (long long)g.nz * g.nx;
        b->w_total += g.nt;
        b->tr_total += (long long)g.ns * g.nr * g.nt;
        b->pt_total += (long long)nzp * nxp;
        build_host_tables(g, nzp, nxp, ztop, rd[r].ht);
        st = st ? st : balloc(b, &rd[r].ax, (size_t)nxp);
        st = st ? st : balloc(b, &rd[r].az, (size_t)nzp);
        st = st ? st : balloc(b, &rd[r].src_pt, (size_t)g.ns);
        st = st ? st : balloc(b, &rd[r].rec_map, (size_t)nzp * nxp);
        st = st ? st : balloc(b, &rd[r].rec_of_col, (size_t)nxp);
        st = st ? st : balloc(b, &rd[r].rec_invw, (size_t)g.nr);
        if (st) break;
        const HostTables& t = rd[r].ht;
        st = hip_ok(hipMemcpy(rd[r].ax, t.ax.data(), nxp * sizeof(float), hipMemcpyHostToDevice));
        st = st ? st : hip_ok(hipMemcpy(rd[r].az, t.az.data(), nzp * sizeof(float), hipMemcpyHostToDevice));
        st = st ? st : hip_ok(hipMemcpy(rd[r].src_pt, t.src_pt.data(), g.ns * sizeof(int), hipMemcpyHostToDevice));
        st = st ? st
                : hip_ok(hipMemcpy(rd[r].rec_map, t.rec_map.data(), t.rec_map.size() * sizeof(int),
                                   hipMemcpyHostToDevice));
        st = st ? st
                : hip_ok(hipMemcpy(rd[r].rec_of_col, t.rec_of_col.data(), nxp * sizeof(int), hipMemcpyHostToDevice));
        st = st ? st
                : hip_ok(hipMemcpy(rd[r].rec_invw, t.rec_invw.data(), g.nr * sizeof(float), hipMemcpyHostToDevice));
        if (st) break;
    }
    st = st ? st : balloc(b, &b->K, (size_t)b->pt_total);
    st = st ? st : balloc(b, &b->counter, 1);
    st = st ? st : balloc(b, &b->flags, 1);
    if (st == FWI_OK && hipMemset(b->flags, 0, sizeof(int)) != hipSuccess) st = FWI_EHIP;
    // kinds: LDS-resident when some variant fits and the receivers share a row
    b->kind.assign(nreq, 1);
    b->variant.assign(nreq, 0);
    b->tuned.assign(nreq, 0);
    for (int r = 0; r < nreq && st == FWI_OK; ++r) {
        int ncg, nstrip;
        if (rd[r].ht.one_row)
            for (int v = 0; v < kBatchLdsVariants; ++v)
                if (lds_var_fits(v, b->nzp[r], b->nxp[r], &ncg, &nstrip)) b->kind[r] = 0;
    }
    // fields too large for one workgroup's LDS run as row bands held in LDS
    // (layout from the split sweep's cost model) when their receivers share a
    // row; in a gradient batch only when the full history of D of those fields
    // fits (at most 60 % of the device memory free at creation), else they are
    // swept from HBM with checkpoints
    b->sp_X.assign(nreq, 0);
    b->sp_P.assign(nreq, 0);
    b->sp_ncg.assign(nreq, 0);
    b->sp_nstrip.assign(nreq, 0);
    b->sp_G.assign(nreq, 0);
    {
        std::vector<std::array<int, 7>> cand;  // r, X, P, ncg, nstrip, G, variant
        size_t dbytes = 0;
        for (int r = 0; r < nreq && st == FWI_OK && o.bands >= 0; ++r) {
            if (b->kind[r] != 1 || !rd[r].ht.one_row) continue;
            int X = 0, P = 0, ncg = 0, nstrip = 0, G = 0, v = -1;
            if (!batch_split_layout(b->nzp[r], b->nxp[r], &X, &P, &ncg, &nstrip, &G, &v) || G > b->n_cu) continue;
            cand.push_back({r, X, P, ncg, nstrip, G, v});
            dbytes += (size_t)b->g[r].ns * b->nzp[r] * b->nxp[r] * (size_t)(b->g[r].nt - 1) * sizeof(float);
        }
        if (o.gradients && !cand.empty()) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
                (void)hipGetLastError();
                free_b = 0;
            }
            if ((double)dbytes > 0.6 * (double)free_b) cand.clear();
        }
        for (const auto& c : cand) {
            const int r = c[0];
            b->kind[r] = 2;
            b->variant[r] = c[6];
            b->sp_X[r] = c[1];
            b->sp_P[r] = c[2];
            b->sp_ncg[r] = c[3];
            b->sp_nstrip[r] = c[4];
            b->sp_G[r] = c[5];
        }
    }

    // autotuning per size class: every candidate on a 64-step sweep of the
    // class's first request, one copy per compute unit
    const int tune_steps = 64;
    for (int r = 0; r < nreq && st == FWI_OK; ++r) {
        if (b->kind[r] == 2) continue;  // layout from the split cost model
        const int nzp = b->nzp[r], nxp = b->nxp[r];
        int ncg, nstrip;
        std::vector<int> cands;
        bool exact = false;
        if (b->kind[r] == 0) {
            for (int v = 0; v < kBatchLdsVariants; ++v)
                if (lds_var_fits(v, nzp, nxp, &ncg, &nstrip)) {
                    cands.push_back(v);
                    exact = exact || kLdsVar[v].exact;
                }
        } else {
            for (int v = 0; v < kBatchGlbVariants; ++v) cands.push_back(v);
        }
        const TuneKey key{nzp, nxp, b->kind[r], exact ? 1 : 0};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end()) {
                b->variant[r] = it->second;
                b->tuned[r] = 1;
                continue;
            }
        }
        if (!o.autotune || cands.size() == 1 || b->g[r].nt - 1 < tune_steps) {
            // cost model: LDS operations per point (LDS kind), fewest tiles (HBM kind)
            int best = cands[0];
            double bc = 1e300;
            for (int v : cands) {
                double c;
                if (b->kind[r] == 0) {
                    const LdsVar& L = kLdsVar[v];
                    lds_var_fits(v, nzp, nxp, &ncg, &nstrip);
                    c = (double)ncg * L.X * nstrip * L.P * ((L.P + 8.0) / L.P + 8.0 / L.X + 1.0);
                } else {
                    // deeper prefetch first, then fewer panel restarts (8 extra rows each)
                    const GlbVar& G = kGlbVar[v];
                    c = 1.0 / G.RB + 0.01 * G.SMUL;
                }
                if (c < bc) {
                    bc = c;
                    best = v;
                }
            }
            b->variant[r] = best;
            continue;
        }
        const fwi_geometry& g = b->g[r];
        const int copies = b->n_cu;
        const size_t npts = (size_t)nzp * nxp;
        float *Kt = nullptr, *wt = nullptr, *trt = nullptr, *stt = nullptr;
        BatchUnit* du = nullptr;
        std::vector<void*> tmp;
        auto talloc = [&](void** p, size_t bytes) {
            if (st) return;
            if (hipMalloc(p, std::max<size_t>(bytes, 4)) != hipSuccess) {
                st = FWI_ENOMEM;
                return;
            }
            tmp.push_back(*p);
        };
        talloc((void**)&Kt, npts * sizeof(float));
        talloc((void**)&wt, (size_t)g.nt * sizeof(float));
        talloc((void**)&trt, (size_t)copies * g.nr * (tune_steps + 1) * sizeof(float));
        talloc((void**)&stt, b->kind[r] == 1 ? (size_t)copies * 3 * npts * sizeof(float) : 4);
        talloc((void**)&du, (size_t)copies * sizeof(BatchUnit));
        if (st == FWI_OK) {
            // a smooth 2000 m/s medium and a unit impulse train stand in for the request's data
            std::vector<float> kh(npts, (float)std::pow(2000.0 * g.dt, 2));
            std::vector<float> wh(g.nt, 0.f);
            wh[1] = 1.f;
            st = hip_ok(hipMemcpy(Kt, kh.data(), npts * sizeof(float), hipMemcpyHostToDevice));
            st = st ? st : hip_ok(hipMemcpy(wt, wh.data(), g.nt * sizeof(float), hipMemcpyHostToDevice));
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (st == FWI_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = FWI_EHIP;
        float best_ms = 1e30f;
        int best = cands[0];
        for (int v : cands) {
            if (st) break;
            std::vector<BatchUnit> hu(copies);
            for (int c = 0; c < copies; ++c)
                hu[c] = make_unit(b, r, 0, b->kind[r], v, rd[r], Kt, 0, (long long)c * g.nr * (tune_steps + 1),
                                  stt + (b->kind[r] == 1 ? (size_t)c * 3 * npts : 0), tune_steps);
            st = hip_ok(hipMemcpy(du, hu.data(), copies * sizeof(BatchUnit), hipMemcpyHostToDevice));
            const size_t lb =
                b->kind[r] == 0 ? lds_bytes(kLdsVar[v].X, kLdsVar[v].P, hu[0].la.ncg, hu[0].la.nstrip) : glb_lds(v, nzp);
            for (int rep = 0; rep < 2 && st == FWI_OK; ++rep) {  // first run warms up
                st = hip_ok(hipEventRecord(e0, nullptr));
                st = st ? st : launch_units(du, copies, b->counter, copies, lb, trt, wt, nullptr);
                st = st ? st : hip_ok(hipEventRecord(e1, nullptr));
                st = st ? st : hip_ok(hipEventSynchronize(e1));
            }
            float ms = 0.f;
            if (st == FWI_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (void* p : tmp) (void)hipFree(p);
        if (st) break;
        b->variant[r] = best;
        b->tuned[r] = 1;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
    }

    // units, longest first.  An HBM-swept field whose time loop alone would
    // outlast the batch's share per compute unit is cut into row parts swept
    // by as many workgroups in lockstep (queued next to each other).
    if (st == FWI_OK) {
        struct Job {
            double cost;  // of one part
            int r, s, part, nparts;
        };
        double total = 0.0;
        for (int r = 0; r < nreq; ++r)
            total += (double)b->g[r].ns * b->nzp[r] * b->nxp[r] * (b->g[r].nt - 1) * (b->kind[r] != 1 ? 0.2 : 1.0);
        const double share = total / std::max(1, b->n_cu);
        std::vector<Job> jobs;
        size_t state_elems = 0, xchg_words = 0;
        int nsplit = 0;
        for (int r = 0; r < nreq; ++r)
            for (int s = 0; s < b->g[r].ns; ++s) {
                const double cost = (double)b->nzp[r] * b->nxp[r] * (b->g[r].nt - 1) * (b->kind[r] != 1 ? 0.2 : 1.0);
                int np = 1;
                if (b->kind[r] == 1 && cost > 1.25 * share)
                    np = std::max(1, std::min({kMaxParts, (int)std::ceil(cost / share), b->nzp[r] / kMinPartRows}));
                if (b->kind[r] == 2) np = b->sp_G[r];
                for (int q = 0; q < np; ++q) jobs.push_back({cost / np, r, s, q, np});
                if (np > 1 && b->kind[r] == 1) ++nsplit;
                // kind 2: exchange rows of the forward sweep, and of the adjoint sweep in gradient batches
                if (b->kind[r] == 2)
                    xchg_words += (o.gradients ? 2 : 1) * (size_t)np * 2 * 2 * 4 * b->sp_ncg[r] * b->sp_X[r];
                if (b->kind[r] == 1) state_elems += 3 * (size_t)b->nzp[r] * b->nxp[r];
            }
        std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& c) { return a.cost > c.cost; });
        float* state = nullptr;
        st = balloc(b, &state, state_elems);
        st = st ? st : balloc(b, &b->bars, (size_t)std::max(nsplit, 1));
        if (xchg_words) {
            st = st ? st : balloc(b, &b->xchg, xchg_words);
            b->xchg_words = xchg_words;
        }
        size_t so = 0, xo = 0;
        int nb = 0;
        std::map<std::pair<int, int>, std::pair<float*, int*>> field;  // (r, s) -> state, barrier
        std::map<std::pair<int, int>, unsigned long long*> fxchg;     // (r, s) -> exchange rows of its bands
        for (const Job& j : jobs) {
            if (st) break;
            const int r = j.r;
            const long long tr_off = b->tr_off[r] + (long long)j.s * b->g[r].nr * b->g[r].nt;
            float* sp = nullptr;
            int* bar = nullptr;
            if (b->kind[r] == 1) {
                auto it = field.find({r, j.s});
                if (it == field.end()) {
                    sp = state + so;
                    so += 3 * (size_t)b->nzp[r] * b->nxp[r];
                    bar = j.nparts > 1 ? b->bars + nb++ : nullptr;
                    field[{r, j.s}] = {sp, bar};
                } else {
                    sp = it->second.first;
                    bar = it->second.second;
                }
            }
            BatchUnit U = make_unit(b, r, j.s, b->kind[r], b->variant[r], rd[r], b->K + b->pt_off[r], b->w_off[r],
                                    tr_off, sp, b->g[r].nt - 1);
            if (b->kind[r] == 2) {
                auto it = fxchg.find({r, j.s});
                unsigned long long* xb;
                const size_t words = (size_t)j.nparts * 2 * 2 * 4 * b->sp_ncg[r] * b->sp_X[r];
                if (it == fxchg.end()) {
                    xb = b->xchg + xo;
                    xo += (o.gradients ? 2 : 1) * words;
                    fxchg[{r, j.s}] = xb;
                } else {
                    xb = it->second;
                }
                U.sp.G = j.nparts;
                U.sp.W = b->sp_ncg[r] * b->sp_X[r];
                U.sp.xchg = xb;
                U.xchg_adj = o.gradients ? xb + words : nullptr;
                U.sp.err = b->flags;
                U.sp.field0 = 0;
                U.part = j.part;
                U.nparts = j.nparts;
            } else if (j.nparts > 1) {
                // rows split evenly; every part takes part of the sweep's panels
                const int nzp = b->nzp[r];
                U.part = j.part;
                U.nparts = j.nparts;
                U.z_lo = (int)((long long)nzp * j.part / j.nparts);
                U.z_hi = (int)((long long)nzp * (j.part + 1) / j.nparts);
                U.bar = bar;
            }
            b->units.push_back(U);
            b->unit_req.push_back(r);
            b->unit_shot.push_back(j.s);
            const size_t lb = b->kind[r] == 0   ? lds_bytes(U.la.X, U.la.P, U.la.ncg, U.la.nstrip)
                              : b->kind[r] == 2 ? split_lds_bytes(U.la.X, U.la.P, U.la.ncg, U.la.nstrip)
                                                : glb_lds(U.variant, U.nzp);
            b->lds_bytes = std::max(b->lds_bytes, lb);
        }
        if (st == FWI_OK && o.gradients) {
            // per field: LDS-resident or row bands -> full history of D; HBM-swept ->
            // adjoint state, checkpoints every C = ceil(sqrt(2 (nt - 1))) steps and one
            // segment of D
            b->gradients = 1;
            long long gtot = 0;
            for (int r = 0; r < nreq; ++r) {
                b->g_off.push_back(gtot);
                gtot += (long long)b->g[r].ns * b->nzp[r] * b->nxp[r];
            }
            st = balloc(b, &b->gpad, (size_t)gtot);
            st = st ? st : balloc(b, &b->tr_scratch, (size_t)b->tr_total);
            b->grad_bytes = (size_t)(gtot + b->tr_total) * sizeof(float);
            std::map<std::pair<int, int>, size_t> first;  // (r, s) -> its first unit: parts share the buffers
            for (size_t ui = 0; ui < b->units.size() && st == FWI_OK; ++ui) {
                BatchUnit& U = b->units[ui];
                const int r = b->unit_req[ui];
                const int shot = b->unit_shot[ui];
                auto f = first.find({r, shot});
                if (f != first.end()) {
                    const BatchUnit& F = b->units[f->second];
                    U.gpad = F.gpad;
                    U.la.Dstore = F.la.Dstore;
                    U.pa = F.pa;
                    U.pb = F.pb;
                    U.pw = F.pw;
                    U.ckpt = F.ckpt;
                    U.dseg = F.dseg;
                    U.ckpt_every = F.ckpt_every;
                    continue;
                }
                first[{r, shot}] = ui;
                const size_t npts = (size_t)b->nzp[r] * b->nxp[r];
                const int nsteps = b->g[r].nt - 1;
                U.gpad = b->gpad + b->g_off[r] + (long long)shot * npts;
                if (U.kind == 0 || U.kind == 2) {
                    float* dst = nullptr;
                    st = balloc(b, &dst, (size_t)nsteps * npts);
                    U.la.Dstore = dst;
                    b->grad_bytes += (size_t)nsteps * npts * sizeof(float);
                } else {
                    const int C = std::max(1, std::min(nsteps, (int)std::ceil(std::sqrt(2.0 * nsteps))));
                    const int nseg = (nsteps + C - 1) / C;
                    float* buf = nullptr;
                    const size_t n = (3 + 2 * (size_t)nseg + C) * npts;
                    st = balloc(b, &buf, n);
                    U.pa = buf;
                    U.pb = buf + npts;
                    U.pw = buf + 2 * npts;
                    U.ckpt = buf + 3 * npts;
                    U.dseg = buf + (3 + 2 * (size_t)nseg) * npts;
                    U.ckpt_every = C;
                    b->grad_bytes += n * sizeof(float);
                }
            }
            std::vector<FoldReq> fr(nreq);
            for (int r = 0; r < nreq; ++r)
                fr[r] = {b->v_off[r], b->pt_off[r], b->g_off[r], b->g[r].nz, b->g[r].nx, b->nzp[r], b->nxp[r],
                         b->g[r].nb, b->ztop[r], b->g[r].ns, (float)b->g[r].dt, b->g[r].free_surface ? 0.5f : 1.f};
            st = st ? st : balloc(b, &b->d_fold, (size_t)nreq);
            st = st ? st : hip_ok(hipMemcpy(b->d_fold, fr.data(), nreq * sizeof(FoldReq), hipMemcpyHostToDevice));
        }
        st = st ? st : balloc(b, &b->d_units, b->units.size());
        st = st ? st
                : hip_ok(hipMemcpy(b->d_units, b->units.data(), b->units.size() * sizeof(BatchUnit),
                                   hipMemcpyHostToDevice));
        std::vector<PrepReq> pr(nreq);
        for (int r = 0; r < nreq; ++r)
            pr[r] = {b->pt_off[r], b->v_off[r], b->g[r].nz, b->g[r].nx, b->nzp[r], b->nxp[r], b->ztop[r], b->g[r].nb,
                     (float)b->g[r].dt, (float)b->g[r].v_max};
        st = st ? st : balloc(b, &b->d_prep, (size_t)nreq);
        st = st ? st : hip_ok(hipMemcpy(b->d_prep, pr.data(), nreq * sizeof(PrepReq), hipMemcpyHostToDevice));
    }
    if (st == FWI_OK && hipDeviceSynchronize() != hipSuccess) st = FWI_EHIP;
    if (st) {
        bfree(b);
        delete b;
        return st;
    }
    *out = b;
    return FWI_OK;
}

int fwi_batch_destroy(fwi_batch* b) {
    if (!b) return FWI_OK;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    bfree(b);
    delete b;
    return FWI_OK;
}

int fwi_batch_get_info(const fwi_batch* b, int r, fwi_batch_request_info* info) {
    if (!b || !info || r < 0 || r >= b->nreq) return FWI_EINVAL;
    info->v_offset = (size_t)b->v_off[r];
    info->wavelet_offset = (size_t)b->w_off[r];
    info->trace_offset = (size_t)b->tr_off[r];
    info->nzp = b->nzp[r];
    info->nxp = b->nxp[r];
    info->kind = b->kind[r];
    if (b->kind[r] == 0) {
        info->tile_x = kLdsVar[b->variant[r]].X;
        info->tile_z = kLdsVar[b->variant[r]].P;
    } else if (b->kind[r] == 2) {
        info->tile_x = b->sp_X[r];
        info->tile_z = b->sp_P[r];
    } else {
        info->tile_x = 64;
        info->tile_z = kGlbVar[b->variant[r]].RB;
    }
    info->tuned = b->tuned[r];
    info->parts = 1;
    for (size_t i = 0; i < b->units.size(); ++i)
        if (b->unit_req[i] == r && b->units[i].kind != 0) info->parts = std::max(info->parts, b->units[i].nparts);
    return FWI_OK;
}

int fwi_batch_sizes(const fwi_batch* b, size_t* v_elems, size_t* wavelet_elems, size_t* trace_elems) {
    if (!b) return FWI_EINVAL;
    if (v_elems) *v_elems = (size_t)b->v_total;
    if (wavelet_elems) *wavelet_elems = (size_t)b->w_total;
    if (trace_elems) *trace_elems = (size_t)b->tr_total;
    return FWI_OK;
}

int fwi_batch_forward(fwi_batch* b, const float* v, const float* wavelets, float* traces, void* stream) {
    if (!b || !v || !wavelets || !traces) return FWI_EINVAL;
    (void)hipSetDevice(b->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const long long total = b->pt_total;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 65535);
    hipLaunchKernelGGL(k_batch_prep, dim3(blocks), dim3(256), 0, st, b->d_prep, b->nreq, total, v, b->K, b->flags);
    if (hipGetLastError() != hipSuccess) return FWI_EHIP;
    if (b->xchg) {  // the bands' exchange rows start at time level 0
        const int rc = launch_fill(reinterpret_cast<float*>(b->xchg), 2 * b->xchg_words, 0.f, st);
        if (rc) return rc;
    }
    const int grid = std::min<int>(b->n_cu, (int)b->units.size());
    return launch_units(b->d_units, (int)b->units.size(), b->counter, grid, b->lds_bytes, traces, wavelets, st);
}

int fwi_batch_gradient(fwi_batch* b, const float* v, const float* wavelets, const float* adj, float* grad,
                       void* stream) {
    if (!b || !v || !wavelets || !adj || !grad) return FWI_EINVAL;
    if (!b->gradients) return FWI_ESTATE;
    (void)hipSetDevice(b->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const long long total = b->pt_total;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 65535);
    hipLaunchKernelGGL(k_batch_prep, dim3(blocks), dim3(256), 0, st, b->d_prep, b->nreq, total, v, b->K, b->flags);
    if (hipGetLastError() != hipSuccess) return FWI_EHIP;
    if (b->xchg) {  // the bands' exchange rows (both sweeps) start at time level 0
        const int rc = launch_fill(reinterpret_cast<float*>(b->xchg), 2 * b->xchg_words, 0.f, st);
        if (rc) return rc;
    }
    const int grid = std::min<int>(b->n_cu, (int)b->units.size());
    int rc = launch_units(b->d_units, (int)b->units.size(), b->counter, grid, b->lds_bytes, b->tr_scratch, wavelets,
                          st, adj, true);
    if (rc) return rc;
    const long long cells = b->v_total;
    hipLaunchKernelGGL(k_batch_fold, dim3((int)std::min<long long>((cells + 255) / 256, 65535)), dim3(256), 0, st,
                       b->d_fold, b->nreq, cells, b->K, b->gpad, grad);
    return hip_ok(hipGetLastError());
}

int fwi_batch_status(fwi_batch* b) {
    if (!b) return FWI_EINVAL;
    (void)hipSetDevice(b->device);
    if (hipDeviceSynchronize() != hipSuccess) return FWI_EHIP;
    int flags = 0;
    if (hipMemcpy(&flags, b->flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return FWI_EHIP;
    if (flags) {
        (void)hipMemset(b->flags, 0, sizeof(int));
        (void)hipDeviceSynchronize();
        return FWI_EDEVICE;
    }
    return FWI_OK;
}

}  // extern "C"
