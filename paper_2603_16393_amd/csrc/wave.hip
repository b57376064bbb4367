// Acoustic wave propagation on gfx950: forward modelling and the adjoint
// sweep with the zero-lag imaging condition.
//
// Scheme (the constant-density acoustic equation of Sec. 2.1 with the solver
// settings of Sec. 6.1; a damping sponge stands in for the PML):
//   D^n     = L u^n + s^n                    (8th-order Laplacian; s^n = f_n/(dx dz) at the source node)
//   u^{n+1} = (1 + a) u^n - a u^{n-1} + K D^n,   K = (v dt)^2,  a = a_x(x) a_z(z) (1 in the model),
// advanced as w^{n+1} = a w^n + K D^n, u^{n+1} = u^n + w^{n+1} with the
// Laplacian summed as differences from the centre value (FP32 rounding then
// neither cancels in L nor feeds back through the second difference).
// Traces: d^n = u^n at the receivers.  With W = diag(1/2 on a reflecting top
// row, 1 elsewhere), W L is symmetric, so the adjoint field psi obeys the same
// recursion backward in time with sources a^n / w at the receivers, and
//   dJ/dv_pad = (2 w / v) sum_n psi^{n+1} D^n,
// folded onto the model by transposing the edge replication.
//
// Two execution paths:
//  * LDS-resident (wave_lds.hip): one workgroup per (sample, shot) keeps the
//    whole padded field in LDS for all nt-1 steps, or, when the batch leaves
//    compute units idle, several workgroups each keep a band of its rows and
//    exchange halos every step (wave_split_body.h).
//  * tiled (this file): fields too large for LDS are swept two time steps per
//    launch in 64 x 16 tiles staged through LDS (k_wave_tile2; k_wave_tile for
//    a single step).  Each
//    sweep's launches are captured once into a hipGraph on a plan-owned
//    stream and replayed on the caller's stream; the graph touches only
//    plan-owned buffers (traces and adjoint sources are staged through them).
//    When the full history of D does not fit the memory budget, the forward
//    sweep saves (u, w) every ckpt_every steps and the adjoint sweep recomputes
//    each segment's D before stepping backward through it.
#include <algorithm>
#include <cmath>

#include "fwi_internal.h"

namespace fwi {

// ---------------------------------------------------------------------------
// Velocity -> padded coefficient K = (v dt)^2, with the device-side check.
__global__ void k_prep_velocity(int B, int nz, int nx, int nzp, int nxp, int ztop, int nb, float dt, float vmax,
                                const float* __restrict__ v, float* __restrict__ K, int* __restrict__ flags) {
    const int npts = nzp * nxp;
    const long total = (long)B * npts;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int b = (int)(i / npts);
        const int p = (int)(i - (long)b * npts);
        const int iz = p / nxp, ix = p - (p / nxp) * nxp;
        const int mz = min(max(iz - ztop, 0), nz - 1);
        const int mx = min(max(ix - nb, 0), nx - 1);
        const float vv = v[(size_t)b * nz * nx + mz * nx + mx];
        if (!(vv > 0.f) || !(vv <= vmax)) atomicOr(flags, kFlagBadVelocity);  // also catches NaN
        const float c = vv * dt;
        K[i] = c * c;
    }
}

int launch_prep_velocity(const Plan& p, int B, const float* v, hipStream_t st) {
    const long total = (long)B * p.npts;
    const int threads = 256;
    const int blocks = (int)std::min<long>((total + threads - 1) / threads, 65535);
    hipLaunchKernelGGL(k_prep_velocity, dim3(blocks), dim3(threads), 0, st, B, p.g.nz, p.g.nx, p.nzp, p.nxp, p.ztop,
                       p.g.nb, (float)p.g.dt, (float)p.g.v_max, v, p.K, p.flags);
    return hip_ok(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Tiled sweep, one time step: block = 64 columns x 4 strips of 4 rows (a
// 64 x 16 tile); the tile of u^n plus a 4-cell halo is staged in LDS.
constexpr int TX = 64, TZ = 16, TSTRIP = 4, TROWS = TZ / TSTRIP;

template <bool ADJ>
__global__ __launch_bounds__(256) void k_wave_tile(TileArgs a, int m, const float* __restrict__ ax_g,
                                                   const float* __restrict__ az_g) {
    constexpr int SS = TX + 8;
    __shared__ float tile[(TZ + 8) * SS];
    const TileIdx ti = tile_of_block();
    const int field = ti.field;
    const int b = field / a.ns;
    const int s = field - b * a.ns;
    const int x0 = ti.tx * TX, zt = ti.tz * TZ;
    const int tx = threadIdx.x % TX, ts = threadIdx.x / TX;
    const int nxp = a.nxp, nzp = a.nzp;
    const float* uc = a.ucur + (size_t)field * a.npts;
    float* un_g = a.unxt + (size_t)field * a.npts;
    float* wg = a.wst + (size_t)field * a.npts;

    for (int i = threadIdx.x; i < (TZ + 8) * SS; i += 256) {
        const int r = i / SS, c = i - (i / SS) * SS;
        int gz = zt + r - 4;
        const int gx = x0 + c - 4;
        if (a.fs && gz < 0) gz = -gz;
        float val = 0.f;
        if (gz >= 0 && gz < nzp && gx >= 0 && gx < nxp) val = uc[gz * nxp + gx];
        tile[i] = val;
    }
    __syncthreads();
    const int gx = x0 + tx;
    if (gx >= nxp) return;
    const float axv = ax_g[gx];
    const int sp = a.src_pt[s];
    const bool check_rec = (zt + TZ > a.rec_z0) && (zt <= a.rec_z1);
#pragma unroll
    for (int j = 0; j < TROWS; ++j) {
        const int lz = ts * TROWS + j;
        const int gz = zt + lz;
        if (gz >= nzp) break;
        const int p = gz * nxp + gx;
        const int li = (lz + 4) * SS + tx + 4;
        const float c = tile[li];
        const float lzs = FWI_LAPD(c, tile[li - 4 * SS], tile[li - 3 * SS], tile[li - 2 * SS], tile[li - SS],
                                   tile[li + SS], tile[li + 2 * SS], tile[li + 3 * SS], tile[li + 4 * SS]);
        const float lxs = FWI_LAPD(c, tile[li - 4], tile[li - 3], tile[li - 2], tile[li - 1], tile[li + 1],
                                   tile[li + 2], tile[li + 3], tile[li + 4]);
        float D = fmaf(lzs, a.idz2, lxs * a.idx2);
        int r = -1;
        if (check_rec) r = a.rec_map[p];
        if (!ADJ && p == sp) D = fmaf(a.wavelet[m], a.src_scale, D);
        if (ADJ && r >= 0) D = fmaf(a.rec_invw[r], a.adj[((size_t)field * a.nr + r) * a.nt + (a.nt - 1 - m)], D);
        const float Kp = a.K[(size_t)b * a.npts + p];
        const float wn = fmaf(Kp, D, (axv * az_g[gz]) * wg[p]);
        const float un = c + wn;
        wg[p] = wn;
        un_g[p] = un;
        if (ADJ) {
            if (a.Din) {
                float* acc = a.acc + (size_t)field * a.npts + p;
                *acc = fmaf(un, a.Din[(size_t)field * a.dstride + p], *acc);
            }
        } else {
            if (a.Dout) a.Dout[(size_t)field * a.dstride + p] = D;
            if (r >= 0 && a.traces) a.traces[((size_t)field * a.nr + r) * a.nt + m + 1] = un;
        }
    }
}

// Two time steps per launch (temporal blocking): the block computes step 1
// on its 64 x 16 tile plus a 4-cell ring (72 x 24 points, from u^n staged with
// an 8-cell ring), keeps u^{n+1} of that region in LDS and w^{n+1} of the tile
// in the registers of the thread that updates the point again in step 2, then
// computes step 2 on the tile.  Every point is updated with the same
// operations as in k_wave_tile (the ring points again by each block that
// needs them), so two launches of k_wave_tile and one of this kernel agree
// bitwise; u, w and K pass through HBM once per two steps and, in the adjoint,
// the imaging sum is read and written once per two steps.  w is not updated in
// place (a neighbour still reads w^n of the ring): w^n from a.wst, w^{n+2} to
// wout.  Step 1 is step m (forward: time index m; adjoint: step m of the
// reversed recursion), step 2 is m + 1; Dout / Din belong to step 1, Dout2 /
// Din2 to step 2.
constexpr int EX = TX + 8, EZ = TZ + 8;   // step-1 region: the tile and a 4-cell ring
constexpr int AX = TX + 16, AZ = TZ + 16; // u^n window: the tile and an 8-cell ring

template <bool ADJ>
__global__ __launch_bounds__(256) void k_wave_tile2(TileArgs a, int m, const float* __restrict__ ax_g,
                                                    const float* __restrict__ az_g, float* __restrict__ wout,
                                                    float* __restrict__ Dout2, const float* __restrict__ Din2) {
    // Each phase first issues a thread's global loads (clamped addresses, so no load sits
    // in a divergent branch; in step 1 four points at a time, which keeps the kernel within
    // 64 VGPRs) and only then uses them: the loads of one thread overlap instead of waiting
    // one by one.  17 KB of LDS and at most 64 VGPRs: 8 waves per SIMD.
    constexpr int NA = (AZ * AX + 255) / 256;  // u^n values staged per thread
    __shared__ float A[AZ * AX];   // u^n
    __shared__ float Bt[EZ * EX];  // u^{n+1}
    const TileIdx ti = tile_of_block();
    const int field = ti.field;
    const int b = field / a.ns;
    const int s = field - b * a.ns;
    const int x0 = ti.tx * TX, zt = ti.tz * TZ;
    const int nxp = a.nxp, nzp = a.nzp;
    const float* uc = a.ucur + (size_t)field * a.npts;
    const float* wg = a.wst + (size_t)field * a.npts;
    const float* Kb = a.K + (size_t)b * a.npts;
    const int sp = a.src_pt[s];
    const size_t trf = (size_t)field * a.nr;
    const int tid = threadIdx.x;

    {
        float va[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int i = tid + k * 256;
            const int r = i / AX, c = i - (i / AX) * AX;
            int gz = zt + r - 8;
            const int gx = x0 + c - 8;
            if (a.fs && gz < 0) gz = -gz;
            const float t = uc[min(max(gz, 0), nzp - 1) * nxp + min(max(gx, 0), nxp - 1)];
            va[k] = (gz >= 0 && gz < nzp && gx >= 0 && gx < nxp) ? t : 0.f;
        }
#pragma unroll
        for (int k = 0; k < NA; ++k)
            if (tid + k * 256 < AZ * AX) A[tid + k * 256] = va[k];
    }
    __syncthreads();

    // step 1 on the tile and its ring: each thread first takes the 4 tile points it updates again in step 2
    // (w^{n+1} stays in its registers), then up to 3 of the 704 ring points
    const bool rec1 = (zt + TZ + 4 > a.rec_z0) && (zt - 4 <= a.rec_z1);
    const int tx = tid % TX, ts = tid / TX;
    float w1[TROWS];
    // step 2 updates the same four tile points: K, the damping product, the receiver and its weight of each,
    // loaded in step 1, stay in registers
    float kt[TROWS], dt[TROWS], it[TROWS];
    int rt[TROWS];
    {
        constexpr int NRING = EZ * EX - TZ * TX;  // 704
        constexpr int NP = TROWS + (NRING + 255) / 256;
        const float src = ADJ ? 0.f : a.wavelet[m];
        // region coordinates (r, c) of this thread's points: the tile points, then the ring points
        auto point = [&](int k, int& r, int& c) -> bool {
            if (k < TROWS) {
                r = 4 + ts * TROWS + k;
                c = 4 + tx;
                return true;
            }
            const int q = tid + (k - TROWS) * 256;
            if (q >= NRING) return false;
            if (q < 4 * EX) {
                r = q / EX;
                c = q - r * EX;
            } else if (q < 8 * EX) {
                r = TZ + 4 + (q - 4 * EX) / EX;
                c = (q - 4 * EX) - (r - TZ - 4) * EX;
            } else {
                const int e = q - 8 * EX;  // rows 4 .. TZ + 3, the 4 columns at each side
                r = 4 + e / 8;
                const int c8 = e - (e / 8) * 8;
                c = c8 < 4 ? c8 : TX + c8;
            }
            return true;
        };
        // the column of u^n a thread's tile points need vertically (rows 4 .. 15 of its strip), in registers
        float ca[TROWS + 8];
#pragma unroll
        for (int i = 0; i < TROWS + 8; ++i) ca[i] = A[(ts * TROWS + 4 + i) * AX + tx + 8];
        constexpr int CH = 4;  // points whose loads are in flight together
#pragma unroll
        for (int k0 = 0; k0 < NP; k0 += CH) {
            float kv[CH], wv[CH], dv[CH], av[CH], iv[CH];
            int rv[CH];
#pragma unroll
            for (int kk = 0; kk < CH; ++kk) {
                const int k = k0 + kk;
                if (k >= NP) break;
                int r = 0, c = 0;
                point(k, r, c);
                const int gz = min(max(zt + r - 4, 0), nzp - 1), gx = min(max(x0 + c - 4, 0), nxp - 1);
                const int p = gz * nxp + gx;
                kv[kk] = Kb[p];
                wv[kk] = wg[p];
                dv[kk] = ax_g[gx] * az_g[gz];
                rv[kk] = -1;
                av[kk] = iv[kk] = 0.f;
                if (rec1) {
                    rv[kk] = a.rec_map[p];
                    if (ADJ) {
                        const int q = max(rv[kk], 0);
                        av[kk] = a.adj[(trf + q) * a.nt + (a.nt - 1 - m)];
                        iv[kk] = a.rec_invw[q];
                    }
                }
            }
#pragma unroll
            for (int kk = 0; kk < CH; ++kk) {
                const int k = k0 + kk;
                if (k >= NP) break;
                int r = 0, c = 0;
                if (!point(k, r, c)) continue;
                const int gz = zt + r - 4, gx = x0 + c - 4;
                float un = 0.f, wn = 0.f;
                if (gz >= 0 && gz < nzp && gx >= 0 && gx < nxp) {
                    const int p = gz * nxp + gx;
                    const int li = (r + 4) * AX + c + 4;
                    const float cc = k < TROWS ? ca[k + 4] : A[li];
                    const float lzs =
                        k < TROWS ? FWI_LAPD(cc, ca[k], ca[k + 1], ca[k + 2], ca[k + 3], ca[k + 5], ca[k + 6],
                                             ca[k + 7], ca[k + 8])
                                  : FWI_LAPD(cc, A[li - 4 * AX], A[li - 3 * AX], A[li - 2 * AX], A[li - AX],
                                             A[li + AX], A[li + 2 * AX], A[li + 3 * AX], A[li + 4 * AX]);
                    const float lxs = FWI_LAPD(cc, A[li - 4], A[li - 3], A[li - 2], A[li - 1], A[li + 1], A[li + 2],
                                               A[li + 3], A[li + 4]);
                    float D = fmaf(lzs, a.idz2, lxs * a.idx2);
                    const int rr = rv[kk];
                    if (!ADJ && p == sp) D = fmaf(src, a.src_scale, D);
                    if (ADJ && rr >= 0) D = fmaf(iv[kk], av[kk], D);
                    wn = fmaf(kv[kk], D, dv[kk] * wv[kk]);
                    un = cc + wn;
                    if (k < TROWS && !ADJ) {
                        if (a.Dout) a.Dout[(size_t)field * a.dstride + p] = D;
                        if (rr >= 0 && a.traces) a.traces[(trf + rr) * a.nt + m + 1] = un;
                    }
                }
                if (k < TROWS) {
                    w1[k] = wn;
                    kt[k] = kv[kk];
                    dt[k] = dv[kk];
                    rt[k] = rv[kk];
                    it[k] = iv[kk];
                }
                Bt[r * EX + c] = un;
            }
        }
    }
    __syncthreads();
    if (a.fs && zt == 0) {  // rows above a reflecting top mirror rows 1..4 of u^{n+1}
        for (int i = tid; i < 4 * EX; i += 256) {
            const int r = i / EX, c = i - (i / EX) * EX;
            Bt[i] = Bt[(8 - r) * EX + c];
        }
        __syncthreads();
    }

    // step 2 on the tile (the mapping of k_wave_tile)
    const int gx = x0 + tx;
    if (gx >= nxp) return;
    const bool rec2 = (zt + TZ > a.rec_z0) && (zt <= a.rec_z1);  // implies rec1
    float* un_g = a.unxt + (size_t)field * a.npts;
    float* wo = wout + (size_t)field * a.npts;
    float av[TROWS], d1[TROWS], d2[TROWS], sv[TROWS];
    int rv[TROWS];
#pragma unroll
    for (int j = 0; j < TROWS; ++j) {
        const int gz = min(zt + ts * TROWS + j, nzp - 1);
        const int p = gz * nxp + gx;
        rv[j] = rec2 ? rt[j] : -1;
        av[j] = d1[j] = d2[j] = sv[j] = 0.f;
        if (ADJ && rec2) av[j] = a.adj[(trf + max(rv[j], 0)) * a.nt + (a.nt - 2 - m)];
        if (ADJ && a.Din) {
            d1[j] = a.Din[(size_t)field * a.dstride + p];
            d2[j] = Din2[(size_t)field * a.dstride + p];
            sv[j] = a.acc[(size_t)field * a.npts + p];
        }
    }
    const float src = ADJ ? 0.f : a.wavelet[m + 1];
    // forward: the column of u^{n+1} the thread's points need vertically, in registers; the adjoint reads it
    // from LDS (with its step-2 loads the column would leave 7 waves per SIMD instead of 8)
    float cb[TROWS + 8] = {};
    if (!ADJ) {
#pragma unroll
        for (int i = 0; i < TROWS + 8; ++i) cb[i] = Bt[(ts * TROWS + i) * EX + tx + 4];
    }
#pragma unroll
    for (int j = 0; j < TROWS; ++j) {
        const int lz = ts * TROWS + j;
        const int gz = zt + lz;
        if (gz >= nzp) break;
        const int p = gz * nxp + gx;
        const int li = (lz + 4) * EX + tx + 4;
        const float cc = ADJ ? Bt[li] : cb[j + 4];
        const float lzs =
            ADJ ? FWI_LAPD(cc, Bt[li - 4 * EX], Bt[li - 3 * EX], Bt[li - 2 * EX], Bt[li - EX], Bt[li + EX],
                           Bt[li + 2 * EX], Bt[li + 3 * EX], Bt[li + 4 * EX])
                : FWI_LAPD(cc, cb[j], cb[j + 1], cb[j + 2], cb[j + 3], cb[j + 5], cb[j + 6], cb[j + 7], cb[j + 8]);
        const float lxs = FWI_LAPD(cc, Bt[li - 4], Bt[li - 3], Bt[li - 2], Bt[li - 1], Bt[li + 1], Bt[li + 2],
                                   Bt[li + 3], Bt[li + 4]);
        float D = fmaf(lzs, a.idz2, lxs * a.idx2);
        const int rr = rv[j];
        if (!ADJ && p == sp) D = fmaf(src, a.src_scale, D);
        if (ADJ && rr >= 0) D = fmaf(it[j], av[j], D);
        const float wn = fmaf(kt[j], D, dt[j] * w1[j]);
        const float un = cc + wn;
        wo[p] = wn;
        un_g[p] = un;
        if (ADJ) {
            if (a.Din) {
                const float s1 = fmaf(cc, d1[j], sv[j]);
                a.acc[(size_t)field * a.npts + p] = fmaf(un, d2[j], s1);
            }
        } else {
            if (Dout2) Dout2[(size_t)field * a.dstride + p] = D;
            if (rr >= 0 && a.traces) a.traces[(trf + rr) * a.nt + m + 2] = un;
        }
    }
}

__global__ void k_fill(float* __restrict__ x, size_t n, float val) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = val;
}

__global__ void k_copy(float* __restrict__ dst, const float* __restrict__ src, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Checkpoint slot c of every field <-> (u, w): ckpt layout [field][seg][2][npts].
template <bool SAVE>
__global__ void k_ckpt(float* __restrict__ ckpt, float* __restrict__ u, float* __restrict__ w, int nf, int nseg,
                       int c, int npts) {
    const size_t n = (size_t)nf * npts;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t f = i / npts, q = i - f * npts;
        float* slot = ckpt + ((f * nseg + c) * 2) * npts;
        if (SAVE) {
            slot[q] = u[i];
            slot[npts + q] = w[i];
        } else {
            u[i] = slot[q];
            w[i] = slot[npts + q];
        }
    }
}

// Receiver sample 0 of every trace is u^0 = 0.
__global__ void k_zero_first_sample(float* __restrict__ traces, int ntr, int nt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntr) traces[(size_t)i * nt] = 0.f;
}

static int grid_for(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

static void fill(float* x, size_t n, float v, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, st, x, n, v);
}

static void copy(float* dst, const float* src, size_t n, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, st, dst, src, n);
}

int launch_fill(float* x, size_t n, float v, hipStream_t st) {
    fill(x, n, v, st);
    return hip_ok(hipGetLastError());
}

int launch_copy(float* dst, const float* src, size_t n, hipStream_t st) {
    copy(dst, src, n, st);
    return hip_ok(hipGetLastError());
}

// plain byte copy: 16-byte vectors for the aligned body, bytes for the tail
__global__ void k_copy_bytes(unsigned char* __restrict__ dst, const unsigned char* __restrict__ src, size_t nvec,
                             size_t tail) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    uint4* d = reinterpret_cast<uint4*>(dst);
    const uint4* s = reinterpret_cast<const uint4*>(src);
    for (size_t i = t0; i < nvec; i += stride) d[i] = s[i];
    for (size_t i = t0; i < tail; i += stride) dst[nvec * 16 + i] = src[nvec * 16 + i];
}

int launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (!bytes) return FWI_OK;
    const bool vec = ((uintptr_t)dst % 16 == 0) && ((uintptr_t)src % 16 == 0);
    const size_t nvec = vec ? bytes / 16 : 0;
    const size_t tail = bytes - nvec * 16;
    const size_t work = std::max(nvec, tail);
    const int grid = (int)std::min<size_t>((work + 255) / 256, 2048 * 8);
    hipLaunchKernelGGL(k_copy_bytes, dim3(grid), dim3(256), 0, st, (unsigned char*)dst, (const unsigned char*)src,
                       nvec, tail);
    return hip_ok(hipGetLastError());
}

static TileArgs make_tile_args(const Plan& p, int B) {
    TileArgs a{};
    a.nzp = p.nzp;
    a.nxp = p.nxp;
    a.npts = p.npts;
    a.fs = p.g.free_surface ? 1 : 0;
    a.nt = p.g.nt;
    a.ns = p.g.ns;
    a.nr = p.g.nr;
    a.nfields = B * p.g.ns;
    a.idz2 = (float)(1.0 / (p.g.dz * p.g.dz));
    a.idx2 = (float)(1.0 / (p.g.dx * p.g.dx));
    a.src_scale = (float)(1.0 / (p.g.dx * p.g.dz));
    a.K = p.K;
    a.src_pt = p.src_pt;
    a.rec_map = p.rec_map;
    a.rec_invw = p.rec_invw;
    a.rec_z0 = p.rec_z0;
    a.rec_z1 = p.rec_z1;
    return a;
}

static dim3 tile_grid(const Plan& p, int nfields) {
    return dim3((p.nxp + TX - 1) / TX, (p.nzp + TZ - 1) / TZ, nfields);
}

// One or two forward steps from (u0, w0) to u1 and, for two steps, w1 (one
// step updates w0 in place).  Returns the number of steps taken.
static int forward_steps(TileArgs a, const dim3& grid, int n, bool two, float* u0, float* u1, float* w0, float* w1,
                         float* D0, float* D1, const Plan& p, hipStream_t st) {
    a.ucur = u0;
    a.unxt = u1;
    a.wst = w0;
    a.Dout = D0;
    if (two) {
        hipLaunchKernelGGL(k_wave_tile2<false>, grid, dim3(256), 0, st, a, n, p.ax, p.az, w1, D1, nullptr);
        return 2;
    }
    hipLaunchKernelGGL(k_wave_tile<false>, grid, dim3(256), 0, st, a, n, p.ax, p.az);
    return 1;
}

// Enqueues the whole forward sweep of B samples on st (reads p.wav, writes p.trace_buf).
// State: p.state = [u][u][w][w] per field, (u, w) ping-pong.
static void enqueue_forward(Plan& p, int B, int keep, hipStream_t st) {
    const int nf = B * p.g.ns;
    const size_t fs = (size_t)nf * p.npts;
    float* u0 = p.state;
    float* u1 = p.state + fs;
    float* w0 = p.state + 2 * fs;
    float* w1 = p.state + 3 * fs;
    fill(p.state, 4 * fs, 0.f, st);
    hipLaunchKernelGGL(k_zero_first_sample, dim3((nf * p.g.nr + 255) / 256), dim3(256), 0, st, p.trace_buf,
                       nf * p.g.nr, p.g.nt);
    TileArgs a = make_tile_args(p, B);
    a.traces = p.trace_buf;
    a.wavelet = p.wav;
    const dim3 grid = tile_grid(p, nf);
    const int nsteps = p.g.nt - 1;
    a.dstride = (size_t)nsteps * p.npts;
    const bool ck = keep && p.store_mode == 1;
    for (int n = 0; n < nsteps;) {
        if (ck && n % p.ckpt_every == 0)
            hipLaunchKernelGGL(k_ckpt<true>, dim3(grid_for(fs)), dim3(256), 0, st, p.ckpt, u0, w0, nf, p.nseg,
                               n / p.ckpt_every, p.npts);
        // a pair never straddles a checkpoint
        const bool two = n + 1 < nsteps && !(ck && (n + 1) % p.ckpt_every == 0);
        const bool full = keep && p.store_mode == 0;
        const int k = forward_steps(a, grid, n, two, u0, u1, w0, w1, full ? p.Dstore + (size_t)n * p.npts : nullptr,
                                    full ? p.Dstore + (size_t)(n + 1) * p.npts : nullptr, p, st);
        std::swap(u0, u1);
        if (k == 2) std::swap(w0, w1);
        n += k;
    }
}

// One or two adjoint steps (m, m + 1) with D slices Da (step m) and Db (step m + 1).
static int adjoint_steps(TileArgs a, const dim3& grid, int m, bool two, float* u0, float* u1, float* w0, float* w1,
                         const float* Da, const float* Db, const Plan& p, hipStream_t st) {
    a.ucur = u0;
    a.unxt = u1;
    a.wst = w0;
    a.Din = Da;
    if (two) {
        hipLaunchKernelGGL(k_wave_tile2<true>, grid, dim3(256), 0, st, a, m, p.ax, p.az, w1, nullptr, Db);
        return 2;
    }
    hipLaunchKernelGGL(k_wave_tile<true>, grid, dim3(256), 0, st, a, m, p.ax, p.az);
    return 1;
}

// Enqueues the whole adjoint sweep (reads p.adj_buf, p.wav; writes p.gpad).
static void enqueue_adjoint(Plan& p, int B, hipStream_t st) {
    const int nf = B * p.g.ns;
    const size_t fs = (size_t)nf * p.npts;
    const int nsteps = p.g.nt - 1;
    float* a0 = p.astate;
    float* a1 = p.astate + fs;
    float* aw0 = p.astate + 2 * fs;
    float* aw1 = p.astate + 3 * fs;
    fill(p.astate, 4 * fs, 0.f, st);
    fill(p.gpad, fs, 0.f, st);
    TileArgs aa = make_tile_args(p, B);
    aa.adj = p.adj_buf;
    aa.acc = p.gpad;
    aa.wavelet = p.wav;
    const dim3 grid = tile_grid(p, nf);
    if (p.store_mode == 0) {
        aa.dstride = (size_t)nsteps * p.npts;
        for (int m = 0; m < nsteps;) {
            const bool two = m + 1 < nsteps;
            const int k = adjoint_steps(aa, grid, m, two, a0, a1, aw0, aw1, p.Dstore + (size_t)(nsteps - 1 - m) * p.npts,
                                        two ? p.Dstore + (size_t)(nsteps - 2 - m) * p.npts : nullptr, p, st);
            std::swap(a0, a1);
            if (k == 2) std::swap(aw0, aw1);
            m += k;
        }
        return;
    }
    // checkpointed: recompute each segment's D, then step the adjoint through it
    TileArgs fa = make_tile_args(p, B);
    fa.wavelet = p.wav;
    fa.traces = nullptr;
    const int K = p.ckpt_every;
    fa.dstride = (size_t)K * p.npts;
    aa.dstride = (size_t)K * p.npts;
    float* f0 = p.state;
    float* f1 = p.state + fs;
    float* fw0 = p.state + 2 * fs;
    float* fw1 = p.state + 3 * fs;
    for (int c = p.nseg - 1; c >= 0; --c) {
        const int n0 = c * K;
        const int n1 = std::min(n0 + K, nsteps);
        float* g0 = f0;
        float* g1 = f1;
        float* gw0 = fw0;
        float* gw1 = fw1;
        hipLaunchKernelGGL(k_ckpt<false>, dim3(grid_for(fs)), dim3(256), 0, st, p.ckpt, g0, gw0, nf, p.nseg, c,
                           p.npts);
        for (int n = n0; n < n1;) {
            const bool two = n + 1 < n1;
            const int k = forward_steps(fa, grid, n, two, g0, g1, gw0, gw1, p.Dstore + (size_t)(n - n0) * p.npts,
                                        p.Dstore + (size_t)(n + 1 - n0) * p.npts, p, st);
            std::swap(g0, g1);
            if (k == 2) std::swap(gw0, gw1);
            n += k;
        }
        for (int n = n1 - 1; n >= n0;) {
            const int m = nsteps - 1 - n;
            const bool two = n - 1 >= n0;
            const int k = adjoint_steps(aa, grid, m, two, a0, a1, aw0, aw1, p.Dstore + (size_t)(n - n0) * p.npts,
                                        two ? p.Dstore + (size_t)(n - 1 - n0) * p.npts : nullptr, p, st);
            std::swap(a0, a1);
            if (k == 2) std::swap(aw0, aw1);
            n -= k;
        }
    }
}

// Captures enqueue(p.cap) into an executable graph.
int capture_graph(Plan& p, hipGraphExec_t* exec, const std::function<void(hipStream_t)>& enqueue) {
    if (*exec) {
        (void)hipGraphExecDestroy(*exec);
        *exec = nullptr;
    }
    if (hipStreamBeginCapture(p.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return FWI_EHIP;
    enqueue(p.cap);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(p.cap, &g) != hipSuccess || !g) return FWI_EHIP;
    const hipError_t e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return hip_ok(e);
}

int tiled_forward(Plan& p, int B, float* traces, const float* wavelet, int keep, hipStream_t st) {
    copy(p.wav, wavelet, (size_t)p.g.nt, st);
    const int k = keep ? 1 : 0;
    if (!p.g_fwd[k] || p.g_fwd_B[k] != B) {
        const int rc = capture_graph(p, &p.g_fwd[k], [&](hipStream_t cs) { enqueue_forward(p, B, keep, cs); });
        if (rc) return rc;
        p.g_fwd_B[k] = B;
    }
    if (hipGraphLaunch(p.g_fwd[k], st) != hipSuccess) return FWI_EHIP;
    copy(traces, p.trace_buf, (size_t)B * p.g.ns * p.g.nr * p.g.nt, st);
    return hip_ok(hipGetLastError());
}

int tiled_adjoint(Plan& p, int B, const float* adj, const float* /*wavelet*/, float* /*unused*/, hipStream_t st) {
    copy(p.adj_buf, adj, (size_t)B * p.g.ns * p.g.nr * p.g.nt, st);
    if (!p.g_adj || p.g_adj_B != B) {
        const int rc = capture_graph(p, &p.g_adj, [&](hipStream_t cs) { enqueue_adjoint(p, B, cs); });
        if (rc) return rc;
        p.g_adj_B = B;
    }
    if (hipGraphLaunch(p.g_adj, st) != hipSuccess) return FWI_EHIP;
    return hip_ok(hipGetLastError());
}

void release_graphs(Plan& p) {
    for (int k = 0; k < 2; ++k)
        if (p.g_fwd[k]) {
            (void)hipGraphExecDestroy(p.g_fwd[k]);
            p.g_fwd[k] = nullptr;
        }
    if (p.g_adj) {
        (void)hipGraphExecDestroy(p.g_adj);
        p.g_adj = nullptr;
    }
}

// ---------------------------------------------------------------------------
// grad[b][iz][ix] = scale[b] * sum_s sum_{padded p -> (iz, ix)} gpad[b, s][p] * 2 w_p dt / sqrt(K_p)
// (2 w / v with v = sqrt(K)/dt): the transpose of the edge replication, done
// as two separable passes (padded columns onto model columns, then padded
// rows onto model rows), each summed in a fixed order.
__global__ void k_fold_columns(int B, int ns, int nx, int nzp, int nxp, int nb, float dt, const float* __restrict__ K,
                               const float* __restrict__ wgt_row, const float* __restrict__ gpad,
                               float* __restrict__ tmp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * nzp * nx) return;
    const int b = i / (nzp * nx);
    const int q = i - b * nzp * nx;
    const int z = q / nx, ix = q - (q / nx) * nx;
    const int xlo = (ix == 0) ? 0 : ix + nb;
    const int xhi = (ix == nx - 1) ? nxp - 1 : ix + nb;
    const int npts = nzp * nxp;
    const float* Kr = K + (size_t)b * npts + z * nxp;
    const float wz = 2.f * wgt_row[z] * dt;
    // columns in chunks of CH whose loads go out together (the edge columns sum the whole sponge width); each
    // column's shots are added in ascending order, then the columns in ascending order.  Every lane runs the
    // same chunk loop (a separate path for the single-column lanes measured slower: a wave holding an edge
    // lane then runs both)
    constexpr int CH = 8;
    float sum = 0.f;
    for (int x0 = xlo; x0 <= xhi; x0 += CH) {
        float gs[CH], kv[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            gs[c] = 0.f;
            kv[c] = Kr[min(x0 + c, xhi)];
        }
        for (int s = 0; s < ns; ++s) {
            const float* g = gpad + ((size_t)b * ns + s) * npts + z * nxp;
#pragma unroll
            for (int c = 0; c < CH; ++c) gs[c] += g[min(x0 + c, xhi)];
        }
#pragma unroll
        for (int c = 0; c < CH; ++c)
            if (x0 + c <= xhi) sum += gs[c] * (wz / sqrtf(kv[c]));
    }
    tmp[i] = sum;
}

__global__ void k_fold_rows(int B, int nz, int nx, int nzp, int ztop, const float* __restrict__ tmp,
                            const float* __restrict__ scale, float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * nz * nx) return;
    const int b = i / (nz * nx);
    const int q = i - b * nz * nx;
    const int iz = q / nx, ix = q - (q / nx) * nx;
    const int zlo = (iz == 0) ? 0 : iz + ztop;
    const int zhi = (iz == nz - 1) ? nzp - 1 : iz + ztop;
    // rows in chunks of CH whose loads go out together, added in ascending order
    constexpr int CH = 8;
    float sum = 0.f;
    for (int z0 = zlo; z0 <= zhi; z0 += CH) {
        float v[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) v[c] = tmp[((size_t)b * nzp + min(z0 + c, zhi)) * nx + ix];
#pragma unroll
        for (int c = 0; c < CH; ++c)
            if (z0 + c <= zhi) sum += v[c];
    }
    grad[i] = sum * (scale ? scale[b] : 1.f);
}

int launch_fold_gradient(const Plan& p, int B, const float* scale, float* grad, hipStream_t st) {
    const int n1 = B * p.nzp * p.g.nx;
    hipLaunchKernelGGL(k_fold_columns, dim3((n1 + 255) / 256), dim3(256), 0, st, B, p.g.ns, p.g.nx, p.nzp, p.nxp,
                       p.g.nb, (float)p.g.dt, p.K, p.wgt_row, p.gpad, p.fold_tmp);
    const int n2 = B * p.g.nz * p.g.nx;
    hipLaunchKernelGGL(k_fold_rows, dim3((n2 + 255) / 256), dim3(256), 0, st, B, p.g.nz, p.g.nx, p.nzp, p.ztop,
                       p.fold_tmp, scale, grad);
    return hip_ok(hipGetLastError());
}

}  // namespace fwi
