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
#include <cmath>

#include "fwi_internal.h"
#include "wave_lds_body.h"
#include "wave_split_body.h"

namespace fwi {

template <int X, int P, bool ADJ, bool EXACT, bool STORE>
__global__ __launch_bounds__(kLdsThreads) void k_wave_lds(LdsArgs a, const float* __restrict__ ax_g,
                                                          const float* __restrict__ az_g) {
    extern __shared__ float lds[];
    lds_field<X, P, ADJ, EXACT, STORE>(a, blockIdx.x, ax_g, az_g, lds);
}

// Threads of a split-sweep workgroup: 2-row interior tiles take 768 (three
// waves per SIMD for the same band), the others 512.
constexpr int split_threads(int PI) { return PI == 2 ? 768 : kLdsThreads; }

// Split sweep: workgroup b holds band g = b % G of field b / G (wave_split_body.h).
// Launched cooperatively, so all F * G workgroups are resident together.
template <int X, int PI, bool ADJ, bool XEXACT, bool STORE>
__global__ __launch_bounds__(split_threads(PI)) void k_wave_split(LdsArgs a, SplitArgs sp, const float* __restrict__ ax_g,
                                                            const float* __restrict__ az_g) {
    extern __shared__ float lds[];
    const int lf = blockIdx.x / sp.G;
    split_field<X, PI, ADJ, XEXACT, STORE>(a, sp, sp.field0 + lf, blockIdx.x - lf * sp.G, ax_g, az_g, lds);
}

// Instantiated tiles (X columns, P rows).  (3, 11) tiles the 110 x 150 padded
// field of a 70 x 70 model with a 40-cell sponge exactly.
#define FWI_LDS_TILES(M) \
    M(1, 8) M(1, 12) M(1, 16) M(1, 20) \
    M(2, 8) M(2, 12)                   \
    M(3, 8) M(3, 11) M(3, 12)          \
    M(4, 8)

// Interior tiles of the split sweep (X columns, PI rows): a band has 8
// boundary rows and nstrip interior strips of PI rows, nstrip <= split_threads(PI) / ncg.
#define FWI_SPLIT_TILES(M) M(3, 2) M(3, 3) M(3, 4)

size_t split_lds_bytes(int X, int PI, int ncg, int nstrip) {
    const size_t S = (size_t)ncg * X + 8;
    const size_t H = 8 + (size_t)nstrip * PI;
    return (2 * (H + 8) * S + H) * sizeof(float);
}

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

// Cycles of one CU per time step: VALU issue (about 33 wave64 FP32
// instructions per point, 4 cycles each, over 4 SIMDs), LDS traffic
// ((P+8)/P + 8/X reads and one write per point, 128 bytes per cycle) and,
// split, the latency of the halo exchange (about 0.6 us measured for one
// tagged message between two workgroups) plus the latency the band's waves
// leave exposed, about 2400 cycles divided by the waves per SIMD (`threads`
// busy threads).  The last term is fitted to the 110 x 150 band of 38 rows:
// 3-row tiles on 500 threads (2 waves per SIMD) took 2.61 us per forward
// step, 2-row tiles on 750 threads (3 waves) 2.47 us and 4-row tiles on 400
// threads about 25 % more than 3-row ones.
static double lds_step_cycles(int X, int P, int ncg, int H, bool split, int threads = kLdsThreads) {
    const double pts = (double)ncg * X * H;
    const double waves = std::ceil(threads / 64.0) / 4.0;
    return pts * (33.0 / 64.0 + ((P + 8.0) / P + 8.0 / X + 1.0) / 32.0) + (split ? 1500.0 + 2400.0 / waves : 0.0);
}

bool lds_choose_split(int nzp, int nxp, int nfields, int ncu, int X1, int P1, int force, int* Xo, int* Po, int* ncgo,
                      int* nstripo, int* Go) {
    if (force < 0) return false;
    const int ncg1 = (nxp + X1 - 1) / X1;
    const double whole = lds_step_cycles(X1, P1, ncg1, ((nzp + P1 - 1) / P1) * P1, false);
    double best = force > 0 ? 1e300 : 0.9 * whole;
    bool found = false;
#define FWI_TRY(XX, PP)                                                                                   \
    {                                                                                                     \
        const int ncg = (nxp + XX - 1) / XX;                                                              \
        const int smax = split_threads(PP) / ncg;                                                         \
        if (smax >= 8) {                                                                                  \
            const int G = (nzp + 8 + smax * PP - 1) / (8 + smax * PP);                                    \
            const int nstrip = std::max(1, ((nzp + G - 1) / G - 8 + PP - 1) / PP);                        \
            const int H = 8 + nstrip * PP;                                                                \
            if (G >= 2 && (long long)nfields * G <= ncu && nstrip <= smax &&                              \
                split_lds_bytes(XX, PP, ncg, nstrip) <= (size_t)kLdsBytes) {                              \
                const double c = lds_step_cycles(XX, PP, ncg, H, true, ncg * std::max(8, nstrip));        \
                if (c < best) {                                                                           \
                    best = c;                                                                             \
                    *Xo = XX;                                                                             \
                    *Po = PP;                                                                             \
                    *ncgo = ncg;                                                                          \
                    *nstripo = nstrip;                                                                    \
                    *Go = G;                                                                              \
                    found = true;                                                                         \
                }                                                                                         \
            }                                                                                             \
        }                                                                                                 \
    }
    FWI_SPLIT_TILES(FWI_TRY)
#undef FWI_TRY
    return found;
}

template <bool ADJ, bool STORE>
static int split_dispatch(const LdsArgs& a, SplitArgs sp, int nfields, hipStream_t st, const float* ax,
                          const float* az) {
    const size_t bytes = split_lds_bytes(a.X, a.P, a.ncg, a.nstrip);
    const bool exact = a.ncg * a.X == a.nxp;  // columns; rows are always guarded
    void* args[] = {(void*)&a, (void*)&sp, (void*)&ax, (void*)&az};
#define FWI_CASE(XX, PP)                                                                                      \
    if (a.X == XX && a.P == PP) {                                                                             \
        auto kern = exact ? k_wave_split<XX, PP, ADJ, true, STORE> : k_wave_split<XX, PP, ADJ, false, STORE>; \
        if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != \
            hipSuccess)                                                                                       \
            return hip_ok(hipGetLastError());                                                                 \
        return hip_ok(hipLaunchCooperativeKernel((const void*)kern, dim3(nfields * sp.G), dim3(split_threads(PP)), \
                                                 args, (unsigned)bytes, st));                                 \
    }
    FWI_SPLIT_TILES(FWI_CASE)
#undef FWI_CASE
    return FWI_EINVAL;
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

// A cooperative launch cannot be recorded into a graph: while the caller's
// stream is capturing, the whole-field kernels run instead (same results, bit
// for bit).
bool stream_capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs != hipStreamCaptureStatusNone;
}

// The split sweep's tile replaces the whole-field one; its exchange buffer is
// cleared to level 0 first.
static int split_args(const Plan& p, int nfields, LdsArgs& a, SplitArgs& sp, hipStream_t st) {
    a.X = p.split_X;
    a.P = p.split_P;
    a.ncg = p.split_ncg;
    a.nstrip = p.split_nstrip;
    a.S = a.ncg * a.X + 8;
    sp.G = p.split_G;
    sp.W = a.ncg * a.X;
    sp.xchg = p.xchg;
    sp.err = p.flags;
    return launch_fill(reinterpret_cast<float*>(p.xchg), (size_t)nfields * sp.G * 2 * 2 * 4 * sp.W * 2, 0.f, st);
}

// When the batch has more fields than CUs and is not split as a whole, the
// whole-field sweep runs in rounds of one field per CU.  The fields of the
// last, partial round are instead split over the idle CUs (tile and band
// count from the cost model for that many fields) in a second launch after
// the full rounds; the results are the same bit for bit.  Returns false
// when no such split applies.
static bool tail_split_args(const Plan& p, int nf, const LdsArgs& a, LdsArgs& ta, SplitArgs& sp, int* head,
                            hipStream_t st, int* rc) {
    *rc = FWI_OK;
    if (!p.tail_xchg || p.ncu <= 0 || nf <= p.ncu || stream_capturing(st)) return false;
    const int h = (nf / p.ncu) * p.ncu, tail = nf - h;
    if (tail <= 0) return false;
    int X = 0, P = 0, ncg = 0, nstrip = 0, G = 1;
    if (!lds_choose_split(p.nzp, p.nxp, tail, p.ncu, p.lds_X, p.lds_P, 0, &X, &P, &ncg, &nstrip, &G) || G < 2 ||
        ncg * X > p.tail_W || (long long)tail * G > p.ncu)
        return false;
    ta = a;
    ta.X = X;
    ta.P = P;
    ta.ncg = ncg;
    ta.nstrip = nstrip;
    ta.S = ncg * X + 8;
    sp = SplitArgs{};
    sp.G = G;
    sp.W = ncg * X;
    sp.xchg = p.tail_xchg;
    sp.err = p.flags;
    sp.field0 = h;
    *head = h;
    *rc = launch_fill(reinterpret_cast<float*>(p.tail_xchg), (size_t)tail * G * 2 * 2 * 4 * sp.W * 2, 0.f, st);
    return true;
}

int launch_lds_forward(const Plan& p, int B, float* traces, const float* wavelet, int store, hipStream_t st) {
    LdsArgs a = make_lds_args(p);
    a.traces = traces;
    a.wavelet = wavelet;
    a.store = store;
    const int nf = B * p.g.ns;
    if (p.split_G > 1 && !stream_capturing(st)) {
        SplitArgs sp{};
        const int rc = split_args(p, nf, a, sp, st);
        if (rc) return rc;
        if (store) return split_dispatch<false, true>(a, sp, nf, st, p.ax, p.az);
        return split_dispatch<false, false>(a, sp, nf, st, p.ax, p.az);
    }
    {
        LdsArgs ta;
        SplitArgs sp;
        int head = 0, rc = FWI_OK;
        if (tail_split_args(p, nf, a, ta, sp, &head, st, &rc)) {
            if (!rc) rc = store ? lds_dispatch<false, true>(a, head, st, p.ax, p.az)
                                : lds_dispatch<false, false>(a, head, st, p.ax, p.az);
            if (!rc) rc = store ? split_dispatch<false, true>(ta, sp, nf - head, st, p.ax, p.az)
                                : split_dispatch<false, false>(ta, sp, nf - head, st, p.ax, p.az);
            return rc;
        }
        if (rc) return rc;
    }
    if (store) return lds_dispatch<false, true>(a, nf, st, p.ax, p.az);
    return lds_dispatch<false, false>(a, nf, st, p.ax, p.az);
}

int launch_lds_adjoint(const Plan& p, int B, const float* adj, const float* wavelet, hipStream_t st) {
    LdsArgs a = make_lds_args(p);
    a.adj = adj;
    a.wavelet = wavelet;
    const int nf = B * p.g.ns;
    if (p.split_G > 1 && !stream_capturing(st)) {
        SplitArgs sp{};
        const int rc = split_args(p, nf, a, sp, st);
        if (rc) return rc;
        return split_dispatch<true, false>(a, sp, nf, st, p.ax, p.az);
    }
    {
        LdsArgs ta;
        SplitArgs sp;
        int head = 0, rc = FWI_OK;
        if (tail_split_args(p, nf, a, ta, sp, &head, st, &rc)) {
            if (!rc) rc = lds_dispatch<true, false>(a, head, st, p.ax, p.az);
            if (!rc) rc = split_dispatch<true, false>(ta, sp, nf - head, st, p.ax, p.az);
            return rc;
        }
        if (rc) return rc;
    }
    return lds_dispatch<true, false>(a, nf, st, p.ax, p.az);
}

}  // namespace fwi
