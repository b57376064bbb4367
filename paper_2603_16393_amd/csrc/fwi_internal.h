// Internal declarations shared by the HIP translation units of libfwi.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <vector>

#include "fwi.h"

namespace fwi {

// Weights of the 8th-order central second derivative, offsets 0..4.
#define FWI_W0 (-205.0f / 72.0f)
#define FWI_W1 (8.0f / 5.0f)
#define FWI_W2 (-1.0f / 5.0f)
#define FWI_W3 (8.0f / 315.0f)
#define FWI_W4 (-1.0f / 560.0f)

// 8th-order second difference of a 9-point window in difference form:
// sum_k W_k [(u(+k) - u) + (u(-k) - u)].  Neighbouring values of a resolved
// field are close, so each difference is (nearly) exact and the sum carries
// no cancellation of the size of u.  The fused multiply-adds are written out
// so every kernel using it rounds identically, accumulating from the smallest
// weight to the largest.
// Each pair is written (u(+k) - u) - (u - u(-k)), equal bit for bit to
// (u(-k) - u) + (u(+k) - u), so that a kernel sweeping along an axis can
// share the first difference of one point with the point k cells further on.
#define FWI_LAPD(c, m4, m3, m2, m1, p1, p2, p3, p4)                                \
    fmaf(FWI_W1, ((p1) - (c)) - ((c) - (m1)),                                      \
         fmaf(FWI_W2, ((p2) - (c)) - ((c) - (m2)),                                 \
              fmaf(FWI_W3, ((p3) - (c)) - ((c) - (m3)), FWI_W4 * (((p4) - (c)) - ((c) - (m4))))))

// Tile of a block, XCD-aware.  Workgroups are dealt to the 8 XCDs in turn
// (hardware block b runs on XCD b mod 8), each with its own L2; the tiles are
// therefore renumbered so that every XCD sweeps one contiguous run of them in
// row-major order (columns, then rows, then fields), and the halo rows and
// columns a tile shares with its neighbours are read from that XCD's L2.
// A bijection of the grid, so every tile is still computed exactly once.
struct TileIdx {
    int tx, tz, field;
};
__device__ __forceinline__ TileIdx tile_of_block() {
    constexpr int kXcd = 8;
    const int nbx = gridDim.x, nby = gridDim.y;
    const int n = nbx * nby * gridDim.z;
    const int b = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
    const int xcd = b % kXcd, q = n / kXcd, r = n - q * kXcd;
    const int t = xcd * q + min(xcd, r) + b / kXcd;
    TileIdx ti;
    ti.tx = t % nbx;
    ti.tz = (t / nbx) % nby;
    ti.field = t / (nbx * nby);
    return ti;
}

// Global-memory view of a generic pointer: accesses through it compile to
// global instructions rather than flat ones.  A flat access is also counted
// as an LDS access, so a wave that waits for its LDS reads would wait for
// every outstanding flat load or store too; this matters where a pointer
// comes from a descriptor in memory (the persistent batch kernels), whose
// address space the compiler cannot infer.
#define FWI_AS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ FWI_AS_GLOBAL T* gmem(T* p) {
    return (FWI_AS_GLOBAL T*)p;
}

// Largest LDS allocation of one workgroup on gfx950.
constexpr int kLdsBytes = 160 * 1024;
constexpr int kLdsThreads = 512;
constexpr int kLdsMaxP = 48;   // rows per thread of the LDS-resident sweep (multiple of 4)

// PML sweep: threads of its workgroup and the most cells one thread owns.
constexpr int kPmlThreads = 1024;
constexpr int kPmlMaxCells = 7;
// PML row bands: threads per band, most cells per thread, auxiliary-update
// cells and received halo words per thread.
constexpr int kPmlBandThreads = 1024;
constexpr int kPmlBandMaxKC = 4;
constexpr int kPmlBandKQ = 1;
constexpr int kPmlBandKH = 2;

// Cell order of the PML sweep.  Slots list (1) the model cells at least 4
// cells from the layer, whose stencils never see the auxiliary fields,
// row-major; (2) the other model cells (the 4-cell ring next to the layer),
// row-major; (3) the layer cells: side strips row by row, then the full rows
// above (no reflecting top) and below the model.  A wavefront of consecutive
// slots then does the same work throughout.
struct PmlOrder {
    int nz, nx, nb, ztop, nxp;
    int zlo, zhi, dw;  // deep rows [zlo, zhi) and columns [4, 4 + dw) of the model
    int ndeep, nint;
    __host__ __device__ PmlOrder(int nz_, int nx_, int nb_, int fs) : nz(nz_), nx(nx_), nb(nb_) {
        ztop = fs ? 0 : nb;
        nxp = nx + 2 * nb;
        zlo = fs ? 0 : 4;
        zhi = nz - 4 > zlo ? nz - 4 : zlo;
        dw = (nx > 8 && zhi > zlo) ? nx - 8 : 0;
        if (dw == 0) zhi = zlo;
        ndeep = dw * (zhi - zlo);
        nint = nz * nx;
    }
    // slot of model cell (zm, xm)
    __host__ __device__ int model_slot(int zm, int xm) const {
        if (zm >= zlo && zm < zhi && xm >= 4 && xm < 4 + dw) return (zm - zlo) * dw + (xm - 4);
        const int rw = nx - dw;  // ring cells of a deep row
        int e;
        if (zm < zlo)
            e = zm * nx + xm;
        else if (zm < zhi)
            e = zlo * nx + (zm - zlo) * rw + (xm < 4 ? xm : xm - dw);
        else
            e = zlo * nx + (zhi - zlo) * rw + (zm - zhi) * nx + xm;
        return ndeep + e;
    }
    // slot of padded cell (iz, ix): the inverse of cell()
    __host__ __device__ int slot_of(int iz, int ix) const {
        const int zm = iz - ztop, xm = ix - nb;
        if (zm >= 0 && zm < nz && xm >= 0 && xm < nx) return model_slot(zm, xm);
        const int w2 = 2 * nb;
        if (zm >= 0 && zm < nz) return nint + zm * w2 + (ix < nb ? ix : ix - nx);
        const int row = iz < ztop ? iz : iz - nz;
        return nint + nz * w2 + row * nxp + ix;
    }
    // padded cell (iz, ix) of slot j
    __host__ __device__ void cell(int j, int& iz, int& ix) const {
        int zm, xm;
        if (j < ndeep) {
            zm = zlo + j / dw;
            xm = 4 + j % dw;
        } else if (j < nint) {
            int e = j - ndeep;
            const int rw = nx - dw, top = zlo * nx, mid = (zhi - zlo) * rw;
            if (e < top) {
                zm = e / nx;
                xm = e % nx;
            } else if (e - top < mid) {
                e -= top;
                zm = zlo + e / rw;
                const int c = e % rw;
                xm = c < 4 ? c : c + dw;
            } else {
                e -= top + mid;
                zm = zhi + e / nx;
                xm = e % nx;
            }
        } else {
            const int e = j - nint, w2 = 2 * nb, nside = nz * w2;
            if (e < nside) {
                const int c = e % w2;
                iz = ztop + e / w2;
                ix = c < nb ? c : nx + c;
                return;
            }
            const int e2 = e - nside, row = e2 / nxp;
            ix = e2 - row * nxp;
            iz = row < ztop ? row : row + nz;
            return;
        }
        iz = ztop + zm;
        ix = nb + xm;
    }
};

// Device flag bits.
constexpr int kFlagBadVelocity = 1;

struct Plan;

// Time stepping keeps (u^n, w^n = u^n - u^{n-1}) and advances
//   D^n     = sum_k W_k [(u(+k) - u) + (u(-k) - u)] / h^2 per axis + s^n
//   w^{n+1} = a w^n + K D^n,   u^{n+1} = u^n + w^{n+1},   a = a_x a_z (1 in the model)
// which is the leapfrog recursion u^{n+1} = (1 + a) u^n - a u^{n-1} + K D^n
// rearranged so that FP32 rounding neither cancels in the Laplacian nor
// feeds back through the second difference.

// Arguments of the LDS-resident time loop (one workgroup per (sample, shot) field).
struct LdsArgs {
    int nzp, nxp, npts;      // padded grid
    int S;                   // LDS row stride (ncg * X + 8)
    int X, P;                // columns and rows of one thread's register tile
    int ncg, nstrip;         // column groups and row strips (threads = ncg * nstrip)
    int fs;                  // reflecting top
    int nt, ns, nr;
    int rec_row;             // padded row holding every receiver
    float rec_invw;          // 1/w on that row (2 on a reflecting top row)
    float idz2, idx2, src_scale;   // 1/dz^2, 1/dx^2, 1/(dx dz)
    const float* K;          // [B][npts] (v dt)^2
    const float* wavelet;    // [nt]
    const int* src_pt;       // [ns] padded linear index
    const int* rec_of_col;   // [nxp] receiver index on rec_row, or -1
    float* traces;           // forward: d_syn out [B][ns][nr][nt]
    const float* adj;        // adjoint: [B][ns][nr][nt]
    float* Dstore;           // [B*ns][nt-1][npts]
    float* gpad;             // adjoint out: [B*ns][npts] sum_n psi^{n+1} D^n
    int store;               // forward: write D
};

// Split LDS-resident sweep: G workgroups share one field, workgroup g owning
// the band of padded rows [g H, g H + H).  In each step a workgroup publishes
// its first and last 4 rows of u^{n+1} and reads its neighbours' into its
// 4-row halos.  Every published value carries its time level in the
// upper half of a 64-bit word (relaxed device-scope stores and loads), so a
// reader checks each value itself and no fences are needed; two slots per
// boundary alternate with the step parity (a workgroup cannot publish level
// n + 2 before its neighbour has read level n, because it first needs that
// neighbour's level n + 1).  The buffer is cleared to level 0 before a sweep.
struct SplitArgs {
    int G;                       // workgroups per field
    int W;                       // values per exchanged row (ncg * X)
    unsigned long long* xchg;    // [fields][G][2: top, bottom rows][2: slot][4][W], a row as [X][ncg]
                                 // (column x0 + c of column group cg at c * ncg + cg: coalesced)
    int* err;                    // |= 2 when a wait gave up (the sweep's results are then invalid)
    int field0;                  // first field of this launch; xchg is indexed from it
};
constexpr int kSplitSpinMax = 1 << 18;  // polls of one value before a wait gives up
constexpr int kBufferRsrcWord3 = 0x00020000;  // buffer resource word 3 for raw 32-bit accesses (gfx9 data format)

// Arguments of one tiled step (fields in HBM).
struct TileArgs {
    int nzp, nxp, npts;
    int fs;
    int nt, ns, nr;
    int nfields;
    float idz2, idx2, src_scale;
    const float* K;
    const float* wavelet;
    const int* src_pt;
    const int* rec_map;      // [npts] receiver index or -1
    const float* rec_invw;
    int rec_z0, rec_z1;      // receiver row range (inclusive) for a block-uniform skip
    const float* ucur;       // [nfields][npts] u^n
    float* unxt;             // [nfields][npts] u^{n+1} (output)
    float* wst;              // [nfields][npts] w^n in, w^{n+1} out
    float* traces;
    const float* adj;
    float* Dout;             // forward: D^n destination [nfields][dstride] slice for this step, or null
    const float* Din;        // adjoint: D^{n} source for the accumulation, or null
    size_t dstride;          // elements between fields in Dout/Din
    float* acc;              // adjoint: [nfields][npts] running sum of psi D
};

struct Plan {
    fwi_geometry g;                      // host copy (index pointers point into vectors below)
    std::vector<int> src_iz, src_ix, rec_iz, rec_ix;
    int nzp, nxp, npts, ztop;
    int max_batch;
    size_t budget;
    int device;
    int path;                            // 0 LDS-resident, 1 tiled, 2 PML LDS-resident, 3 PML HBM sweep
    int store_mode;                      // 0 full, 1 checkpointed
    int ckpt_every;
    int nseg;
    int lds_X = 0, lds_P = 0, lds_ncg = 0, lds_nstrip = 0;
    int split_G = 1;                     // LDS path: workgroups per field (1: whole field in one workgroup)
    int split_X = 0, split_P = 0, split_ncg = 0, split_nstrip = 0;
    unsigned long long* xchg = nullptr;  // split halo exchange [max_batch*ns][G][2][2][4][ncg*X]
    int ncu = 0;                         // LDS path: CUs of the device when cooperative launches work, else 0
    unsigned long long* tail_xchg = nullptr;  // exchange of the split tail launch: [ncu][2][2][4][tail_W]
    int tail_W = 0;                      // capacity of one exchanged row in tail_xchg
    size_t device_bytes;
    std::vector<void*> allocs;

    // device buffers
    float* K = nullptr;          // [max_batch][npts]
    float* pml_tx = nullptr;     // PML: [nxp] zeta_x dt / 2 per padded column
    float* pml_tz = nullptr;     // PML: [nzp] zeta_z dt / 2 per padded row
    int* pml_rec = nullptr;      // PML: [npts] receiver index of each slot of the sweep's cell order, or -1
    // PML row bands (several workgroups per field, section of wave_pml.hip): bands, rows per band, cells per
    // thread, words per exchanged edge; per band the cell lists and the published-cell counts
    int pml_G = 1, pml_H = 0, pml_KC = 0, pml_NW = 0;
    int* pml_cells = nullptr;    // [G][KC * kPmlBandThreads] own cells, iz << 16 | ix (published first), or -1
    int* pml_qcells = nullptr;   // [G][kPmlBandKQ * kPmlBandThreads] cells of the auxiliary update, or -1
    int* pml_npub = nullptr;     // [G]
    unsigned long long* pml_xchg = nullptr;  // [max_batch*ns][G][2 edges][2 parity][NW]
    // PML HBM sweep (path 3): padded cells outside the model (each has psi_x, psi_z); its u, w, psi and y, nu,
    // mu, phi live in state and astate, the traces in trace_buf and adj_buf, the checkpoints in ckpt
    int pml_nl = 0;
    int* pml_tiles = nullptr;    // tiles (tz << 16 | tx): the pml_ntp plain ones, then the pml_ntl with layer cells
    int pml_ntp = 0, pml_ntl = 0;  // within 4 cells
    float* ax = nullptr;         // [nxp] sponge damping factor per padded column
    float* az = nullptr;         // [nzp] sponge damping factor per padded row
    float* wgt_row = nullptr;    // [nzp]
    int* src_pt = nullptr;       // [ns]
    int* rec_pt = nullptr;       // [nr]
    int* rec_map = nullptr;      // [npts] (tiled path)
    int* rec_of_col = nullptr;   // [nxp] (LDS path)
    int rec_row = -1;            // padded row of the receivers when they share one row
    float* rec_invw = nullptr;   // [nr]
    float* Dstore = nullptr;     // full: [max_batch*ns][nt-1][npts]; ckpt: [max_batch*ns][ckpt_every][npts]
    float* ckpt = nullptr;       // ckpt: [max_batch*ns][nseg][2][npts] (u^n, w^n); PML HBM sweep:
                                 // [max_batch*ns][nseg][(nzp + 8) (nxp + 8) + npts + 2 pml_nl] (u plane, w, psi)
    float* state = nullptr;      // tiled: [4][max_batch*ns][npts] u and w, each ping-pong; PML HBM sweep:
                                 // two bordered u planes, w, two psi buffers (offsets by max_batch)
    float* astate = nullptr;     // tiled adjoint: [4][max_batch*ns][npts]; PML HBM sweep: two mu buffers, nu,
                                 // two phi buffers
    float* acc = nullptr;        // tiled adjoint: [max_batch*ns][npts]
    float* gpad = nullptr;       // [max_batch*ns][npts]
    float* fold_tmp = nullptr;   // [max_batch][nzp][nx] column-folded gradient
    int* flags = nullptr;        // [1]
    float* wav = nullptr;        // [nt] copy of the kept forward's wavelet (segment recomputation)
    int rec_z0 = 0, rec_z1 = -1;

    // observation cache
    int have_obs = 0;
    fwi_w2_params w2p;
    double* omega = nullptr;     // [ns*nr*nt]
    double* cprime = nullptr;    // [ns*nr]
    double* qobs = nullptr;      // [ns*nr*n_xi]
    double* qnorm = nullptr;     // [ns*nr] per-trace (int Q_obs^2) (squared) or its root
    double* sobs = nullptr;      // [1]
    double* w2pair = nullptr;    // [max_batch*ns*nr] per-pair terms (W2 and least-squares misfits)
    double* l2stat = nullptr;    // [2*ns*nr + 2] least squares: per-trace max|d_obs|, weighted energies; max, S
    int qobs_cap = 0;            // n_xi capacity of qobs

    int stored_B = 0;            // batch of the forward state kept for the adjoint (0 = none)
    unsigned long long n_forward = 0;  // forward calls so far (each gets the next number)
    unsigned long long history = 0;    // number of the forward call whose state is kept (0 = none)

    // tiled path: sweeps captured as graphs on a private stream, replayed on the caller's
    hipStream_t cap = nullptr;
    hipGraphExec_t g_fwd[2] = {nullptr, nullptr};  // keep = 0 / 1
    int g_fwd_B[2] = {0, 0};
    hipGraphExec_t g_adj = nullptr;
    int g_adj_B = 0;
    float* trace_buf = nullptr;  // [max_batch*ns][nr][nt] traces written by the forward graph
    float* adj_buf = nullptr;    // [max_batch*ns][nr][nt] adjoint source read by the adjoint graph

    // optional HIP events around forward / adjoint sweeps: rings of start/stop
    // pairs; n_*_rec counts the sweeps recorded since the last query
    static constexpr int kTimingRing = 256;
    int timing = 0;
    std::vector<hipEvent_t> ev_fwd, ev_adj;  // [2 * kTimingRing] each
    int n_fwd_rec = 0, n_adj_rec = 0;
};

void release_graphs(Plan& p);

// Argument checks shared by plans and batches (FWI_OK, FWI_EINVAL or FWI_ECFL).
int validate_geometry(const fwi_geometry* g, int max_batch);

// Host tables of one geometry on its padded grid (ztop = rows of sponge above
// the model): sponge factors per axis, row weights (1/2 on a reflecting top),
// source and receiver points, receiver lookup by point and, when every
// receiver shares one row, by column.
struct HostTables {
    std::vector<float> ax, az, wrow, rec_invw;
    std::vector<int> src_pt, rec_pt, rec_map, rec_of_col;
    int rec_z0 = 0, rec_z1 = -1, rec_row = -1;
    bool one_row = true;
};
void build_host_tables(const fwi_geometry& g, int nzp, int nxp, int ztop, HostTables& t);
// PML damping tables t = zeta dt / 2 per padded column (tx) and row (tz).
void pml_profiles(const fwi_geometry& g, int nzp, int nxp, int ztop, std::vector<float>& tx, std::vector<float>& tz);

// Register-tile layout of the LDS-resident sweep for an nzp x nxp padded
// field (false if the field does not fit in LDS).
// req_X, req_P > 0 restrict the choice to that tile.
bool lds_choose_layout(int nzp, int nxp, int req_X, int req_P, int* X, int* P, int* ncg, int* nstrip);
size_t lds_bytes(int X, int P, int ncg, int nstrip);
// LDS of one band of the split sweep: H = 8 + nstrip * PI rows.
size_t split_lds_bytes(int X, int PI, int ncg, int nstrip);
// Split sweep for `nfields` fields on `ncu` CUs: picks the tile and the
// workgroups per field when that beats the whole-field tile (X1, P1) by the
// cost model (force > 0: whenever feasible; force < 0: never).
bool lds_choose_split(int nzp, int nxp, int nfields, int ncu, int X1, int P1, int force, int* Xo, int* Po, int* ncgo,
                      int* nstripo, int* Go);
int launch_fill(float* x, size_t n, float v, hipStream_t st);

// Launchers (return FWI_OK or FWI_EHIP).
int launch_prep_velocity(const Plan& p, int B, const float* v, hipStream_t st);
int launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t st);
int launch_lds_forward(const Plan& p, int B, float* traces, const float* wavelet, int store, hipStream_t st);
int launch_lds_adjoint(const Plan& p, int B, const float* adj, const float* wavelet, hipStream_t st);
int tiled_forward(Plan& p, int B, float* traces, const float* wavelet, int keep, hipStream_t st);
int tiled_adjoint(Plan& p, int B, const float* adj, const float* wavelet, float* traces_scratch, hipStream_t st);
int launch_fold_gradient(const Plan& p, int B, const float* scale, float* grad, hipStream_t st);
// PML sweeps (path 2): the field of an nzp x nxp padded grid in one workgroup's LDS.
size_t pml_lds_bytes(int nzp, int nxp);
bool pml_fits(int nzp, int nxp);
int launch_pml_forward(const Plan& p, int B, float* traces, const float* wavelet, int store, hipStream_t st);
int launch_pml_adjoint(const Plan& p, int B, const float* adj, hipStream_t st);
// PML HBM sweep (path 3): tile classes (no layer cell within 4 cells, and the others) and the sweeps (captured
// graphs).
void pml_tile_classes(const fwi_geometry& g, int nzp, int nxp, int ztop, std::vector<int>& plain,
                      std::vector<int>& layer);
int pml_hbm_forward(Plan& p, int B, float* traces, const float* wavelet, int keep, hipStream_t st);
int pml_hbm_adjoint(Plan& p, int B, const float* adj, hipStream_t st);
// Captures enqueue(p.cap) into an executable graph (replacing *exec).
int capture_graph(Plan& p, hipGraphExec_t* exec, const std::function<void(hipStream_t)>& enqueue);
// PML row bands for `nfields` fields on `ncu` CUs: bands G and rows per band H
// (false when no split into 2 or more bands applies; force > 0: the largest
// feasible G, force < 0: never).  Host tables for the chosen split.
bool pml_choose_bands(const fwi_geometry& g, int nzp, int nxp, int ztop, int nfields, int ncu, int force, int* G,
                      int* H, int* KC, int* NW);
void pml_band_tables(const fwi_geometry& g, int nzp, int nxp, int ztop, int G, int H, int KC, std::vector<int>& cells,
                     std::vector<int>& qcells, std::vector<int>& npub);
// true while the stream is capturing a graph (cooperative launches cannot be captured)
bool stream_capturing(hipStream_t st);
int launch_copy(float* dst, const float* src, size_t n, hipStream_t st);
int launch_w2_obs(Plan& p, const float* d_obs, hipStream_t st);
int launch_w2_misfit(const Plan& p, int B, const float* d_syn, double* J, float* adj, hipStream_t st);
int launch_w2_misfit_noalloc(const Plan& p, int B, const float* d_syn, double* J, float* adj, hipStream_t st);
int launch_l2_misfit(const Plan& p, int B, const float* d_syn, const float* d_obs, const fwi_l2_params& lp, double* J,
                     float* adj, hipStream_t st);
int launch_tv_subgradient(int B, int nz, int nx, const float* v, const float* g, double alpha, float* out,
                          hipStream_t st);
int launch_guidance(int B, int nz, int nx, const float* v_prop, const float* h, const float* g, const float* v0hat,
                    const fwi_guidance_params& gp, float* v_next, float* rho_out, hipStream_t st);

inline int hip_ok(hipError_t e) { return e == hipSuccess ? FWI_OK : FWI_EHIP; }

}  // namespace fwi
