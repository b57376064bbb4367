// C ABI of libfwi: plan management, argument validation and dispatch to the
// HIP kernels.  Every step of the guidance path runs in the kernels of
// wave.hip, w2.hip and guidance.hip; this file only checks arguments, owns
// device workspaces and enqueues launches on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <set>
#include <utility>

#include "fwi_internal.h"

struct fwi_plan : public fwi::Plan {};

namespace fwi {

size_t w2_lds_requirement(int nt, int nxi);

static int dev_alloc(Plan& p, void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) return FWI_OK;
    if (hipMalloc(ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return FWI_ENOMEM;
    }
    p.allocs.push_back(*ptr);
    p.device_bytes += bytes;
    return FWI_OK;
}

template <class T>
static int alloc_n(Plan& p, T** ptr, size_t n) {
    return dev_alloc(p, (void**)ptr, n * sizeof(T));
}

static void free_all(Plan& p) {
    release_graphs(p);
    for (auto* ring : {&p.ev_fwd, &p.ev_adj}) {
        for (hipEvent_t e : *ring)
            if (e) (void)hipEventDestroy(e);
        ring->clear();
    }
    if (p.cap) {
        (void)hipStreamDestroy(p.cap);
        p.cap = nullptr;
    }
    for (void* a : p.allocs) (void)hipFree(a);
    p.allocs.clear();
    p.device_bytes = 0;
}

int validate_geometry(const fwi_geometry* g, int max_batch) {
    if (!g || max_batch < 1) return FWI_EINVAL;
    if (g->nz < 1 || g->nx < 1 || g->nt < 2 || g->nb < 0 || g->ns < 1 || g->nr < 1) return FWI_EINVAL;
    if (!(g->dz > 0) || !(g->dx > 0) || !(g->dt > 0) || !(g->v_max > 0)) return FWI_EINVAL;
    if (!std::isfinite(g->dz) || !std::isfinite(g->dx) || !std::isfinite(g->dt) || !std::isfinite(g->v_max))
        return FWI_EINVAL;
    if (!g->src_iz || !g->src_ix || !g->rec_iz || !g->rec_ix) return FWI_EINVAL;
    if (g->pml != 0 && g->pml != 1) return FWI_EINVAL;
    for (int s = 0; s < g->ns; ++s)
        if (g->src_iz[s] < 0 || g->src_iz[s] >= g->nz || g->src_ix[s] < 0 || g->src_ix[s] >= g->nx) return FWI_EINVAL;
    std::set<std::pair<int, int>> seen;
    for (int r = 0; r < g->nr; ++r) {
        if (g->rec_iz[r] < 0 || g->rec_iz[r] >= g->nz || g->rec_ix[r] < 0 || g->rec_ix[r] >= g->nx) return FWI_EINVAL;
        if (!seen.insert({g->rec_iz[r], g->rec_ix[r]}).second) return FWI_EINVAL;  // distinct receiver nodes
    }
    const double r = g->v_max * g->dt * std::sqrt(2048.0 / 315.0 * (1.0 / (g->dx * g->dx) + 1.0 / (g->dz * g->dz)));
    if (!(r < 2.0)) return FWI_ECFL;
    const long nzp = (long)g->nz + g->nb + (g->free_surface ? 0 : g->nb);
    const long nxp = (long)g->nx + 2L * g->nb;
    if (nzp * nxp > (1L << 30)) return FWI_EINVAL;
    return FWI_OK;
}

// PML damping per axis, as t = zeta dt / 2: the same quadratic profile and
// strength as the sponge, zeta = 3 v_max ln(1/R)/(2 nb h) (delta/nb)^2, R = 1e-3.
void pml_profiles(const fwi_geometry& g, int nzp, int nxp, int ztop, std::vector<float>& tx, std::vector<float>& tz) {
    tx.assign(nxp, 0.f);
    tz.assign(nzp, 0.f);
    if (g.nb <= 0) return;
    const double base = 3.0 * g.v_max * std::log(1e3) / (2.0 * g.nb);
    auto t = [&](int d, double h) {
        const double r = (double)d / g.nb;
        return (float)(base * r * r / h * g.dt / 2.0);
    };
    for (int ix = 0; ix < nxp; ++ix) {
        int d = 0;
        if (ix < g.nb) d = g.nb - ix;
        if (ix >= g.nb + g.nx) d = ix - (g.nb + g.nx - 1);
        tx[ix] = d > 0 ? t(d, g.dx) : 0.f;
    }
    for (int iz = 0; iz < nzp; ++iz) {
        int d = 0;
        if (iz >= ztop + g.nz) d = iz - (ztop + g.nz - 1);
        if (!g.free_surface && iz < ztop) d = ztop - iz;
        tz[iz] = d > 0 ? t(d, g.dz) : 0.f;
    }
}

void build_host_tables(const fwi_geometry& g, int nzp, int nxp, int ztop, HostTables& t) {
    // sponge: per axis the quadratic profile eta = 3 v_max ln(1/R)/(2 nb h) (delta/nb)^2,
    // R = 1e-3, as the velocity-damping factor (1 - eta dt/2)/(1 + eta dt/2)
    t.ax.assign(nxp, 1.f);
    t.az.assign(nzp, 1.f);
    t.wrow.assign(nzp, 1.f);
    if (g.nb > 0) {
        const double base = 3.0 * g.v_max * std::log(1e3) / (2.0 * g.nb);
        auto factor = [&](int d, double h) {
            const double r = (double)d / g.nb;
            const double e = base * r * r / h * g.dt / 2.0;
            return (float)((1.0 - e) / (1.0 + e));
        };
        for (int ix = 0; ix < nxp; ++ix) {
            int d = 0;
            if (ix < g.nb) d = g.nb - ix;
            if (ix >= g.nb + g.nx) d = ix - (g.nb + g.nx - 1);
            t.ax[ix] = d > 0 ? factor(d, g.dx) : 1.f;
        }
        for (int iz = 0; iz < nzp; ++iz) {
            int d = 0;
            if (iz >= ztop + g.nz) d = iz - (ztop + g.nz - 1);
            if (!g.free_surface && iz < ztop) d = ztop - iz;
            t.az[iz] = d > 0 ? factor(d, g.dz) : 1.f;
        }
    }
    if (g.free_surface) t.wrow[0] = 0.5f;
    const int ns = g.ns, nr = g.nr;
    t.src_pt.resize(ns);
    t.rec_pt.resize(nr);
    t.rec_invw.resize(nr);
    for (int s = 0; s < ns; ++s) t.src_pt[s] = (g.src_iz[s] + ztop) * nxp + g.src_ix[s] + g.nb;
    t.rec_z0 = 1 << 30;
    t.rec_z1 = -1;
    t.one_row = true;
    for (int r = 0; r < nr; ++r) {
        const int z = g.rec_iz[r] + ztop;
        t.rec_pt[r] = z * nxp + g.rec_ix[r] + g.nb;
        t.rec_invw[r] = 1.0f / t.wrow[z];
        t.rec_z0 = std::min(t.rec_z0, z);
        t.rec_z1 = std::max(t.rec_z1, z);
        t.one_row = t.one_row && g.rec_iz[r] == g.rec_iz[0];
    }
    t.rec_map.assign((size_t)nzp * nxp, -1);
    for (int r = 0; r < nr; ++r) t.rec_map[t.rec_pt[r]] = r;
    t.rec_row = t.one_row ? g.rec_iz[0] + ztop : -1;
    t.rec_of_col.assign(nxp, -1);
    if (t.one_row)
        for (int r = 0; r < nr; ++r) t.rec_of_col[g.rec_ix[r] + g.nb] = r;
}

static int create(const fwi_geometry* geom, int max_batch, size_t budget, const fwi_plan_options* opt,
                  fwi_plan** out) {
    if (!out) return FWI_EINVAL;
    *out = nullptr;
    int st = validate_geometry(geom, max_batch);
    if (st) return st;
    fwi_plan_options o{-1, 0, 0, 0, 0, 0};
    if (opt) o = *opt;
    if (o.force_path < -1 || o.force_path > 1 || o.ckpt_every < 0 || o.timing < 0 || o.timing > 1 || o.split < -1 ||
        o.split > 1)
        return FWI_EINVAL;

    fwi_plan* pp = new (std::nothrow) fwi_plan();
    if (!pp) return FWI_ENOMEM;
    Plan& p = *pp;
    p.g = *geom;
    p.src_iz.assign(geom->src_iz, geom->src_iz + geom->ns);
    p.src_ix.assign(geom->src_ix, geom->src_ix + geom->ns);
    p.rec_iz.assign(geom->rec_iz, geom->rec_iz + geom->nr);
    p.rec_ix.assign(geom->rec_ix, geom->rec_ix + geom->nr);
    p.g.src_iz = p.src_iz.data();
    p.g.src_ix = p.src_ix.data();
    p.g.rec_iz = p.rec_iz.data();
    p.g.rec_ix = p.rec_ix.data();
    p.g.free_surface = geom->free_surface ? 1 : 0;
    p.ztop = p.g.free_surface ? 0 : p.g.nb;
    p.nzp = p.g.nz + p.g.nb + (p.g.free_surface ? 0 : p.g.nb);
    p.nxp = p.g.nx + 2 * p.g.nb;
    p.npts = p.nzp * p.nxp;
    p.max_batch = max_batch;
    p.budget = budget;
    p.device_bytes = 0;
    (void)hipGetDevice(&p.device);

    const int ns = p.g.ns, nr = p.g.nr, nt = p.g.nt;
    const size_t nf = (size_t)max_batch * ns;
    const size_t npts = (size_t)p.npts;
    const size_t nsteps = (size_t)nt - 1;

    // the LDS-resident sweep needs every receiver on one row (the surface
    // spread of Sec. 2.1, or one buried row)
    bool one_row = true;
    for (int r = 1; r < nr; ++r) one_row = one_row && (p.rec_iz[r] == p.rec_iz[0]);
    std::vector<int> pml_rec;
    if (p.g.pml) {
        // the PML sweep keeps the field in LDS (one workgroup, or row bands over several) with the full
        // history of D (path 2), or sweeps it from HBM (path 3: fields too large for that, a history that
        // does not fit, checkpoints, or force_path = 1)
        if (o.lds_tile_x > 0 || o.lds_tile_z > 0 || (o.force_path == 0 && o.ckpt_every > 0) ||
            (o.split > 0 && (o.force_path == 1 || o.ckpt_every > 0))) {
            delete pp;
            return FWI_EINVAL;
        }
        p.path = (o.force_path == 1 || o.ckpt_every > 0) ? 3 : 2;
    } else {
        bool lds_ok = one_row && lds_choose_layout(p.nzp, p.nxp, o.lds_tile_x, o.lds_tile_z, &p.lds_X, &p.lds_P,
                                                   &p.lds_ncg, &p.lds_nstrip);
        if ((o.lds_tile_x > 0 || o.lds_tile_z > 0) && !lds_ok) {
            delete pp;
            return FWI_EINVAL;
        }
        if (o.force_path == 0 && (!lds_ok || o.ckpt_every > 0)) {
            delete pp;
            return FWI_EINVAL;
        }
        p.path = (o.force_path == 1 || !lds_ok || o.ckpt_every > 0) ? 1 : 0;
    }
    // PML path: row bands when the batch leaves CUs idle (cooperative launches); the whole-field sweep needs
    // the field in one workgroup's LDS
    std::vector<int> band_cells, band_qcells, band_npub;
    if (p.path == 2) {
        int ncu = 0, coop = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p.device) != hipSuccess ||
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, p.device) != hipSuccess) {
            (void)hipGetLastError();
            ncu = coop = 0;
        }
        int G = 1, H = 0, KC = 0, NW = 0;
        const bool bands = coop && pml_choose_bands(p.g, p.nzp, p.nxp, p.ztop, (int)nf, ncu, o.split, &G, &H, &KC, &NW);
        if ((o.split > 0 && !bands) || (!bands && !pml_fits(p.nzp, p.nxp) && o.force_path == 0)) {
            delete pp;
            return FWI_EINVAL;
        }
        if (!bands && !pml_fits(p.nzp, p.nxp)) {
            p.path = 3;
        } else if (bands) {
            p.pml_G = G;
            p.pml_H = H;
            p.pml_KC = KC;
            p.pml_NW = NW;
            pml_band_tables(p.g, p.nzp, p.nxp, p.ztop, G, H, KC, band_cells, band_qcells, band_npub);
        }
    }

    p.timing = o.timing;
    if (p.timing)
        for (auto* ring : {&p.ev_fwd, &p.ev_adj}) {
            ring->assign(2 * Plan::kTimingRing, nullptr);
            for (hipEvent_t& e : *ring)
                if (hipEventCreate(&e) != hipSuccess) {
                    free_all(p);
                    delete pp;
                    return FWI_EHIP;
                }
        }

    // fixed-size buffers
    size_t fixed = (nf * npts + max_batch * npts) * sizeof(float) + npts * sizeof(int) + (size_t)ns * nr * nt * 8 +
                   nf * nr * 8 + (size_t)ns * nr * 1000 * 8;
    // PML HBM sweep: two bordered u planes, w, nu, mu (two), psi and phi (two each), traces, tile table
    const size_t plane = (size_t)(p.nzp + 8) * (p.nxp + 8);
    const size_t nl = (size_t)(p.nzp * p.nxp - p.g.nz * p.g.nx);
    const size_t ntiles = (size_t)((p.nzp + 15) / 16) * ((p.nxp + 63) / 64);
    const size_t fixed_hbm_pml =
        (2 * nf * plane + 4 * nf * npts + 8 * nf * nl + 2 * nf * nr * (size_t)nt + npts + ntiles) * sizeof(float);
    if (p.path == 1) fixed += (8 * nf * npts + 2 * nf * nr * (size_t)nt) * sizeof(float);
    if (p.path == 3) fixed += fixed_hbm_pml;
    const size_t full_store = nf * nsteps * npts * sizeof(float);
    size_t avail = budget;
    if (avail == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = 0;
        }
        avail = free_b > ((size_t)2 << 30) ? free_b - ((size_t)2 << 30) : free_b / 2;
    }
    if (o.ckpt_every > 0) {
        p.store_mode = 1;
        p.ckpt_every = std::min<int>(o.ckpt_every, (int)nsteps);
    } else if (fixed + full_store <= avail) {
        p.store_mode = 0;
        p.ckpt_every = 0;
    } else if (p.path == 2 && o.force_path == 0) {
        free_all(p);
        delete pp;
        return FWI_ENOMEM;
    } else {
        if (p.path == 0) p.path = 1;  // checkpointing runs on the tiled sweep
        if (p.path == 2) {            // and, for the PML, on its HBM sweep
            p.path = 3;
            p.pml_G = 1;
            fixed += fixed_hbm_pml;
        }
        p.store_mode = 1;
        int K = (int)std::ceil(std::sqrt(2.0 * (double)nsteps));
        p.ckpt_every = std::max(1, std::min<int>(K, (int)nsteps));
    }
    if (p.store_mode == 1) {
        p.nseg = (int)((nsteps + p.ckpt_every - 1) / p.ckpt_every);
        const size_t need = p.path == 3 ? fixed + nf * ((size_t)p.ckpt_every * npts +
                                                        (size_t)p.nseg * (plane + npts + 2 * nl)) * sizeof(float)
                                        : fixed + 8 * nf * npts * sizeof(float) +
                                              nf * ((size_t)p.ckpt_every + 2 * (size_t)p.nseg) * npts * sizeof(float);
        if (need > avail) {
            free_all(p);
            delete pp;
            return FWI_ENOMEM;
        }
    }

    // LDS-resident path: several workgroups per field when the batch leaves CUs idle
    if (o.split > 0 && (p.path == 1 || p.path == 3)) {
        free_all(p);
        delete pp;
        return FWI_EINVAL;
    }
    if (p.path == 0) {
        int ncu = 0, coop = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p.device) != hipSuccess ||
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, p.device) != hipSuccess) {
            (void)hipGetLastError();
            ncu = coop = 0;
        }
        const int force = (o.split == 0 && (o.lds_tile_x > 0 || o.lds_tile_z > 0)) ? -1 : o.split;
        if (coop && lds_choose_split(p.nzp, p.nxp, (int)nf, ncu, p.lds_X, p.lds_P, force, &p.split_X, &p.split_P,
                                     &p.split_ncg, &p.split_nstrip, &p.split_G)) {
        } else if (o.split > 0) {
            free_all(p);
            delete pp;
            return FWI_EINVAL;
        } else {
            p.split_G = 1;
            // more fields than CUs: the last partial round may be split (wave_lds.hip)
            if (coop && force == 0 && (long long)nf > ncu) {
                p.ncu = ncu;
                p.tail_W = p.nxp + 8;
            }
        }
    }

    // host-side tables
    HostTables ht;
    build_host_tables(p.g, p.nzp, p.nxp, p.ztop, ht);
    const std::vector<float>& axf = ht.ax;
    const std::vector<float>& azf = ht.az;
    const std::vector<float>& wrow = ht.wrow;
    const std::vector<int>& src_pt = ht.src_pt;
    const std::vector<int>& rec_pt = ht.rec_pt;
    const std::vector<float>& rec_invw = ht.rec_invw;
    p.rec_z0 = ht.rec_z0;
    p.rec_z1 = ht.rec_z1;
    std::vector<int> rec_of_col, rec_map;
    if (p.path == 2) {
        // receiver of each slot of the LDS-resident PML sweep's cell order
        pml_rec.assign(npts, -1);
        const PmlOrder ord(p.g.nz, p.g.nx, p.g.nb, p.g.free_surface);
        for (int r = 0; r < nr; ++r) pml_rec[ord.model_slot(p.rec_iz[r], p.rec_ix[r])] = r;
    }
    std::vector<int> tiles_plain, tiles_layer;
    if (p.path == 3) {
        p.pml_nl = (int)nl;
        pml_tile_classes(p.g, p.nzp, p.nxp, p.ztop, tiles_plain, tiles_layer);
        p.pml_ntp = (int)tiles_plain.size();
        p.pml_ntl = (int)tiles_layer.size();
        tiles_plain.insert(tiles_plain.end(), tiles_layer.begin(), tiles_layer.end());
    }
    if (p.path == 1 || p.path == 3) {
        rec_map = ht.rec_map;
    } else {
        p.rec_row = ht.rec_row;
        rec_of_col = ht.rec_of_col;
    }

    // device allocations
    st = FWI_OK;
    st = st ? st : alloc_n(p, &p.K, (size_t)max_batch * npts);
    st = st ? st : alloc_n(p, &p.ax, (size_t)p.nxp);
    st = st ? st : alloc_n(p, &p.az, (size_t)p.nzp);
    st = st ? st : alloc_n(p, &p.wgt_row, (size_t)p.nzp);
    st = st ? st : alloc_n(p, &p.src_pt, (size_t)ns);
    st = st ? st : alloc_n(p, &p.rec_pt, (size_t)nr);
    st = st ? st : alloc_n(p, &p.rec_invw, (size_t)nr);
    st = st ? st : alloc_n(p, &p.gpad, nf * npts);
    st = st ? st : alloc_n(p, &p.fold_tmp, (size_t)max_batch * p.nzp * p.g.nx);
    st = st ? st : alloc_n(p, &p.flags, 1);
    st = st ? st : alloc_n(p, &p.wav, (size_t)nt);
    st = st ? st : alloc_n(p, &p.omega, (size_t)ns * nr * nt);
    st = st ? st : alloc_n(p, &p.cprime, (size_t)ns * nr);
    st = st ? st : alloc_n(p, &p.qnorm, (size_t)ns * nr);
    st = st ? st : alloc_n(p, &p.sobs, 2);
    st = st ? st : alloc_n(p, &p.w2pair, nf * nr);
    st = st ? st : alloc_n(p, &p.l2stat, (size_t)2 * ns * nr + 2);
    if (p.path == 1) {
        st = st ? st : alloc_n(p, &p.rec_map, npts);
        st = st ? st : alloc_n(p, &p.state, 4 * nf * npts);   // u, u, w, w (two-step launches do not update w in place)
        st = st ? st : alloc_n(p, &p.astate, 4 * nf * npts);
        st = st ? st : alloc_n(p, &p.trace_buf, nf * nr * (size_t)nt);
        st = st ? st : alloc_n(p, &p.adj_buf, nf * nr * (size_t)nt);
        if (!st && hipStreamCreateWithFlags(&p.cap, hipStreamNonBlocking) != hipSuccess) st = FWI_EHIP;
    } else if (p.path == 3) {
        const size_t nl2 = 2 * (size_t)p.pml_nl;
        st = st ? st : alloc_n(p, &p.rec_map, npts);
        st = st ? st : alloc_n(p, &p.pml_tx, (size_t)p.nxp);
        st = st ? st : alloc_n(p, &p.pml_tz, (size_t)p.nzp);
        st = st ? st : alloc_n(p, &p.state, nf * (2 * plane + npts + 2 * nl2));
        st = st ? st : alloc_n(p, &p.astate, nf * (3 * npts + 2 * nl2));
        st = st ? st : alloc_n(p, &p.pml_tiles, tiles_plain.size());
        st = st ? st : alloc_n(p, &p.trace_buf, nf * nr * (size_t)nt);
        st = st ? st : alloc_n(p, &p.adj_buf, nf * nr * (size_t)nt);
        if (!st && hipStreamCreateWithFlags(&p.cap, hipStreamNonBlocking) != hipSuccess) st = FWI_EHIP;
    } else if (p.path == 2) {
        st = st ? st : alloc_n(p, &p.pml_rec, npts);
        st = st ? st : alloc_n(p, &p.pml_tx, (size_t)p.nxp);
        st = st ? st : alloc_n(p, &p.pml_tz, (size_t)p.nzp);
        if (p.pml_G > 1) {
            st = st ? st : alloc_n(p, &p.pml_cells, band_cells.size());
            st = st ? st : alloc_n(p, &p.pml_qcells, band_qcells.size());
            st = st ? st : alloc_n(p, &p.pml_npub, band_npub.size());
            st = st ? st : alloc_n(p, &p.pml_xchg, nf * p.pml_G * 4 * (size_t)p.pml_NW);
        }
    } else {
        st = st ? st : alloc_n(p, &p.rec_of_col, (size_t)p.nxp);
        if (p.split_G > 1)
            st = st ? st : alloc_n(p, &p.xchg, nf * p.split_G * 2 * 2 * 4 * (size_t)p.split_ncg * p.split_X);
        if (p.tail_W > 0) st = st ? st : alloc_n(p, &p.tail_xchg, (size_t)p.ncu * 2 * 2 * 4 * p.tail_W);
    }
    if (p.store_mode == 0) {
        st = st ? st : alloc_n(p, &p.Dstore, nf * nsteps * npts);
    } else {
        st = st ? st : alloc_n(p, &p.Dstore, nf * (size_t)p.ckpt_every * npts);
        const size_t per = p.path == 3 ? plane + npts + 2 * (size_t)p.pml_nl : 2 * npts;
        st = st ? st : alloc_n(p, &p.ckpt, nf * (size_t)p.nseg * per);
    }
    if (!st) {
        st = hip_ok(hipMemcpy(p.ax, axf.data(), axf.size() * sizeof(float), hipMemcpyHostToDevice));
        st = st ? st : hip_ok(hipMemcpy(p.az, azf.data(), azf.size() * sizeof(float), hipMemcpyHostToDevice));
        st = st ? st : hip_ok(hipMemcpy(p.wgt_row, wrow.data(), wrow.size() * sizeof(float), hipMemcpyHostToDevice));
        st = st ? st : hip_ok(hipMemcpy(p.src_pt, src_pt.data(), ns * sizeof(int), hipMemcpyHostToDevice));
        st = st ? st : hip_ok(hipMemcpy(p.rec_pt, rec_pt.data(), nr * sizeof(int), hipMemcpyHostToDevice));
        st = st ? st : hip_ok(hipMemcpy(p.rec_invw, rec_invw.data(), nr * sizeof(float), hipMemcpyHostToDevice));
        if (p.path == 2 || p.path == 3) {
            std::vector<float> tx, tz;
            pml_profiles(p.g, p.nzp, p.nxp, p.ztop, tx, tz);
            st = st ? st : hip_ok(hipMemcpy(p.pml_tx, tx.data(), tx.size() * sizeof(float), hipMemcpyHostToDevice));
            st = st ? st : hip_ok(hipMemcpy(p.pml_tz, tz.data(), tz.size() * sizeof(float), hipMemcpyHostToDevice));
        }
        if (p.path == 3)
            st = st ? st : hip_ok(hipMemcpy(p.pml_tiles, tiles_plain.data(), tiles_plain.size() * sizeof(int),
                                            hipMemcpyHostToDevice));
        if (p.path == 2) {
            st = st ? st : hip_ok(hipMemcpy(p.pml_rec, pml_rec.data(), pml_rec.size() * sizeof(int),
                                            hipMemcpyHostToDevice));
            if (p.pml_G > 1) {
                st = st ? st : hip_ok(hipMemcpy(p.pml_cells, band_cells.data(), band_cells.size() * sizeof(int),
                                                hipMemcpyHostToDevice));
                st = st ? st : hip_ok(hipMemcpy(p.pml_qcells, band_qcells.data(), band_qcells.size() * sizeof(int),
                                                hipMemcpyHostToDevice));
                st = st ? st : hip_ok(hipMemcpy(p.pml_npub, band_npub.data(), band_npub.size() * sizeof(int),
                                                hipMemcpyHostToDevice));
            }
        }
        if (p.path == 1 || p.path == 3)
            st = st ? st : hip_ok(hipMemcpy(p.rec_map, rec_map.data(), npts * sizeof(int), hipMemcpyHostToDevice));
        else if (p.path == 0)
            st = st ? st
                    : hip_ok(hipMemcpy(p.rec_of_col, rec_of_col.data(), p.nxp * sizeof(int), hipMemcpyHostToDevice));
        st = st ? st : hip_ok(hipMemset(p.flags, 0, sizeof(int)));
        st = st ? st : hip_ok(hipDeviceSynchronize());
    }
    if (st) {
        (void)hipGetLastError();
        free_all(p);
        delete pp;
        return st;
    }
    *out = pp;
    return FWI_OK;
}

}  // namespace fwi

using namespace fwi;

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

int fwi_plan_create(const fwi_geometry* geom, int max_batch, size_t mem_budget_bytes, fwi_plan** plan) {
    return create(geom, max_batch, mem_budget_bytes, nullptr, plan);
}

int fwi_plan_create_ex(const fwi_geometry* geom, int max_batch, size_t mem_budget_bytes,
                       const fwi_plan_options* options, fwi_plan** plan) {
    return create(geom, max_batch, mem_budget_bytes, options, plan);
}

int fwi_plan_destroy(fwi_plan* plan) {
    if (!plan) return FWI_EINVAL;
    (void)hipSetDevice(plan->device);
    int st = hip_ok(hipDeviceSynchronize());
    free_all(*plan);
    delete plan;
    return st;
}

int fwi_plan_get_info(const fwi_plan* plan, fwi_plan_info* info) {
    if (!plan || !info) return FWI_EINVAL;
    info->nzp = plan->nzp;
    info->nxp = plan->nxp;
    info->path = plan->path;
    info->store_mode = plan->store_mode;
    info->ckpt_every = plan->ckpt_every;
    info->max_batch = plan->max_batch;
    info->device_bytes = plan->device_bytes;
    const bool split = plan->path == 0 && plan->split_G > 1;
    info->lds_tile_x = plan->path == 0 ? (split ? plan->split_X : plan->lds_X) : 0;
    info->lds_tile_z = plan->path == 0 ? (split ? plan->split_P : plan->lds_P) : 0;
    info->lds_split = plan->path == 0 ? plan->split_G : (plan->path == 2 ? plan->pml_G : 0);
    return FWI_OK;
}

int fwi_set_obs(fwi_plan* plan, const float* d_obs, const fwi_w2_params* params, void* stream) {
    if (!plan || !d_obs || !params) return FWI_EINVAL;
    const fwi_w2_params& w = *params;
    if (!(w.k >= 0) || !(w.eps_prime >= 0) || w.n_xi < 2 || !(w.c_factor >= 0) || (w.squared != 0 && w.squared != 1) ||
        (w.reduction != 0 && w.reduction != 1))
        return FWI_EINVAL;
    if (w2_lds_requirement(plan->g.nt, w.n_xi) > (size_t)kLdsBytes) return FWI_EINVAL;
    (void)hipSetDevice(plan->device);
    Plan& p = *plan;
    if (p.qobs_cap < w.n_xi) {
        if (p.qobs) {
            (void)hipStreamSynchronize(as_stream(stream));
            auto it = std::find(p.allocs.begin(), p.allocs.end(), (void*)p.qobs);
            if (it != p.allocs.end()) p.allocs.erase(it);
            (void)hipFree(p.qobs);
            p.device_bytes -= (size_t)p.qobs_cap * p.g.ns * p.g.nr * sizeof(double);
            p.qobs = nullptr;
        }
        int st = alloc_n(p, &p.qobs, (size_t)w.n_xi * p.g.ns * p.g.nr);
        if (st) return st;
        p.qobs_cap = w.n_xi;
    }
    p.w2p = w;
    int st = launch_w2_obs(p, d_obs, as_stream(stream));
    if (st) return st;
    p.have_obs = 1;
    return FWI_OK;
}

int fwi_forward(fwi_plan* plan, int B, const float* v, const float* wavelet, float* d_syn, int keep_for_adjoint,
                void* stream) {
    if (!plan || B < 0 || B > plan->max_batch) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (!v || !wavelet || !d_syn) return FWI_EINVAL;
    (void)hipSetDevice(plan->device);
    Plan& p = *plan;
    hipStream_t st = as_stream(stream);
    int rc = launch_prep_velocity(p, B, v, st);
    if (rc) return rc;
    p.stored_B = 0;
    p.history = 0;
    const unsigned long long call = ++p.n_forward;
    if (keep_for_adjoint) {
        rc = launch_copy(p.wav, wavelet, (size_t)p.g.nt, st);
        if (rc) return rc;
    }
    const int slot_f = p.n_fwd_rec % Plan::kTimingRing;
    if (p.timing && hipEventRecord(p.ev_fwd[2 * slot_f], st) != hipSuccess) return FWI_EHIP;
    if (p.path == 0)
        rc = launch_lds_forward(p, B, d_syn, wavelet, keep_for_adjoint ? 1 : 0, st);
    else if (p.path == 2)
        rc = launch_pml_forward(p, B, d_syn, wavelet, keep_for_adjoint ? 1 : 0, st);
    else if (p.path == 3)
        rc = pml_hbm_forward(p, B, d_syn, wavelet, keep_for_adjoint ? 1 : 0, st);
    else
        rc = tiled_forward(p, B, d_syn, wavelet, keep_for_adjoint ? 1 : 0, st);
    if (rc) return rc;
    if (p.timing) {
        if (hipEventRecord(p.ev_fwd[2 * slot_f + 1], st) != hipSuccess) return FWI_EHIP;
        ++p.n_fwd_rec;
    }
    p.stored_B = keep_for_adjoint ? B : 0;
    p.history = keep_for_adjoint ? call : 0;
    return FWI_OK;
}

int fwi_w2_misfit(fwi_plan* plan, int B, const float* d_syn, double* J, float* adj_src, void* stream) {
    if (!plan || B < 0 || B > plan->max_batch) return FWI_EINVAL;
    if (!plan->have_obs) return FWI_ESTATE;
    if (B == 0) return FWI_OK;
    if (!d_syn || !J) return FWI_EINVAL;
    (void)hipSetDevice(plan->device);
    return launch_w2_misfit(*plan, B, d_syn, J, adj_src, as_stream(stream));
}

int fwi_w2_misfit_noalloc(fwi_plan* plan, int B, const float* d_syn, double* J, float* adj_src, void* stream) {
    if (!plan || B < 0 || B > plan->max_batch) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (!d_syn || !J) return FWI_EINVAL;
    if ((long long)B * plan->g.ns * plan->g.nr > FWI_W2_SCRATCH_PAIRS) return FWI_ENOMEM;
    if (!plan->have_obs) return FWI_ESTATE;
    (void)hipSetDevice(plan->device);
    return launch_w2_misfit_noalloc(*plan, B, d_syn, J, adj_src, as_stream(stream));
}

int fwi_adjoint_gradient(fwi_plan* plan, int B, const float* v, const float* adj_src, const float* scale, float* grad,
                         void* stream) {
    if (!plan || B < 0 || B > plan->max_batch) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (!v || !adj_src || !grad) return FWI_EINVAL;
    if (plan->stored_B != B) return FWI_ESTATE;
    (void)hipSetDevice(plan->device);
    Plan& p = *plan;
    hipStream_t st = as_stream(stream);
    int rc = launch_prep_velocity(p, B, v, st);
    if (rc) return rc;
    const int slot_a = p.n_adj_rec % Plan::kTimingRing;
    if (p.timing && hipEventRecord(p.ev_adj[2 * slot_a], st) != hipSuccess) return FWI_EHIP;
    if (p.path == 0)
        rc = launch_lds_adjoint(p, B, adj_src, p.wav, st);
    else if (p.path == 2)
        rc = launch_pml_adjoint(p, B, adj_src, st);
    else if (p.path == 3)
        rc = pml_hbm_adjoint(p, B, adj_src, st);
    else
        rc = tiled_adjoint(p, B, adj_src, p.wav, nullptr, st);
    if (rc) return rc;
    if (p.timing) {
        if (hipEventRecord(p.ev_adj[2 * slot_a + 1], st) != hipSuccess) return FWI_EHIP;
        ++p.n_adj_rec;
    }
    return launch_fold_gradient(p, B, scale, grad, st);
}

int fwi_plan_history(const fwi_plan* plan, unsigned long long* history) {
    if (!plan || !history) return FWI_EINVAL;
    *history = plan->history;
    return FWI_OK;
}

int fwi_adjoint_gradient_of(fwi_plan* plan, unsigned long long history, int B, const float* v, const float* adj_src,
                            const float* scale, float* grad, void* stream) {
    if (!plan) return FWI_EINVAL;
    if (history == 0 || plan->history != history) return FWI_ESTATE;
    return fwi_adjoint_gradient(plan, B, v, adj_src, scale, grad, stream);
}

int fwi_l2_misfit(fwi_plan* plan, int B, const float* d_syn, const float* d_obs, const fwi_l2_params* params,
                  double* J, float* adj_src, void* stream) {
    if (!plan || !params || B < 0 || B > plan->max_batch) return FWI_EINVAL;
    const fwi_l2_params& lp = *params;
    if (!(lp.k >= 0) || !std::isfinite(lp.k) || (lp.normalize != 0 && lp.normalize != 1) ||
        (lp.normalize == 0 && !(lp.sigma > 0 && std::isfinite(lp.sigma))))
        return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (!d_syn || !d_obs || !J) return FWI_EINVAL;
    (void)hipSetDevice(plan->device);
    return launch_l2_misfit(*plan, B, d_syn, d_obs, lp, J, adj_src, as_stream(stream));
}

int fwi_tv_subgradient(int B, int nz, int nx, const float* v, const float* g, double alpha, float* out, void* stream) {
    if (B < 0 || nz < 1 || nx < 1 || !std::isfinite(alpha)) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (!v || !out || out == v) return FWI_EINVAL;
    return launch_tv_subgradient(B, nz, nx, v, g, alpha, out, as_stream(stream));
}

int fwi_guidance_step(int B, int nz, int nx, const float* v_prop, const float* h, const float* g, const float* v0hat,
                      const fwi_guidance_params* params, float* v_next, float* rho_out, void* stream) {
    if (B < 0 || nz < 1 || nx < 1 || !params) return FWI_EINVAL;
    if (B == 0) return FWI_OK;
    if (!v_prop || !h || !g || !v0hat || !v_next) return FWI_EINVAL;
    const fwi_guidance_params& gp = *params;
    if (!(gp.c > 0) || !(gp.eps > 0) || !(gp.gamma >= 0) || !std::isfinite(gp.rho0) || !std::isfinite(gp.tau) ||
        !std::isfinite(gp.unit_scale))
        return FWI_EINVAL;
    return launch_guidance(B, nz, nx, v_prop, h, g, v0hat, gp, v_next, rho_out, as_stream(stream));
}

static int ring_mean(const std::vector<hipEvent_t>& ring, int& n_rec, float* out) {
    if (n_rec == 0) return FWI_ESTATE;
    const int n = std::min(n_rec, Plan::kTimingRing);
    const int first = n_rec - n;
    double sum = 0.0;
    for (int i = first; i < n_rec; ++i) {
        const int s = i % Plan::kTimingRing;
        float ms = 0.f;
        if (hipEventSynchronize(ring[2 * s + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, ring[2 * s], ring[2 * s + 1]) != hipSuccess)
            return FWI_EHIP;
        sum += ms;
    }
    *out = (float)(sum / n);
    n_rec = 0;
    return FWI_OK;
}

int fwi_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (bytes && (!dst || !src)) return FWI_EINVAL;
    return launch_copy_bytes(dst, src, bytes, as_stream(stream));
}

int fwi_plan_sweep_ms(fwi_plan* plan, float* forward_ms, float* adjoint_ms) {
    if (!plan) return FWI_EINVAL;
    Plan& p = *plan;
    if (!p.timing) return FWI_ESTATE;
    if ((forward_ms && p.n_fwd_rec == 0) || (adjoint_ms && p.n_adj_rec == 0)) return FWI_ESTATE;
    (void)hipSetDevice(p.device);
    int rc = forward_ms ? ring_mean(p.ev_fwd, p.n_fwd_rec, forward_ms) : FWI_OK;
    if (rc == FWI_OK && adjoint_ms) rc = ring_mean(p.ev_adj, p.n_adj_rec, adjoint_ms);
    return rc;
}

int fwi_status(fwi_plan* plan) {
    if (!plan) return FWI_EINVAL;
    (void)hipSetDevice(plan->device);
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return FWI_EHIP;
    }
    int flags = 0;
    if (hipMemcpy(&flags, plan->flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return FWI_EHIP;
    if (flags) {
        (void)hipMemset(plan->flags, 0, sizeof(int));
        (void)hipDeviceSynchronize();
        return FWI_EDEVICE;
    }
    return FWI_OK;
}

const char* fwi_error_string(int code) {
    switch (code) {
        case FWI_OK: return "ok";
        case FWI_EINVAL: return "invalid argument";
        case FWI_ECFL: return "CFL condition violated for the declared v_max";
        case FWI_ENOMEM: return "out of device memory, memory budget or fixed scratch capacity";
        case FWI_EHIP: return "HIP runtime error";
        case FWI_ESTATE: return "call out of order (observations or forward state missing)";
        case FWI_EDEVICE: return "device-side check failed (velocity not finite, <= 0 or > v_max)";
        default: return "unknown status";
    }
}

}  // extern "C"
