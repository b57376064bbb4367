// Host-side check of the PML row-band tables (pml_choose_bands, pml_band_tables of libfwi):
// every padded cell belongs to exactly one band, published cells come first and map one to one
// onto the halo words the neighbouring band reads, every value a band reads outside its rows is
// received, mirrored or outside the grid, ghost rows cover the layer cells past each inner edge,
// and every LDS and exchange-buffer index stays in bounds.  The device-side index formulas of
// k_wave_pml_band (published word, received word, LDS offsets) are restated here.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <map>
#include <vector>
#include "fwi_internal.h"
using namespace fwi;

static int pub_word(int r, int ix, int H, int nxp, int nb, int nx, int ndc, int NW) {
    const int dc = ix < nb ? ix : ix - nx;
    if (r < 4) return r * nxp + ix;
    if (r < 8) return 4 * nxp + (r - 4) * ndc + dc;
    if (r >= H - 4) return 2 * NW + (r - (H - 4)) * nxp + ix;
    return 2 * NW + 4 * nxp + (r - (H - 8)) * ndc + dc;
}

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails < 20) { printf("FAIL %s:%d: ", __FILE__, __LINE__); printf(__VA_ARGS__); printf("\n"); } ++fails; } } while (0)

static int check(int nz, int nx, int nb, int fs, int nfields, int force) {
    fwi_geometry g{};
    g.nz = nz; g.nx = nx; g.nb = nb; g.free_surface = fs; g.pml = 1;
    const int ztop = fs ? 0 : nb, nzp = nz + nb + (fs ? 0 : nb), nxp = nx + 2 * nb;
    int G, H, KC, NW;
    if (!pml_choose_bands(g, nzp, nxp, ztop, nfields, 256, force, &G, &H, &KC, &NW)) {
        printf("nz %d nx %d nb %d fs %d nf %d: no bands\n", nz, nx, nb, fs, nfields);
        return 1;
    }
    std::vector<int> cells, qcells, npub;
    pml_band_tables(g, nzp, nxp, ztop, G, H, KC, cells, qcells, npub);
    const int T = kPmlBandThreads, KQ = kPmlBandKQ, KH = kPmlBandKH, S = nxp + 8, ndc = 2 * nb;
    const int plane = (H + 16) * S;
    const PmlOrder ord(nz, nx, nb, fs);
    printf("nz %d nx %d nb %d fs %d nf %d: G %d H %d KC %d NW %d npub", nz, nx, nb, fs, nfields, G, H, KC, NW);
    for (int b = 0; b < G; ++b) printf(" %d", npub[b]);
    printf("\n");
    auto side = [&](int ix) { return ix < nb || ix >= nb + nx; };
    // slot_of is the inverse of cell
    for (int j = 0; j < nzp * nxp; ++j) { int iz, ix; ord.cell(j, iz, ix); CHECK(ord.slot_of(iz, ix) == j, "slot_of(cell(%d))", j); }
    long long xsize = (long long)nfields * G * 4 * NW;
    const int field = nfields - 1;
    // per band: position of each cell in the list (for published-word checks)
    std::vector<std::map<int, int>> where(G);
    for (int b = 0; b < G; ++b)
        for (int j = 0; j < KC * T; ++j) { int c = cells[(size_t)b * KC * T + j]; if (c >= 0) where[b][c] = j; }
    for (int b = 0; b < G; ++b) {
        const int z0 = b * H, z1 = std::min(z0 + H, nzp);
        std::set<int> own;
        std::map<int, int> pubcount;
        // own cells
        for (int j = 0; j < KC * T; ++j) {
            int c = cells[(size_t)b * KC * T + j];
            if (c < 0) continue;
            int iz = c >> 16, ix = c & 0xffff;
            CHECK(iz >= z0 && iz < z1 && ix >= 0 && ix < nxp, "cell out of band");
            CHECK(own.insert(c).second, "duplicate cell");
            int off = (iz - z0 + 8) * S + ix + 4;
            CHECK(off - 4 * S >= 0 && off + 4 * S < plane && off - 4 >= 0 && off + 4 < plane, "own read bounds");
            int mir = (fs && iz >= 1 && iz <= 4) ? 2 * iz * S : 0;
            CHECK(off - mir >= 0, "mirror bounds");
            if (mir) CHECK(b == 0, "mirror outside band 0");
            if (j < npub[b]) {
                int pw = pub_word(iz - z0, ix, H, nxp, nb, nx, ndc, NW);
                CHECK(pw >= 0 && pw < 4 * NW, "pub word range %d", pw);
                int edge = pw / (2 * NW), w = pw % (2 * NW);
                CHECK(w < NW, "pub word beyond NW");
                CHECK(edge == 0 ? b > 0 : b < G - 1, "edge without neighbour");
                CHECK(pubcount[pw]++ == 0, "pub word duplicate");
                long long idx = ((long long)field * G + b) * 4 * NW + pw + NW;
                CHECK(idx < xsize, "xchg bounds");
            } else {
                int r = iz - z0;
                bool pub = (b > 0 && (r < 4 || (r < 8 && side(ix)))) || (b < G - 1 && (r >= H - 4 || (r >= H - 8 && side(ix))));
                CHECK(!pub, "published cell after npub");
            }
        }
        CHECK((int)own.size() == (z1 - z0) * nxp, "band cell count %zu vs %d", own.size(), (z1 - z0) * nxp);
        // q cells
        std::set<int> qset;
        for (int j = 0; j < KQ * T; ++j) {
            int c = qcells[(size_t)b * KQ * T + j];
            if (c < 0) continue;
            int iz = c >> 16, ix = c & 0xffff;
            CHECK(qset.insert(c).second, "dup q");
            int off = (iz - z0 + 8) * S + ix + 4;
            CHECK(off - 4 * S >= 0 && off + 4 * S < plane, "q read bounds z");
            bool ownq = iz >= z0 && iz < z0 + H;
            if (ownq) CHECK(ord.slot_of(iz, ix) >= ord.nint, "own q not layer");
            else CHECK(side(ix) && ((b > 0 && iz >= z0 - 4 && iz < z0) || (b < G - 1 && iz >= z1 && iz < z1 + 4)), "bad ghost");
        }
        for (int iz = z0; iz < z1; ++iz) for (int ix = 0; ix < nxp; ++ix)
            if (ord.slot_of(iz, ix) >= ord.nint) CHECK(qset.count((iz << 16) | ix), "layer cell missing from q");
        // every layer cell within 4 rows past an inner edge must be a ghost
        for (int iz = z0 - 4; iz < z1 + 4; ++iz) {
            if (iz >= z0 && iz < z1) continue;
            if (iz < 0 || iz >= nzp) continue;
            if ((iz < z0 && b == 0) || (iz >= z1 && b == G - 1)) continue;
            for (int ix = 0; ix < nxp; ++ix)
                if (ord.slot_of(iz, ix) >= ord.nint) CHECK(qset.count((iz << 16) | ix), "ghost missing iz %d ix %d", iz, ix);
        }
        // halo words
        std::set<int> recv;  // (lds row, ix) as iz<<16|ix
        for (int tid = 0; tid < T; ++tid) for (int k = 0; k < KH; ++k) {
            const int i = tid + k * T;
            const bool top = i < NW && b > 0, bot = i >= NW && i < 2 * NW && b < G - 1;
            if (!(top || bot)) continue;
            const int wd = top ? i : i - NW;
            int lr, ix;
            if (wd < 4 * nxp) { ix = wd % nxp; lr = top ? 4 + wd / nxp : 8 + H + wd / nxp; }
            else { const int e = wd - 4 * nxp, dc = e % ndc; ix = dc < nb ? dc : dc + nx; lr = top ? e / ndc : 8 + H + 4 + e / ndc; }
            int hdst = lr * S + ix + 4;
            CHECK(hdst >= 0 && hdst < plane, "hdst bounds");
            long long hsrc = (((long long)field * G + (top ? b - 1 : b + 1)) * 2 + (top ? 1 : 0)) * 2 * NW + wd;
            CHECK(hsrc + NW < xsize, "hsrc bounds");
            int iz = lr - 8 + z0;
            CHECK(iz >= 0 && iz < nzp, "halo row outside grid");
            int gg = top ? b - 1 : b + 1;
            int c = (iz << 16) | ix;
            CHECK(where[gg].count(c), "halo cell not in neighbour");
            if (where[gg].count(c)) {
                int j = where[gg][c];
                CHECK(j < npub[gg], "halo cell not published by neighbour");
                int pw = pub_word(iz - gg * H, ix, H, nxp, nb, nx, ndc, NW);
                CHECK(pw == (top ? 2 * NW : 0) + wd, "pub word mismatch");
            }
            CHECK(recv.insert(c).second, "dup recv");
        }
        // every value read from outside the band rows is received, a mirror, or outside the grid
        auto need = [&](int iz, int ix, const char* what) {
            if (iz >= z0 && iz < z1) return;
            if (iz >= nzp) return;
            if (iz < 0) { CHECK(b == 0, "negative row outside band 0"); if (!fs) return; CHECK(iz >= -4, "mirror depth"); return; }
            CHECK(recv.count((iz << 16) | ix), "%s needs (%d,%d) not received (band %d)", what, iz, ix, b);
        };
        for (int c : own) { int iz = c >> 16, ix = c & 0xffff; for (int d = -4; d <= 4; ++d) need(iz + d, ix, "lap"); }
        for (int c : qset) { int iz = c >> 16, ix = c & 0xffff; for (int d = -4; d <= 4; ++d) need(iz + d, ix, "dz"); }
    }
    // LDS size
    CHECK((size_t)4 * plane * 4 <= (size_t)kLdsBytes, "lds");
    return G;
}

int main() {
    // the 16-sample, 5-shot, 70 x 70 workload with the 6-cell PML: 3 bands
    CHECK(check(70, 70, 6, 1, 80, 0) == 3, "workload bands");
    check(40, 50, 6, 1, 6, 1);
    check(40, 50, 6, 0, 6, 1);
    check(62, 70, 6, 1, 6, 0);
    check(37, 53, 6, 0, 6, 0);
    check(70, 70, 6, 1, 5, 0);
    check(70, 70, 6, 1, 10, 0);
    check(70, 70, 6, 0, 80, 0);
    check(70, 70, 6, 0, 5, 1);
    check(23, 37, 6, 1, 5, 1);
    check(40, 33, 4, 1, 5, 1);
    check(64, 48, 6, 0, 8, 1);
    check(70, 70, 0, 1, 20, 1);
    check(100, 90, 10, 1, 40, 0);
    check(120, 128, 6, 1, 30, 0);
    check(150, 60, 8, 0, 12, 0);
    printf("fails: %d\n", fails);
    return fails != 0;
}
