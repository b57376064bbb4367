/*
 * fwi_oracle.c -- plain FP64 CPU oracle for the likelihood-guidance path of
 * "Robust Physics-Guided Diffusion for Full-Waveform Inversion" (arXiv 2603.16393).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP product library; both are fed by the
 * same seeded input generators and nothing else.
 *
 * Everything is double precision and written as directly as the definitions
 * allow: the forward operator is the explicit time stepping of the acoustic
 * wave equation (Sec. 2.1, Eq. "solving"; solver settings of Sec. 6.1), the
 * misfit is the weighted, shift-rescaled, quantile-based Wasserstein-2
 * objective (Sec. 5.1, Eqs. omega_def, weighted_traces, pdf_map, Wp_1d,
 * final_objective; numerics of Sec. 6.2), the gradient is the literal
 * reverse-mode derivative of that discrete objective (discretise, then
 * differentiate), and the guidance update is Eqs. precond_step, tv, rho and
 * kappa of Sec. 5.2 / Algorithm 2.  OpenMP runs independent (sample, shot)
 * units in parallel; each unit is a serial loop.
 *
 * Discrete choices the paper leaves open (each is listed in the design notes):
 *   - 8th-order central weights for the second derivative; mirror (even)
 *     ghosts above row 0 implement the reflecting top boundary d_n u = 0;
 *   - a damping sponge (separable velocity-damping factor with the quadratic
 *     textbook profile) is the default absorbing layer; the PML section at the
 *     end of the file gives the paper's layer type in an unsplit form;
 *   - the point source f(t) delta(x - xi) is injected as f(t_n)/(dx dz) at the
 *     source node; sample n of a trace is u^n at the receiver node, t_n = n dt;
 *   - quantile = first crossing of the linearly interpolated trapezoid CDF,
 *     with xi clamped to the largest CDF value (eps' keeps F below 1).
 *
 * Status codes: 0 ok, -1 invalid argument, -2 CFL violated, -3 out of memory.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ECFL (-2)
#define ORC_ENOMEM (-3)

/* Weights of the 8th-order central second-derivative stencil, offsets 0..4
 * (standard Fornberg weights). */
static const double W8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

/* Reflection target of the sponge profile (textbook damping-layer formula). */
static const double SPONGE_R = 1e-3;

typedef struct {
    int nz, nx, nb, fs; /* model rows/cols, sponge width, reflecting top */
    int nzp, nxp, ztop; /* padded rows/cols, padded row of model row 0 */
    double dz, dx, dt;
    int nt;
} Grid;

static int grid_init(Grid* g, int nz, int nx, double dz, double dx, double dt, int nt, int nb,
                     int fs) {
    if (nz < 1 || nx < 1 || nb < 0 || nt < 2 || !(dz > 0) || !(dx > 0) || !(dt > 0)) return ORC_EINVAL;
    g->nz = nz;
    g->nx = nx;
    g->nb = nb;
    g->fs = fs ? 1 : 0;
    g->ztop = g->fs ? 0 : nb;
    g->nzp = nz + nb + (g->fs ? 0 : nb);
    g->nxp = nx + 2 * nb;
    g->dz = dz;
    g->dx = dx;
    g->dt = dt;
    g->nt = nt;
    return ORC_OK;
}

static int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* Padded velocity: every padded node takes the value of the nearest model node. */
static void pad_velocity(const Grid* g, const double* v, double* vp) {
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            int mz = clampi(iz - g->ztop, 0, g->nz - 1);
            int mx = clampi(ix - g->nb, 0, g->nx - 1);
            vp[iz * g->nxp + ix] = v[mz * g->nx + mx];
        }
}

/* Damping sponge (replaces the paper's PML): per axis the classic quadratic
 * profile eta = 3 vmax ln(1/R) / (2 nb h) (delta/nb)^2 (delta = cells into the
 * layer), turned into a velocity-damping factor a = (1 - eta dt/2)/(1 + eta dt/2)
 * per axis; the factor of a node is the product of its two axis factors
 * (1 in the model region). */
static double axis_damping(int delta, int nb, double h, double vmax, double dt) {
    if (nb <= 0 || delta <= 0) return 1.0;
    double r = (double)delta / nb;
    double eta = 3.0 * vmax * log(1.0 / SPONGE_R) / (2.0 * nb * h) * r * r;
    double e = eta * dt / 2.0;
    return (1.0 - e) / (1.0 + e);
}

static void sponge_factor(const Grid* g, double vmax, double* a) {
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            int dzc = 0, dxc = 0;
            if (iz >= g->ztop + g->nz) dzc = iz - (g->ztop + g->nz - 1);
            if (!g->fs && iz < g->ztop) dzc = g->ztop - iz;
            if (ix < g->nb) dxc = g->nb - ix;
            if (ix >= g->nb + g->nx) dxc = ix - (g->nb + g->nx - 1);
            a[iz * g->nxp + ix] = axis_damping(dzc, g->nb, g->dz, vmax, g->dt) *
                                  axis_damping(dxc, g->nb, g->dx, vmax, g->dt);
        }
}

/* Field value with the boundary rules: zero outside the padded grid, and an
 * even mirror across row 0 when the top is reflecting. */
static double uat(const Grid* g, const double* u, int iz, int ix) {
    if (g->fs && iz < 0) iz = -iz;
    if (iz < 0 || iz >= g->nzp || ix < 0 || ix >= g->nxp) return 0.0;
    return u[iz * g->nxp + ix];
}

/* (L u)(iz, ix) = sum_k w_|k| [u(iz+k, ix)/dz^2 + u(iz, ix+k)/dx^2], k = -4..4. */
static double lap_at(const Grid* g, const double* u, int iz, int ix) {
    double sz = 0.0, sx = 0.0;
    for (int k = -4; k <= 4; ++k) {
        int a = k < 0 ? -k : k;
        sz += W8[a] * uat(g, u, iz + k, ix);
        sx += W8[a] * uat(g, u, iz, ix + k);
    }
    return sz / (g->dz * g->dz) + sx / (g->dx * g->dx);
}

/* out = L^T y, written as the scatter that transposes lap_at term by term. */
static void lap_transpose(const Grid* g, const double* y, double* out) {
    int np = g->nzp * g->nxp;
    memset(out, 0, sizeof(double) * (size_t)np);
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            double val = y[iz * g->nxp + ix];
            if (val == 0.0) continue;
            for (int k = -4; k <= 4; ++k) {
                int a = k < 0 ? -k : k;
                int tz = iz + k;
                if (g->fs && tz < 0) tz = -tz;
                if (tz >= 0 && tz < g->nzp) out[tz * g->nxp + ix] += W8[a] * val / (g->dz * g->dz);
                int tx = ix + k;
                if (tx >= 0 && tx < g->nxp) out[iz * g->nxp + tx] += W8[a] * val / (g->dx * g->dx);
            }
        }
}

/* Stability (leapfrog with the 8th-order symbol, whose extreme value is
 * 2048/315 at the Nyquist wavenumber): vmax dt sqrt(2048/315 (1/dx^2+1/dz^2)) < 2. */
static int cfl_ok(const Grid* g, double vmax) {
    double r = vmax * g->dt * sqrt(2048.0 / 315.0 * (1.0 / (g->dx * g->dx) + 1.0 / (g->dz * g->dz)));
    return r < 2.0;
}

double orc_cfl_number(double vmax, double dt, double dz, double dx) {
    return vmax * dt * sqrt(2048.0 / 315.0 * (1.0 / (dx * dx) + 1.0 / (dz * dz))) / 2.0;
}

/* Per-unit coefficient fields: C = dt^2 v^2 and the sponge factor a. */
typedef struct {
    double *vp, *C, *a;
} Coefs;

static int coefs_make(const Grid* g, const double* v, double vmax_decl, Coefs* cf) {
    int np = g->nzp * g->nxp;
    cf->vp = (double*)malloc(sizeof(double) * np);
    cf->C = (double*)malloc(sizeof(double) * np);
    cf->a = (double*)malloc(sizeof(double) * np);
    if (!cf->vp || !cf->C || !cf->a) return ORC_ENOMEM;
    sponge_factor(g, vmax_decl, cf->a);
    pad_velocity(g, v, cf->vp);
    for (int p = 0; p < np; ++p) cf->C[p] = g->dt * g->dt * cf->vp[p] * cf->vp[p];
    return ORC_OK;
}

static void coefs_free(Coefs* cf) {
    free(cf->vp);
    free(cf->C);
    free(cf->a);
}

/* One time step: D = L u^n + s^n (s^n = f_n/(dx dz) at the source node),
 * u^{n+1} = (1 + a) u^n - a u^{n-1} + C D, i.e. leapfrog (a = 1) in the model
 * and a damped velocity u^{n+1} - u^n = a (u^n - u^{n-1}) + C D in the sponge.
 * D is returned when requested. */
static void fwd_step(const Grid* g, const Coefs* cf, const double* ucur, const double* uprev,
                     double* unext, int src_p, double src_amp, double* Dout) {
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            int p = iz * g->nxp + ix;
            double D = lap_at(g, ucur, iz, ix);
            if (p == src_p) D += src_amp / (g->dx * g->dz);
            if (Dout) Dout[p] = D;
            unext[p] = (1.0 + cf->a[p]) * ucur[p] - cf->a[p] * uprev[p] + cf->C[p] * D;
        }
}

/* Forward modelling of one (sample, shot) unit; trace[r*nt + n] = u^n(rec_r).
 * If ck != NULL, states (u^{cK-1}, u^{cK}) are saved every K steps for the
 * reverse sweep: ck[(2c)*np] = u^{cK-1}, ck[(2c+1)*np] = u^{cK}. */
static int forward_unit(const Grid* g, const Coefs* cf, const double* wavelet, int src_p, int nr,
                        const int* rec_p, double* trace, double* ck, int K) {
    int np = g->nzp * g->nxp;
    double* u0 = (double*)calloc((size_t)np, sizeof(double)); /* u^{n-1} */
    double* u1 = (double*)calloc((size_t)np, sizeof(double)); /* u^n */
    double* u2 = (double*)calloc((size_t)np, sizeof(double)); /* u^{n+1} */
    if (!u0 || !u1 || !u2) {
        free(u0);
        free(u1);
        free(u2);
        return ORC_ENOMEM;
    }
    for (int r = 0; r < nr; ++r) trace[(size_t)r * g->nt] = u1[rec_p[r]];
    for (int n = 0; n + 1 < g->nt; ++n) {
        if (ck && n % K == 0) {
            int c = n / K;
            memcpy(ck + (size_t)(2 * c) * np, u0, sizeof(double) * np);
            memcpy(ck + (size_t)(2 * c + 1) * np, u1, sizeof(double) * np);
        }
        fwd_step(g, cf, u1, u0, u2, src_p, wavelet[n], NULL);
        for (int r = 0; r < nr; ++r) trace[(size_t)r * g->nt + n + 1] = u2[rec_p[r]];
        double* t = u0;
        u0 = u1;
        u1 = u2;
        u2 = t;
    }
    free(u0);
    free(u1);
    free(u2);
    return ORC_OK;
}

/* Reverse-mode derivative of one unit.  Given a^n = dJ/d(trace sample n),
 * returns gC[p] = dJ/dC[p] and, optionally, gw[n] = dJ/df_n.
 * The forward recursion is u^{n+1} = (1+a) u^n - a u^{n-1} + C (L u^n + s^n),
 * n = 0..N-2, with u^0 = u^{-1} = 0 and trace samples d^n = u^n(rec).
 * Adjoint variables ub^n = dJ/du^n satisfy
 *   ub^n = R^T a^n + (1+a) ub^{n+1} + L^T(C ub^{n+1}) - a ub^{n+2},
 * and dJ/dC += ub^{n+1} (L u^n + s^n) for every step n. */
static int reverse_unit(const Grid* g, const Coefs* cf, const double* wavelet, int src_p, int nr,
                        const int* rec_p, const double* adj, double* gC, double* gw) {
    int np = g->nzp * g->nxp;
    int N = g->nt;
    int K = (int)ceil(sqrt((double)N));
    if (K < 1) K = 1;
    int nseg = (N - 1 + K - 1) / K; /* segments over steps n = 0..N-2 */
    size_t cknum = (size_t)2 * nseg * np;
    double* ck = (double*)malloc(sizeof(double) * cknum);
    double* seg = (double*)malloc(sizeof(double) * (size_t)(K + 1) * np); /* u^{a-1}..u^{a+K-1} */
    double* trace = (double*)malloc(sizeof(double) * (size_t)nr * N);
    double* ub0 = (double*)calloc((size_t)np, sizeof(double));
    double* ub1 = (double*)calloc((size_t)np, sizeof(double));
    double* ub2 = (double*)calloc((size_t)np, sizeof(double));
    double* q = (double*)malloc(sizeof(double) * np);
    double* Cq = (double*)malloc(sizeof(double) * np);
    double* LTq = (double*)malloc(sizeof(double) * np);
    double* D = (double*)malloc(sizeof(double) * np);
    int st = ORC_OK;
    if (!ck || !seg || !trace || !ub0 || !ub1 || !ub2 || !q || !Cq || !LTq || !D) {
        st = ORC_ENOMEM;
        goto done;
    }
    /* forward sweep that keeps the checkpoints */
    st = forward_unit(g, cf, wavelet, src_p, nr, rec_p, trace, ck, K);
    if (st) goto done;
    memset(gC, 0, sizeof(double) * np);
    if (gw) memset(gw, 0, sizeof(double) * N);

    /* n = N-1: only the receiver term */
    for (int r = 0; r < nr; ++r) ub1[rec_p[r]] += adj[(size_t)r * N + (N - 1)];
    /* ub1 = ub^{n+1}, ub2 = ub^{n+2} while processing n */
    for (int c = nseg - 1; c >= 0; --c) {
        int a = c * K;
        int e = a + K;
        if (e > N - 1) e = N - 1;
        /* recompute u^{a-1} .. u^{e-1} into seg[0..] (seg[i] = u^{a-1+i}) */
        memcpy(seg, ck + (size_t)(2 * c) * np, sizeof(double) * np);
        memcpy(seg + (size_t)np, ck + (size_t)(2 * c + 1) * np, sizeof(double) * np);
        for (int n = a; n + 1 < e; ++n) {
            int i = n - (a - 1); /* seg index of u^n */
            fwd_step(g, cf, seg + (size_t)i * np, seg + (size_t)(i - 1) * np, seg + (size_t)(i + 1) * np,
                     src_p, wavelet[n], NULL);
        }
        for (int n = e - 1; n >= a; --n) {
            const double* un = seg + (size_t)(n - (a - 1)) * np;
            /* D^n = L u^n + s^n */
            for (int iz = 0; iz < g->nzp; ++iz)
                for (int ix = 0; ix < g->nxp; ++ix) {
                    int p = iz * g->nxp + ix;
                    double d = lap_at(g, un, iz, ix);
                    if (p == src_p) d += wavelet[n] / (g->dx * g->dz);
                    D[p] = d;
                }
            for (int p = 0; p < np; ++p) {
                q[p] = ub1[p];
                Cq[p] = cf->C[p] * q[p];
                gC[p] += q[p] * D[p];
            }
            if (gw) gw[n] += q[src_p] * cf->C[src_p] / (g->dx * g->dz);
            lap_transpose(g, Cq, LTq);
            for (int p = 0; p < np; ++p)
                ub0[p] = (1.0 + cf->a[p]) * q[p] + LTq[p] - cf->a[p] * ub2[p];
            for (int r = 0; r < nr; ++r) ub0[rec_p[r]] += adj[(size_t)r * N + n];
            double* t = ub2;
            ub2 = ub1;
            ub1 = ub0;
            ub0 = t;
        }
    }
done:
    free(ck);
    free(seg);
    free(trace);
    free(ub0);
    free(ub1);
    free(ub2);
    free(q);
    free(Cq);
    free(LTq);
    free(D);
    return st;
}

/* Shared validation of the acquisition and the velocity model. */
static int check_inputs(const Grid* g, int B, const double* v, double vmax_decl, int ns, const int* src_iz,
                        const int* src_ix, int nr, const int* rec_iz, const int* rec_ix) {
    if (B < 0 || ns < 1 || nr < 0 || !(vmax_decl > 0)) return ORC_EINVAL;
    for (int s = 0; s < ns; ++s)
        if (src_iz[s] < 0 || src_iz[s] >= g->nz || src_ix[s] < 0 || src_ix[s] >= g->nx) return ORC_EINVAL;
    for (int r = 0; r < nr; ++r)
        if (rec_iz[r] < 0 || rec_iz[r] >= g->nz || rec_ix[r] < 0 || rec_ix[r] >= g->nx) return ORC_EINVAL;
    double vmax = 0.0;
    for (long i = 0; i < (long)B * g->nz * g->nx; ++i) {
        if (!(v[i] > 0) || !isfinite(v[i])) return ORC_EINVAL;
        if (v[i] > vmax) vmax = v[i];
    }
    if (vmax > vmax_decl) return ORC_EINVAL;
    if (!cfl_ok(g, vmax_decl)) return ORC_ECFL;
    return ORC_OK;
}

static int padded_index(const Grid* g, int iz, int ix) { return (iz + g->ztop) * g->nxp + (ix + g->nb); }

/* Forward modelling F(v): d[b][s][r][n] = u^n at receiver r for shot s of sample b. */
int orc_forward(int nz, int nx, double dz, double dx, double dt, int nt, int nb, int fs, double vmax_decl,
                int ns, const int* src_iz, const int* src_ix, int nr, const int* rec_iz, const int* rec_ix,
                int B, const double* v, const double* wavelet, double* d) {
    Grid g;
    int st = grid_init(&g, nz, nx, dz, dx, dt, nt, nb, fs);
    if (st) return st;
    st = check_inputs(&g, B, v, vmax_decl, ns, src_iz, src_ix, nr, rec_iz, rec_ix);
    if (st) return st;
    int* rec_p = (int*)malloc(sizeof(int) * (nr > 0 ? nr : 1));
    for (int r = 0; r < nr; ++r) rec_p[r] = padded_index(&g, rec_iz[r], rec_ix[r]);
    int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int u = 0; u < B * ns; ++u) {
        int b = u / ns, s = u % ns;
        Coefs cf;
        int e = coefs_make(&g, v + (size_t)b * nz * nx, vmax_decl, &cf);
        if (!e)
            e = forward_unit(&g, &cf, wavelet, padded_index(&g, src_iz[s], src_ix[s]), nr, rec_p,
                             d + (size_t)u * nr * nt, NULL, 1);
        coefs_free(&cf);
        if (e) {
#pragma omp critical
            err = e;
        }
    }
    free(rec_p);
    return err;
}

/* Reverse-mode gradient: given adj[b][s][r][n] = dJ/dd, returns
 * grad[b][iz][ix] = dJ/dv (summed over shots) and optionally
 * gwav[b][s][n] = dJ/df_n for the wavelet seen by each shot. */
int orc_gradient(int nz, int nx, double dz, double dx, double dt, int nt, int nb, int fs, double vmax_decl,
                 int ns, const int* src_iz, const int* src_ix, int nr, const int* rec_iz, const int* rec_ix,
                 int B, const double* v, const double* wavelet, const double* adj, double* grad, double* gwav) {
    Grid g;
    int st = grid_init(&g, nz, nx, dz, dx, dt, nt, nb, fs);
    if (st) return st;
    st = check_inputs(&g, B, v, vmax_decl, ns, src_iz, src_ix, nr, rec_iz, rec_ix);
    if (st) return st;
    int np = g.nzp * g.nxp;
    int* rec_p = (int*)malloc(sizeof(int) * (nr > 0 ? nr : 1));
    for (int r = 0; r < nr; ++r) rec_p[r] = padded_index(&g, rec_iz[r], rec_ix[r]);
    double* gvp = (double*)calloc((size_t)B * ns * np, sizeof(double)); /* dJ/dv_pad per unit */
    if (!gvp) {
        free(rec_p);
        return ORC_ENOMEM;
    }
    int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int u = 0; u < B * ns; ++u) {
        int b = u / ns, s = u % ns;
        Coefs cf;
        double* gC = (double*)malloc(sizeof(double) * np);
        int e = gC ? coefs_make(&g, v + (size_t)b * nz * nx, vmax_decl, &cf) : ORC_ENOMEM;
        if (!e)
            e = reverse_unit(&g, &cf, wavelet, padded_index(&g, src_iz[s], src_ix[s]), nr, rec_p,
                             adj + (size_t)u * nr * nt, gC, gwav ? gwav + (size_t)u * nt : NULL);
        if (!e) /* C = dt^2 vp^2  =>  dC/dvp = 2 dt^2 vp */
            for (int p = 0; p < np; ++p) gvp[(size_t)u * np + p] = gC[p] * 2.0 * dt * dt * cf.vp[p];
        if (gC) coefs_free(&cf);
        free(gC);
        if (e) {
#pragma omp critical
            err = e;
        }
    }
    if (!err) {
        /* transpose of the edge replication, summed over shots */
        memset(grad, 0, sizeof(double) * (size_t)B * nz * nx);
        for (int b = 0; b < B; ++b)
            for (int s = 0; s < ns; ++s)
                for (int iz = 0; iz < g.nzp; ++iz)
                    for (int ix = 0; ix < g.nxp; ++ix) {
                        int mz = clampi(iz - g.ztop, 0, nz - 1);
                        int mx = clampi(ix - g.nb, 0, nx - 1);
                        grad[(size_t)b * nz * nx + mz * nx + mx] += gvp[((size_t)b * ns + s) * np + iz * g.nxp + ix];
                    }
    }
    free(gvp);
    free(rec_p);
    return err;
}

/* ------------------------------------------------------------------------ */
/* Wasserstein-2 misfit (Sec. 5.1 and Sec. 6.2)                               */
/* ------------------------------------------------------------------------ */

/* Trapezoid mass Z of a shifted trace, density rho = h/(Z + eps'), and the
 * trapezoid CDF F_0 = 0, F_{k+1} = F_k + dt (rho_k + rho_{k+1})/2. */
static void w2_cdf(int nt, double dt, double epsp, const double* h, double* rho, double* F, double* Zout) {
    double Z = 0.0;
    for (int k = 0; k + 1 < nt; ++k) Z += dt * (h[k] + h[k + 1]) / 2.0;
    for (int k = 0; k < nt; ++k) rho[k] = h[k] / (Z + epsp);
    F[0] = 0.0;
    for (int k = 0; k + 1 < nt; ++k) F[k + 1] = F[k] + dt * (rho[k] + rho[k + 1]) / 2.0;
    *Zout = Z;
}

/* Quantiles Q_j = inf{t : F(t) >= x_j} of the linearly interpolated CDF at
 * x_j = min(xi_j, max F), xi_j = j/(nxi-1).  Records the bracket k*_j (first
 * node with F >= x_j), the interpolation weight and whether xi_j was clamped.
 * The search pointer never moves backwards because x_j is non-decreasing in
 * j and the first index with F >= x is non-decreasing in x. */
static void w2_quantiles(int nt, double dt, const double* F, int nxi, double* Q, int* kst, int* clamped) {
    double Fmax = F[0];
    for (int k = 1; k < nt; ++k)
        if (F[k] > Fmax) Fmax = F[k];
    int k = 0;
    for (int j = 0; j < nxi; ++j) {
        double xi = (nxi > 1) ? (double)j / (double)(nxi - 1) : 0.0;
        int cl = 0;
        double x = xi;
        if (x > Fmax) {
            x = Fmax;
            cl = 1;
        }
        while (F[k] < x) ++k; /* terminates: some node holds Fmax >= x */
        if (k == 0)
            Q[j] = 0.0;
        else
            Q[j] = dt * ((double)(k - 1) + (x - F[k - 1]) / (F[k] - F[k - 1]));
        if (kst) kst[j] = k;
        if (clamped) clamped[j] = cl;
    }
}

/* Trapezoid weights on the uniform xi grid. */
static double xi_weight(int j, int nxi) {
    if (nxi < 2) return 1.0;
    double w = 1.0 / (double)(nxi - 1);
    return (j == 0 || j == nxi - 1) ? w / 2.0 : w;
}

/* Observation side: omega (Eq. omega_def), c' = cfac |min_t omega d_obs|,
 * Q_obs at the xi grid, and the scale S_obs = sum_{s,r} (int Q_obs^2)^(1/2)
 * (squared = 0) or sum_{s,r} int Q_obs^2 (squared = 1). */
int orc_w2_prepare(int ntr, int nt, double dt, const double* dobs, double kw, double epsp, int nxi,
                   double cfac, int squared, double* omega, double* cprime, double* Qobs, double* S_obs) {
    if (ntr < 1 || nt < 2 || nxi < 2 || !(dt > 0) || kw < 0 || !(epsp >= 0)) return ORC_EINVAL;
    double M = 0.0;
    for (long i = 0; i < (long)ntr * nt; ++i) {
        if (!isfinite(dobs[i])) return ORC_EINVAL;
        double a = fabs(dobs[i]);
        if (a > M) M = a;
    }
    for (long i = 0; i < (long)ntr * nt; ++i) {
        double a = (M > 0.0) ? fabs(dobs[i]) / M : 0.0;
        omega[i] = 1.0 / (1.0 + kw * a);
    }
    double* h = (double*)malloc(sizeof(double) * nt);
    double* rho = (double*)malloc(sizeof(double) * nt);
    double* F = (double*)malloc(sizeof(double) * nt);
    double S = 0.0;
    for (int t = 0; t < ntr; ++t) {
        const double* o = dobs + (size_t)t * nt;
        const double* w = omega + (size_t)t * nt;
        double mn = w[0] * o[0];
        for (int k = 1; k < nt; ++k)
            if (w[k] * o[k] < mn) mn = w[k] * o[k];
        double cp = cfac * fabs(mn);
        cprime[t] = cp;
        for (int k = 0; k < nt; ++k) h[k] = w[k] * o[k] + cp;
        double Z;
        w2_cdf(nt, dt, epsp, h, rho, F, &Z);
        w2_quantiles(nt, dt, F, nxi, Qobs + (size_t)t * nxi, NULL, NULL);
        double m2 = 0.0;
        for (int j = 0; j < nxi; ++j) m2 += xi_weight(j, nxi) * Qobs[(size_t)t * nxi + j] * Qobs[(size_t)t * nxi + j];
        S += squared ? m2 : sqrt(m2);
    }
    *S_obs = S;
    free(h);
    free(rho);
    free(F);
    return ORC_OK;
}

/* Synthetic side for B samples of ntr traces each.  J[b] is
 *   reduction 0: sum_{s,r} W / S_obs                 (Eq. final_objective)
 *   reduction 1: sum_{s,r} W / ntr                   (average over pairs)
 * with W = W2 (squared = 0) or W2^2 (squared = 1).  adj (optional) is dJ/dd_syn
 * by reverse-mode differentiation of every step with the brackets k* fixed;
 * a pair with W2 = 0 contributes zero (subgradient).  w2 (optional) gets the
 * per-pair W2. */
int orc_w2_misfit(int B, int ntr, int nt, double dt, const double* dsyn, const double* omega,
                  const double* cprime, const double* Qobs, double S_obs, double epsp, int nxi, int squared,
                  int reduction, double* J, double* adj, double* w2) {
    if (B < 0 || ntr < 1 || nt < 2 || nxi < 2 || !(dt > 0)) return ORC_EINVAL;
    double norm = reduction ? (double)ntr : S_obs;
    if (!(norm > 0)) return ORC_EINVAL;
    int err = ORC_OK;
    for (int b = 0; b < B; ++b) J[b] = 0.0;
    double* Jpair = (double*)malloc(sizeof(double) * (size_t)B * ntr);
#pragma omp parallel
    {
        double* h = (double*)malloc(sizeof(double) * nt);
        double* rho = (double*)malloc(sizeof(double) * nt);
        double* F = (double*)malloc(sizeof(double) * nt);
        double* Fb = (double*)malloc(sizeof(double) * nt);
        double* rb = (double*)malloc(sizeof(double) * nt);
        double* hb = (double*)malloc(sizeof(double) * nt);
        double* Q = (double*)malloc(sizeof(double) * nxi);
        int* kst = (int*)malloc(sizeof(int) * nxi);
        int* cl = (int*)malloc(sizeof(int) * nxi);
#pragma omp for schedule(static)
        for (long u = 0; u < (long)B * ntr; ++u) {
            int t = (int)(u % ntr);
            const double* y = dsyn + (size_t)u * nt;
            const double* w = omega + (size_t)t * nt;
            const double* qo = Qobs + (size_t)t * nxi;
            double cp = cprime[t];
            for (int k = 0; k < nt; ++k) h[k] = w[k] * y[k] + cp;
            double Z;
            w2_cdf(nt, dt, epsp, h, rho, F, &Z);
            w2_quantiles(nt, dt, F, nxi, Q, kst, cl);
            double m2 = 0.0;
            for (int j = 0; j < nxi; ++j) m2 += xi_weight(j, nxi) * (Q[j] - qo[j]) * (Q[j] - qo[j]);
            double W2 = sqrt(m2);
            if (w2) w2[u] = W2;
            Jpair[u] = (squared ? m2 : W2) / norm;
            if (!adj) continue;
            double* ab = adj + (size_t)u * nt;
            /* dJ/dm2 */
            double dm2 = 0.0;
            if (squared)
                dm2 = 1.0 / norm;
            else if (W2 > 0.0)
                dm2 = 1.0 / (2.0 * W2 * norm);
            /* Q_j -> F (brackets fixed) */
            for (int k = 0; k < nt; ++k) Fb[k] = 0.0;
            double Fmax = F[0];
            int kmax = 0;
            for (int k = 1; k < nt; ++k)
                if (F[k] > Fmax) {
                    Fmax = F[k];
                    kmax = k;
                }
            for (int j = 0; j < nxi; ++j) {
                double Qb = dm2 * 2.0 * xi_weight(j, nxi) * (Q[j] - qo[j]);
                int k = kst[j];
                if (k == 0) continue;
                /* Q = dt (k-1 + (x - F[k-1]) / (F[k] - F[k-1])) */
                double den = F[k] - F[k - 1];
                double num = cl[j] ? (Fmax - F[k - 1]) : ((double)j / (double)(nxi - 1) - F[k - 1]);
                double dQ_dnum = dt / den;
                double dQ_dden = -dt * num / (den * den);
                /* num = x - F[k-1]; den = F[k] - F[k-1]; x = Fmax = F[kmax] when clamped */
                Fb[k - 1] += Qb * (-dQ_dnum - dQ_dden);
                Fb[k] += Qb * dQ_dden;
                if (cl[j]) Fb[kmax] += Qb * dQ_dnum;
            }
            /* F_{k+1} = F_k + dt (rho_k + rho_{k+1})/2, reversed */
            for (int k = 0; k < nt; ++k) rb[k] = 0.0;
            for (int k = nt - 2; k >= 0; --k) {
                Fb[k] += Fb[k + 1];
                rb[k] += dt / 2.0 * Fb[k + 1];
                rb[k + 1] += dt / 2.0 * Fb[k + 1];
            }
            /* rho_k = h_k / (Z + eps') */
            double Zb = 0.0;
            for (int k = 0; k < nt; ++k) {
                hb[k] = rb[k] / (Z + epsp);
                Zb += -rb[k] * h[k] / ((Z + epsp) * (Z + epsp));
            }
            /* Z = sum_k dt (h_k + h_{k+1})/2 */
            for (int k = 0; k + 1 < nt; ++k) {
                hb[k] += Zb * dt / 2.0;
                hb[k + 1] += Zb * dt / 2.0;
            }
            /* h = omega d_syn + c' */
            for (int k = 0; k < nt; ++k) ab[k] = w[k] * hb[k];
        }
        free(h);
        free(rho);
        free(F);
        free(Fb);
        free(rb);
        free(hb);
        free(Q);
        free(kst);
        free(cl);
    }
    for (int b = 0; b < B; ++b)
        for (int t = 0; t < ntr; ++t) J[b] += Jpair[(size_t)b * ntr + t];
    free(Jpair);
    return err;
}

/* Quantile function of one raw density (used by closed-form checks). */
int orc_quantiles(int nt, double dt, const double* h, double epsp, int nxi, double* Q, double* F) {
    if (nt < 2 || nxi < 2) return ORC_EINVAL;
    double* rho = (double*)malloc(sizeof(double) * nt);
    double Z;
    w2_cdf(nt, dt, epsp, h, rho, F, &Z);
    w2_quantiles(nt, dt, F, nxi, Q, NULL, NULL);
    free(rho);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Preconditioned guidance update (Sec. 5.2, Algorithm 2)                     */
/* ------------------------------------------------------------------------ */

/* Per sample b (fields [nz][nx]):
 *   TV = (1/(nz nx)) sum (|v[z][x+1]-v[z][x]| + |v[z+1][x]-v[z][x]|) over v0hat
 *        (forward differences that exist)                          Eq. tv
 *   rho = rho0 exp(-max(TV - tau, 0)/c)                             Eq. rho
 *   g~ = s g, h~ = s h  (s: chain factor from the gradient's units to the
 *        diffusion state's units)
 *   kappa_j = ((max|g~| + eps)/(|g~_j| + eps))^gamma, optionally
 *        min(kappa, kappa_max) when kappa_max > 0                   Eq. kappa
 *   v_next = v_prop - rho kappa h~                                  Eq. precond_step */
int orc_guidance(int B, int nz, int nx, const double* vprop, const double* h, const double* g,
                 const double* v0hat, double rho0, double c, double tau, double gamma, double eps,
                 double kappa_max, double unit_scale, double* vnext, double* rho_out, double* tv_out,
                 double* kappa_out) {
    if (B < 0 || nz < 1 || nx < 1 || !(c > 0) || !(eps > 0) || gamma < 0) return ORC_EINVAL;
    size_t n = (size_t)nz * nx;
    for (int b = 0; b < B; ++b) {
        const double* x = v0hat + b * n;
        double tv = 0.0;
        for (int iz = 0; iz < nz; ++iz)
            for (int ix = 0; ix < nx; ++ix) {
                if (ix + 1 < nx) tv += fabs(x[iz * nx + ix + 1] - x[iz * nx + ix]);
                if (iz + 1 < nz) tv += fabs(x[(iz + 1) * nx + ix] - x[iz * nx + ix]);
            }
        tv /= (double)n;
        double ex = tv - tau;
        if (ex < 0.0) ex = 0.0;
        double rho = rho0 * exp(-ex / c);
        double gmax = 0.0;
        for (size_t j = 0; j < n; ++j) {
            double a = fabs(unit_scale * g[b * n + j]);
            if (a > gmax) gmax = a;
        }
        for (size_t j = 0; j < n; ++j) {
            double kap = pow((gmax + eps) / (fabs(unit_scale * g[b * n + j]) + eps), gamma);
            if (kappa_max > 0.0 && kap > kappa_max) kap = kappa_max;
            if (kappa_out) kappa_out[b * n + j] = kap;
            vnext[b * n + j] = vprop[b * n + j] - rho * kap * unit_scale * h[b * n + j];
        }
        rho_out[b] = rho;
        if (tv_out) tv_out[b] = tv;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Least-squares potential of baseline DPS (Sec. 4, Phi_l2 with Sigma =       */
/* sigma^2 I; Sec. 6 ablation: MSE guidance, optionally with the wavefield    */
/* enhancement of Sec. 5.1 (I) and a misfit-scale normalisation)              */
/* ------------------------------------------------------------------------ */

/* Observations dobs [ntr][nt] shared by the B samples dsyn [B][ntr][nt]:
 *   w = 1/(1 + k |dobs| / max|dobs|)                      Eq. omega_def
 *       (w = 1 when k = 0 or every observation is zero)
 *   r = dsyn_b - dobs
 *   S = sigma^2                   (normalize = 0: Phi_l2 = |r|^2_{Sigma^-1} / 2)
 *     = sum (w dobs)^2            (normalize = 1; 1 if that sum is 0)
 *   J_b   = (1/2) sum (w r)^2 / S
 *   adj_b = dJ_b / d dsyn_b = w^2 r / S                                     */
int orc_l2_misfit(int B, int ntr, int nt, const double* dsyn, const double* dobs, double sigma, double k,
                  int normalize, double* J, double* adj) {
    if (B < 0 || ntr < 1 || nt < 1 || !(k >= 0) || (!normalize && !(sigma > 0))) return ORC_EINVAL;
    size_t n = (size_t)ntr * nt;
    double amax = 0.0;
    for (size_t j = 0; j < n; ++j)
        if (fabs(dobs[j]) > amax) amax = fabs(dobs[j]);
    double* w = (double*)malloc(n * sizeof(double));
    if (!w) return ORC_ENOMEM;
    for (size_t j = 0; j < n; ++j) w[j] = (k > 0.0 && amax > 0.0) ? 1.0 / (1.0 + k * fabs(dobs[j]) / amax) : 1.0;
    double S = sigma * sigma;
    if (normalize) {
        S = 0.0;
        for (size_t j = 0; j < n; ++j) S += (w[j] * dobs[j]) * (w[j] * dobs[j]);
        if (S == 0.0) S = 1.0;
    }
    for (int b = 0; b < B; ++b) {
        double acc = 0.0;
        for (size_t j = 0; j < n; ++j) {
            double r = dsyn[(size_t)b * n + j] - dobs[j];
            acc += (w[j] * r) * (w[j] * r);
            if (adj) adj[(size_t)b * n + j] = w[j] * w[j] * r / S;
        }
        J[b] = 0.5 * acc / S;
    }
    free(w);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Total-variation subgradient (Eq. tv; the TV-regularised descent baselines  */
/* W2+TV and OT-WE+TV of Sec. 6)                                              */
/* ------------------------------------------------------------------------ */

/* For each sample b, x and g [nz][nx]:
 *   out = g + alpha q,  q a subgradient of TV(x) = (1/(nz nx)) sum |x_m - x_l|
 *   over the forward differences (l -> m = right or lower neighbour) that exist:
 *   each difference adds sign(x_m - x_l) / (nz nx) to q_m and subtracts it from
 *   q_l, with sign(0) = 0.  g may be NULL (zero).                            */
int orc_tv_subgradient(int B, int nz, int nx, const double* x, const double* g, double alpha, double* out) {
    if (B < 0 || nz < 1 || nx < 1) return ORC_EINVAL;
    size_t n = (size_t)nz * nx;
    for (int b = 0; b < B; ++b) {
        const double* xb = x + (size_t)b * n;
        double* ob = out + (size_t)b * n;
        for (size_t j = 0; j < n; ++j) ob[j] = g ? g[(size_t)b * n + j] : 0.0;
        for (int iz = 0; iz < nz; ++iz)
            for (int ix = 0; ix < nx; ++ix) {
                int l = iz * nx + ix;
                if (ix + 1 < nx) {
                    double d = xb[l + 1] - xb[l];
                    double s = (d > 0.0) - (d < 0.0);
                    ob[l + 1] += alpha * s / (double)n;
                    ob[l] -= alpha * s / (double)n;
                }
                if (iz + 1 < nz) {
                    double d = xb[l + nx] - xb[l];
                    double s = (d > 0.0) - (d < 0.0);
                    ob[l + nx] += alpha * s / (double)n;
                    ob[l] -= alpha * s / (double)n;
                }
            }
    }
    return ORC_OK;
}

/* Small helpers exposed for the self-checks. */
void orc_stencil_weights(double* w) {
    for (int i = 0; i < 5; ++i) w[i] = W8[i];
}

/* Applies L (with the boundary rules) to a padded field, for operator checks. */
int orc_apply_laplacian(int nzp, int nxp, double dz, double dx, int fs, const double* u, double* out, int transpose) {
    Grid g;
    g.nz = nzp;
    g.nx = nxp;
    g.nb = 0;
    g.fs = fs ? 1 : 0;
    g.nzp = nzp;
    g.nxp = nxp;
    g.ztop = 0;
    g.dz = dz;
    g.dx = dx;
    g.dt = 1.0;
    g.nt = 2;
    if (transpose) {
        lap_transpose(&g, u, out);
    } else {
        for (int iz = 0; iz < nzp; ++iz)
            for (int ix = 0; ix < nxp; ++ix) out[iz * nxp + ix] = lap_at(&g, u, iz, ix);
    }
    return ORC_OK;
}

/* Sponge damping factor a of the padded grid, for checks of the profile. */
int orc_sponge(int nz, int nx, double dz, double dx, double dt, int nb, int fs, double vmax, double* a) {
    Grid g;
    int st = grid_init(&g, nz, nx, dz, dx, dt, 2, nb, fs);
    if (st) return st;
    sponge_factor(&g, vmax, a);
    return ORC_OK;
}

/* Full wavefield snapshot u^n (padded grid) after n steps, for checks that need
 * the field itself (stability, energy). */
int orc_wavefield(int nz, int nx, double dz, double dx, double dt, int nt, int nb, int fs, double vmax_decl,
                  int src_iz, int src_ix, const double* v, const double* wavelet, int nsteps, int check_cfl,
                  double* u_out) {
    Grid g;
    int st = grid_init(&g, nz, nx, dz, dx, dt, nt, nb, fs);
    if (st) return st;
    if (check_cfl && !cfl_ok(&g, vmax_decl)) return ORC_ECFL;
    int np = g.nzp * g.nxp;
    Coefs cf;
    st = coefs_make(&g, v, vmax_decl, &cf);
    if (st) return st;
    double* u0 = (double*)calloc((size_t)np, sizeof(double));
    double* u1 = (double*)calloc((size_t)np, sizeof(double));
    double* u2 = (double*)calloc((size_t)np, sizeof(double));
    int sp = padded_index(&g, src_iz, src_ix);
    for (int n = 0; n < nsteps; ++n) {
        double amp = (n < nt) ? wavelet[n] : 0.0;
        fwd_step(&g, &cf, u1, u0, u2, sp, amp, NULL);
        double* t = u0;
        u0 = u1;
        u1 = u2;
        u2 = t;
    }
    memcpy(u_out, u1, sizeof(double) * np);
    free(u0);
    free(u1);
    free(u2);
    coefs_free(&cf);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Perfectly matched layer (Sec. 2.1 absorbing boundary; Sec. 6.1: PML of 6
 * grid points on the left, right and bottom).  The paper does not state its
 * PML equations; this is the unsplit second-order PML of Grote and Sim
 * ("Efficient PML for the wave equation", 2010) in the form obtained from the
 * complex coordinate stretch s_x = 1 + zeta_x/(i w), s_z = 1 + zeta_z/(i w):
 *
 *   u_tt + (zeta_x + zeta_z) u_t + zeta_x zeta_z u = v^2 (Lap u + d_x psi_x + d_z psi_z + s)
 *   psi_x,t = -zeta_x psi_x + (zeta_z - zeta_x) d_x u
 *   psi_z,t = -zeta_z psi_z + (zeta_x - zeta_z) d_z u
 *
 * with v^2 outside the divergence (exact here because the padded velocity is
 * constant along the normal of each layer).  zeta uses the quadratic profile
 * of the sponge with the same strength formula; it does not depend on v.
 * Discretisation (8th-order central first derivatives d_k = 4/5, -1/5, 4/105,
 * -1/280; psi at half steps, advanced by the trapezoid rule):
 *
 *   g_x = Dx u^n, g_z = Dz u^n                         (u even across a reflecting top)
 *   Q   = c (psi^{n-1/2} + h g),  c = 1/(1 + zeta dt/2), h_x = dt/2 (zeta_z - zeta_x),
 *                                  h_z = dt/2 (zeta_x - zeta_z)   (Q = psi at step n)
 *   psi^{n+1/2} = 2 Q - psi^{n-1/2}
 *   D   = L u^n + Dx Q_x + Dz Q_z + s^n                (Q_z odd across a reflecting top)
 *   u^{n+1} = p u^n - q u^{n-1} + r D,  E = 1/(1 + alpha dt/2), alpha = zeta_x + zeta_z,
 *             p = (2 - dt^2 zeta_x zeta_z) E, q = (1 - alpha dt/2) E, r = dt^2 v^2 E.
 *
 * In the model region zeta = 0, so p = 2, q = 1, r = dt^2 v^2 and Q = 0: the
 * interior update is the leapfrog of the sponge scheme, operation for
 * operation.  Outside the padded grid every field is zero. */

static const double D8[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
static const double PML_R = 1e-3;

static double pml_zeta(int delta, int nb, double h, double vmax) {
    if (nb <= 0 || delta <= 0) return 0.0;
    double r = (double)delta / nb;
    return 3.0 * vmax * log(1.0 / PML_R) / (2.0 * nb * h) * r * r;
}

typedef struct {
    double *vp, *p, *q, *r, *E, *cx, *cz, *hx, *hz;
} PmlCoefs;

static void pml_free(PmlCoefs* c) {
    free(c->vp);
    free(c->p);
    free(c->q);
    free(c->r);
    free(c->E);
    free(c->cx);
    free(c->cz);
    free(c->hx);
    free(c->hz);
}

static int pml_make(const Grid* g, const double* v, double vmax, PmlCoefs* c) {
    int np = g->nzp * g->nxp;
    double** arr[9] = {&c->vp, &c->p, &c->q, &c->r, &c->E, &c->cx, &c->cz, &c->hx, &c->hz};
    int bad = 0;
    for (int i = 0; i < 9; ++i) {
        *arr[i] = (double*)malloc(sizeof(double) * np);
        if (!*arr[i]) bad = 1;
    }
    if (bad) return ORC_ENOMEM;
    pad_velocity(g, v, c->vp);
    double dt = g->dt;
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            int dzc = 0, dxc = 0;
            if (iz >= g->ztop + g->nz) dzc = iz - (g->ztop + g->nz - 1);
            if (!g->fs && iz < g->ztop) dzc = g->ztop - iz;
            if (ix < g->nb) dxc = g->nb - ix;
            if (ix >= g->nb + g->nx) dxc = ix - (g->nb + g->nx - 1);
            double zx = pml_zeta(dxc, g->nb, g->dx, vmax), zz = pml_zeta(dzc, g->nb, g->dz, vmax);
            int p = iz * g->nxp + ix;
            double alpha = zx + zz;
            c->E[p] = 1.0 / (1.0 + alpha * dt / 2.0);
            c->p[p] = (2.0 - dt * dt * zx * zz) * c->E[p];
            c->q[p] = (1.0 - alpha * dt / 2.0) * c->E[p];
            c->r[p] = dt * dt * c->vp[p] * c->vp[p] * c->E[p];
            c->cx[p] = 1.0 / (1.0 + zx * dt / 2.0);
            c->cz[p] = 1.0 / (1.0 + zz * dt / 2.0);
            c->hx[p] = dt / 2.0 * (zz - zx);
            c->hz[p] = dt / 2.0 * (zx - zz);
        }
    return ORC_OK;
}

/* Q_z with the odd extension across a reflecting top. */
static double qz_at(const Grid* g, const double* q, int iz, int ix) {
    double sgn = 1.0;
    if (g->fs && iz < 0) {
        iz = -iz;
        sgn = -1.0;
    }
    if (iz < 0 || iz >= g->nzp || ix < 0 || ix >= g->nxp) return 0.0;
    return sgn * q[iz * g->nxp + ix];
}

static double dx_at(const Grid* g, const double* f, int iz, int ix) {
    double s = 0.0;
    for (int k = 1; k <= 4; ++k) s += D8[k] * (uat(g, f, iz, ix + k) - uat(g, f, iz, ix - k));
    return s / g->dx;
}

static double dz_even_at(const Grid* g, const double* f, int iz, int ix) {
    double s = 0.0;
    for (int k = 1; k <= 4; ++k) s += D8[k] * (uat(g, f, iz + k, ix) - uat(g, f, iz - k, ix));
    return s / g->dz;
}

static double dz_odd_at(const Grid* g, const double* f, int iz, int ix) {
    double s = 0.0;
    for (int k = 1; k <= 4; ++k) s += D8[k] * (qz_at(g, f, iz + k, ix) - qz_at(g, f, iz - k, ix));
    return s / g->dz;
}

/* State of one unit between steps: u^n, u^{n-1}, psi_x^{n-1/2}, psi_z^{n-1/2}. */
typedef struct {
    double *u, *um, *px, *pz;
} PmlState;

/* One step.  Q_x, Q_z and D of the step are returned in the work arrays;
 * the state advances in place (un receives u^{n+1}). */
static void pml_step(const Grid* g, const PmlCoefs* c, const double* u, const double* um, double* px, double* pz,
                     double* un, int src_p, double src_amp, double* Qx, double* Qz, double* D) {
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            int p = iz * g->nxp + ix;
            Qx[p] = c->cx[p] * (px[p] + c->hx[p] * dx_at(g, u, iz, ix));
            Qz[p] = c->cz[p] * (pz[p] + c->hz[p] * dz_even_at(g, u, iz, ix));
        }
    for (int p = 0; p < g->nzp * g->nxp; ++p) {
        px[p] = 2.0 * Qx[p] - px[p];
        pz[p] = 2.0 * Qz[p] - pz[p];
    }
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            int p = iz * g->nxp + ix;
            double d = lap_at(g, u, iz, ix) + dx_at(g, Qx, iz, ix) + dz_odd_at(g, Qz, iz, ix);
            if (p == src_p) d += src_amp / (g->dx * g->dz);
            D[p] = d;
            un[p] = c->p[p] * u[p] - c->q[p] * um[p] + c->r[p] * d;
        }
}

/* Forward of one unit; if ck != NULL the state before step n is saved for
 * every n that is a multiple of K, as 4 planes (u^n, u^{n-1}, psi_x, psi_z). */
static int pml_forward_unit(const Grid* g, const PmlCoefs* c, const double* wavelet, int src_p, int nr,
                            const int* rec_p, double* trace, double* ck, int K) {
    size_t np = (size_t)g->nzp * g->nxp;
    double* buf = (double*)calloc(8 * np, sizeof(double));
    if (!buf) return ORC_ENOMEM;
    double *u = buf, *um = buf + np, *un = buf + 2 * np, *px = buf + 3 * np, *pz = buf + 4 * np;
    double *Qx = buf + 5 * np, *Qz = buf + 6 * np, *D = buf + 7 * np;
    for (int r = 0; r < nr; ++r) trace[(size_t)r * g->nt] = u[rec_p[r]];
    for (int n = 0; n + 1 < g->nt; ++n) {
        if (ck && n % K == 0) {
            double* dst = ck + (size_t)(n / K) * 4 * np;
            memcpy(dst, u, sizeof(double) * np);
            memcpy(dst + np, um, sizeof(double) * np);
            memcpy(dst + 2 * np, px, sizeof(double) * np);
            memcpy(dst + 3 * np, pz, sizeof(double) * np);
        }
        pml_step(g, c, u, um, px, pz, un, src_p, wavelet[n], Qx, Qz, D);
        for (int r = 0; r < nr; ++r) trace[(size_t)r * g->nt + n + 1] = un[rec_p[r]];
        double* t = um;
        um = u;
        u = un;
        un = t;
    }
    free(buf);
    return ORC_OK;
}

/* Scatter transposes of the first-derivative gathers (each term of dx_at,
 * dz_even_at and dz_odd_at sent back to the node it read). */
static void dx_transpose_add(const Grid* g, const double* y, double* out) {
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            double val = y[iz * g->nxp + ix] / g->dx;
            if (val == 0.0) continue;
            for (int k = 1; k <= 4; ++k) {
                if (ix + k < g->nxp) out[iz * g->nxp + ix + k] += D8[k] * val;
                if (ix - k >= 0) out[iz * g->nxp + ix - k] -= D8[k] * val;
            }
        }
}

static void dz_even_transpose_add(const Grid* g, const double* y, double* out) {
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            double val = y[iz * g->nxp + ix] / g->dz;
            if (val == 0.0) continue;
            for (int k = 1; k <= 4; ++k) {
                if (iz + k < g->nzp) out[(iz + k) * g->nxp + ix] += D8[k] * val;
                int t = iz - k;
                if (g->fs && t < 0) t = -t;
                if (t >= 0 && t < g->nzp) out[t * g->nxp + ix] -= D8[k] * val;
            }
        }
}

static void dz_odd_transpose_add(const Grid* g, const double* y, double* out) {
    for (int iz = 0; iz < g->nzp; ++iz)
        for (int ix = 0; ix < g->nxp; ++ix) {
            double val = y[iz * g->nxp + ix] / g->dz;
            if (val == 0.0) continue;
            for (int k = 1; k <= 4; ++k) {
                if (iz + k < g->nzp) out[(iz + k) * g->nxp + ix] += D8[k] * val;
                int t = iz - k;
                if (t >= 0)
                    out[t * g->nxp + ix] -= D8[k] * val;
                else if (g->fs && -t < g->nzp)
                    out[(-t) * g->nxp + ix] += D8[k] * val; /* the read was -Q_z(-t) */
            }
        }
}

/* Reverse mode of pml_forward_unit: gC[p] = dJ/d(dt^2 v_p^2) given a^n = dJ/d(trace sample n).
 * Per step n (reverse order), with ub1 = dJ/du^{n+1} complete, ub2 = dJ/du^{n+2}
 * and (bx, bz) = dJ/d psi^{n+1/2}:
 *   dJ/dC += ub1 E D;  Db = r ub1;
 *   Qb = D^T-gather of Db (x: Dx^T, z: odd-extension transpose) + 2 (bx, bz);
 *   (bx, bz) <- c Qb - (bx, bz);  gb = c h Qb;
 *   ub^n = R^T a^n + p ub1 - q ub2 + L^T Db + Dx^T gb_x + Dz^T gb_z (even-extension transpose). */
static int pml_reverse_unit(const Grid* g, const PmlCoefs* c, const double* wavelet, int src_p, int nr,
                            const int* rec_p, const double* adj, double* gC) {
    size_t np = (size_t)g->nzp * g->nxp;
    int N = g->nt;
    int K = (int)ceil(sqrt((double)N));
    if (K < 1) K = 1;
    int nseg = (N - 1 + K - 1) / K;
    double* ck = (double*)malloc(sizeof(double) * (size_t)nseg * 4 * np);
    double* seg = (double*)malloc(sizeof(double) * (size_t)(K + 1) * 4 * np); /* state before each step */
    double* trace = (double*)malloc(sizeof(double) * (size_t)nr * N);
    double* w = (double*)calloc(12 * np, sizeof(double));
    int st = ORC_OK;
    if (!ck || !seg || !trace || !w) {
        st = ORC_ENOMEM;
        goto done;
    }
    {
        double *ub0 = w, *ub1 = w + np, *ub2 = w + 2 * np, *bx = w + 3 * np, *bz = w + 4 * np;
        double *Db = w + 5 * np, *Qbx = w + 6 * np, *Qbz = w + 7 * np, *Qx = w + 8 * np, *Qz = w + 9 * np;
        double *D = w + 10 * np, *un = w + 11 * np;
        st = pml_forward_unit(g, c, wavelet, src_p, nr, rec_p, trace, ck, K);
        if (st) goto done;
        memset(gC, 0, sizeof(double) * np);
        for (int r = 0; r < nr; ++r) ub1[rec_p[r]] += adj[(size_t)r * N + (N - 1)];
        for (int s = nseg - 1; s >= 0; --s) {
            int a = s * K, e = a + K;
            if (e > N - 1) e = N - 1;
            /* seg[i] = state before step a + i (4 planes each) */
            memcpy(seg, ck + (size_t)s * 4 * np, sizeof(double) * 4 * np);
            for (int n = a; n + 1 < e; ++n) {
                double* cur = seg + (size_t)(n - a) * 4 * np;
                double* nxt = cur + 4 * np;
                memcpy(nxt + 2 * np, cur + 2 * np, sizeof(double) * 2 * np);
                pml_step(g, c, cur, cur + np, nxt + 2 * np, nxt + 3 * np, nxt, src_p, wavelet[n], Qx, Qz, D);
                memcpy(nxt + np, cur, sizeof(double) * np);
            }
            for (int n = e - 1; n >= a; --n) {
                double* cur = seg + (size_t)(n - a) * 4 * np;
                /* recompute Q and D of step n from the state before it */
                memcpy(Qbx, cur + 2 * np, sizeof(double) * np); /* scratch copies of psi */
                memcpy(Qbz, cur + 3 * np, sizeof(double) * np);
                pml_step(g, c, cur, cur + np, Qbx, Qbz, un, src_p, wavelet[n], Qx, Qz, D);
                for (size_t p = 0; p < np; ++p) {
                    gC[p] += ub1[p] * c->E[p] * D[p];
                    Db[p] = c->r[p] * ub1[p];
                    Qbx[p] = 2.0 * bx[p];
                    Qbz[p] = 2.0 * bz[p];
                }
                dx_transpose_add(g, Db, Qbx);
                dz_odd_transpose_add(g, Db, Qbz);
                lap_transpose(g, Db, ub0); /* overwrites ub0 */
                for (size_t p = 0; p < np; ++p) {
                    bx[p] = c->cx[p] * Qbx[p] - bx[p];
                    bz[p] = c->cz[p] * Qbz[p] - bz[p];
                    ub0[p] += c->p[p] * ub1[p] - c->q[p] * ub2[p];
                    Qbx[p] *= c->cx[p] * c->hx[p]; /* gb_x */
                    Qbz[p] *= c->cz[p] * c->hz[p]; /* gb_z */
                }
                dx_transpose_add(g, Qbx, ub0);
                dz_even_transpose_add(g, Qbz, ub0);
                for (int r = 0; r < nr; ++r) ub0[rec_p[r]] += adj[(size_t)r * N + n];
                double* t = ub2;
                ub2 = ub1;
                ub1 = ub0;
                ub0 = t;
            }
        }
    }
done:
    free(ck);
    free(seg);
    free(trace);
    free(w);
    return st;
}

/* Forward modelling with the PML as the absorbing layer (nb cells); arguments as orc_forward. */
int orc_forward_pml(int nz, int nx, double dz, double dx, double dt, int nt, int nb, int fs, double vmax_decl,
                    int ns, const int* src_iz, const int* src_ix, int nr, const int* rec_iz, const int* rec_ix,
                    int B, const double* v, const double* wavelet, double* d) {
    Grid g;
    int st = grid_init(&g, nz, nx, dz, dx, dt, nt, nb, fs);
    if (st) return st;
    st = check_inputs(&g, B, v, vmax_decl, ns, src_iz, src_ix, nr, rec_iz, rec_ix);
    if (st) return st;
    int* rec_p = (int*)malloc(sizeof(int) * (nr > 0 ? nr : 1));
    for (int r = 0; r < nr; ++r) rec_p[r] = padded_index(&g, rec_iz[r], rec_ix[r]);
    int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int u = 0; u < B * ns; ++u) {
        int b = u / ns, s = u % ns;
        PmlCoefs c;
        memset(&c, 0, sizeof(c));
        int e = pml_make(&g, v + (size_t)b * nz * nx, vmax_decl, &c);
        if (!e)
            e = pml_forward_unit(&g, &c, wavelet, padded_index(&g, src_iz[s], src_ix[s]), nr, rec_p,
                                 d + (size_t)u * nr * nt, NULL, 1);
        pml_free(&c);
        if (e) {
#pragma omp critical
            err = e;
        }
    }
    free(rec_p);
    return err;
}

/* Reverse-mode gradient dJ/dv with the PML (summed over shots); arguments as orc_gradient
 * without the wavelet gradient. */
int orc_gradient_pml(int nz, int nx, double dz, double dx, double dt, int nt, int nb, int fs, double vmax_decl,
                     int ns, const int* src_iz, const int* src_ix, int nr, const int* rec_iz, const int* rec_ix,
                     int B, const double* v, const double* wavelet, const double* adj, double* grad) {
    Grid g;
    int st = grid_init(&g, nz, nx, dz, dx, dt, nt, nb, fs);
    if (st) return st;
    st = check_inputs(&g, B, v, vmax_decl, ns, src_iz, src_ix, nr, rec_iz, rec_ix);
    if (st) return st;
    int np = g.nzp * g.nxp;
    int* rec_p = (int*)malloc(sizeof(int) * (nr > 0 ? nr : 1));
    for (int r = 0; r < nr; ++r) rec_p[r] = padded_index(&g, rec_iz[r], rec_ix[r]);
    double* gvp = (double*)calloc((size_t)B * ns * np, sizeof(double));
    if (!gvp) {
        free(rec_p);
        return ORC_ENOMEM;
    }
    int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int u = 0; u < B * ns; ++u) {
        int b = u / ns, s = u % ns;
        PmlCoefs c;
        memset(&c, 0, sizeof(c));
        double* gC = (double*)malloc(sizeof(double) * np);
        int e = gC ? pml_make(&g, v + (size_t)b * nz * nx, vmax_decl, &c) : ORC_ENOMEM;
        if (!e)
            e = pml_reverse_unit(&g, &c, wavelet, padded_index(&g, src_iz[s], src_ix[s]), nr, rec_p,
                                 adj + (size_t)u * nr * nt, gC);
        if (!e) /* C = dt^2 vp^2  =>  dC/dvp = 2 dt^2 vp */
            for (int p = 0; p < np; ++p) gvp[(size_t)u * np + p] = gC[p] * 2.0 * dt * dt * c.vp[p];
        pml_free(&c);
        free(gC);
        if (e) {
#pragma omp critical
            err = e;
        }
    }
    if (!err) {
        memset(grad, 0, sizeof(double) * (size_t)B * nz * nx);
        for (int b = 0; b < B; ++b)
            for (int s = 0; s < ns; ++s)
                for (int iz = 0; iz < g.nzp; ++iz)
                    for (int ix = 0; ix < g.nxp; ++ix) {
                        int mz = clampi(iz - g.ztop, 0, nz - 1);
                        int mx = clampi(ix - g.nb, 0, nx - 1);
                        grad[(size_t)b * nz * nx + mz * nx + mx] += gvp[((size_t)b * ns + s) * np + iz * g.nxp + ix];
                    }
    }
    free(gvp);
    free(rec_p);
    return err;
}
