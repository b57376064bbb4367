/*
 * fwi.h -- C ABI of the MI355X (gfx950) likelihood-guidance library for
 * physics-guided diffusion full-waveform inversion
 * ("Robust Physics-Guided Diffusion for Full-Waveform Inversion", arXiv 2603.16393).
 *
 * One call of the guidance path per reverse-diffusion step (Algorithm 2, the
 * gradient, preconditioner and update lines) is
 *
 *     fwi_forward            d_syn = F(v)                    (Sec. 2.1, Sec. 6.1)
 *     fwi_w2_misfit          J(v), dJ/dd_syn                 (Sec. 5.1, Sec. 6.2)
 *     fwi_adjoint_gradient   g = dJ/dv                       (adjoint of F applied to dJ/dd_syn)
 *     fwi_guidance_step      v_{i-1} = v'_{i-1} - rho_i D_i h (Sec. 5.2, Eqs. tv, rho, kappa, precond_step)
 *
 * after a one-time fwi_set_obs (weights, shift constants, observed quantiles
 * and S_obs of Sec. 5.1 (I)-(III)).  The comparison variants of Sec. 6 swap
 * single calls: fwi_l2_misfit for fwi_w2_misfit (baseline DPS, Algorithm 1,
 * and the MSE ablations), and fwi_tv_subgradient before fwi_guidance_step
 * (the TV-regularised descent baselines).  fwi_ddpm_step gives the other
 * lines of a reverse step of Algorithm 2 (clean estimator, posterior mean
 * plus noise) around the score network.  The absorbing layer of F is a
 * damping sponge, or the perfectly matched layer of Sec. 2.1 / Sec. 6.1 when
 * fwi_geometry.pml is set.
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers unless marked HOST; they are owned by
 *     the caller, must stay valid until the work queued on `stream` has run,
 *     and are row-major with the last index contiguous.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream); all
 *     calls only enqueue work on it and return without synchronising, except
 *     fwi_plan_create / fwi_plan_destroy / fwi_status.
 *   - Velocities are in m/s, lengths in m, times in s; model row 0 is the
 *     surface (the reflecting top boundary), x is the fast axis.
 *   - Return value: FWI_OK (0) or a negative fwi_status_code.  Argument errors
 *     are detected on the host before anything is enqueued.  Conditions that
 *     can only be seen on the device (a velocity outside (0, v_max], NaN/Inf)
 *     raise a sticky flag that fwi_status reports.  Nothing throws.
 *   - A plan is not thread-safe: use one plan per host thread and stream.
 */
#ifndef FWI_H
#define FWI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FWI_OK = 0,
    FWI_EINVAL = -1,   /* invalid argument (shape, index, NULL pointer, parameter range) */
    FWI_ECFL = -2,     /* v_max dt sqrt(2048/315 (1/dx^2 + 1/dz^2)) >= 2: explicit scheme unstable */
    FWI_ENOMEM = -3,   /* device allocation failed or the memory budget is too small */
    FWI_EHIP = -4,     /* a HIP runtime call failed */
    FWI_ESTATE = -5,   /* call out of order (no observations set, no stored forward state, ...) */
    FWI_EDEVICE = -6   /* device-side check failed (velocity not finite, <= 0 or > v_max) */
} fwi_status_code;

/* Grid, time axis and acquisition (Sec. 2.1: grid V of nodal velocities,
 * receiver restriction R, data array N_s x N_r x N_T; Sec. 6.3.1 geometry).
 * Index arrays are HOST pointers, copied by fwi_plan_create.  Source and
 * receiver nodes must lie in the model grid; receiver nodes must be distinct. */
typedef struct {
    int nz, nx;            /* model grid rows (depth) and columns */
    double dz, dx;         /* grid spacings (m) */
    double dt;             /* time step (s); trace sample n is the field at t_n = n dt */
    int nt;                /* samples per trace (>= 2); nt - 1 time steps are taken */
    int nb;                /* absorbing-layer width in cells on the left, right and bottom
                              (and the top when free_surface == 0); the layer is the damping
                              sponge unless `pml` is set */
    int free_surface;      /* 1: reflecting top, d_n u = 0 by even mirroring (Eq. solving) */
    double v_max;          /* declared upper bound of v: sets the layer strength and is
                              checked against the CFL limit at plan creation */
    int ns;                /* shots */
    const int* src_iz;     /* HOST [ns] source rows */
    const int* src_ix;     /* HOST [ns] source columns */
    int nr;                /* receivers, one spread shared by all shots */
    const int* rec_iz;     /* HOST [nr] receiver rows */
    const int* rec_ix;     /* HOST [nr] receiver columns */
    int pml;               /* 0: the nb-cell layer is the damping sponge; 1: it is a perfectly matched layer
                              (Sec. 2.1 absorbing boundary, Sec. 6.1: 6 cells on the left, right and bottom),
                              the unsplit second-order form of a complex coordinate stretch with the sponge's
                              quadratic profile and strength.  Plans only (fwi_batch_create rejects it).
                              The field stays in LDS when it can (plan path 2, full forward history): in one
                              workgroup (about 7,000 padded cells, e.g. a 70 x 70 model with 6 cells) or, when
                              max_batch * ns fields leave CUs idle, split into row bands held by several
                              workgroups (launched cooperatively; see `split` of fwi_plan_options).  Larger
                              fields, a history that does not fit, ckpt_every > 0 and force_path = 1 take the
                              HBM sweep (path 3, full history or checkpoints), with the same results bit for
                              bit where both apply.  While the caller's stream is capturing a graph, path 2
                              runs its one-workgroup sweep: FWI_EINVAL at the call if the field only fits as
                              row bands. */
} fwi_geometry;

/* Misfit settings (Sec. 5.1 and Sec. 6.2).  Paper values: k = 100,
 * eps_prime = 1e-9, n_xi = 1000, c_factor = 1.1, squared = 0, reduction = 0. */
typedef struct {
    double k;          /* amplitude weight omega = 1/(1 + k |d_obs| / max|d_obs|) (Eq. omega_def); 0 = raw traces */
    double eps_prime;  /* added to the trapezoid mass before normalising (Sec. 6.2) */
    int n_xi;          /* uniform xi grid j/(n_xi-1) for the quantile integral (>= 2) */
    double c_factor;   /* c' = c_factor |min_t omega d_obs| per trace (Sec. 5.1 (II)) */
    int squared;       /* 0: sum W2 / sum ||Q_obs||  (Eq. final_objective)
                          1: sum W2^2 / sum ||Q_obs||^2 (raw-trace W2 baseline, Sec. 6) */
    int reduction;     /* 0: divide by the observation scale S_obs; 1: average over pairs */
} fwi_w2_params;

/* Least-squares misfit settings: the potential Phi_l2 of baseline DPS (Sec. 4,
 * Algorithm 1; Sigma = sigma^2 I, paper sigma = 0.05) and the ablation's MSE
 * guidance with wavefield enhancement (Sec. 6: the amplitude weight of
 * Sec. 5.1 (I) and a misfit-scale normalisation). */
typedef struct {
    double sigma;   /* noise standard deviation; S = sigma^2 when normalize = 0 (> 0 then) */
    double k;       /* amplitude weight w = 1/(1 + k |d_obs| / max|d_obs|) (Eq. omega_def); 0: w = 1 */
    int normalize;  /* 1: S = sum (w d_obs)^2 over all traces (1 if that is 0) instead of sigma^2 */
} fwi_l2_params;

/* Guidance-update settings (Sec. 5.2).  Paper fixed values: c = 0.1,
 * tau = 0, eps = 1e-4 (Sec. 6.3); gamma and rho0 per dataset (Table 'parameter'). */
typedef struct {
    double rho0;        /* base guidance strength */
    double c;           /* TV decay scale of rho (Eq. rho), > 0 */
    double tau;         /* TV tolerance of rho (Eq. rho) */
    double gamma;       /* exponent of the diagonal scaling (Eq. kappa), >= 0 */
    double eps;         /* regulariser of the diagonal scaling (Eq. kappa), > 0 */
    double kappa_max;   /* optional cap on kappa (the optional clipping of Algorithm 2); <= 0: off */
    double unit_scale;  /* chain factor from the gradients' units to the diffusion state's
                           (e.g. 1500 when v = 1500 + 1500 (x + 1) m/s and g is per m/s) */
} fwi_guidance_params;

typedef struct fwi_plan fwi_plan;

/* Read-only description of a plan's layout. */
typedef struct {
    int nzp, nxp;              /* padded grid */
    int path;                  /* 0: field resident in LDS (one workgroup per (sample, shot), or lds_split
                                  workgroups per field each holding a band of rows);
                                  1: tiled sweep from HBM, two time steps per launch;
                                  2: PML sweep, field and auxiliary fields resident in LDS, one workgroup
                                  per (sample, shot), or lds_split workgroups per field each holding a band
                                  of rows;
                                  3: PML sweep from HBM, one time step per two launches (auxiliary fields
                                  of the layer, then every cell) */
    int store_mode;            /* 0: full history of D = L u + s kept for the adjoint;
                                  1: checkpoints every `ckpt_every` steps plus recomputation */
    int ckpt_every;
    int max_batch;
    size_t device_bytes;       /* device memory held by the plan */
    int lds_tile_x, lds_tile_z;  /* register tile of the LDS-resident path (0 on the tiled path) */
    int lds_split;             /* LDS-resident paths (0, 2): workgroups sharing one field (1: one per field;
                                  0 on the tiled and PML HBM paths) */
} fwi_plan_info;

/* Creates a plan for up to `max_batch` velocity samples on the current device.
 * Validates the geometry (FWI_EINVAL), the CFL condition for v_max (FWI_ECFL),
 * and allocates every workspace up front: padded coefficients, the forward
 * history (full or checkpointed, whichever fits `mem_budget_bytes`; 0 = no
 * limit beyond device memory) and the observation cache.  FWI_ENOMEM if even
 * the checkpointed layout does not fit.  *plan receives the handle. */
int fwi_plan_create(const fwi_geometry* geom, int max_batch, size_t mem_budget_bytes, fwi_plan** plan);

/* Execution options for fwi_plan_create_ex. */
typedef struct {
    int force_path;     /* -1: automatic; 0: LDS-resident (FWI_EINVAL if the field does not fit);
                           1: tiled sweep (PML: its HBM sweep) */
    int ckpt_every;     /* 0: automatic (full history when it fits the budget, else checkpoints);
                           > 0: checkpoint every ckpt_every steps and recompute (tiled sweep, or the PML's
                           HBM sweep; FWI_EINVAL with force_path = 0) */
    int lds_tile_x;     /* LDS-resident path: columns x rows of one thread's register tile;   */
    int lds_tile_z;     /* 0, 0 = the built-in cost model's choice; FWI_EINVAL if not available */
    int timing;         /* 1: record HIP events around each forward and adjoint sweep on the caller's
                           stream (read with fwi_plan_sweep_ms); 0: off */
    int split;          /* LDS-resident and PML paths, when max_batch * ns fields leave CUs idle: 0 = split
                           each field over several workgroups (row bands exchanging halos every step, launched
                           cooperatively) if the cost model prefers it (PML: whenever feasible), and never with
                           an explicit lds tile; 1 = split whenever feasible (FWI_EINVAL if not); -1 = never.
                           While the caller's stream is capturing a graph the unsplit kernels run (same
                           results bit for bit). */
} fwi_plan_options;

/* fwi_plan_create with explicit execution options (NULL = automatic). */
int fwi_plan_create_ex(const fwi_geometry* geom, int max_batch, size_t mem_budget_bytes,
                       const fwi_plan_options* options, fwi_plan** plan);

/* Frees the plan's device memory after synchronising the device. */
int fwi_plan_destroy(fwi_plan* plan);

int fwi_plan_get_info(const fwi_plan* plan, fwi_plan_info* info);

/* Observation side of the misfit (Sec. 5.1 (I)-(III), Sec. 6.2): from
 * d_obs [ns][nr][nt] computes the weights omega, the per-trace shift c', the
 * observed quantiles on the xi grid and the scale S_obs, all kept by the plan
 * (d_obs itself is not retained).  Must precede fwi_w2_misfit. */
int fwi_set_obs(fwi_plan* plan, const float* d_obs, const fwi_w2_params* params, void* stream);

/* Forward modelling (Eq. solving with the discretisation of Sec. 6.1):
 * 8th-order central differences in space, leapfrog in time, damping sponge,
 * even mirror at the top, point source wavelet[n] / (dx dz) at the shot node,
 * d_syn[b][s][r][n] = u^n at receiver r (so d_syn[..][0] = 0).
 *   v        [B][nz][nx]  velocity (m/s)
 *   wavelet  [nt]         source time function f(t_n)
 *   d_syn    [B][ns][nr][nt] output
 *   keep_for_adjoint: 1 keeps the forward history (or its checkpoints) for a
 *   following fwi_adjoint_gradient with the same v and B.  B <= max_batch. */
int fwi_forward(fwi_plan* plan, int B, const float* v, const float* wavelet, float* d_syn,
                int keep_for_adjoint, void* stream);

/* Wasserstein-2 misfit per sample and its adjoint source (Eqs. pdf_map,
 * Wp_1d, final_objective; numerics of Sec. 6.2): weighted, shifted traces
 * -> densities -> trapezoid CDFs -> quantiles on the xi grid -> W2 per pair,
 * summed and normalised.  Scans and quantiles run in FP64.
 *   d_syn    [B][ns][nr][nt]
 *   J        [B] output (double)
 *   adj_src  [B][ns][nr][nt] output dJ/dd_syn, or NULL to skip the adjoint. */
int fwi_w2_misfit(fwi_plan* plan, int B, const float* d_syn, double* J, float* adj_src, void* stream);

/* Largest B * ns * nr that fwi_w2_misfit_noalloc accepts (2 MiB of FP64
 * per-pair terms per GPU). */
#define FWI_W2_SCRATCH_PAIRS 262144

/* fwi_w2_misfit that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results
 * (bit for bit) as fwi_w2_misfit; the per-pair W2 terms go to a fixed
 * device array of FWI_W2_SCRATCH_PAIRS doubles that the library holds once
 * per GPU until the process ends, instead of the plan's workspace.  The
 * array's address is looked up on the first call on each device; no call
 * allocates or frees memory.  Every call on a GPU reuses that GPU's array
 * (each term is written before it is read, so nothing carries over), so
 * calls that overlap on one GPU, e.g. on two streams, race and must be
 * ordered by the caller.  FWI_ENOMEM when B * ns * nr > FWI_W2_SCRATCH_PAIRS;
 * otherwise the errors of fwi_w2_misfit. */
int fwi_w2_misfit_noalloc(fwi_plan* plan, int B, const float* d_syn, double* J, float* adj_src, void* stream);

/* Least-squares misfit and its adjoint source (fwi_l2_params), per sample b:
 *   J[b]        = (1/2) sum (w (d_syn[b] - d_obs))^2 / S
 *   adj_src[b]  = dJ[b]/dd_syn[b] = w^2 (d_syn[b] - d_obs) / S
 *   d_obs [ns][nr][nt] (shared by the batch), d_syn and adj_src [B][ns][nr][nt],
 *   J [B] FP64; adj_src may be NULL.  w and S come from d_obs on every call
 *   (no fwi_set_obs needed).  FP64 sums in a fixed order (deterministic).
 *   Uses the plan's scratch: not concurrent with fwi_w2_misfit on the plan. */
int fwi_l2_misfit(fwi_plan* plan, int B, const float* d_syn, const float* d_obs, const fwi_l2_params* params,
                  double* J, float* adj_src, void* stream);

/* Adjoint-state gradient (the transpose of the linearised forward map
 * applied to the adjoint source): the adjoint field is stepped backward in
 * time with the receivers as sources and correlated at zero lag with the
 * stored forward term D = L u + s, then padded cells are folded onto their
 * edge cells and shots are summed.
 *   v        [B][nz][nx]  must equal the v of the preceding keep_for_adjoint forward
 *   adj_src  [B][ns][nr][nt]  dJ/dd_syn
 *   scale    [B] per-sample factor applied to the gradient (e.g. dL/dJ), or NULL for 1
 *   grad     [B][nz][nx] output dJ/dv per m/s, summed over shots.
 * FWI_ESTATE if no forward state of this batch size is stored. */
int fwi_adjoint_gradient(fwi_plan* plan, int B, const float* v, const float* adj_src, const float* scale,
                         float* grad, void* stream);

/* Number of the forward call whose state the plan keeps for the adjoint:
 * every fwi_forward call takes the next number (1, 2, ...), and the number is
 * kept while the call's history is (keep_for_adjoint = 1); 0 when no history
 * is kept.  Host-side, no device work. */
int fwi_plan_history(const fwi_plan* plan, unsigned long long* history);

/* fwi_adjoint_gradient for the forward call numbered `history` (from
 * fwi_plan_history right after that call): FWI_ESTATE, with nothing
 * enqueued, when a later fwi_forward has replaced that call's history.  For
 * callers that keep several forward results alive at once (an autograd
 * graph with two misfit evaluations on one plan before one backward pass),
 * where the plain call would correlate with the newer history. */
int fwi_adjoint_gradient_of(fwi_plan* plan, unsigned long long history, int B, const float* v,
                            const float* adj_src, const float* scale, float* grad, void* stream);

/* Preconditioned guidance update (Eqs. tv, rho, kappa, precond_step), per sample b:
 *   TV   = (1/(nz nx)) sum of |forward differences| of v0hat in x and z (those that exist)
 *   rho  = rho0 exp(-max(TV - tau, 0) / c)
 *   kappa_j = ((max_j |s g_j| + eps) / (|s g_j| + eps))^gamma   (capped at kappa_max if > 0)
 *   v_next = v_prop - rho kappa (s h),   s = unit_scale
 * All fields [B][nz][nx]: v_prop = v'_{i-1}, h = grad wrt the diffusion state
 * v_i (the caller's chain rule through the clean estimate), g = grad wrt the
 * clean estimate, v0hat = the clean estimate in diffusion-state units.
 * rho_out [B] (may be NULL).  Needs no plan. */
int fwi_guidance_step(int B, int nz, int nx, const float* v_prop, const float* h, const float* g,
                      const float* v0hat, const fwi_guidance_params* params, float* v_next, float* rho_out,
                      void* stream);

/* Total-variation subgradient for the TV-regularised descent baselines
 * (Sec. 6: W2+TV and OT-WE+TV, with TV of Eq. tv), per sample of [B][nz][nx]:
 *   out = g + alpha q,  q_l = (1/(nz nx)) sum over the forward differences
 *   x_m - x_l' (m the right or lower neighbour of l') that contain l of
 *   sign(x_m - x_l') (+ at the head m, - at the tail l'), sign(0) = 0.
 * g may be NULL (zero) and may equal out; out must not alias v.  Needs no
 * plan.  The descent steps are then fwi_guidance_step with h = out:
 * W2+TV is gamma = 0 and tau above any TV (rho = rho0), OT-WE+TV uses the
 * preconditioner evaluated at v (v_prop = v0hat = v). */
int fwi_tv_subgradient(int B, int nz, int nx, const float* v, const float* g, double alpha, float* out, void* stream);

/* One reverse DDPM step of Algorithm 2 without its guidance term (VP schedule in DDPM indexing, Sec. 5.3):
 *   v0hat = (v + (1 - abar_i) s) / sqrt(abar_i)                                   (Eq. v0hat)
 *   v_prop = sqrt(alpha_i)(1 - abar_{i-1})/(1 - abar_i) v + sqrt(abar_{i-1}) beta_i/(1 - abar_i) v0hat + sigma z
 * with alpha_i = 1 - beta_i, over n elements (any layout; all arrays [n] f32, 16-byte aligned).  `score` = s
 * (the score network's output at (v, i)), or NULL: then v0hat is an INPUT (a clean estimate from elsewhere, e.g.
 * a denoiser).  `z` = standard normal draws (passed in; NULL = no noise).  The guidance update that completes
 * the step is fwi_guidance_step with v_prop.  FWI_EINVAL unless 0 < beta < 1, 0 < abar < abar_prev <= 1,
 * sigma >= 0, pointers non-NULL (except score, z) and aligned. */
int fwi_ddpm_step(long n, const float* v, const float* score, const float* z, double beta, double abar,
                  double abar_prev, double sigma, float* v0hat, float* v_prop, void* stream);

/* ------------------------------------------------------------------------
 * Building blocks of the learned surrogate (BF16 storage, FP32 accumulation).
 * ------------------------------------------------------------------------ */

/* Batched GEMM on the matrix cores: for b < batch,
 *   C[b] = alpha op(A[b]) op(B[b]) + beta C[b] (+ bias[n]),
 * or with reduce_batch = 1 a single C = alpha sum_b op(A[b]) op(B[b]) + beta C.
 * A, B: BF16 bit patterns (uint16); op(A)[m][k] = transA ? A[k lda + m] : A[m lda + k],
 * op(B)[k][n] = transB ? B[n ldb + k] : B[k ldb + n]; batch b starts at A + b strideA
 * (elements), likewise B and C.  Exactly one of C32 (FP32) and C16 (BF16) is
 * non-NULL.  bias: FP32 [N] or NULL.  splitk > 1 (batch == 1 or reduce_batch
 * only) splits the reduction into splitk partial sums kept in work
 * (FP32, splitk * M * N elements, caller-owned) and added in a fixed order.
 * Accumulation is FP32; results are deterministic.  FWI_EINVAL on bad shapes. */
int fwi_nn_gemm(int M, int N, int K, int batch, const void* A, long lda, long strideA, int transA, const void* B,
                long ldb, long strideB, int transB, float* C32, void* C16, long ldc, long strideC, float alpha,
                float beta, const float* bias, int reduce_batch, int splitk, float* work, void* stream);

/* Mixing along x of the surrogate's decoder blocks, per slab s < S of
 * [72][64] BF16 (a (sample, time row) of the decoder's NHWC activations),
 * Xm [72][72] BF16, R() rounding to BF16:
 *   forward  g1[s] = R(g[s] + R(Xm g[s]))
 *   VJP      d32[s] += Xm^T d1[s] (FP32, in place),  d16[s] = R(d32[s])
 * Bitwise equal to the tiled GEMM with its residual / dual-output epilogues.
 * g and d1 16-byte aligned (else FWI_EINVAL); g1 must not overlap g, nor d16
 * d1.  Asynchronous. */
int fwi_nn_mix_forward(long S, const void* Xm, const void* g, void* g1, void* stream);
int fwi_nn_mix_vjp(long S, const void* Xm, const void* d1, float* d32, void* d16, void* stream);

/* Fused pointwise MLP of the surrogate's blocks (64 -> 128 GELU -> 64 per row,
 * the 1x1 convolutions of the encoder and decoder blocks), R rows, BF16
 * row-major operands: a, res, h, dg [R][64]; W1 [64][128]; W2 [128][64]; FP32
 * b1 [128], b2 [64], da [R][64].  With R() rounding to BF16 and
 * p = R(a W1 + b1):
 *   forward  h  = R(res + R(R(gelu(p)) W2 + b2))          (gelu: erf form)
 *   VJP      da = R((dg W2^T) gelu'(p)) W1^T              (p recomputed from a)
 * One kernel each; the 128-wide hidden activation never leaves the chip.
 * Results equal, bit for bit, those of the same block as two fwi_nn_gemm-style
 * GEMMs with the roundings above.  BF16 and FP32 arrays 16-byte aligned, else
 * FWI_EINVAL; h must not overlap a or res, nor da dg or a.  Asynchronous,
 * except that the first call on a device fills a 384 KB table of GELU values
 * and waits for it on `stream` (FWI_ESTATE if `stream` is capturing a graph
 * then; fwi_sur_create fills it too). */
int fwi_nn_mlp_forward(long R, const void* a, const void* W1, const float* b1, const void* W2, const float* b2,
                       const void* res, void* h, void* stream);
int fwi_nn_mlp_vjp(long R, const void* dg, const void* a, const void* W1, const float* b1, const void* W2, float* da,
                   void* stream);

/* ------------------------------------------------------------------------
 * Learned surrogate of the forward map (Sec. 7, future work: a cheaper stand-in for
 * the wave solver inside guidance), fixed shapes: v [B][70][70] m/s ->
 * traces [B][5][70][1000] in the layout of fwi_forward's d_syn.
 *
 * Network: lift of (v, z, x) features to 64 channels on a 72 x 72 grid;
 * 4 encoder blocks {depthwise 3x3, 64->128 GELU 128->64, residual};
 * a learned depth->time map (72 -> 256 rows); 4 decoder blocks {mixing along
 * x, depthwise 3x3, 64->128 GELU 128->64, residuals}; a 64->8 head; a learned
 * time up-sampling 256 -> 1000; traces = out_scale * (channels 0..4, columns
 * 0..69).  GEMM operands and stored activations are BF16, accumulation FP32.
 *
 * Parameters are one FP32 vector of fwi_sur_param_count() entries in the
 * order lift_w[3][64], lift_b[64], encoder blocks 0..3 {dw_k[64][3][3],
 * dw_b[64], w1[64][128], b1[128], w2[128][64], b2[64]}, d2t[256][72],
 * decoder blocks 0..3 {xm[72][72], dw_k, dw_b, w1, b1, w2, b2}, proj_w[64][8],
 * proj_b[8], up[1000][256], out_scale[1].  out_scale is not trained (its
 * gradient entry stays 0).
 *
 * The object owns its parameters, Adam state and activation buffers (about
 * 135 MB per sample of max_batch); it lives on the device current at creation
 * and is not thread-safe (one stream at a time).  Device arrays are the
 * caller's.  Calls marked asynchronous return after enqueueing on `stream`.
 * ------------------------------------------------------------------------ */
typedef struct fwi_surrogate fwi_surrogate;

typedef struct {
    float lr, beta1, beta2, eps; /* Adam */
    float loss_k;                /* trace weight 1/(1 + loss_k |target| / max_sample |target|) */
    float pair_weight;           /* > 0: B is even and samples B/2..B-1 perturb samples 0..B/2-1 (see
                                    fwi_sur_train_step) */
} fwi_sur_train_params;

/* dims[5] <- {nz, nx, ns, nr, nt} = {70, 70, 5, 70, 1000}. */
int fwi_sur_shape(int* dims);
long fwi_sur_param_count(void);
/* max_batch in [1, 128]; parameters start at zero (set them before use). */
int fwi_sur_create(int max_batch, fwi_surrogate** out);
int fwi_sur_destroy(fwi_surrogate* s);
/* Synchronous host <-> device copies of the FP32 parameter vector; set also
 * refreshes the BF16 copies and resets the Adam state. */
int fwi_sur_set_params(fwi_surrogate* s, const float* host_params);
int fwi_sur_get_params(fwi_surrogate* s, float* host_params);
/* Weight gradients of the last fwi_sur_backward(want_weight_grads = 1) or
 * training step (synchronous). */
int fwi_sur_get_grads(fwi_surrogate* s, float* host_grads);
/* Adam moments and step count (synchronous): with the parameters, the state
 * a resumed training run needs. */
int fwi_sur_get_adam(fwi_surrogate* s, float* host_m, float* host_v, int* step);
int fwi_sur_set_adam(fwi_surrogate* s, const float* host_m, const float* host_v, int step);
/* fused = 1 (the default): each block's pointwise MLP runs as one kernel
 * (fwi_nn_mlp_forward / fwi_nn_mlp_vjp) and the forward keeps no 128-wide
 * hidden activations (a backward with want_weight_grads recomputes them); an
 * input-only backward also runs each decoder block's depthwise-convolution
 * and mixing VJP as one kernel.  fused = 0: two GEMMs per MLP, hidden
 * activations kept, separate depthwise and mixing kernels.  Both give
 * identical results; the setting applies from the next forward.  FWI_EINVAL
 * unless 0 or 1. */
int fwi_sur_set_fused_mlp(fwi_surrogate* s, int fused);
/* traces = S(v) for B <= max_batch samples (asynchronous).  Keeps the
 * activations for fwi_sur_backward. */
int fwi_sur_forward(fwi_surrogate* s, int B, const float* v, float* traces, void* stream);
/* Vector-Jacobian product of the last fwi_sur_forward (same B, else
 * FWI_ESTATE): dv = (dS/dv)^T dtraces (dv may be NULL), and with
 * want_weight_grads the parameter gradient (asynchronous). */
int fwi_sur_backward(fwi_surrogate* s, int B, const float* dtraces, float* dv, int want_weight_grads, void* stream);
/* One Adam step on the weighted mean-square trace loss
 *   L = (1/(B 5 70 1000)) sum (w (S(v) - target))^2,
 *   w = 1/(1 + loss_k |target| / max over the sample of |target|),
 * plus, with pair_weight > 0 (B even, h = B/2, sample h + b a perturbation of
 * sample b), the finite-difference term that trains directional derivatives
 *   pair_weight (1/(h 5 70 1000)) sum_b (w_b ((S(v_{h+b}) - S(v_b)) - (target_{h+b} - target_b)))^2
 * with w_b the weight of sample b;
 * loss_out (device float, may be NULL) receives L before the step
 * (asynchronous). */
int fwi_sur_train_step(fwi_surrogate* s, int B, const float* v, const float* target,
                       const fwi_sur_train_params* params, float* loss_out, void* stream);

/* Judge of a stand-in gradient against the solver's (Sec. 7, future work), per
 * sample b < B over n entries: cos_out[b] = <g_a, g_b> / (|g_a| |g_b|) (0 if
 * either is zero) and, if jerr_out is non-NULL, jerr_out[b] =
 * |J_a[b] - J_b[b]| / |J_b[b]| (0 if J_b[b] = 0).  Device arrays; FP64 sums in
 * a fixed order (asynchronous). */
int fwi_judge(int B, int n, const float* g_a, const float* g_b, const double* J_a, const double* J_b,
              float* cos_out, float* jerr_out, void* stream);

/* Multi-fidelity prediction (Sec. 7, future work: multi-fidelity surrogate
 * strategies): the exact solver's value at an anchor model plus the
 * surrogate's change since that anchor,
 *   g_out = g_anchor + (s_now - s_anchor)            [B][n] FP32,
 *   J_out = J_anchor + (Js_now - Js_anchor)          [B] FP64 (all four NULL or non-NULL).
 * g_out may alias g_anchor or s_now (element-wise).  Asynchronous. */
int fwi_mf_predict(int B, int n, const float* g_anchor, const float* s_now, const float* s_anchor, float* g_out,
                   const double* J_anchor, const double* Js_now, const double* Js_anchor, double* J_out,
                   void* stream);

/* ---- score network of the reverse-diffusion loop (Algorithm 2) ----------
 *
 * A noise-prediction network eps_theta(x, t) for the 70 x 70 diffusion state
 * (the score model of Sec. 3 in the form s = -eps / sqrt(1 - abar_i),
 * trained by denoising score matching, Eq. L2_rewrite with the weight
 * 1 - abar), its vector-Jacobian product and an Adam step, on the BF16
 * matrix cores (FP32 accumulation):
 *   time embedding (FP32): e = [sin(1000 t f_k), cos(1000 t f_k)],
 *     f_k = 10000^(-k/16), k < 16; tb = W_t2^T gelu(W_t1^T e + b_t1) + b_t2
 *     (320 per-channel biases of the five blocks, in their order);
 *   lift: 32 channels on a 72 x 72 grid holding x in rows/columns 1..70 (zero
 *     ring): h = W_l^T [x, (i - 35.5)/36, (j - 35.5)/36] + b_l;
 *   block(C): p = conv3(h; W1) + b1 + tb, q = gelu(p),
 *     h' = h + conv3(q; W2) + b2 (3 x 3, zero padding; W [9 C][C], row
 *     (3 dy + dx) C + c_in holds the tap at offset (dy - 1, dx - 1));
 *   U-Net: block b0a (C 32, 72^2); 2 x 2 mean, 1 x 1 32 -> 64; b1a (64, 36^2);
 *     mean, 1 x 1 64 -> 128; b2 (128, 18^2); 1 x 1 128 -> 64, nearest x 2,
 *     + b1a output; b1b (64); 1 x 1 64 -> 32, nearest x 2, + b0a output;
 *     b0b (32); head eps = w_h . h + b_h on rows/columns 1..70;
 *   output map: out = skip_b x + scale_b eps per sample (skip, scale NULL:
 *     0 and 1).  skip = 0, scale = -1/sqrt(1 - abar) gives the score;
 *     skip = 1/sqrt(abar), scale = -sqrt(1 - abar)/sqrt(abar) gives the
 *     clean estimate v0hat of Eq. v0hat.
 * Activations and GEMM weights are BF16, FP32 elsewhere.  Parameters are one
 * FP32 vector of fwi_score_param_count() entries: temb_w1 [32][128], temb_b1,
 * temb_w2 [128][320], temb_b2, lift_w [3][32], lift_b, then per block
 * W1, b1, W2, b2 with the 1 x 1 maps between them (b0a, down0 [32][64] + b,
 * b1a, down1 [64][128] + b, b2, up1 [128][64] + b, b1b, up0 [64][32] + b,
 * b0b), head_w [32], head_b [1]. */
typedef struct fwi_score_net fwi_score_net;

typedef struct {
    float lr, beta1, beta2, eps; /* Adam */
} fwi_score_train_params;

long fwi_score_param_count(void);
/* max_batch in [1, 256]; parameters start at zero (set them before use). */
int fwi_score_create(int max_batch, fwi_score_net** net);
int fwi_score_destroy(fwi_score_net* net);
/* Synchronous host <-> device copies of the FP32 parameter vector; set also
 * refreshes the BF16 copies and resets the Adam state (moments and step). */
int fwi_score_set_params(fwi_score_net* net, const float* host_params);
int fwi_score_get_params(fwi_score_net* net, float* host_params);
/* Parameter gradient of the last fwi_score_backward(want_weight_grads = 1)
 * or training step (synchronous). */
int fwi_score_get_grads(fwi_score_net* net, float* host_grads);
/* Adam moments and step count (synchronous): with the parameters, the state
 * a resumed training run needs. */
int fwi_score_get_adam(fwi_score_net* net, float* host_m, float* host_v, int* step);
int fwi_score_set_adam(fwi_score_net* net, const float* host_m, const float* host_v, int step);
/* out = skip_b x + scale_b eps_theta(x, t_b) for B <= max_batch states
 * x [B][70][70] at conditioning times tcond [B] (t = i / N for step i of N);
 * skip, scale [B] or NULL.  Keeps the activations for fwi_score_backward
 * (asynchronous). */
int fwi_score_forward(fwi_score_net* net, int B, const float* x, const float* tcond, const float* skip,
                      const float* scale, float* out, void* stream);
/* Vector-Jacobian product of the last fwi_score_forward (same B, else
 * FWI_ESTATE): dx = (d out / d x)^T dout (dx may be NULL), and with
 * want_weight_grads the parameter gradient.  For the clean estimate this is
 * the chain rule of Eq. chain_rule, h = (d v0hat / d x_i)^T g (asynchronous). */
int fwi_score_backward(fwi_score_net* net, int B, const float* dout, float* dx, int want_weight_grads,
                       void* stream);
/* One denoising score-matching step: x_t = sqrt_abar_b x0 + sqrt_1m_abar_b noise,
 * L = mean over samples and nodes of (eps_theta(x_t, tcond_b) - noise)^2, its
 * parameter gradient and one Adam update.  x0, noise [B][70][70]; tcond,
 * sqrt_abar, sqrt_1m_abar [B]; loss_out (device float, may be NULL) receives
 * L before the update (asynchronous). */
int fwi_score_train_step(fwi_score_net* net, int B, const float* x0, const float* noise, const float* tcond,
                         const float* sqrt_abar, const float* sqrt_1m_abar, const fwi_score_train_params* params,
                         float* loss_out, void* stream);

/* Mean device time, in ms, of the forward sweeps (the nt - 1 time steps of
 * fwi_forward, without the velocity preparation) and of the adjoint sweeps
 * (of fwi_adjoint_gradient, without the gradient fold) enqueued since the
 * previous call (at most the last 256 of each), from the HIP events of a plan
 * created with options.timing = 1; then starts counting afresh.  Waits for
 * those events.  Either pointer may be NULL.  FWI_ESTATE if timing is off or
 * a requested kind of sweep has not run since the previous call. */
int fwi_plan_sweep_ms(fwi_plan* plan, float* forward_ms, float* adjoint_ms);

/* ------------------------------------------------------------------------
 * Uneven batches: requests with their own grids, trace lengths and shots
 * (the same scheme as fwi_forward, Sec. 2.1 and Sec. 6.1), swept by one
 * persistent launch.  Every (request, shot) field is one work unit run to
 * completion by one workgroup; units are queued longest first.  Fields whose
 * padded grid fits the LDS (and whose receivers share a row) run LDS-resident;
 * larger ones are swept from HBM tile by tile.  The tile of each size class is
 * chosen at creation by timing the compiled candidates (autotune = 1; results
 * are kept for the process) or by a cost model (autotune = 0).
 *
 * Packed layouts (offsets from fwi_batch_get_info, in elements):
 *   v, grad  request r: [nz_r][nx_r] at v_offset
 *   wavelets request r: [nt_r] at wavelet_offset (one wavelet for its shots)
 *   traces   request r: [ns_r][nr_r][nt_r] at trace_offset
 * ------------------------------------------------------------------------ */
typedef struct fwi_batch fwi_batch;

typedef struct {
    int autotune;   /* 1: time the candidate tiles per size class at creation; 0: cost model */
    int gradients;  /* 1: also allocate what fwi_batch_gradient needs (per field: the full history of D for
                       LDS-resident fields and row bands; checkpoints every ceil(sqrt(2 (nt - 1))) steps, one
                       segment of D and the adjoint state for HBM-swept ones) */
    int bands;      /* 0: fields too large for one workgroup's LDS whose receivers share a row run as
                       LDS-resident row bands (in a gradient batch only when the full history of D of those
                       fields takes at most 60 % of the device memory free at creation); -1: never, they are
                       swept from HBM */
} fwi_batch_options;

typedef struct {
    size_t v_offset, wavelet_offset, trace_offset;
    int nzp, nxp;           /* padded grid */
    int kind;               /* 0: LDS-resident, 1: swept from HBM, 2: LDS-resident row bands on several
                               workgroups (fields too large for one workgroup's LDS whose receivers share a
                               row; see fwi_batch_options.bands) */
    int tile_x, tile_z;     /* kinds 0 and 2: register tile (columns, rows); kind 1: sweep tile */
    int tuned;              /* 1 if the tile was picked by timing (kind 2: by the cost model, 0) */
    int parts;              /* workgroups per field: kind 1 row parts swept in lockstep, kind 2 row bands
                               exchanging halos (1: one workgroup per field) */
} fwi_batch_request_info;

/* Validates every geometry (FWI_EINVAL / FWI_ECFL as fwi_plan_create), builds
 * the tables and the unit queue, allocates per-unit state (about 12 bytes per
 * padded point for each HBM-swept field) and runs the autotuner on the
 * current device (synchronous). */
int fwi_batch_create(int nreq, const fwi_geometry* geoms, const fwi_batch_options* options, fwi_batch** batch);
int fwi_batch_destroy(fwi_batch* batch);
int fwi_batch_get_info(const fwi_batch* batch, int request, fwi_batch_request_info* info);
/* Total elements of the packed v, wavelet and trace buffers (any may be NULL). */
int fwi_batch_sizes(const fwi_batch* batch, size_t* v_elems, size_t* wavelet_elems, size_t* trace_elems);
/* Forward modelling of every request (traces as fwi_forward's d_syn, sample 0
 * = 0) in one persistent launch after one coefficient launch (asynchronous).
 * Velocities outside (0, v_max_r] raise the flag read by fwi_batch_status. */
int fwi_batch_forward(fwi_batch* batch, const float* v, const float* wavelets, float* traces, void* stream);
/* dJ/dv of every request for given adjoint sources a = dJ/dd (packed like the
 * traces), as fwi_adjoint_gradient computes it for one plan (the transpose of
 * the linearised forward map, Sec. 4, summed over shots and folded onto the
 * model): grad packed like v.  Each field runs its forward sweep and its
 * adjoint sweep in the same persistent launch (HBM-swept fields recompute
 * each checkpoint segment; row bands run both sweeps band by band, exchanging
 * halos in each), then one launch folds the imaging sums.
 * FWI_ESTATE unless the batch was created with options.gradients = 1.
 * Asynchronous. */
int fwi_batch_gradient(fwi_batch* batch, const float* v, const float* wavelets, const float* adj, float* grad,
                       void* stream);
/* Synchronises; FWI_OK or FWI_EDEVICE (and clears the flag). */
int fwi_batch_status(fwi_batch* batch);

/* Plain device-to-device copy of `bytes` bytes by one kernel (16-byte vector
 * loads and stores when both pointers are 16-byte aligned), asynchronous on
 * `stream`.  The buffers must not overlap.  It reads and writes exactly
 * `bytes` bytes each, which makes it the reference kernel for calibrating
 * hardware traffic counters. */
int fwi_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Synchronises the plan's device and returns FWI_OK, or the first recorded
 * device-side error (FWI_EDEVICE for an invalid velocity) and clears it. */
int fwi_status(fwi_plan* plan);

/* Static description of a status code. */
const char* fwi_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* FWI_H */
