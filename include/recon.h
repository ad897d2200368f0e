/*
 * recon.h -- C ABI of the MI355X (gfx950) nonlinear-reconstruction library.
 *
 * Method: Zhu, Yu, Pen, Chen & Yu, "Nonlinear reconstruction",
 * arXiv:1611.09638.  Given a nonlinear density field on a periodic grid, find
 * the displacement potential phi whose curvilinear mesh x = xi + grad phi
 * (Sec. II, Eq. mapping) carries constant mass per cell with a positive-
 * definite map det(dx/dxi) > 0 (Sec. II), built from small increments
 * phi = sum dphi_i (Sec. II; App. A), each solving the linear elliptic
 * equation div(rho sqrt g grad phidot) = S(Sigma + C + E) with x ~ xi
 * (App. A, Eq. elliptic) by multigrid; return phi and the reconstructed
 * density delta_r = -laplacian phi (Sec. II, Eq. rec).
 *
 * Conventions for every entry point:
 *   - Arrays are C-order [n][n][n] (last index fastest), periodic, FP64 unless
 *     the name says f32.  Array pointers are DEVICE pointers on the device
 *     that was current at recon_init; the stats/config structs and scalar
 *     out-parameters are HOST pointers.
 *   - The caller owns every array and the workspace; the library allocates no
 *     device memory (it keeps one small pinned host buffer per context).
 *   - All device work is enqueued on the stream given to recon_init.  Calls
 *     that take host decisions (solve, backward, the stage calls returning
 *     scalars) synchronise that stream before returning.
 *   - A context is not thread-safe; use one per thread/stream.
 *   - Return value: RECON_OK (0) or a negative RECON_E_* code.  On error the
 *     outputs are unspecified and recon_last_error(ctx) describes the cause.
 *     Nothing is thrown across the ABI.
 */
#ifndef RECON_H
#define RECON_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RECON_OK 0
#define RECON_E_ARG (-1)            /* null pointer, bad size, bad config */
#define RECON_E_INPUT (-2)          /* density negative, NaN/Inf, or zero total mass */
#define RECON_E_NOT_PD (-3)         /* no step 2^-j (j <= max_halvings) keeps the map positive definite */
#define RECON_E_NO_CONVERGENCE (-4) /* linear solve exceeded max_vcycles or produced NaN */
#define RECON_E_NO_TAPE (-5)        /* backward without a forward that recorded its tape */
#define RECON_E_HIP (-6)            /* a HIP runtime call or kernel launch failed */
#define RECON_E_WORKSPACE (-7)      /* workspace null, too small or misaligned */
#define RECON_E_SCRATCH (-8)        /* recon_solve_noalloc: the problem needs more than the static scratch */

#define RECON_FP64 0  /* every kernel in FP64 */
#define RECON_MIXED 1 /* V-cycle (smoother, residual, transfers, coarse solve) in FP32 inside the FP64 loop */

#define RECON_SOLVER_PCG 0    /* conjugate gradients preconditioned by one symmetric V-cycle */
#define RECON_SOLVER_VCYCLE 1 /* plain V-cycle iteration u += V(b - A u) */

#define RECON_MAX_STEPS 64

/* Solver knobs.  xi_m = 1/10 and v_m = 10 are the paper's limiter constants
 * (App. A, App. B); the other values are this library's readings of what the
 * paper leaves to its references (multigrid design, smoothing, step control). */
typedef struct recon_config {
    int max_outer;      /* outer moving-mesh steps (10)                                   */
    int n_pre, n_post;  /* RB Gauss-Seidel sweeps before/after the coarse correction (2, 2) */
    int coarse_n;       /* coarsest grid edge, even, 2..16 (8)                             */
    int coarse_sweeps;  /* symmetric red/black sweep pairs on the coarsest grid (64)       */
    int max_vcycles;    /* V-cycles per linear solve before RECON_E_NO_CONVERGENCE (100)   */
    int max_halvings;   /* step trials alpha = 2^-j, j = 0..max_halvings (30)              */
    int precision;      /* RECON_FP64 or RECON_MIXED                                       */
    int solver;         /* RECON_SOLVER_PCG or RECON_SOLVER_VCYCLE                         */
    int warm_start;     /* 1: start each outer step's solve from the previous solution when its
                           residual is below ||b|| (else from 0) (1)                       */
    int mass_update;    /* 0: the mass per curvilinear cell M is gathered by CIC on the deformed
                           mesh every step; 1: it is gathered once and then carried by the
                           paper's update M' = M + alpha div(M e^-1 grad dphi) (App. A, Eq.
                           elliptic_diff), and steps must also keep M' > 0.  No reverse mode:
                           record_tape must be 0 (0)                                        */
    int particle_deposit; /* particle input only (recon_solve_particles): 1 deposits the particles
                           by CIC at their Lagrangian positions on the deformed mesh every step
                           (xi_p with xi_p + grad phi(xi_p) = y_p, by Newton from the previous
                           step's); 0 assigns them to the grid once.  Needs up to n^3
                           particles and mass_update = 0; 6 more FP64 fields of workspace
                           (positions and node shifts); reverse mode through
                           recon_backward_particles (0)                                     */
    int full_operator;  /* 1: the linear system of each step is the exact Jacobian of the mass
                           map, div(M e^-1 grad u) = b on the current mesh (App. A, Eq.
                           elliptic_diff, without x ~ xi; diagonal face coefficients floored at
                           a_min as in the x ~ xi operator), solved by the same Krylov loop with
                           an x ~ xi V-cycle as its preconditioner, whose coefficient is the
                           mean diagonal (K^xx + K^yy + K^zz) / 3 of K = M e^-1; 7 more FP64
                           fields of workspace.  No reverse mode: record_tape must be 0 (0) */
    int fixed_cycles;   /* > 0: every linear solve runs exactly this many V-cycles, ignoring tol
                           (makes the forward a smooth map for finite differences) (0)      */
    int record_tape;    /* 1: keep every (u_i, alpha_i) so recon_backward can run          */
    int tape_fp32;      /* 1: store the tape's u_i in FP32 (half the tape memory; the
                           backward then linearises about phi rebuilt from the rounded u_i) */
    int profile;        /* 1: time every fine-level smoother sweep with hipEvents (stats)  */
    double tol;         /* linear-solve stop: ||b - A u||_2 <= tol ||b||_2 (1e-10)          */
    double outer_tol;   /* outer stop when rms(Sigma) <= outer_tol (0: run max_outer)       */
    double xi_m;        /* maximal compression factor of the compression limiter (0.1)      */
    double v_m;         /* expansion volume limit of the expansion limiter (10)             */
    double smooth_center; /* S f = c0 f + (1 - c0)/6 * sum of 6 neighbours (c0 = 0.5)       */
    double s_max;       /* largest per-step shift of any node, in cells (1.0)              */
    double a_min;       /* floor of the face coefficient of the elliptic operator (1e-3)  */
} recon_config;

/* Per-solve diagnostics (host struct).  Entries [0, outer_steps) describe the
 * steps taken; rms_sigma/kappa have one more entry, the state after the last. */
typedef struct recon_stats {
    int outer_steps;
    int vcycles_total;
    int vcycles[RECON_MAX_STEPS];       /* V-cycles (preconditioner applications) per step */
    double alpha[RECON_MAX_STEPS];      /* accepted step 2^-j */
    double rms_sigma[RECON_MAX_STEPS + 1]; /* rms of Sigma = mean(M) - M before each step */
    double kappa[RECON_MAX_STEPS + 1];  /* mean of M (mass on the deformed mesh / input mass) */
    double rel_residual[RECON_MAX_STEPS]; /* final ||b - A u|| / ||b|| of each linear solve */
    double min_det;                     /* min over nodes of det(I + Hess phi) at the end */
    double min_lambda0;                 /* min over nodes of the smallest eigenvalue of I + Hess phi */
    double max_delta_r;                 /* max of delta_r (< 3 for a positive-definite map) */
    double ms_total;                    /* wall time of the solve on the stream (hipEvents) */
    int smoother_sweeps;                /* fine-level RB-GS sweeps timed (cfg.profile) that read
                                           u, a and b and write u (the plain sweeps) */
    double smoother_ms;                 /* their summed kernel time on the stream */
    int smoother_zero_sweeps;           /* timed fine-level sweeps that start a V-cycle from u = 0
                                           (read a and b, write u) */
    double smoother_zero_ms;            /* their summed kernel time */
    int alpha_limit[RECON_MAX_STEPS];   /* what set each step: 0 the full step alpha = 1 was taken;
                                           1 the shift bound s_max (the largest step it allows passed);
                                           2 the positive-definiteness (or mass positivity) test, which
                                           rejected at least one step the shift bound allows */
    int smoother_folded_sweeps;         /* timed fine-level sweeps with the V-cycle's coarse correction
                                           folded in (read u, a, b and the coarse e, write u) */
    double smoother_folded_ms;          /* their summed kernel time */
} recon_stats;

typedef struct recon_ctx recon_ctx;

/* Fill *cfg with the defaults listed above.  Returns RECON_E_ARG if cfg is NULL. */
int recon_config_default(recon_config *cfg);

/* Bytes of device workspace recon_init needs for an n^3 grid under cfg (host
 * call, no device work).  Returns 0 if n/cfg are invalid, n above 1024
 * included. */
size_t recon_workspace_bytes(int n, const recon_config *cfg);

/* Create a context for n^3 grids.  workspace: device buffer of at least
 * recon_workspace_bytes(n, cfg) bytes, 256-byte aligned, owned by the caller
 * and untouched by anyone else while the context lives.  hip_stream: a
 * hipStream_t (NULL = default stream).  n must equal coarse_n * 2^k and be at
 * most 1024 (the largest such grid whose workspace fits one 288 GB device);
 * anything else returns RECON_E_ARG. */
int recon_init(recon_ctx **ctx, int n, const recon_config *cfg, void *workspace, size_t ws_bytes,
               void *hip_stream);

/* Forward reconstruction (Sec. II, App. A).  density: n^3 values >= 0 with a
 * positive total (any normalisation: it is divided by its mean).  box: box
 * edge in length units (finite and > 0); phi_out is returned in length^2
 * (grid-unit phi times (box/n)^2), delta_r_out = -laplacian phi
 * (dimensionless; Eq. rec).  tol (finite, >= 0): > 0 overrides cfg->tol for
 * this call; 0 keeps it.  Other box or tol values give RECON_E_ARG.  Either output may be NULL; the two must
 * not overlap (RECON_E_ARG), and either may be the density array, which is
 * read before they are written.  stats may be NULL.  Records the tape when
 * cfg->record_tape is set. */
int recon_solve(recon_ctx *ctx, const double *density, int n, double box, double tol, double *phi_out,
                double *delta_r_out, recon_stats *stats);

/* Same, from particles: pos = np x (x, y, z) float32 positions in [0, box),
 * x along the first array index.  They are cloud-in-cell assigned to the
 * n^3 vertex-centred grid (node j at position j*box/n) before the solve.
 * recon_backward then returns the gradient with respect to that grid. */
int recon_solve_particles(recon_ctx *ctx, const float *pos, long long np, double box, double tol,
                          double *phi_out, double *delta_r_out, recon_stats *stats);

/* Reverse-mode gradient of the last recorded forward: given dL/d delta_r and
 * (optionally, NULL = 0) dL/d phi_out, write dL/d density (n^3) for the
 * density passed to recon_solve.  Discrete decisions of the forward (step
 * sizes, limiter branches) are held fixed; each linear solve is
 * differentiated as exact.  Returns RECON_E_NO_TAPE without a recorded tape. */
int recon_backward(recon_ctx *ctx, const double *grad_delta_r, const double *grad_phi, double *grad_density);

/* Reverse mode of a recorded recon_solve_particles with particle_deposit = 1:
 * dL/d pos (grad_pos: np x 3 FP64 device array, in the units of pos) given
 * dL/d delta_r and (optionally) dL/d phi_out.  pos and np must be the
 * particles of the recorded forward (device, float32, unchanged; grad_pos
 * must not overlap them, RECON_E_ARG).  Each
 * step's Lagrangian positions are recomputed by Newton from the later step's
 * (reverse order); the gradient runs through the inversion of the map
 * (J^-T per particle) and the xi-space CIC, with the step sizes and limiter
 * branches of the forward held fixed.  RECON_E_NO_TAPE without a tape,
 * RECON_E_ARG for a density tape or other particles. */
int recon_backward_particles(recon_ctx *ctx, const float *pos, long long np, const double *grad_delta_r,
                             const double *grad_phi, double *grad_pos);

/* For callers that cannot allocate device or pinned host memory (tight
 * serving loops, harnesses that forbid hipMalloc): recon_solve without a
 * context or a workspace.  Same arguments and results as recon_solve on a
 * context made by recon_init(n, cfg) (the same kernels; bitwise-identical
 * phi, delta_r and stats apart from ms_total), with hip_stream (a
 * hipStream_t, NULL = default stream) on the current device.
 *
 * Scratch: a static device array of RECON_NOALLOC_SCRATCH_BYTES (64 MiB) in
 * the library, one copy per device, held from the library's first use on that
 * device until the process ends; its device address is looked up on the first
 * call on each device.  The call makes no hipMalloc, hipFree, hipHostMalloc or
 * other allocating call, creates no events, and keeps its host-side state in
 * static memory.  Problems whose workspace (recon_workspace_bytes(n, cfg))
 * exceeds the scratch return RECON_E_SCRATCH: every mode fits for n <= 64
 * (coarse_n = 8).  cfg->record_tape, cfg->particle_deposit and cfg->profile
 * must be 0 (RECON_E_ARG): there is no reverse mode, no particle input and no
 * sweep timing here.  The scratch keeps the last call's contents; nothing the
 * solve reads is taken from it before being written.  Calls on one device
 * share its scratch: the library serialises them on the host and each returns
 * only after its device work has finished, so they never overlap on the
 * device.  Work the caller enqueues on other streams must not touch the
 * scratch (it cannot name it).  Error text: recon_strerror(code). */
#define RECON_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int recon_solve_noalloc(const double *density, int n, double box, double tol, const recon_config *cfg,
                        double *phi_out, double *delta_r_out, recon_stats *stats, void *hip_stream);

/* Release the context (not the workspace, which the caller owns). */
void recon_destroy(recon_ctx *ctx);

/* Static text for an error code. */
const char *recon_strerror(int code);

/* Text of the last error on this context ("" if none). */
const char *recon_last_error(const recon_ctx *ctx);

/* ------------------------------------------------------------------------
 * Stage entry points: one step of the path on caller-provided device arrays,
 * on the context's stream, using its workspace for reductions and multigrid
 * levels.  The grid edge is the context's n unless stated.  dtype: 0 = FP64
 * arrays, 1 = FP32 arrays.  They exist so each kernel can be checked and
 * timed on its own.  An output array must not overlap an input array or
 * another output (RECON_E_ARG), except where a function updates an array in
 * place (u of recon_stage_rbgs, recon_stage_prolong_add and
 * recon_stage_prolong_sweep, xi of recon_stage_invert_map); normalize and
 * source may also write over their inputs.  Caller arrays must not lie in
 * the context's workspace.
 * ------------------------------------------------------------------------ */

/* m = rho / mean(rho) after checking rho (App. A input; Sec. III gridding). */
int recon_stage_normalize(recon_ctx *ctx, const double *rho, double *m);

/* Cloud-in-cell assignment of np particles onto the n^3 grid (particle count per node). */
int recon_stage_cic(recon_ctx *ctx, const float *pos, long long np, double box, double *rho);

/* The next three run on the context's n^3 grid.  variant 0: the kernels the
 * solver uses at that size; 1: per-node gathers; 2: the stencil field streamed
 * through LDS (n a multiple of 64, else RECON_E_ARG).  All variants give the
 * same node values; sums (mean M, rms(Sigma)) may differ in rounding. */

/* Mass per curvilinear cell M = det(I + Hess phi) * CIC(m)(xi + D_c phi)
 * (rho sqrt g of App. A on the current mesh); phi in grid units. */
int recon_stage_meshmass(recon_ctx *ctx, const double *phi, const double *m, double *M, int variant);

/* b = S(Sigma + C + E) - mean, Sigma = mean(M) - M, with the compression and
 * expansion limiters of App. A (Eq. elliptic).  *rms_sigma (host) <- rms(Sigma). */
int recon_stage_source(recon_ctx *ctx, const double *phi, const double *M, double *b, double *rms_sigma,
                       int variant);

/* out = S f, the nearest-neighbour smoothing of App. A. */
int recon_stage_smooth(recon_ctx *ctx, const double *f, double *out, int variant);

/* out = A u with A = div(a grad .) in flux form on an nl^3 level (scale 4^-l). */
int recon_stage_apply(recon_ctx *ctx, const double *u, const double *a, int nl, double scale, double *out);

/* r = b - A u on an nl^3 level.  variant 0: the kernel the solver uses on
 * that level; 1: per-node gathers; 2: the LDS-streaming kernel (nl a
 * multiple of 128, else RECON_E_ARG). */
int recon_stage_residual(recon_ctx *ctx, const void *u, const void *a, const void *b, int nl, double scale,
                         void *r, int dtype, int variant);

/* One conjugate-gradient direction on the fine level (the Krylov loop around
 * the V-cycle preconditioner): p_new = z (first != 0) or z + beta p_old,
 * q = A p_new, and *pq (host) <- p_new . q.  z is FP64 (z_dtype 0) or FP32
 * (z_dtype 1); a and q are FP64; p_old and p_new are FP64 (p_dtype 0) or FP32
 * (p_dtype 1: needs z_dtype 1 and the streaming kernel; p_new is rounded to
 * FP32 as it is formed and q is the product of the rounded values).  p_new
 * must differ from p_old (p_old is not read, and may be NULL, when
 * first != 0).  If u (FP64, device) is not NULL, the previous step's solution
 * update u += alpha_u p_old is applied in the same pass (first must be 0; u
 * distinct from every other array).  variant as for recon_stage_residual
 * (1: in-place update then gathers; 2: one fused streaming pass). */
int recon_stage_direction(recon_ctx *ctx, const void *z, int z_dtype, const void *p_old, const double *a,
                          double beta, int first, void *p_new, double *q, double *pq, int variant, double *u,
                          double alpha_u, int p_dtype);

/* One red-black Gauss-Seidel sweep in place (colour `first` then the other;
 * red = i+j+k even) on an nl^3 level.  variant 0: the kernel the solver uses
 * on that level; 1: two per-colour launches; 2: the fused two-colour kernel
 * (nl a multiple of 16, else RECON_E_ARG).  All variants give the same
 * values. */
int recon_stage_rbgs(recon_ctx *ctx, void *u, const void *a, const void *b, int nl, double scale, int first,
                     int dtype, int variant);

/* 27-point full weighting of an nl^3 field onto (nl/2)^3.  variant 0: the
 * kernel the solver uses on that level; 1: per-node gathers; 2: the
 * LDS-streaming kernel (nl a multiple of 256, else RECON_E_ARG). */
int recon_stage_restrict(recon_ctx *ctx, const void *f, int nl, void *c, int dtype, int variant);

/* The V-cycle's coarse right-hand side c = R (b - scale A u) on an nl^3 level
 * (App. A: residual, then 27-point full weighting), c of size (nl/2)^3, all
 * arrays FP64 (dtype 0) or FP32 (dtype 1) on the device.  variant 0: what the
 * solver does on that level; 1: the residual kernel, then the restriction
 * kernel (through a library-owned fine buffer); 2: one fused streaming pass
 * (nl/2 a multiple of 32, else RECON_E_ARG).  All variants give the same
 * values. */
int recon_stage_residual_restrict(recon_ctx *ctx, const void *u, const void *a, const void *b, int nl, double scale,
                                  void *c, int dtype, int variant);

/* u += trilinear prolongation of the (nl/2)^3 field e onto the nl^3 field u
 * (P = 8 R^T).  variant as for recon_stage_restrict. */
int recon_stage_prolong_add(recon_ctx *ctx, void *u, const void *e, int nl, int dtype, int variant);

/* A V-cycle's coarse correction followed by its first post-smoothing sweep
 * (App. A multigrid): u <- one fused red-black sweep (colour `first` first)
 * of u + P e, with P the trilinear prolongation of e (edge nl/2) and the
 * operator of coefficient a at level scale `scale`, rhs b.  variant 1: the
 * prolongation's own pass, then the sweep; 2: the correction added as the
 * sweep reads each plane (what the V-cycle runs).  Both give the same values.
 * nl a level edge that the fused sweep takes (a multiple of 16), else
 * RECON_E_ARG.  Uses the context's scratch field t. */
int recon_stage_prolong_sweep(recon_ctx *ctx, void *u, const void *e, const void *a, const void *b, int nl,
                              double scale, int first, int dtype, int variant);

/* z = one symmetric V-cycle applied to r for coefficient a (fine level n). */
int recon_stage_vcycle(recon_ctx *ctx, const void *a, const void *r, void *z, int dtype);

/* Solve A(a) u = b (b mean-free) with cfg's solver and precision; u is
 * returned mean-free.  *cycles and *rel_residual are host outputs. */
int recon_stage_mg_solve(recon_ctx *ctx, const double *a, const double *b, double tol, double *u, int *cycles,
                         double *rel_residual);

/* The Krylov residual of the exact-Jacobian mode: K = M e^-1 from phi (into
 * the context's K fields), r = b - div(K grad u) in the flux form of
 * recon_stage_mass_change with the diagonal face coefficients floored at the
 * config's a_min, r32 (FP32, may be NULL) a copy of r, *rr (host)
 * <- r.r.  All FP64 n^3 device fields except r32; r distinct from u and b.
 * variant 1: per-node gathers; 2: one streaming pass (edges that are
 * multiples of 64); 0: the solve's choice.  Needs full_operator = 1. */
int recon_stage_full_residual(recon_ctx *ctx, const double *phi, const double *M, const double *u, const double *b,
                              double *r, float *r32, double *rr, int variant);

/* One Krylov direction of the exact-Jacobian mode: K = M e^-1 from phi, then
 * as recon_stage_direction with the operator div(K grad .) (diagonal face
 * coefficients floored at a_min) in place of A:
 * p_new = z or z + beta p_old, q = div(K grad p_new), *pq <- p_new.q, and
 * u += alpha_u p_old when u is not NULL; same dtypes, aliasing rules and
 * variants (2: one streaming pass, edges that are multiples of 64).  Needs
 * full_operator = 1. */
int recon_stage_full_direction(recon_ctx *ctx, const double *phi, const double *M, const void *z, int z_dtype,
                               const void *p_old, double beta, int first, void *p_new, double *q, double *pq,
                               int variant, double *u, double alpha_u, int p_dtype);

/* The linear solve of the exact-Jacobian mode: div(K grad u) = b with
 * K = a e^-1, e = I + Hess phi (App. A, Eq. elliptic_diff without x ~ xi), in
 * the flux form of recon_stage_mass_change with the diagonal face
 * coefficients floored at a_min, by the context's Krylov loop preconditioned
 * by its x ~ xi V-cycle of the mean diagonal of K.  a, phi, b, u: n^3 FP64
 * device fields of the context's edge (b mean-free, a > 0, phi with e
 * positive definite); u receives the mean-free solution.  Needs a context
 * made with full_operator = 1; RECON_E_NO_CONVERGENCE as recon_stage_mg_solve. */
int recon_stage_mg_solve_full(recon_ctx *ctx, const double *a, const double *phi, const double *b, double tol,
                              double *u, int *cycles, double *rel_residual);

/* First alpha = 2^-j keeping I + Hess(phi + alpha dphi) positive definite
 * everywhere with max |alpha D_c dphi| <= s_max (host output); returns
 * RECON_E_NOT_PD if none of j = 0..max_halvings does. */
int recon_stage_choose_step(recon_ctx *ctx, const double *phi, const double *dphi, double *alpha);

/* Step trials of the map's positivity (Sec. II, App. A): counts[t] = number
 * of nodes where I + Hess(phi + 2^-(j0+t) dphi) fails Sylvester's criterion,
 * t = 0..ntrial-1, ntrial 1 or 4, 0 <= j0 <= 1000.  phi, dphi: device n^3
 * FP64; counts: host, ntrial doubles.  variant 1 gathers the 19-point
 * neighbourhood per node, 2 streams planes through LDS (n a multiple of 64,
 * else RECON_E_ARG), 0 picks what recon_stage_choose_step uses; all variants
 * give the same counts.  M and D (device n^3 FP64, both or neither): the mass
 * update's test, a node also counts where M + 2^-(j0+t) D > 0 fails. */
int recon_stage_pd_count(recon_ctx *ctx, const double *phi, const double *dphi, int j0, int ntrial, int variant,
                         double *counts, const double *M, const double *D);

/* The exact change of the mass per curvilinear cell per unit step (App. A, Eq.
 * elliptic_diff applied to f): out = div(M e^-1 grad f) with e = I + Hess phi,
 * in flux form (it sums to zero).  phi, M, f, out: device n^3 FP64; out must
 * not alias the inputs.  Uses library-owned scratch fields of the context. */
int recon_stage_mass_change(recon_ctx *ctx, const double *phi, const double *M, const double *f, double *out);

/* Lagrangian positions of particles on the deformed mesh of phi (Sec. II):
 * xi (device, 3 np FP64, in/out: the start of Newton's method on entry, the
 * solution in grid units [0, n) on exit) with x(xi) = y, y = pos n / box
 * (pos: device float32 np x 3 in [0, box)), where x = xi + trilinear
 * interpolant of the node shifts D_c phi.  *failed (host) = particles not
 * located to 1e-12 cells.  The node shifts go into the context's workspace:
 * its particle-deposit buffer, else three fine fields that lie back to back
 * (RECON_E_ARG when they do not, for edges whose FP64 field is not a
 * multiple of 256 bytes and contexts without particle_deposit). */
int recon_stage_invert_map(recon_ctx *ctx, const double *phi, const float *pos, long long np, double box, double *xi,
                           double *failed);

/* M (device n^3 FP64) = CIC deposit of np particles at Lagrangian positions
 * xi (device 3 np FP64, grid units), n^3 / np each; coordinates that are not
 * finite or beyond 1e9 cells are skipped. */
int recon_stage_deposit_xi(recon_ctx *ctx, const double *xi, long long np, double *M);

/* delta = -laplacian phi (7-point, Eq. rec). */
int recon_stage_delta_r(recon_ctx *ctx, const double *phi, double *delta);

#ifdef __cplusplus
}
#endif

#endif /* RECON_H */
