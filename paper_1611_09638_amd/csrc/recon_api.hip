// Host driver and C ABI of the reconstruction library (include/recon.h).
//
// Outer moving-mesh iteration (Sec. II; App. A):
//   m = rho / mean(rho); phi = 0
//   repeat max_outer times:
//     M   = det(I + Hess phi) * CIC(m)(xi + D_c phi)         rho sqrt g on the mesh
//     t   = Sigma + C + E, Sigma = mean(M) - M                Eq. (elliptic) source
//     b   = S t - mean                                        smoothed, mean-free
//     u   = A(M)^-1 b, A = div(M grad .) with x ~ xi          multigrid (App. A)
//     dphi = S u; alpha = first 2^-j keeping I + Hess phi PD  step limiting
//     phi += alpha dphi
//   delta_r = -laplacian phi                                  Eq. (rec)
// Every step runs in the kernels of recon_kernels.hip on the context stream;
// the host only takes the scalar decisions (step size, convergence).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/recon.h"
#include "kernels.h"

using namespace recon;

// Static scratch of recon_solve_noalloc, one copy per device.  In host code
// this name is only a handle for hipGetSymbolAddress: its device address is
// looked up once per device and used everywhere instead.
static __device__ __align__(256) char scratch[RECON_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxLevels = 16;
constexpr int kScal = 64;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <typename T>
struct Levels {
    int L = 0;
    int n[kMaxLevels];
    T *a[kMaxLevels];    // coefficient (level 0: M or its FP32 copy)
    T *u[kMaxLevels];    // V-cycle iterate (level 0: z)
    T *b[kMaxLevels];    // right-hand side (level 0: the caller's residual)
    T *res[kMaxLevels];  // residual inside the cycle
    T *tmp[kMaxLevels];  // second buffer for out-of-place sweeps
};

// Byte layout of the caller's workspace.  Computed identically by
// recon_workspace_bytes and recon_init.
struct Layout {
    size_t total = 0;
    size_t part, scal;
    size_t m, phi, M, t, b, u, r, z, p, q, dphi;
    size_t lv64_a[kMaxLevels], lv64_u[kMaxLevels], lv64_b[kMaxLevels], lv64_res[kMaxLevels], lv64_tmp[kMaxLevels];
    size_t lv32_a[kMaxLevels], lv32_u[kMaxLevels], lv32_b[kMaxLevels], lv32_res[kMaxLevels], lv32_tmp[kMaxLevels];
    size_t tape;
    size_t adj[8];
    size_t xi;  // particle deposit: Lagrangian positions, 3 per particle (up to n^3 particles)
    size_t shifts;  // particle deposit: node shifts D_c phi, 3 per node
    size_t K;   // exact-Jacobian solve: K = M e^-1, 6 fields, and its mean diagonal
    int levels = 0;
};

int num_levels(int n, int coarse_n)
{
    if (n <= 0 || coarse_n < 2 || coarse_n > 16 || (coarse_n & 1)) return -1;
    int L = 1;
    while (n > coarse_n) {
        if (n & 1) return -1;
        n /= 2;
        ++L;
    }
    return (n == coarse_n && L <= kMaxLevels) ? L : -1;
}

bool config_ok(const recon_config *c)
{
    return c && c->max_outer >= 0 && c->max_outer <= RECON_MAX_STEPS && c->n_pre >= 0 && c->n_post >= 0 &&
           c->n_pre <= 16 && c->n_post <= 16 && c->coarse_sweeps >= 0 && c->max_vcycles >= 1 &&
           c->max_halvings >= 0 && c->max_halvings <= 60 && c->fixed_cycles >= 0 && (c->warm_start == 0 || c->warm_start == 1) &&
           (c->mass_update == 0 || c->mass_update == 1) && !(c->mass_update && c->record_tape) &&
           (c->particle_deposit == 0 || c->particle_deposit == 1) &&
           !(c->particle_deposit && c->mass_update) &&
           (c->full_operator == 0 || c->full_operator == 1) && !(c->full_operator && c->record_tape) &&
           (c->tape_fp32 == 0 || c->tape_fp32 == 1) && (c->precision == RECON_FP64 || c->precision == RECON_MIXED) &&
           (c->solver == RECON_SOLVER_PCG || c->solver == RECON_SOLVER_VCYCLE) && c->tol > 0 && c->outer_tol >= 0 &&
           c->xi_m >= 0 && c->v_m > 0 && c->smooth_center >= 0 && c->smooth_center <= 1 && c->s_max > 0 &&
           c->a_min > 0 && std::isfinite(c->tol) && std::isfinite(c->a_min);
}

bool make_layout(int n, const recon_config *cfg, Layout &Lo)
{
    if (!config_ok(cfg) || n > 1024) return false;
    int L = num_levels(n, cfg->coarse_n);
    if (L < 1) return false;
    Lo.levels = L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    const size_t n3 = (size_t)n * n * n;
    const size_t f64 = n3 * 8;
    Lo.part = take(sizeof(double) * kPartCap);
    Lo.scal = take(sizeof(double) * kScal);
    Lo.m = take(f64);
    Lo.phi = take(f64);
    Lo.M = take(f64);
    Lo.t = take(f64);
    Lo.b = take(f64);
    Lo.u = take(f64);
    Lo.r = take(f64);
    Lo.z = take(f64);
    Lo.p = take(f64);
    Lo.q = take(f64);
    Lo.dphi = take(f64);
    int nl = n;
    for (int l = 0; l < L; ++l, nl /= 2) {
        const size_t c3 = (size_t)nl * nl * nl;
        Lo.lv64_a[l] = l ? take(c3 * 8) : Lo.M;
        Lo.lv64_u[l] = l ? take(c3 * 8) : Lo.z;
        Lo.lv64_b[l] = l ? take(c3 * 8) : 0;
        Lo.lv64_res[l] = take(c3 * 8);
        Lo.lv64_tmp[l] = take(c3 * 8);
    }
    nl = n;
    for (int l = 0; l < L; ++l, nl /= 2) {
        const size_t c3 = (size_t)nl * nl * nl;
        if (cfg->precision == RECON_MIXED) {
            Lo.lv32_a[l] = take(c3 * 4);
            Lo.lv32_u[l] = take(c3 * 4);
            Lo.lv32_b[l] = take(c3 * 4);
            Lo.lv32_res[l] = take(c3 * 4);
            Lo.lv32_tmp[l] = take(c3 * 4);
        } else {
            Lo.lv32_a[l] = Lo.lv32_u[l] = Lo.lv32_b[l] = Lo.lv32_res[l] = Lo.lv32_tmp[l] = (size_t)-1;
        }
    }
    const size_t tape_field = cfg->tape_fp32 ? n3 * 4 : f64;
    Lo.tape = cfg->record_tape ? take(tape_field * (size_t)std::max(cfg->max_outer, 1)) : (size_t)-1;
    // adjoint: phibar, Mbar, mbar, replayed phi, ebar (6 fields), xbar (3 fields).
    // The last three are live only between the end of a step's adjoint solve
    // and the end of that step, when the forward's phi, the six fields b..q
    // and dphi with the two fine-level V-cycle buffers are idle; they reuse
    // that memory whenever those fields are packed back to back (f64 a
    // multiple of the alignment), else they get their own.
    const size_t adj_fields[6] = {1, 1, 1, 1, 6, 3};
    for (int i = 0; i < 8; ++i) Lo.adj[i] = (size_t)-1;
    if (cfg->record_tape) {
        const bool packed = f64 % kAlign == 0 && Lo.u == Lo.b + f64 && Lo.q == Lo.b + 5 * f64 &&
                            Lo.lv64_res[0] == Lo.dphi + f64 && Lo.lv64_tmp[0] == Lo.dphi + 2 * f64;
        for (int i = 0; i < 6; ++i) Lo.adj[i] = (packed && i >= 3) ? (size_t)-1 : take(f64 * adj_fields[i]);
        if (packed) {
            Lo.adj[3] = Lo.phi;
            Lo.adj[4] = Lo.b;
            Lo.adj[5] = Lo.dphi;
        }
    }
    Lo.xi = cfg->particle_deposit ? take(3 * f64) : (size_t)-1;
    Lo.shifts = cfg->particle_deposit ? take(3 * f64) : (size_t)-1;
    Lo.K = cfg->full_operator ? take(7 * f64) : (size_t)-1;
    Lo.total = off;
    return true;
}

}  // namespace

struct recon_ctx {
    int n = 0;
    long n3 = 0;
    recon_config cfg;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Layout lo;
    Part part;
    double *scal = nullptr;       // device scalars (reduction results)
    double *host_scal = nullptr;  // pinned host mirror
    double *m, *phi, *M, *t, *b, *u, *r, *z, *p, *q, *dphi;
    Levels<double> L64;
    Levels<float> L32;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_ks = nullptr;  // marks the Krylov scalars' copy to host_scal
    // cfg.profile: event pairs around each fine-level smoother sweep
    hipEvent_t *prof = nullptr;
    unsigned char prof_zero[4096];  // 0: a plain sweep (reads u, a, b, writes u); 1: from u = 0 (reads a
                                    // and b only); 2: with the coarse correction folded in (also reads e)
    int prof_count = 0;
    // tape of the last recorded forward
    int tape_steps = 0;
    double tape_alpha[RECON_MAX_STEPS];
    double input_mean = 0.0;
    double box = 0.0;
    // particle deposit: the particles of the running solve and their
    // Lagrangian positions (null outside such a solve)
    const float *part_pos = nullptr;
    long long part_np = 0;
    double *xi = nullptr;
    double *shifts = nullptr;  // node shifts of the particle deposit (3 per node)
    // exact-Jacobian solve: K = M e^-1 of the current step (six fields)
    MassTensor Kf{};
    double last_tol = 0.0;
    int tape_valid = 0;
    long long tape_np = 0;  // particles of a recorded particle-deposit forward (0: density input)
    char err[512];
};

namespace {

int fail(recon_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHK(x)                                                                                        \
    do {                                                                                                 \
        hipError_t e_ = (x);                                                                             \
        if (e_ != hipSuccess) return fail(ctx, RECON_E_HIP, "%s: %s", #x, hipGetErrorString(e_));        \
    } while (0)

#define TRY(x)                                                                                           \
    do {                                                                                                 \
        int rc_ = (x);                                                                                   \
        if (rc_ != RECON_OK) return rc_;                                                                 \
    } while (0)

template <typename T>
T *wsp(recon_ctx *ctx, size_t off)
{
    return off == (size_t)-1 ? nullptr : reinterpret_cast<T *>(ctx->ws + off);
}

// Fold the partials of the last reducing launch and read K scalars to the host.
int fetch(recon_ctx *ctx, const int *ops, double *out)
{
    const int K = ctx->part.k;
    HIPCHK(reduce_finalize(ctx->part, ops, ctx->scal, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->host_scal, ctx->scal, sizeof(double) * K, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < K; ++c) out[c] = ctx->host_scal[c];
    return RECON_OK;
}

// Newton's method for the particles' Lagrangian positions: at most this many
// steps, to this max-norm residual in cells.
constexpr int kInvertIters = 100;
constexpr double kInvertTol = 1e-12;

// The device scalars of the conjugate-gradient loop (KS_* in kernels.h) sit at
// this offset of ctx->scal; fetch_krylov copies all of them to the host.
constexpr int kKrylovScal = 32;
// The next V-cycle is queued ahead of the stop test while the extrapolated
// residual norm is above this multiple of the target.
constexpr double kAheadMargin = 8.0;
static_assert(kKrylovScal + KS_COUNT <= kScal, "the scalar block fits");

// In two halves, so that work queued between them overlaps the round trip:
// the copy is enqueued with an event behind it, and the host later waits for
// that event only.  Nothing queued in between may read host_scal.
// A context without events (recon_solve_noalloc) waits for the whole stream
// instead: the same results, without the overlap.
int wait_copy_begin(recon_ctx *ctx)
{
    if (ctx->ev_ks) HIPCHK(hipEventRecord(ctx->ev_ks, ctx->stream));
    return RECON_OK;
}

int wait_copy_end(recon_ctx *ctx)
{
    if (ctx->ev_ks) HIPCHK(hipEventSynchronize(ctx->ev_ks));
    else HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int fetch_krylov_begin(recon_ctx *ctx)
{
    HIPCHK(hipMemcpyAsync(ctx->host_scal, ctx->scal + kKrylovScal, sizeof(double) * KS_COUNT,
                          hipMemcpyDeviceToHost, ctx->stream));
    return wait_copy_begin(ctx);
}

int fetch_krylov_end(recon_ctx *ctx, double *out)
{
    TRY(wait_copy_end(ctx));
    for (int c = 0; c < KS_COUNT; ++c) out[c] = ctx->host_scal[c];
    return RECON_OK;
}

int fetch_sum(recon_ctx *ctx, double *out)
{
    static const int ops[8] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM};
    return fetch(ctx, ops, out);
}

// fetch_sum in two halves, as fetch_krylov_begin/_end; the end reads the
// first sum only.
int fetch_sum1_begin(recon_ctx *ctx)
{
    static const int ops[8] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM};
    HIPCHK(reduce_finalize(ctx->part, ops, ctx->scal, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->host_scal, ctx->scal, sizeof(double) * ctx->part.k, hipMemcpyDeviceToHost,
                          ctx->stream));
    return wait_copy_begin(ctx);
}

int fetch_sum1_end(recon_ctx *ctx, double *out)
{
    TRY(wait_copy_end(ctx));
    out[0] = ctx->host_scal[0];
    return RECON_OK;
}

double level_scale(int l) { return std::ldexp(1.0, -2 * l); }

// ------------------------------------------------------------- multigrid

constexpr int kProfPairs = 4096;  // size of recon_ctx::prof_zero

// Every level whose edge a fused shape divides (multiples of 16) is swept by
// the fused two-colour kernel: from 256^3 with the wide streaming tiles,
// below with narrow tiles and short chunks, where one launch instead of two
// per sweep is most of the gain.  Other edges (ragged hierarchies) take two
// per-colour launches.
template <typename T>
bool use_fused(int n)
{
    return rbgs_fused_supported<T>(n);
}

// One red-black sweep on level l: fused levels out of place between `cur` and
// `alt` (the pointers are swapped), the others in place.
template <typename T>
int sweep(recon_ctx *ctx, Levels<T> &S, int l, T *&cur, T *&alt, const T *rhs, int first, bool zero_init,
          const T *coarse = nullptr)
{
    const int n = S.n[l];
    const T sc = (T)level_scale(l), amin = (T)ctx->cfg.a_min;
    const bool timed = l == 0 && ctx->prof && ctx->prof_count < kProfPairs;
    if (timed) HIPCHK(hipEventRecord(ctx->prof[2 * ctx->prof_count], ctx->stream));
    if (use_fused<T>(n)) {
        HIPCHK(launch_rbgs_fused<T>(cur, alt, S.a[l], rhs, n, sc, amin, first, zero_init, ctx->stream, coarse));
        std::swap(cur, alt);
    } else {
        HIPCHK(launch_rbgs_half<T>(cur, S.a[l], rhs, n, sc, amin, first, zero_init, ctx->stream, l == 0));
        HIPCHK(launch_rbgs_half<T>(cur, S.a[l], rhs, n, sc, amin, 1 - first, false, ctx->stream, l == 0));
    }
    if (timed) {
        ctx->prof_zero[ctx->prof_count] = zero_init ? 1 : (coarse && use_fused<T>(n) ? 2 : 0);
        HIPCHK(hipEventRecord(ctx->prof[2 * ctx->prof_count++ + 1], ctx->stream));
    }
    return RECON_OK;
}

// Levels of at least 256^3 whose edge is a multiple of 128 apply the operator
// with the LDS-streaming kernels; smaller levels (resident in L2/MALL) with
// per-node gathers.  variant: 0 = that choice, 1 = gather, 2 = streaming.
template <typename T>
bool use_stream(int n)
{
    return n >= 256 && stencil25_supported<T>(n);
}

template <typename T>
hipError_t residual_level(const T *u, const T *a, const T *b, T *r, int n, T scale, T a_min, hipStream_t s,
                          int variant = 0)
{
    if (variant == 2 || (variant == 0 && use_stream<T>(n))) return launch_residual25<T>(u, a, b, r, n, scale, a_min, s);
    return launch_residual<T>(u, a, b, r, n, scale, a_min, s);
}

// Grid transfers from fine levels of at least 256^3: streaming kernels;
// otherwise per-node gathers.  variant as for residual_level.
template <typename T>
bool use_transfer_stream(int n)
{
    return n >= 256 && transfer25_supported<T>(n);
}

template <typename T>
hipError_t restrict_level(const T *f, T *c, int n, hipStream_t s, int variant = 0)
{
    if (variant == 2 || (variant == 0 && use_transfer_stream<T>(n))) return launch_restrict25<T>(f, c, n, s);
    return launch_restrict<T>(f, c, n, s);
}

// Coarse right-hand side c = R (b - scale A u): streaming levels whose coarse
// edge is a multiple of 32 form it in one fused pass; otherwise the residual
// goes through `res` (a fine-level buffer) and is then restricted.  variant:
// 0 = that choice, 1 = the two passes, 2 = the fused pass.
template <typename T>
hipError_t coarse_rhs(const T *u, const T *a, const T *b, T *res, T *c, int n, T scale, T a_min, hipStream_t s,
                      int variant = 0)
{
    if (variant == 2 || (variant == 0 && use_stream<T>(n) && resrestrict25_supported<T>(n)))
        return launch_resrestrict25<T>(u, a, b, c, n, scale, a_min, s);
    hipError_t e = residual_level<T>(u, a, b, res, n, scale, a_min, s);
    if (e != hipSuccess) return e;
    return restrict_level<T>(res, c, n, s);
}

template <typename T>
hipError_t prolong_level(T *u, const T *e, int n, hipStream_t s, int variant = 0)
{
    if (variant == 2 || (variant == 0 && use_transfer_stream<T>(n))) return launch_prolong25<T>(u, e, n, s);
    return launch_prolong_add<T>(u, e, n, s);
}

// The outer step's per-node passes (deformed-mesh mass, source, smoothing):
// from 256^3 on edges that are multiples of 64 the stencil field streams
// through LDS; otherwise per-node gathers.  Both give the same node values;
// the sums are grouped differently.  variant: 0 = that choice, 1 = gather,
// 2 = streaming.
bool use_outer_stream(int n, int variant = 0)
{
    return variant == 2 || (variant == 0 && n >= 256 && outer25_supported(n));
}

hipError_t meshmass_pass(const double *phi, const double *m, double *M, int n, Part &p, hipStream_t s,
                         int variant = 0)
{
    if (use_outer_stream(n, variant)) return launch_meshmass25(phi, m, M, n, p, s);
    return launch_meshmass(phi, m, M, n, p, s);
}

hipError_t source_pass(const double *phi, const double *M, double rho_bar, double xi_m, double v_m, double *t, int n,
                       Part &p, hipStream_t s, int variant = 0)
{
    if (use_outer_stream(n, variant)) return launch_source25(phi, M, rho_bar, xi_m, v_m, t, n, p, s);
    return launch_source(phi, M, rho_bar, xi_m, v_m, t, n, p, s);
}

hipError_t smooth_pass(const double *f, double *out, int n, double c0, double sub, hipStream_t s, int variant = 0)
{
    if (use_outer_stream(n, variant)) return launch_smooth25(f, out, n, c0, sub, s);
    return launch_smooth(f, out, n, c0, sub, s);
}

// r = b - A u on the fine level in FP64, its squared norm, and optionally r
// in FP32 (the mixed preconditioner's input).
hipError_t residual_norm(recon_ctx *ctx, const double *u, const double *a, const double *b, double *r, float *r32,
                         const MassTensor *Kf = nullptr)
{
    if (Kf && use_stream<double>(ctx->n) && full25_supported(ctx->n))
        return launch_full_residual_norm25(*Kf, u, b, r, r32, ctx->n, ctx->cfg.a_min, ctx->part, ctx->stream);
    if (Kf) return launch_full_residual_norm(*Kf, u, b, r, r32, ctx->n, ctx->cfg.a_min, ctx->part, ctx->stream);
    if (use_stream<double>(ctx->n))
        return launch_residual_norm25(u, a, b, r, r32, ctx->n, ctx->cfg.a_min, ctx->part, ctx->stream);
    return launch_residual_norm(u, a, b, r, r32, ctx->n, ctx->cfg.a_min, ctx->part, ctx->stream);
}

// Sum the recorded fine-level sweep times (stream already synchronised).
int collect_profile(recon_ctx *ctx, recon_stats *st)
{
    double ms[3] = {0.0, 0.0, 0.0};
    int count[3] = {0, 0, 0};
    for (int i = 0; i < ctx->prof_count; ++i) {
        float e = 0.0f;
        HIPCHK(hipEventElapsedTime(&e, ctx->prof[2 * i], ctx->prof[2 * i + 1]));
        ms[ctx->prof_zero[i]] += e;
        ++count[ctx->prof_zero[i]];
    }
    st->smoother_sweeps = count[0];
    st->smoother_ms = ms[0];
    st->smoother_zero_sweeps = count[1];
    st->smoother_zero_ms = ms[1];
    st->smoother_folded_sweeps = count[2];
    st->smoother_folded_ms = ms[2];
    ctx->prof_count = 0;
    return RECON_OK;
}

// out = V(rhs) on level l from a zero initial guess: n_pre sweeps red->black,
// residual, full weighting, recursion, trilinear correction, n_post sweeps
// black->red; the coarsest level is relaxed in one workgroup.
template <typename T>
int vcycle(recon_ctx *ctx, Levels<T> &S, int l, const T *rhs, T *out)
{
    const int n = S.n[l];
    const T sc = (T)level_scale(l), amin = (T)ctx->cfg.a_min;
    if (l == S.L - 1) {
        HIPCHK(launch_coarse_solve<T>(out, S.a[l], rhs, n, sc, amin, ctx->cfg.coarse_sweeps, ctx->stream));
        return RECON_OK;
    }
    T *cur = out, *alt = S.tmp[l];
    const long n3 = (long)n * n * n;
    if (ctx->cfg.n_pre == 0) HIPCHK(launch_zero(out, n3 * sizeof(T), ctx->stream));
    for (int s = 0; s < ctx->cfg.n_pre; ++s) TRY(sweep<T>(ctx, S, l, cur, alt, rhs, 0, s == 0));
    HIPCHK(coarse_rhs<T>(cur, S.a[l], rhs, S.res[l], S.b[l + 1], n, sc, amin, ctx->stream));
    TRY(vcycle<T>(ctx, S, l + 1, S.b[l + 1], S.u[l + 1]));
    // on fused levels the coarse correction enters the first post-smoothing
    // sweep's planes as they are read (no pass of its own over u)
    const bool fold = ctx->cfg.n_post >= 1 && use_fused<T>(n);
    if (!fold) HIPCHK(prolong_level<T>(cur, S.u[l + 1], n, ctx->stream));
    for (int s = 0; s < ctx->cfg.n_post; ++s)
        TRY(sweep<T>(ctx, S, l, cur, alt, rhs, 1, false, fold && s == 0 ? S.u[l + 1] : nullptr));
    if (cur != out) HIPCHK(hipMemcpyAsync(out, cur, n3 * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    return RECON_OK;
}

// Coefficient hierarchy from a0 (= M): a_{l+1} = R a_l in FP64, and the FP32
// copies when the V-cycle runs in FP32.
int build_hierarchy(recon_ctx *ctx, const double *a0)
{
    Levels<double> &S = ctx->L64;
    S.a[0] = const_cast<double *>(a0);
    for (int l = 0; l + 1 < S.L; ++l) HIPCHK(restrict_level<double>(S.a[l], S.a[l + 1], S.n[l], ctx->stream));
    if (ctx->cfg.precision == RECON_MIXED) {
        for (int l = 0; l < S.L; ++l)
            HIPCHK(launch_cast_f32(S.a[l], ctx->L32.a[l], (long)S.n[l] * S.n[l] * S.n[l], ctx->stream));
    }
    return RECON_OK;
}

// z = V(r) in the configured precision (r FP64 in, z FP64 out for FP64 mode;
// FP32 r32 -> z32 for mixed mode, the FP32 rhs being written by the caller).
int precondition(recon_ctx *ctx)
{
    if (ctx->cfg.precision == RECON_MIXED) return vcycle<float>(ctx, ctx->L32, 0, ctx->L32.b[0], ctx->L32.u[0]);
    return vcycle<double>(ctx, ctx->L64, 0, ctx->r, ctx->z);
}

// Solve A(a0) u = b (b mean-free) into ctx->u; hierarchy must be built.  With
// warm set, ctx->u holds the previous solution and is kept as the starting
// guess when ||b - A u|| < ||b||; otherwise the solve starts from u = 0.
// With Kf the operator is L_K = div(K grad .) instead (the exact Jacobian of
// the mass map, K = M e^-1 filled by the caller), still preconditioned by the
// x ~ xi V-cycle of the built hierarchy (the caller builds it on K's mean
// diagonal).
int mg_solve(recon_ctx *ctx, const double *a0, const double *b, double tol, int *cycles_out, double *rel_out,
             bool warm = false, const MassTensor *Kf = nullptr)
{
    const int n = ctx->n;
    const long n3 = ctx->n3;
    const bool mixed = ctx->cfg.precision == RECON_MIXED;
    float *r32 = mixed ? ctx->L32.b[0] : nullptr;
    double v[KS_COUNT];
    HIPCHK(launch_dot(b, b, n3, ctx->part, ctx->stream));
    TRY(fetch_sum(ctx, v));
    const double bn = std::sqrt(v[0]);
    bool started = false;
    if (warm && bn > 0.0) {
        HIPCHK(residual_norm(ctx, ctx->u, a0, b, ctx->r, r32, Kf));
        TRY(fetch_sum(ctx, v));
        started = std::sqrt(v[0]) < bn;
    }
    if (!started) {
        // u = 0, so the residual kernel gives r = b
        HIPCHK(launch_zero(ctx->u, n3 * 8, ctx->stream));
        HIPCHK(residual_norm(ctx, ctx->u, a0, b, ctx->r, r32, Kf));
    }
    int cycles = 0;
    int status = RECON_E_NO_CONVERGENCE;
    // fixed_cycles > 0: exactly that many V-cycles, no tolerance test
    const int fixed = ctx->cfg.fixed_cycles;
    const int max_cycles = fixed > 0 ? fixed : ctx->cfg.max_vcycles;
    if (bn == 0.0) {
        status = RECON_OK;
    } else if (ctx->cfg.solver == RECON_SOLVER_VCYCLE) {
        // As in the Krylov loop below, the next V-cycle is queued ahead of the
        // stop test when this cycle cannot be the last; it writes only z and
        // the level scratch, and u changes only in the correction after it.
        bool queued = false;
        double rn_last = 0.0, rn_next = 0.0;
        for (int c = 1; c <= max_cycles; ++c) {
            cycles = c;
            if (!queued) TRY(precondition(ctx));
            if (mixed) HIPCHK(launch_add_correction<float>(ctx->u, ctx->L32.u[0], n3, ctx->stream));
            else HIPCHK(launch_add_correction<double>(ctx->u, ctx->z, n3, ctx->stream));
            HIPCHK(residual_norm(ctx, ctx->u, a0, b, ctx->r, r32, Kf));
            queued = cycles < max_cycles && (fixed > 0 ? cycles < fixed : rn_next > kAheadMargin * tol * bn);
            TRY(fetch_sum1_begin(ctx));
            if (queued) TRY(precondition(ctx));
            TRY(fetch_sum1_end(ctx, v));
            const double rn = std::sqrt(v[0]);
            if (!std::isfinite(rn)) break;
            if (fixed > 0 ? cycles >= fixed : rn <= tol * bn) {
                status = RECON_OK;
                break;
            }
            rn_next = rn_last > 0.0 ? rn * (rn / rn_last) : 0.0;
            rn_last = rn;
        }
    } else {
        // Conjugate gradients on A u = b preconditioned by one symmetric V-cycle,
        // flexible form: beta = z_new.(r_new - r_old) / (z_old.r_old)
        //                     = -alpha (z_new.q) / (z_old.r_old).
        // The dot products land in the device scalar block ks, and the kernels
        // form alpha and beta from it themselves (same operations as on the
        // host), so the host waits once per step, for its stop test.
        double *ks = ctx->scal + kKrylovScal;
        static const int sums[2] = {RED_SUM, RED_SUM};
        TRY(precondition(ctx));
        cycles = 1;
        if (mixed) HIPCHK(launch_dots_zr_zq<float>(ctx->L32.u[0], ctx->r, nullptr, n3, ctx->part, ctx->stream));
        else HIPCHK(launch_dots_zr_zq<double>(ctx->z, ctx->r, nullptr, n3, ctx->part, ctx->stream));
        HIPCHK(reduce_finalize(ctx->part, sums, ks + KS_RZ, ctx->stream));
        bool first = true;
        // Streaming levels form the new direction out of place, fused with its
        // operator product; it alternates between p and t (idle during a solve),
        // stored in FP32 when the preconditioner is FP32.  The solution update
        // u += alpha p of one step is deferred into the next direction pass there
        // (it reads p anyway), and applied after the loop for the last step.
        const bool stream = use_stream<double>(n) && (!Kf || full25_supported(n));
        double *pc = ctx->p, *pn = ctx->t;
        auto f32 = [](double *x) { return reinterpret_cast<float *>(x); };
        bool due = false;
        // residual norms: the last one seen and the next one extrapolated
        double rn_last = 0.0, rn_next = 0.0;
        while (true) {
            if (stream && Kf) {
                double *ud = due ? ctx->u : nullptr;
                if (mixed)
                    HIPCHK(launch_full_direction25(ctx->L32.u[0], f32(pc), f32(pn), *Kf, ctx->q, 0.0, n,
                                                   ctx->cfg.a_min, first, ud, 0.0, ks, ctx->part, ctx->stream));
                else
                    HIPCHK(launch_full_direction25(ctx->z, pc, pn, *Kf, ctx->q, 0.0, n, ctx->cfg.a_min, first, ud,
                                                   0.0, ks, ctx->part, ctx->stream));
                due = false;
                std::swap(pc, pn);
            } else if (stream) {
                double *ud = due ? ctx->u : nullptr;
                if (mixed)
                    HIPCHK(launch_direction25(ctx->L32.u[0], f32(pc), f32(pn), a0, ctx->q, 0.0, n, ctx->cfg.a_min,
                                              first, ud, 0.0, ks, ctx->part, ctx->stream));
                else
                    HIPCHK(launch_direction25(ctx->z, pc, pn, a0, ctx->q, 0.0, n, ctx->cfg.a_min, first, ud, 0.0, ks,
                                              ctx->part, ctx->stream));
                due = false;
                std::swap(pc, pn);
            } else if (Kf) {
                if (mixed) HIPCHK(launch_update_p<float>(ctx->L32.u[0], pc, 0.0, n3, first, ks, ctx->stream));
                else HIPCHK(launch_update_p<double>(ctx->z, pc, 0.0, n3, first, ks, ctx->stream));
                HIPCHK(launch_full_apply_dot(*Kf, pc, ctx->q, n, ctx->cfg.a_min, ctx->part, ctx->stream));
            } else if (mixed) {
                HIPCHK(launch_update_pq<float>(ctx->L32.u[0], a0, pc, ctx->q, 0.0, n, ctx->cfg.a_min, first, ks,
                                               ctx->part, ctx->stream));
            } else {
                HIPCHK(launch_update_pq<double>(ctx->z, a0, pc, ctx->q, 0.0, n, ctx->cfg.a_min, first, ks, ctx->part,
                                                ctx->stream));
            }
            first = false;
            HIPCHK(reduce_finalize(ctx->part, sums, ks + KS_PQ, ctx->stream));
            HIPCHK(launch_update_ur(stream ? nullptr : ctx->u, ctx->r, pc, ctx->q, 0.0, r32, n3, ks, ctx->part,
                                    ctx->stream));
            due = stream;
            HIPCHK(reduce_finalize(ctx->part, sums, ks + KS_RR, ctx->stream));
            // The stop test needs ||r|| on the host.  When this step cannot be
            // the last (a fixed count not yet reached, or the residual norm
            // extrapolated from the last two steps still well above the
            // target), the next V-cycle is queued before the host waits, so
            // the device does not idle through the round trip.  The V-cycle
            // writes only z and the level scratch, never u, r or the current
            // direction, so a wrong guess costs one V-cycle and changes no
            // result.
            const bool ahead =
                cycles < max_cycles && (fixed > 0 ? cycles < fixed : rn_next > kAheadMargin * tol * bn);
            TRY(fetch_krylov_begin(ctx));
            if (ahead) TRY(precondition(ctx));
            TRY(fetch_krylov_end(ctx, v));
            const double rn = std::sqrt(v[KS_RR]);
            if (!std::isfinite(rn) || !std::isfinite(v[KS_ALPHA])) break;
            if (fixed > 0 ? cycles >= fixed : rn <= tol * bn) {
                status = RECON_OK;
                break;
            }
            if (cycles >= max_cycles) break;
            if (!ahead) TRY(precondition(ctx));
            rn_next = rn_last > 0.0 ? rn * (rn / rn_last) : 0.0;
            rn_last = rn;
            ++cycles;
            if (mixed) HIPCHK(launch_dots_zr_zq<float>(ctx->L32.u[0], ctx->r, ctx->q, n3, ctx->part, ctx->stream));
            else HIPCHK(launch_dots_zr_zq<double>(ctx->z, ctx->r, ctx->q, n3, ctx->part, ctx->stream));
            HIPCHK(reduce_finalize(ctx->part, sums, ks + KS_RZ, ctx->stream));
        }
        if (due && mixed) HIPCHK(launch_axpy(ctx->u, f32(pc), 0.0, n3, ctx->stream, ks + KS_ALPHA));
        else if (due) HIPCHK(launch_axpy(ctx->u, pc, 0.0, n3, ctx->stream, ks + KS_ALPHA));
    }
    // mean-free solution, then the true residual
    HIPCHK(launch_sum(ctx->u, n3, ctx->part, ctx->stream));
    TRY(fetch_sum(ctx, v));
    HIPCHK(launch_fill(ctx->scal + 16, 1, v[0] / (double)n3, ctx->stream));
    HIPCHK(launch_add_scalar(ctx->u, ctx->scal + 16, -1.0, 1.0, n3, ctx->stream));
    HIPCHK(residual_norm(ctx, ctx->u, a0, b, ctx->r, nullptr, Kf));
    TRY(fetch_sum(ctx, v));
    const double rel = bn > 0.0 ? std::sqrt(v[0]) / bn : 0.0;
    if (cycles_out) *cycles_out = cycles;
    if (rel_out) *rel_out = rel;
    if (status != RECON_OK)
        return fail(ctx, RECON_E_NO_CONVERGENCE, "linear solve did not reach tol %.3g in %d V-cycles (rel %.3g)", tol,
                    cycles, rel);
    return RECON_OK;
}

// ------------------------------------------------------------ step control

// Failing-node counts of `ntrial` step trials from 2^-j0; variant 1 gathers
// per node, 2 streams planes through LDS, 0 takes 2 where it applies.  With M
// and D (mass update) a node also fails where M + alpha D > 0 does not hold.
hipError_t pd_trials(recon_ctx *ctx, const double *phi, const double *dphi, int j0, int ntrial, int variant,
                     const double *M = nullptr, const double *D = nullptr)
{
    if (variant == 0) variant = pd25_supported(ctx->n) ? 2 : 1;
    if (variant == 2) return launch_pd25(phi, dphi, ctx->n, j0, ntrial, ctx->part, ctx->stream, M, D);
    return launch_pd_trials(phi, dphi, ctx->n, j0, ntrial, ctx->part, ctx->stream, M, D);
}

int choose_step(recon_ctx *ctx, const double *phi, const double *dphi, double *alpha_out,
                const double *M = nullptr, const double *D = nullptr, int *limit_out = nullptr)
{
    static const int opmax[1] = {RED_MAX};
    double v[8];
    HIPCHK(launch_max_shift(dphi, ctx->n, ctx->part, ctx->stream));
    TRY(fetch(ctx, opmax, v));
    const double shift = v[0];
    if (!std::isfinite(shift)) return fail(ctx, RECON_E_NO_CONVERGENCE, "non-finite increment");
    int j0 = 0;
    while (j0 <= ctx->cfg.max_halvings && std::ldexp(1.0, -j0) * shift > ctx->cfg.s_max) ++j0;
    // four halvings per launch, from the largest step the shift bound allows
    for (int j = j0, batch = 4; j <= ctx->cfg.max_halvings; j += batch) {
        HIPCHK(pd_trials(ctx, phi, dphi, j, batch, 0, M, D));
        TRY(fetch_sum(ctx, v));
        for (int t = 0; t < batch && j + t <= ctx->cfg.max_halvings; ++t) {
            if (v[t] == 0.0) {
                *alpha_out = std::ldexp(1.0, -(j + t));
                if (limit_out) *limit_out = j + t > j0 ? 2 : (j0 > 0 ? 1 : 0);
                return RECON_OK;
            }
        }
    }
    return fail(ctx, RECON_E_NOT_PD, "no step 2^-j, j <= %d, keeps the map positive definite%s",
                ctx->cfg.max_halvings, M ? " and the mass positive" : "");
}

// ------------------------------------------------------------ forward

int normalize(recon_ctx *ctx, const double *rho, double *m, double *mean_out)
{
    double v[2];
    HIPCHK(launch_check_input(rho, ctx->n3, ctx->part, ctx->stream));
    TRY(fetch_sum(ctx, v));
    if (v[1] != 0.0) return fail(ctx, RECON_E_INPUT, "density has %.0f negative or non-finite values", v[1]);
    if (!(v[0] > 0.0)) return fail(ctx, RECON_E_INPUT, "density has zero total mass");
    const double mean = v[0] / (double)ctx->n3;
    HIPCHK(launch_fill(ctx->scal + 8, 1, mean, ctx->stream));
    HIPCHK(launch_scale(rho, m, ctx->n3, ctx->scal + 8, ctx->stream));
    if (mean_out) *mean_out = mean;
    return RECON_OK;
}

// Particle deposit: M = CIC of the particles at their Lagrangian positions for
// the current phi, found by Newton from the previous ones; the node shifts
// go into their own buffer (ctx->shifts), which the reverse mode reads.
int deposit_particles(recon_ctx *ctx)
{
    double v[1];
    HIPCHK(launch_invert_map(ctx->phi, ctx->part_pos, ctx->part_np, ctx->n, ctx->box, ctx->xi, ctx->shifts,
                             kInvertIters, kInvertTol, ctx->part, ctx->stream));
    TRY(fetch_sum(ctx, v));
    if (v[0] != 0.0)
        return fail(ctx, RECON_E_NO_CONVERGENCE, "%.0f particles not located on the deformed mesh", v[0]);
    HIPCHK(launch_deposit_xi(ctx->xi, ctx->part_np, ctx->n, ctx->M, ctx->stream));
    return RECON_OK;
}

// rho_bar = mean(M), rms(Sigma) and the source for the current phi; M is
// gathered on the deformed mesh when `gather` (or, in a particle-deposit solve,
// deposited from the particles), else (mass update) kept.
int mass_state(recon_ctx *ctx, double *rho_bar, double *rms, double *mean_t, bool gather = true)
{
    double v[2];
    if (ctx->part_pos) {
        TRY(deposit_particles(ctx));
        HIPCHK(launch_sum(ctx->M, ctx->n3, ctx->part, ctx->stream));
    } else if (gather) {
        HIPCHK(meshmass_pass(ctx->phi, ctx->m, ctx->M, ctx->n, ctx->part, ctx->stream));
    } else {
        HIPCHK(launch_sum(ctx->M, ctx->n3, ctx->part, ctx->stream));
    }
    TRY(fetch_sum(ctx, v));
    *rho_bar = v[0] / (double)ctx->n3;
    HIPCHK(source_pass(ctx->phi, ctx->M, *rho_bar, ctx->cfg.xi_m, ctx->cfg.v_m, ctx->t, ctx->n, ctx->part,
                         ctx->stream));
    TRY(fetch_sum(ctx, v));
    *rms = std::sqrt(v[0] / (double)ctx->n3);
    *mean_t = v[1] / (double)ctx->n3;
    return RECON_OK;
}

// RECON_LOG set to anything but "0": one line per outer step on stderr.
bool log_steps()
{
    const char *e = std::getenv("RECON_LOG");
    return e && *e && !(e[0] == '0' && e[1] == 0);
}

int forward(recon_ctx *ctx, double box, double tol, double *phi_out, double *delta_out, recon_stats *st)
{
    const recon_config &c = ctx->cfg;
    const long n3 = ctx->n3;
    HIPCHK(launch_zero(ctx->phi, n3 * 8, ctx->stream));
    ctx->tape_valid = 0;
    ctx->tape_steps = 0;
    ctx->tape_np = 0;
    // Mass update: after the first gather (at phi = 0, where it gives M = m) M
    // is carried by M += alpha D.  D goes into m's field, which is not read
    // again in that mode, and K into six fields idle between the solve and
    // the next step's source.
    // With the exact-Jacobian solve, K = M e^-1 of the step sits in its own
    // fields, and the mass update reuses it (same mesh, same M).
    const bool carry = c.mass_update != 0;
    const bool full = c.full_operator != 0;
    double *D = ctx->m;
    const MassTensor K = full ? ctx->Kf : MassTensor{ctx->t, ctx->b, ctx->r, ctx->z, ctx->p, ctx->q, nullptr};
    int it = 0;
    for (; it < c.max_outer; ++it) {
        double rho_bar, rms, mean_t;
        TRY(mass_state(ctx, &rho_bar, &rms, &mean_t, !carry || it == 0));
        st->rms_sigma[it] = rms;
        st->kappa[it] = rho_bar;
        if (!std::isfinite(rms)) return fail(ctx, RECON_E_NO_CONVERGENCE, "non-finite mass deviation");
        if (rms <= c.outer_tol) break;
        HIPCHK(smooth_pass(ctx->t, ctx->b, ctx->n, c.smooth_center, mean_t, ctx->stream));
        // the exact-Jacobian solve preconditions with the x ~ xi V-cycle of
        // the mean diagonal of K = M e^-1
        if (full) HIPCHK(launch_mass_tensor(ctx->phi, ctx->M, K, ctx->n, ctx->stream));
        TRY(build_hierarchy(ctx, full ? K.tr : ctx->M));
        int cyc = 0;
        double rel = 0.0;
        TRY(mg_solve(ctx, ctx->M, ctx->b, tol, &cyc, &rel, c.warm_start && it > 0, full ? &K : nullptr));
        st->vcycles[it] = cyc;
        st->vcycles_total += cyc;
        st->rel_residual[it] = rel;
        HIPCHK(smooth_pass(ctx->u, ctx->dphi, ctx->n, c.smooth_center, 0.0, ctx->stream));
        if (carry && full) HIPCHK(launch_full_apply(K, ctx->dphi, D, ctx->n, ctx->stream));
        else if (carry) HIPCHK(launch_mass_change(ctx->phi, ctx->M, ctx->dphi, K, D, ctx->n, ctx->stream));
        double alpha = 0.0;
        TRY(choose_step(ctx, ctx->phi, ctx->dphi, &alpha, carry ? ctx->M : nullptr, carry ? D : nullptr,
                        &st->alpha_limit[it]));
        if (carry) HIPCHK(launch_axpy(ctx->M, D, alpha, n3, ctx->stream));
        HIPCHK(launch_axpy(ctx->phi, ctx->dphi, alpha, n3, ctx->stream));
        st->alpha[it] = alpha;
        st->outer_steps = it + 1;
        if (log_steps())
            std::fprintf(stderr, "recon step %d: rms(Sigma) %.6e, mean M %.12f, V-cycles %d, residual %.3e, alpha %.6e\n",
                         it, rms, rho_bar, cyc, rel, alpha);
        if (c.record_tape) {
            if (c.tape_fp32) HIPCHK(launch_cast_f32(ctx->u, wsp<float>(ctx, ctx->lo.tape) + (size_t)it * n3, n3, ctx->stream));
            else HIPCHK(launch_copy(wsp<double>(ctx, ctx->lo.tape) + (size_t)it * n3, ctx->u, n3, ctx->stream));
            ctx->tape_alpha[it] = alpha;
            ctx->tape_steps = it + 1;
        }
    }
    if (it == c.max_outer) {
        double rho_bar, rms, mean_t;
        TRY(mass_state(ctx, &rho_bar, &rms, &mean_t, !carry));
        st->rms_sigma[it] = rms;
        st->kappa[it] = rho_bar;
    }
    static const int opmin[3] = {RED_MIN, RED_MIN, RED_MIN};
    double v[3];
    const double h = box / ctx->n;
    HIPCHK(launch_output(ctx->phi, delta_out, phi_out, h * h, ctx->n, ctx->part, ctx->stream));
    TRY(fetch(ctx, opmin, v));
    st->min_det = v[0];
    st->min_lambda0 = v[1];
    st->max_delta_r = -v[2];
    if (c.record_tape) {
        ctx->tape_valid = 1;
        ctx->tape_np = ctx->part_pos ? ctx->part_np : 0;
    }
    return RECON_OK;
}

// Reverse sweep over the tape (transposes of the forward maps, in reverse
// order); the discrete decisions of the forward are held fixed and each
// linear solve is differentiated as exact.
// pos, gpos (particle-deposit tapes): the particles of the forward and the
// gradient with respect to their positions (3 per particle); else grad is
// the gradient with respect to the input density.
int backward(recon_ctx *ctx, const double *gd, const double *gp, double *grad, const float *pos = nullptr,
             double *gpos = nullptr)
{
    const recon_config &c = ctx->cfg;
    const int n = ctx->n;
    const long n3 = ctx->n3;
    const double h = ctx->box / n;
    double *phibar = wsp<double>(ctx, ctx->lo.adj[0]);
    double *Mbar = wsp<double>(ctx, ctx->lo.adj[1]);
    double *mbar = wsp<double>(ctx, ctx->lo.adj[2]);
    double *phi = wsp<double>(ctx, ctx->lo.adj[3]);
    double *hb = wsp<double>(ctx, ctx->lo.adj[4]);
    double *xb = wsp<double>(ctx, ctx->lo.adj[5]);
    double *ubar = ctx->b, *tbar = ctx->t;
    double v[2];
    // u_q of the tape as FP64; an FP32 tape is widened into z, which is idle
    // whenever this is called (before a step's solve and right after it)
    auto tape_u = [&](int q) -> const double * {
        if (!c.tape_fp32) return wsp<double>(ctx, ctx->lo.tape) + (size_t)q * n3;
        return launch_cast_f64(wsp<float>(ctx, ctx->lo.tape) + (size_t)q * n3, ctx->z, n3, ctx->stream) == hipSuccess
                   ? ctx->z
                   : nullptr;
    };

    const long long np = ctx->tape_np;
    HIPCHK(launch_out_adj(gd, gp, h * h, phibar, n, ctx->stream));
    HIPCHK(launch_zero(mbar, n3 * 8, ctx->stream));
    if (gpos) HIPCHK(launch_zero(gpos, np * 3 * 8, ctx->stream));
    for (int s = ctx->tape_steps - 1; s >= 0; --s) {
        // phi_s, rebuilt from the increments exactly as the forward built it
        HIPCHK(launch_zero(phi, n3 * 8, ctx->stream));
        for (int q = 0; q < s; ++q) {
            const double *u_q = tape_u(q);
            if (!u_q) return fail(ctx, RECON_E_HIP, "tape widening launch failed");
            HIPCHK(smooth_pass(u_q, ctx->dphi, n, c.smooth_center, 0.0, ctx->stream));
            HIPCHK(launch_axpy(phi, ctx->dphi, ctx->tape_alpha[q], n3, ctx->stream));
        }
        if (gpos) {
            // the step's Lagrangian positions, warm-started from the later
            // step's (ctx->xi holds those of the final mesh after the forward)
            HIPCHK(launch_invert_map(phi, pos, np, n, ctx->box, ctx->xi, ctx->shifts, kInvertIters,
                                     kInvertTol, ctx->part, ctx->stream));
            TRY(fetch_sum(ctx, v));
            if (v[0] != 0.0)
                return fail(ctx, RECON_E_NO_CONVERGENCE, "%.0f particles not located on the mesh of step %d", v[0], s);
            HIPCHK(launch_deposit_xi(ctx->xi, np, n, ctx->M, ctx->stream));
            HIPCHK(launch_sum(ctx->M, n3, ctx->part, ctx->stream));
        } else {
            HIPCHK(meshmass_pass(phi, ctx->m, ctx->M, n, ctx->part, ctx->stream));
        }
        TRY(fetch_sum(ctx, v));
        const double rho_bar = v[0] / (double)n3;
        // phi_{s+1} = phi_s + alpha S u:  ubar = alpha S phibar, made mean-free
        HIPCHK(launch_smooth_scaled(phibar, ubar, n, c.smooth_center, ctx->tape_alpha[s], ctx->stream));
        HIPCHK(launch_sum(ubar, n3, ctx->part, ctx->stream));
        TRY(fetch_sum(ctx, v));
        HIPCHK(launch_fill(ctx->scal + 16, 1, v[0] / (double)n3, ctx->stream));
        HIPCHK(launch_add_scalar(ubar, ctx->scal + 16, -1.0, 1.0, n3, ctx->stream));
        // u = A(M)^+ b:  lambda = A^+ ubar (same symmetric operator and solver)
        TRY(build_hierarchy(ctx, ctx->M));
        int cyc = 0;
        double rel = 0.0;
        TRY(mg_solve(ctx, ctx->M, ubar, ctx->last_tol, &cyc, &rel));
        const double *lam = ctx->u;
        const double *u_s = tape_u(s);
        if (!u_s) return fail(ctx, RECON_E_HIP, "tape widening launch failed");
        HIPCHK(launch_coefgrad(lam, u_s, ctx->M, c.a_min, Mbar, n, ctx->stream));
        // b = S t - mean:  tbar = S (lambda - mean lambda)
        HIPCHK(launch_sum(lam, n3, ctx->part, ctx->stream));
        TRY(fetch_sum(ctx, v));
        HIPCHK(smooth_pass(lam, tbar, n, c.smooth_center, v[0] / (double)n3, ctx->stream));
        // source, then Sigma = mean(M) - M
        HIPCHK(launch_source_adj(phi, ctx->M, rho_bar, tbar, c.xi_m, c.v_m, Mbar, hb, n, ctx->part, ctx->stream));
        TRY(fetch_sum(ctx, v));
        HIPCHK(launch_fill(ctx->scal + 16, 1, v[0] / (double)n3, ctx->stream));
        HIPCHK(launch_add_scalar(Mbar, ctx->scal + 16, 1.0, 1.0, n3, ctx->stream));
        if (gpos) {
            // M = CIC(xi), xi = X^-1(y; D_c phi): xb <- adjoint of the node
            // shifts (still those of this step's phi, from the inversion)
            HIPCHK(launch_zero(xb, 3 * n3 * 8, ctx->stream));
            HIPCHK(launch_deposit_adj(ctx->xi, np, n, ctx->shifts, Mbar, xb, gpos, (double)n / ctx->box,
                                      ctx->stream));
        } else {
            // M = det(e) rho~(x), then phibar through e and x
            HIPCHK(launch_meshmass_adj(phi, ctx->m, Mbar, hb, xb, mbar, n, ctx->stream));
        }
        HIPCHK(launch_phibar_update(hb, xb, phibar, n, ctx->stream));
    }
    if (gpos) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return RECON_OK;
    }
    // m = rho / mean(rho)
    HIPCHK(launch_dot(mbar, ctx->m, n3, ctx->part, ctx->stream));
    TRY(fetch_sum(ctx, v));
    HIPCHK(launch_rho_grad(mbar, v[0] / (double)n3, ctx->input_mean, grad, n3, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int check_ctx(recon_ctx *ctx) { return ctx ? RECON_OK : RECON_E_ARG; }

// Point a fresh context at its workspace (laid out by lo) and stream.  Host
// resources (the scalar mirror, events) are the caller's to attach.
void bind_context(recon_ctx *ctx, int n, const recon_config *cfg, void *workspace, size_t ws_bytes,
                  void *hip_stream, const Layout &lo)
{
    ctx->err[0] = 0;
    ctx->n = n;
    ctx->n3 = (long)n * n * n;
    ctx->cfg = *cfg;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    ctx->ws = reinterpret_cast<char *>(workspace);
    ctx->ws_bytes = ws_bytes;
    ctx->lo = lo;
    ctx->part.part = wsp<double>(ctx, lo.part);
    ctx->part.blocks = 0;
    ctx->part.k = 0;
    ctx->scal = wsp<double>(ctx, lo.scal);
    ctx->m = wsp<double>(ctx, lo.m);
    ctx->phi = wsp<double>(ctx, lo.phi);
    ctx->M = wsp<double>(ctx, lo.M);
    ctx->t = wsp<double>(ctx, lo.t);
    ctx->b = wsp<double>(ctx, lo.b);
    ctx->u = wsp<double>(ctx, lo.u);
    ctx->r = wsp<double>(ctx, lo.r);
    ctx->z = wsp<double>(ctx, lo.z);
    ctx->p = wsp<double>(ctx, lo.p);
    ctx->q = wsp<double>(ctx, lo.q);
    ctx->dphi = wsp<double>(ctx, lo.dphi);
    ctx->xi = ctx->cfg.particle_deposit ? wsp<double>(ctx, lo.xi) : nullptr;
    ctx->shifts = ctx->cfg.particle_deposit ? wsp<double>(ctx, lo.shifts) : nullptr;
    if (ctx->cfg.full_operator) {
        double *k0 = wsp<double>(ctx, lo.K);
        ctx->Kf = MassTensor{k0,
                             k0 + ctx->n3,
                             k0 + 2 * ctx->n3,
                             k0 + 3 * ctx->n3,
                             k0 + 4 * ctx->n3,
                             k0 + 5 * ctx->n3,
                             k0 + 6 * ctx->n3};
    }
    ctx->L64.L = ctx->L32.L = lo.levels;
    int nl = n;
    for (int l = 0; l < lo.levels; ++l, nl /= 2) {
        ctx->L64.n[l] = ctx->L32.n[l] = nl;
        ctx->L64.a[l] = wsp<double>(ctx, lo.lv64_a[l]);
        ctx->L64.u[l] = wsp<double>(ctx, lo.lv64_u[l]);
        ctx->L64.b[l] = l ? wsp<double>(ctx, lo.lv64_b[l]) : ctx->r;
        ctx->L64.res[l] = wsp<double>(ctx, lo.lv64_res[l]);
        ctx->L64.tmp[l] = wsp<double>(ctx, lo.lv64_tmp[l]);
        ctx->L32.a[l] = wsp<float>(ctx, lo.lv32_a[l]);
        ctx->L32.u[l] = wsp<float>(ctx, lo.lv32_u[l]);
        ctx->L32.b[l] = wsp<float>(ctx, lo.lv32_b[l]);
        ctx->L32.res[l] = wsp<float>(ctx, lo.lv32_res[l]);
        ctx->L32.tmp[l] = wsp<float>(ctx, lo.lv32_tmp[l]);
    }
}

// recon_solve on a bound context.  Wall time from the context's events, or
// from the host clock around a drained stream when it has none.
// True when the byte ranges [p, p + np) and [q, q + nq) share a byte: an
// output written while other lanes still read an overlapping input would
// race, so the entry points reject such calls.
static bool overlap(const void *p, size_t np, const void *q, size_t nq)
{
    if (!p || !q) return false;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p), b = reinterpret_cast<uintptr_t>(q);
    return a < b + nq && b < a + np;
}

int solve_density(recon_ctx *ctx, const double *density, int n, double box, double tol, double *phi_out,
                  double *delta_r_out, recon_stats *stats)
{
    ctx->err[0] = 0;
    // a failed or partial solve leaves no tape behind
    ctx->tape_valid = 0;
    if (!density || n != ctx->n || !(box > 0.0) || !std::isfinite(box) || !(tol >= 0.0) || !std::isfinite(tol))
        return fail(ctx, RECON_E_ARG, "bad argument (density %p, n %d vs %d, box %g, tol %g)", (const void *)density,
                    n, ctx->n, box, tol);
    if (ctx->cfg.particle_deposit)
        return fail(ctx, RECON_E_ARG, "particle_deposit needs particle input (recon_solve_particles)");
    if (overlap(phi_out, ctx->n3 * 8, delta_r_out, ctx->n3 * 8))
        return fail(ctx, RECON_E_ARG, "phi_out overlaps delta_r_out");
    recon_stats local;
    recon_stats *st = stats ? stats : &local;
    std::memset(st, 0, sizeof(*st));
    ctx->prof_count = 0;
    std::chrono::steady_clock::time_point t0;
    if (ctx->ev0) {
        HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
    } else {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        t0 = std::chrono::steady_clock::now();
    }
    double mean = 0.0;
    TRY(normalize(ctx, density, ctx->m, &mean));
    ctx->input_mean = mean;
    ctx->box = box;
    ctx->last_tol = tol > 0.0 ? tol : ctx->cfg.tol;
    TRY(forward(ctx, box, ctx->last_tol, phi_out, delta_r_out, st));
    if (ctx->ev0) {
        HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
        HIPCHK(hipEventSynchronize(ctx->ev1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        st->ms_total = ms;
    } else {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        st->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    TRY(collect_profile(ctx, st));
    return RECON_OK;
}

// ------------------------------------------- the allocation-free entry point

constexpr int kNoallocDevices = 64;

struct NoallocSlot {
    std::mutex mu;       // serialises the calls on this device
    bool ready = false;  // device address looked up
    char *ptr = nullptr; // device address of `scratch` on this device
    double host_scal[kScal];
    recon_ctx ctx;
};

NoallocSlot g_noalloc[kNoallocDevices];

}  // namespace

// ================================================================= C ABI

extern "C" {

int recon_config_default(recon_config *c)
{
    if (!c) return RECON_E_ARG;
    c->max_outer = 10;
    c->n_pre = 2;
    c->n_post = 2;
    c->coarse_n = 8;
    c->coarse_sweeps = 64;
    c->max_vcycles = 100;
    c->max_halvings = 30;
    c->precision = RECON_FP64;
    c->solver = RECON_SOLVER_PCG;
    c->warm_start = 1;
    c->mass_update = 0;
    c->particle_deposit = 0;
    c->full_operator = 0;
    c->fixed_cycles = 0;
    c->record_tape = 0;
    c->tape_fp32 = 0;
    c->profile = 0;
    c->tol = 1e-10;
    c->outer_tol = 0.0;
    c->xi_m = 0.1;
    c->v_m = 10.0;
    c->smooth_center = 0.5;
    c->s_max = 1.0;
    c->a_min = 1e-3;
    return RECON_OK;
}

size_t recon_workspace_bytes(int n, const recon_config *cfg)
{
    Layout lo;
    return make_layout(n, cfg, lo) ? lo.total : 0;
}

int recon_init(recon_ctx **out, int n, const recon_config *cfg, void *workspace, size_t ws_bytes, void *hip_stream)
{
    if (!out) return RECON_E_ARG;
    *out = nullptr;
    Layout lo;
    if (!make_layout(n, cfg, lo)) return RECON_E_ARG;
    if (!workspace || ws_bytes < lo.total || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
        return RECON_E_WORKSPACE;
    recon_ctx *ctx = new (std::nothrow) recon_ctx();
    if (!ctx) return RECON_E_ARG;
    bind_context(ctx, n, cfg, workspace, ws_bytes, hip_stream, lo);
    if (hipHostMalloc(reinterpret_cast<void **>(&ctx->host_scal), sizeof(double) * kScal, hipHostMallocDefault) !=
            hipSuccess ||
        hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_ks, hipEventDisableTiming) != hipSuccess) {
        recon_destroy(ctx);
        return RECON_E_HIP;
    }
    if (cfg->profile) {
        ctx->prof = new (std::nothrow) hipEvent_t[2 * kProfPairs]();
        if (!ctx->prof) {
            recon_destroy(ctx);
            return RECON_E_ARG;
        }
        for (int i = 0; i < 2 * kProfPairs; ++i)
            if (hipEventCreate(&ctx->prof[i]) != hipSuccess) {
                recon_destroy(ctx);
                return RECON_E_HIP;
            }
    }
    *out = ctx;
    return RECON_OK;
}

void recon_destroy(recon_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->host_scal) (void)hipHostFree(ctx->host_scal);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->ev_ks) (void)hipEventDestroy(ctx->ev_ks);
    if (ctx->prof) {
        for (int i = 0; i < 2 * kProfPairs; ++i)
            if (ctx->prof[i]) (void)hipEventDestroy(ctx->prof[i]);
        delete[] ctx->prof;
    }
    delete ctx;
}

const char *recon_strerror(int code)
{
    switch (code) {
    case RECON_OK: return "ok";
    case RECON_E_ARG: return "invalid argument";
    case RECON_E_INPUT: return "invalid density (negative, non-finite, or zero total mass)";
    case RECON_E_NOT_PD: return "no step size keeps the map positive definite";
    case RECON_E_NO_CONVERGENCE: return "linear solve did not converge";
    case RECON_E_NO_TAPE: return "backward called without a recorded forward";
    case RECON_E_HIP: return "HIP runtime error";
    case RECON_E_WORKSPACE: return "workspace missing, too small or misaligned";
    case RECON_E_SCRATCH:
        return "the problem needs more workspace than the static scratch of recon_solve_noalloc "
               "(RECON_NOALLOC_SCRATCH_BYTES, 64 MiB: n <= 64)";
    default: return "unknown error";
    }
}

const char *recon_last_error(const recon_ctx *ctx) { return ctx ? ctx->err : "null context"; }

int recon_solve(recon_ctx *ctx, const double *density, int n, double box, double tol, double *phi_out,
                double *delta_r_out, recon_stats *stats)
{
    TRY(check_ctx(ctx));
    return solve_density(ctx, density, n, box, tol, phi_out, delta_r_out, stats);
}

int recon_solve_noalloc(const double *density, int n, double box, double tol, const recon_config *cfg,
                        double *phi_out, double *delta_r_out, recon_stats *stats, void *hip_stream)
{
    Layout lo;
    if (!cfg || !make_layout(n, cfg, lo) || cfg->record_tape || cfg->particle_deposit || cfg->profile)
        return RECON_E_ARG;
    if (lo.total > RECON_NOALLOC_SCRATCH_BYTES) return RECON_E_SCRATCH;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return RECON_E_HIP;
    if (dev < 0 || dev >= kNoallocDevices) return RECON_E_ARG;
    NoallocSlot &slot = g_noalloc[dev];
    std::lock_guard<std::mutex> lock(slot.mu);
    if (!slot.ready) {
        // set-up, once per device, with that device current
        if (hipGetSymbolAddress(reinterpret_cast<void **>(&slot.ptr), HIP_SYMBOL(scratch)) != hipSuccess ||
            !slot.ptr)
            return RECON_E_HIP;
        slot.ready = true;
    }
    recon_ctx *ctx = &slot.ctx;
    *ctx = recon_ctx();
    bind_context(ctx, n, cfg, slot.ptr, RECON_NOALLOC_SCRATCH_BYTES, hip_stream, lo);
    ctx->host_scal = slot.host_scal;  // pageable static mirror; every read waits for its copy
    return solve_density(ctx, density, n, box, tol, phi_out, delta_r_out, stats);
}

int recon_solve_particles(recon_ctx *ctx, const float *pos, long long np, double box, double tol, double *phi_out,
                          double *delta_r_out, recon_stats *stats)
{
    TRY(check_ctx(ctx));
    ctx->err[0] = 0;
    ctx->tape_valid = 0;
    if (!pos || np <= 0 || !(box > 0.0) || !std::isfinite(box) || !(tol >= 0.0) || !std::isfinite(tol))
        return fail(ctx, RECON_E_ARG, "bad particle arguments");
    if (overlap(phi_out, ctx->n3 * 8, delta_r_out, ctx->n3 * 8))
        return fail(ctx, RECON_E_ARG, "phi_out overlaps delta_r_out");
    if (ctx->cfg.particle_deposit && np > ctx->n3)
        return fail(ctx, RECON_E_ARG, "the particle deposit takes at most n^3 particles");
    recon_stats local;
    recon_stats *st = stats ? stats : &local;
    std::memset(st, 0, sizeof(*st));
    ctx->prof_count = 0;
    HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
    // the deposit lands in t, then is normalised into m
    HIPCHK(launch_zero(ctx->t, ctx->n3 * 8, ctx->stream));
    HIPCHK(launch_cic(pos, np, ctx->n, box, ctx->t, ctx->stream));
    double mean = 0.0;
    TRY(normalize(ctx, ctx->t, ctx->m, &mean));
    ctx->input_mean = mean;
    ctx->box = box;
    ctx->last_tol = tol > 0.0 ? tol : ctx->cfg.tol;
    if (ctx->cfg.particle_deposit) {
        // every step deposits the particles at their Lagrangian positions,
        // starting from xi = y (the map is the identity at phi = 0)
        ctx->part_pos = pos;
        ctx->part_np = np;
        HIPCHK(launch_init_xi(pos, np, ctx->n, box, ctx->xi, ctx->stream));
    }
    const int rc = forward(ctx, box, ctx->last_tol, phi_out, delta_r_out, st);
    ctx->part_pos = nullptr;
    ctx->part_np = 0;
    TRY(rc);
    HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
    HIPCHK(hipEventSynchronize(ctx->ev1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    st->ms_total = ms;
    TRY(collect_profile(ctx, st));
    return RECON_OK;
}

int recon_backward(recon_ctx *ctx, const double *grad_delta_r, const double *grad_phi, double *grad_density)
{
    TRY(check_ctx(ctx));
    ctx->err[0] = 0;
    if (!ctx->cfg.record_tape || !ctx->tape_valid)
        return fail(ctx, RECON_E_NO_TAPE, "no forward with record_tape has completed on this context");
    if (!grad_delta_r || !grad_density) return fail(ctx, RECON_E_ARG, "null gradient array");
    if (ctx->tape_np > 0)
        return fail(ctx, RECON_E_ARG, "the recorded forward deposited particles: use recon_backward_particles");
    return backward(ctx, grad_delta_r, grad_phi, grad_density);
}

int recon_backward_particles(recon_ctx *ctx, const float *pos, long long np, const double *grad_delta_r,
                             const double *grad_phi, double *grad_pos)
{
    TRY(check_ctx(ctx));
    ctx->err[0] = 0;
    if (!ctx->cfg.record_tape || !ctx->tape_valid)
        return fail(ctx, RECON_E_NO_TAPE, "no forward with record_tape has completed on this context");
    if (ctx->tape_np <= 0)
        return fail(ctx, RECON_E_ARG, "the recorded forward did not deposit particles: use recon_backward");
    if (!pos || np != ctx->tape_np || !grad_delta_r || !grad_pos)
        return fail(ctx, RECON_E_ARG, "the particles must be those of the recorded forward");
    if (overlap(grad_pos, (size_t)np * 24, pos, (size_t)np * 12))
        return fail(ctx, RECON_E_ARG, "grad_pos overlaps pos");
    return backward(ctx, grad_delta_r, grad_phi, nullptr, pos, grad_pos);
}

// ------------------------------------------------------------- stage calls

int recon_stage_normalize(recon_ctx *ctx, const double *rho, double *m)
{
    TRY(check_ctx(ctx));
    if (!rho || !m) return fail(ctx, RECON_E_ARG, "null array");
    return normalize(ctx, rho, m, nullptr);
}

int recon_stage_cic(recon_ctx *ctx, const float *pos, long long np, double box, double *rho)
{
    TRY(check_ctx(ctx));
    if (!pos || !rho || np < 0 || !(box > 0.0) || !std::isfinite(box))
        return fail(ctx, RECON_E_ARG, "bad particle arguments");
    if (overlap(rho, ctx->n3 * 8, pos, (size_t)np * 12)) return fail(ctx, RECON_E_ARG, "rho overlaps pos");
    HIPCHK(launch_zero(rho, ctx->n3 * 8, ctx->stream));
    if (np > 0) HIPCHK(launch_cic(pos, np, ctx->n, box, rho, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

static int outer_variant_ok(recon_ctx *ctx, int variant)
{
    if (variant < 0 || variant > 2) return fail(ctx, RECON_E_ARG, "bad variant");
    if (variant == 2 && !outer25_supported(ctx->n))
        return fail(ctx, RECON_E_ARG, "the streaming outer-step passes need an edge that is a multiple of 64");
    return RECON_OK;
}

int recon_stage_meshmass(recon_ctx *ctx, const double *phi, const double *m, double *M, int variant)
{
    TRY(check_ctx(ctx));
    if (!phi || !m || !M) return fail(ctx, RECON_E_ARG, "null array");
    const size_t F = ctx->n3 * 8;
    if (overlap(M, F, phi, F) || overlap(M, F, m, F)) return fail(ctx, RECON_E_ARG, "M overlaps phi or m");
    TRY(outer_variant_ok(ctx, variant));
    HIPCHK(meshmass_pass(phi, m, M, ctx->n, ctx->part, ctx->stream, variant));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_source(recon_ctx *ctx, const double *phi, const double *M, double *b, double *rms_sigma, int variant)
{
    TRY(check_ctx(ctx));
    if (!phi || !M || !b) return fail(ctx, RECON_E_ARG, "null array");
    TRY(outer_variant_ok(ctx, variant));
    double v[2];
    HIPCHK(launch_sum(M, ctx->n3, ctx->part, ctx->stream));
    TRY(fetch_sum(ctx, v));
    const double rho_bar = v[0] / (double)ctx->n3;
    HIPCHK(source_pass(phi, M, rho_bar, ctx->cfg.xi_m, ctx->cfg.v_m, ctx->t, ctx->n, ctx->part, ctx->stream,
                       variant));
    TRY(fetch_sum(ctx, v));
    if (rms_sigma) *rms_sigma = std::sqrt(v[0] / (double)ctx->n3);
    HIPCHK(smooth_pass(ctx->t, b, ctx->n, ctx->cfg.smooth_center, v[1] / (double)ctx->n3, ctx->stream, variant));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_smooth(recon_ctx *ctx, const double *f, double *out, int variant)
{
    TRY(check_ctx(ctx));
    if (!f || !out) return fail(ctx, RECON_E_ARG, "null array");
    if (overlap(out, ctx->n3 * 8, f, ctx->n3 * 8)) return fail(ctx, RECON_E_ARG, "out overlaps f");
    TRY(outer_variant_ok(ctx, variant));
    HIPCHK(smooth_pass(f, out, ctx->n, ctx->cfg.smooth_center, 0.0, ctx->stream, variant));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

static bool level_ok(recon_ctx *ctx, int nl)
{
    for (int l = 0; l < ctx->L64.L; ++l)
        if (ctx->L64.n[l] == nl) return true;
    return false;
}

int recon_stage_apply(recon_ctx *ctx, const double *u, const double *a, int nl, double scale, double *out)
{
    TRY(check_ctx(ctx));
    if (!u || !a || !out || !level_ok(ctx, nl)) return fail(ctx, RECON_E_ARG, "bad arguments");
    const size_t L = (size_t)nl * nl * nl * 8;
    if (overlap(out, L, u, L) || overlap(out, L, a, L)) return fail(ctx, RECON_E_ARG, "out overlaps u or a");
    HIPCHK(launch_apply<double>(u, a, out, nl, scale, ctx->cfg.a_min, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_residual(recon_ctx *ctx, const void *u, const void *a, const void *b, int nl, double scale, void *r,
                         int dtype, int variant)
{
    TRY(check_ctx(ctx));
    if (!u || !a || !b || !r || !level_ok(ctx, nl) || (dtype != 0 && dtype != 1) || variant < 0 || variant > 2)
        return fail(ctx, RECON_E_ARG, "bad arguments");
    {
        const size_t L = (size_t)nl * nl * nl * (dtype ? 4 : 8);
        if (overlap(r, L, u, L) || overlap(r, L, a, L) || overlap(r, L, b, L))
            return fail(ctx, RECON_E_ARG, "r overlaps u, a or b");
    }
    if (variant == 2 && !(dtype == 0 ? stencil25_supported<double>(nl) : stencil25_supported<float>(nl)))
        return fail(ctx, RECON_E_ARG, "the streaming residual needs an edge that is a multiple of 128");
    if (dtype == 0)
        HIPCHK(residual_level<double>((const double *)u, (const double *)a, (const double *)b, (double *)r, nl, scale,
                                      ctx->cfg.a_min, ctx->stream, variant));
    else
        HIPCHK(residual_level<float>((const float *)u, (const float *)a, (const float *)b, (float *)r, nl,
                                     (float)scale, (float)ctx->cfg.a_min, ctx->stream, variant));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_direction(recon_ctx *ctx, const void *z, int z_dtype, const void *p_old, const double *a,
                          double beta, int first, void *p_new, double *q, double *pq, int variant, double *u,
                          double alpha_u, int p_dtype)
{
    TRY(check_ctx(ctx));
    const int n = ctx->n;
    const long n3 = ctx->n3;
    if (!z || !a || !p_new || !q || !pq || (!first && !p_old) || (z_dtype != 0 && z_dtype != 1) || variant < 0 ||
        variant > 2 || (p_old && p_old == p_new) || (void *)q == p_new || (p_dtype != 0 && p_dtype != 1) ||
        (u && (first || (const void *)u == p_old || (void *)u == p_new || u == q || u == a || (const void *)u == z)))
        return fail(ctx, RECON_E_ARG, "bad arguments");
    {
        const size_t F = (size_t)n3 * 8, Z = (size_t)n3 * (z_dtype ? 4 : 8), P = (size_t)n3 * (p_dtype ? 4 : 8);
        const void *po = first ? nullptr : p_old;
        if (overlap(q, F, z, Z) || overlap(q, F, po, P) || overlap(q, F, a, F) || overlap(q, F, p_new, P) ||
            overlap(p_new, P, z, Z) || overlap(p_new, P, po, P) || overlap(p_new, P, a, F) ||
            (u && (overlap(u, F, z, Z) || overlap(u, F, po, P) || overlap(u, F, a, F) || overlap(u, F, p_new, P) ||
                   overlap(u, F, q, F))))
            return fail(ctx, RECON_E_ARG, "the outputs overlap each other or the inputs");
    }
    const bool stream = variant == 2 || (variant == 0 && use_stream<double>(n));
    if (stream && !stencil25_supported<double>(n))
        return fail(ctx, RECON_E_ARG, "the streaming direction update needs an edge that is a multiple of 128");
    if (p_dtype == 1 && (!stream || z_dtype != 1))
        return fail(ctx, RECON_E_ARG, "FP32 directions need an FP32 z and the streaming kernel");
    if (stream) {
        const void *po = first ? (const void *)q : p_old;  // not read when first; any array other than p_new
        if (p_dtype == 1)
            HIPCHK(launch_direction25((const float *)z, (const float *)po, (float *)p_new, a, q, beta, n,
                                      ctx->cfg.a_min, first != 0, u, alpha_u, nullptr, ctx->part, ctx->stream));
        else if (z_dtype == 0)
            HIPCHK(launch_direction25((const double *)z, (const double *)po, (double *)p_new, a, q, beta, n,
                                      ctx->cfg.a_min, first != 0, u, alpha_u, nullptr, ctx->part, ctx->stream));
        else
            HIPCHK(launch_direction25((const float *)z, (const double *)po, (double *)p_new, a, q, beta, n,
                                      ctx->cfg.a_min, first != 0, u, alpha_u, nullptr, ctx->part, ctx->stream));
    } else {
        double *pn = (double *)p_new;
        if (u) HIPCHK(launch_axpy(u, (const double *)p_old, alpha_u, n3, ctx->stream));
        if (!first) HIPCHK(launch_copy(pn, (const double *)p_old, n3, ctx->stream));
        if (z_dtype == 0)
            HIPCHK(launch_update_pq<double>((const double *)z, a, pn, q, beta, n, ctx->cfg.a_min, first != 0,
                                            nullptr, ctx->part, ctx->stream));
        else
            HIPCHK(launch_update_pq<float>((const float *)z, a, pn, q, beta, n, ctx->cfg.a_min, first != 0,
                                           nullptr, ctx->part, ctx->stream));
    }
    return fetch_sum(ctx, pq);
}

int recon_stage_full_residual(recon_ctx *ctx, const double *phi, const double *M, const double *u, const double *b,
                              double *r, float *r32, double *rr, int variant)
{
    TRY(check_ctx(ctx));
    const int n = ctx->n;
    if (!phi || !M || !u || !b || !r || !rr || variant < 0 || variant > 2 || r == u || r == b)
        return fail(ctx, RECON_E_ARG, "bad arguments");
    {
        const size_t F = ctx->n3 * 8, H = ctx->n3 * 4;
        if (overlap(r, F, phi, F) || overlap(r, F, M, F) || overlap(r, F, u, F) || overlap(r, F, b, F) ||
            overlap(r32, H, phi, F) || overlap(r32, H, M, F) || overlap(r32, H, u, F) || overlap(r32, H, b, F) ||
            overlap(r32, H, r, F))
            return fail(ctx, RECON_E_ARG, "r or r32 overlaps an input or each other");
    }
    if (!ctx->cfg.full_operator) return fail(ctx, RECON_E_ARG, "the context was made without full_operator");
    const bool stream = variant == 2 || (variant == 0 && use_stream<double>(n) && full25_supported(n));
    if (stream && !full25_supported(n))
        return fail(ctx, RECON_E_ARG, "the streaming full operator needs an edge that is a multiple of 64");
    HIPCHK(launch_mass_tensor(phi, M, ctx->Kf, n, ctx->stream));
    if (stream) HIPCHK(launch_full_residual_norm25(ctx->Kf, u, b, r, r32, n, ctx->cfg.a_min, ctx->part, ctx->stream));
    else HIPCHK(launch_full_residual_norm(ctx->Kf, u, b, r, r32, n, ctx->cfg.a_min, ctx->part, ctx->stream));
    return fetch_sum(ctx, rr);
}

int recon_stage_full_direction(recon_ctx *ctx, const double *phi, const double *M, const void *z, int z_dtype,
                               const void *p_old, double beta, int first, void *p_new, double *q, double *pq,
                               int variant, double *u, double alpha_u, int p_dtype)
{
    TRY(check_ctx(ctx));
    const int n = ctx->n;
    const long n3 = ctx->n3;
    if (!phi || !M || !z || !p_new || !q || !pq || (!first && !p_old) || (z_dtype != 0 && z_dtype != 1) ||
        variant < 0 || variant > 2 || (p_old && p_old == p_new) || (void *)q == p_new ||
        (p_dtype != 0 && p_dtype != 1) ||
        (u && (first || (const void *)u == p_old || (void *)u == p_new || u == q || (const void *)u == z)))
        return fail(ctx, RECON_E_ARG, "bad arguments");
    {
        const size_t F = (size_t)n3 * 8, Z = (size_t)n3 * (z_dtype ? 4 : 8), P = (size_t)n3 * (p_dtype ? 4 : 8);
        const void *po = first ? nullptr : p_old;
        auto hits = [&](const void *o, size_t no) {
            return overlap(o, no, z, Z) || overlap(o, no, po, P) || overlap(o, no, phi, F) || overlap(o, no, M, F);
        };
        if (hits(q, F) || hits(p_new, P) || overlap(q, F, p_new, P) ||
            (u && (hits(u, F) || overlap(u, F, p_new, P) || overlap(u, F, q, F))))
            return fail(ctx, RECON_E_ARG, "the outputs overlap each other or the inputs");
    }
    if (!ctx->cfg.full_operator) return fail(ctx, RECON_E_ARG, "the context was made without full_operator");
    const bool stream = variant == 2 || (variant == 0 && use_stream<double>(n) && full25_supported(n));
    if (stream && !full25_supported(n))
        return fail(ctx, RECON_E_ARG, "the streaming full operator needs an edge that is a multiple of 64");
    if (p_dtype == 1 && (!stream || z_dtype != 1))
        return fail(ctx, RECON_E_ARG, "FP32 directions need an FP32 z and the streaming kernel");
    HIPCHK(launch_mass_tensor(phi, M, ctx->Kf, n, ctx->stream));
    if (stream) {
        const void *po = first ? (const void *)q : p_old;  // not read when first; any array other than p_new
        if (p_dtype == 1)
            HIPCHK(launch_full_direction25((const float *)z, (const float *)po, (float *)p_new, ctx->Kf, q, beta, n,
                                           ctx->cfg.a_min, first != 0, u, alpha_u, nullptr, ctx->part, ctx->stream));
        else if (z_dtype == 0)
            HIPCHK(launch_full_direction25((const double *)z, (const double *)po, (double *)p_new, ctx->Kf, q, beta,
                                           n, ctx->cfg.a_min, first != 0, u, alpha_u, nullptr, ctx->part, ctx->stream));
        else
            HIPCHK(launch_full_direction25((const float *)z, (const double *)po, (double *)p_new, ctx->Kf, q, beta,
                                           n, ctx->cfg.a_min, first != 0, u, alpha_u, nullptr, ctx->part, ctx->stream));
    } else {
        double *pn = (double *)p_new;
        if (u) HIPCHK(launch_axpy(u, (const double *)p_old, alpha_u, n3, ctx->stream));
        if (!first) HIPCHK(launch_copy(pn, (const double *)p_old, n3, ctx->stream));
        if (z_dtype == 0)
            HIPCHK(launch_update_p<double>((const double *)z, pn, beta, n3, first != 0, nullptr, ctx->stream));
        else
            HIPCHK(launch_update_p<float>((const float *)z, pn, beta, n3, first != 0, nullptr, ctx->stream));
        HIPCHK(launch_full_apply_dot(ctx->Kf, pn, q, n, ctx->cfg.a_min, ctx->part, ctx->stream));
    }
    return fetch_sum(ctx, pq);
}

extern "C++" {
template <typename T>
static int stage_rbgs_fused(recon_ctx *ctx, T *u, const T *a, const T *b, int nl, double scale, int first)
{
    T *scratch = reinterpret_cast<T *>(ctx->t);  // n^3 doubles >= nl^3 values of T
    HIPCHK(launch_rbgs_fused<T>(u, scratch, a, b, nl, (T)scale, (T)ctx->cfg.a_min, first, false, ctx->stream));
    HIPCHK(hipMemcpyAsync(u, scratch, (size_t)nl * nl * nl * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    return RECON_OK;
}
}

int recon_stage_rbgs(recon_ctx *ctx, void *u, const void *a, const void *b, int nl, double scale, int first, int dtype,
                     int variant)
{
    TRY(check_ctx(ctx));
    if (!u || !a || !b || !level_ok(ctx, nl) || (dtype != 0 && dtype != 1) || (first != 0 && first != 1) ||
        variant < 0 || variant > 2)
        return fail(ctx, RECON_E_ARG, "bad arguments");
    {
        const size_t L = (size_t)nl * nl * nl * (dtype ? 4 : 8);
        if (overlap(u, L, a, L) || overlap(u, L, b, L)) return fail(ctx, RECON_E_ARG, "u overlaps a or b");
    }
    const bool can_fuse = dtype == 0 ? rbgs_fused_supported<double>(nl) : rbgs_fused_supported<float>(nl);
    if (variant == 2 && !can_fuse)
        return fail(ctx, RECON_E_ARG, "the fused sweep needs an edge that is a multiple of 16");
    const bool fused = variant == 2 || (variant == 0 && (dtype == 0 ? use_fused<double>(nl) : use_fused<float>(nl)));
    if (fused) {
        if (dtype == 0) TRY(stage_rbgs_fused<double>(ctx, (double *)u, (const double *)a, (const double *)b, nl, scale, first));
        else TRY(stage_rbgs_fused<float>(ctx, (float *)u, (const float *)a, (const float *)b, nl, scale, first));
    } else if (dtype == 0) {
        HIPCHK(launch_rbgs_half<double>((double *)u, (const double *)a, (const double *)b, nl, scale, ctx->cfg.a_min,
                                        first, false, ctx->stream));
        HIPCHK(launch_rbgs_half<double>((double *)u, (const double *)a, (const double *)b, nl, scale, ctx->cfg.a_min,
                                        1 - first, false, ctx->stream));
    } else {
        HIPCHK(launch_rbgs_half<float>((float *)u, (const float *)a, (const float *)b, nl, (float)scale,
                                       (float)ctx->cfg.a_min, first, false, ctx->stream));
        HIPCHK(launch_rbgs_half<float>((float *)u, (const float *)a, (const float *)b, nl, (float)scale,
                                       (float)ctx->cfg.a_min, 1 - first, false, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

extern "C++" {
template <typename T>
static int stage_prolong_sweep(recon_ctx *ctx, T *u, const T *e, const T *a, const T *b, int nl, double scale,
                               int first, int variant)
{
    T *scratch = reinterpret_cast<T *>(ctx->t);  // n^3 doubles >= nl^3 values of T
    if (variant == 1) {
        HIPCHK(prolong_level<T>(u, e, nl, ctx->stream));
        HIPCHK(launch_rbgs_fused<T>(u, scratch, a, b, nl, (T)scale, (T)ctx->cfg.a_min, first, false, ctx->stream));
    } else {
        HIPCHK(launch_rbgs_fused<T>(u, scratch, a, b, nl, (T)scale, (T)ctx->cfg.a_min, first, false, ctx->stream, e));
    }
    HIPCHK(hipMemcpyAsync(u, scratch, (size_t)nl * nl * nl * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}
}

int recon_stage_prolong_sweep(recon_ctx *ctx, void *u, const void *e, const void *a, const void *b, int nl,
                              double scale, int first, int dtype, int variant)
{
    TRY(check_ctx(ctx));
    if (!u || !e || !a || !b || !level_ok(ctx, nl) || nl % 2 || (dtype != 0 && dtype != 1) ||
        (first != 0 && first != 1) || (variant != 1 && variant != 2))
        return fail(ctx, RECON_E_ARG, "bad arguments");
    {
        const size_t L = (size_t)nl * nl * nl * (dtype ? 4 : 8), C = L / 8;
        if (overlap(u, L, e, C) || overlap(u, L, a, L) || overlap(u, L, b, L))
            return fail(ctx, RECON_E_ARG, "u overlaps e, a or b");
    }
    if (dtype == 0 ? !rbgs_fused_supported<double>(nl) : !rbgs_fused_supported<float>(nl))
        return fail(ctx, RECON_E_ARG, "the fused sweep needs an edge that is a multiple of 16");
    if (dtype == 0)
        return stage_prolong_sweep<double>(ctx, (double *)u, (const double *)e, (const double *)a, (const double *)b,
                                           nl, scale, first, variant);
    return stage_prolong_sweep<float>(ctx, (float *)u, (const float *)e, (const float *)a, (const float *)b, nl,
                                      scale, first, variant);
}

int recon_stage_restrict(recon_ctx *ctx, const void *f, int nl, void *c, int dtype, int variant)
{
    TRY(check_ctx(ctx));
    if (!f || !c || !level_ok(ctx, nl) || nl < 4 || (nl & 1) || (dtype != 0 && dtype != 1) || variant < 0 ||
        variant > 2)
        return fail(ctx, RECON_E_ARG, "bad arguments");
    if (overlap(c, (size_t)nl * nl * nl * (dtype ? 4 : 8) / 8, f, (size_t)nl * nl * nl * (dtype ? 4 : 8)))
        return fail(ctx, RECON_E_ARG, "c overlaps f");
    if (variant == 2 && !(dtype == 0 ? transfer25_supported<double>(nl) : transfer25_supported<float>(nl)))
        return fail(ctx, RECON_E_ARG, "the streaming transfers need a fine edge that is a multiple of 256");
    if (dtype == 0) HIPCHK(restrict_level<double>((const double *)f, (double *)c, nl, ctx->stream, variant));
    else HIPCHK(restrict_level<float>((const float *)f, (float *)c, nl, ctx->stream, variant));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_residual_restrict(recon_ctx *ctx, const void *u, const void *a, const void *b, int nl, double scale,
                                  void *c, int dtype, int variant)
{
    TRY(check_ctx(ctx));
    if (!u || !a || !b || !c || !level_ok(ctx, nl) || nl < 4 || (nl & 1) || (dtype != 0 && dtype != 1) ||
        variant < 0 || variant > 2)
        return fail(ctx, RECON_E_ARG, "bad arguments");
    {
        const size_t L = (size_t)nl * nl * nl * (dtype ? 4 : 8), C = L / 8;
        if (overlap(c, C, u, L) || overlap(c, C, a, L) || overlap(c, C, b, L))
            return fail(ctx, RECON_E_ARG, "c overlaps u, a or b");
    }
    if (variant == 2 && !(dtype == 0 ? resrestrict25_supported<double>(nl) : resrestrict25_supported<float>(nl)))
        return fail(ctx, RECON_E_ARG, "the fused residual-restriction needs a coarse edge that is a multiple of 32");
    if (dtype == 0)
        HIPCHK(coarse_rhs<double>((const double *)u, (const double *)a, (const double *)b, ctx->t, (double *)c, nl,
                                  scale, ctx->cfg.a_min, ctx->stream, variant));
    else
        HIPCHK(coarse_rhs<float>((const float *)u, (const float *)a, (const float *)b, reinterpret_cast<float *>(ctx->t),
                                 (float *)c, nl, (float)scale, (float)ctx->cfg.a_min, ctx->stream, variant));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_prolong_add(recon_ctx *ctx, void *u, const void *e, int nl, int dtype, int variant)
{
    TRY(check_ctx(ctx));
    if (!u || !e || !level_ok(ctx, nl) || nl < 4 || (nl & 1) || (dtype != 0 && dtype != 1) || variant < 0 ||
        variant > 2)
        return fail(ctx, RECON_E_ARG, "bad arguments");
    if (overlap(u, (size_t)nl * nl * nl * (dtype ? 4 : 8), e, (size_t)nl * nl * nl * (dtype ? 4 : 8) / 8))
        return fail(ctx, RECON_E_ARG, "u overlaps e");
    if (variant == 2 && !(dtype == 0 ? transfer25_supported<double>(nl) : transfer25_supported<float>(nl)))
        return fail(ctx, RECON_E_ARG, "the streaming transfers need a fine edge that is a multiple of 256");
    if (dtype == 0) HIPCHK(prolong_level<double>((double *)u, (const double *)e, nl, ctx->stream, variant));
    else HIPCHK(prolong_level<float>((float *)u, (const float *)e, nl, ctx->stream, variant));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_vcycle(recon_ctx *ctx, const void *a, const void *r, void *z, int dtype)
{
    TRY(check_ctx(ctx));
    if (!a || !r || !z || (dtype != 0 && dtype != 1)) return fail(ctx, RECON_E_ARG, "bad arguments");
    if (overlap(z, ctx->n3 * (dtype ? 4 : 8), r, ctx->n3 * (dtype ? 4 : 8))) return fail(ctx, RECON_E_ARG, "z overlaps r");
    if (dtype == 1 && ctx->cfg.precision != RECON_MIXED)
        return fail(ctx, RECON_E_ARG, "FP32 V-cycle needs a context created with precision RECON_MIXED");
    const long n3 = ctx->n3;
    if (dtype == 0) {
        HIPCHK(launch_copy(ctx->M, (const double *)a, n3, ctx->stream));
        recon_config saved = ctx->cfg;
        ctx->cfg.precision = RECON_FP64;
        int rc = build_hierarchy(ctx, ctx->M);
        ctx->cfg = saved;
        TRY(rc);
        TRY(vcycle<double>(ctx, ctx->L64, 0, (const double *)r, (double *)z));
    } else {
        // FP32 coefficient given: build the FP32 hierarchy directly
        Levels<float> &S = ctx->L32;
        HIPCHK(hipMemcpyAsync(S.a[0], a, n3 * 4, hipMemcpyDeviceToDevice, ctx->stream));
        for (int l = 0; l + 1 < S.L; ++l) HIPCHK(launch_restrict<float>(S.a[l], S.a[l + 1], S.n[l], ctx->stream));
        TRY(vcycle<float>(ctx, S, 0, (const float *)r, (float *)z));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_mg_solve(recon_ctx *ctx, const double *a, const double *b, double tol, double *u, int *cycles,
                         double *rel_residual)
{
    TRY(check_ctx(ctx));
    if (!a || !b || !u || !(tol > 0.0)) return fail(ctx, RECON_E_ARG, "bad arguments");
    HIPCHK(launch_copy(ctx->M, a, ctx->n3, ctx->stream));
    TRY(build_hierarchy(ctx, ctx->M));
    TRY(mg_solve(ctx, ctx->M, b, tol, cycles, rel_residual));
    HIPCHK(launch_copy(u, ctx->u, ctx->n3, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_mg_solve_full(recon_ctx *ctx, const double *a, const double *phi, const double *b, double tol,
                              double *u, int *cycles, double *rel_residual)
{
    TRY(check_ctx(ctx));
    if (!a || !phi || !b || !u || !(tol > 0.0)) return fail(ctx, RECON_E_ARG, "bad arguments");
    if (!ctx->cfg.full_operator) return fail(ctx, RECON_E_ARG, "the context was made without full_operator");
    HIPCHK(launch_copy(ctx->M, a, ctx->n3, ctx->stream));
    HIPCHK(launch_mass_tensor(phi, ctx->M, ctx->Kf, ctx->n, ctx->stream));
    TRY(build_hierarchy(ctx, ctx->Kf.tr));
    TRY(mg_solve(ctx, ctx->Kf.tr, b, tol, cycles, rel_residual, false, &ctx->Kf));
    HIPCHK(launch_copy(u, ctx->u, ctx->n3, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_choose_step(recon_ctx *ctx, const double *phi, const double *dphi, double *alpha)
{
    TRY(check_ctx(ctx));
    if (!phi || !dphi || !alpha) return fail(ctx, RECON_E_ARG, "null argument");
    return choose_step(ctx, phi, dphi, alpha);
}

int recon_stage_pd_count(recon_ctx *ctx, const double *phi, const double *dphi, int j0, int ntrial, int variant,
                         double *counts, const double *M, const double *D)
{
    TRY(check_ctx(ctx));
    if (!phi || !dphi || !counts || j0 < 0 || j0 > 1000 || (ntrial != 1 && ntrial != 4) || variant < 0 ||
        variant > 2 || (M == nullptr) != (D == nullptr))
        return fail(ctx, RECON_E_ARG, "bad arguments");
    if (variant == 2 && !pd25_supported(ctx->n))
        return fail(ctx, RECON_E_ARG, "the streaming step trials need an edge that is a multiple of 64");
    double v[8];
    HIPCHK(pd_trials(ctx, phi, dphi, j0, ntrial, variant, M, D));
    TRY(fetch_sum(ctx, v));
    for (int t = 0; t < ntrial; ++t) counts[t] = v[t];
    return RECON_OK;
}

int recon_stage_mass_change(recon_ctx *ctx, const double *phi, const double *M, const double *f, double *out)
{
    TRY(check_ctx(ctx));
    if (!phi || !M || !f || !out) return fail(ctx, RECON_E_ARG, "null array");
    {
        const size_t F = ctx->n3 * 8;
        if (overlap(out, F, phi, F) || overlap(out, F, M, F) || overlap(out, F, f, F))
            return fail(ctx, RECON_E_ARG, "out overlaps phi, M or f");
    }
    const MassTensor K{ctx->t, ctx->b, ctx->r, ctx->z, ctx->p, ctx->q, nullptr};
    HIPCHK(launch_mass_change(phi, M, f, K, out, ctx->n, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_invert_map(recon_ctx *ctx, const double *phi, const float *pos, long long np, double box, double *xi,
                           double *failed)
{
    TRY(check_ctx(ctx));
    if (!phi || !pos || np <= 0 || !(box > 0.0) || !std::isfinite(box) || !xi || !failed)
        return fail(ctx, RECON_E_ARG, "bad arguments");
    if (overlap(xi, (size_t)np * 24, phi, ctx->n3 * 8) || overlap(xi, (size_t)np * 24, pos, (size_t)np * 12))
        return fail(ctx, RECON_E_ARG, "xi overlaps phi or pos");
    // the node shifts need 3 n^3 contiguous doubles: the particle deposit's
    // own buffer, else r, z and p where they lie back to back
    double *s3 = ctx->shifts;
    if (!s3 && ctx->z == ctx->r + ctx->n3 && ctx->p == ctx->r + 2 * ctx->n3) s3 = ctx->r;
    if (!s3) return fail(ctx, RECON_E_ARG, "no room for the node shifts: make the context with particle_deposit = 1");
    double v[1];
    HIPCHK(launch_invert_map(phi, pos, np, ctx->n, box, xi, s3, kInvertIters, kInvertTol, ctx->part, ctx->stream));
    TRY(fetch_sum(ctx, v));
    *failed = v[0];
    return RECON_OK;
}

int recon_stage_deposit_xi(recon_ctx *ctx, const double *xi, long long np, double *M)
{
    TRY(check_ctx(ctx));
    if (!xi || np <= 0 || !M) return fail(ctx, RECON_E_ARG, "bad arguments");
    if (overlap(M, ctx->n3 * 8, xi, (size_t)np * 24)) return fail(ctx, RECON_E_ARG, "M overlaps xi");
    HIPCHK(launch_deposit_xi(xi, np, ctx->n, M, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

int recon_stage_delta_r(recon_ctx *ctx, const double *phi, double *delta)
{
    TRY(check_ctx(ctx));
    if (!phi || !delta) return fail(ctx, RECON_E_ARG, "null array");
    if (overlap(delta, ctx->n3 * 8, phi, ctx->n3 * 8)) return fail(ctx, RECON_E_ARG, "delta overlaps phi");
    HIPCHK(launch_output(phi, delta, nullptr, 1.0, ctx->n, ctx->part, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RECON_OK;
}

}  // extern "C"
