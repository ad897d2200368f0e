// Internal launch interface of the gfx950 kernels (not part of the C ABI).
// Every launcher enqueues on `s` and returns hipGetLastError().
#pragma once
#include <hip/hip_runtime.h>

namespace recon {

// Reductions: kernels that reduce write one row of K partials per block into
// `part` (capacity kPartCap doubles); reduce_finalize() then folds the rows
// in a fixed order into out[0..K).  Results are bitwise reproducible for a
// given launch shape.
constexpr long kPartCap = 1L << 21;

// Device-resident scalars of the conjugate-gradient loop (8 doubles): the dot
// products land here from the reductions, and the kernels that need the step
// sizes form them from these values themselves, so the host reads back only
// what its stop test needs.
enum KrylovScalar {
    KS_RZ = 0,      // z . r of the current step (written by the reduction)
    KS_ZQ = 1,      // z . q_old (written with KS_RZ)
    KS_PQ = 2,      // p . q
    KS_RR = 3,      // ||r||^2 after the update
    KS_ALPHA = 4,   // alpha = rz / pq (written by the residual update)
    KS_RZ_OLD = 5,  // rz of the previous step (written by the residual update)
    KS_COUNT = 8
};
enum RedOp { RED_SUM = 0, RED_MAX = 1, RED_MIN = 2 };

struct Part {
    double *part;   // device partials
    int blocks;     // rows written by the last reducing launch
    int k;          // partials per row
};

hipError_t reduce_finalize(const Part &p, const int *ops, double *out, hipStream_t s);

// ---------------------------------------------------------------- input
hipError_t launch_check_input(const double *rho, long n3, Part &p, hipStream_t s);  // K=2: sum, bad count
hipError_t launch_scale(const double *rho, double *m, long n3, const double *mean_dev, hipStream_t s);
hipError_t launch_fill(double *f, long n3, double v, hipStream_t s);
hipError_t launch_zero(void *f, long bytes, hipStream_t s);
hipError_t launch_copy(double *dst, const double *src, long n3, hipStream_t s);
hipError_t launch_cic(const float *pos, long long np, int n, double box, double *rho, hipStream_t s);

// ------------------------------------------------------- outer-step kernels
// M = det(I + H) * CIC(m)(x); partial K=1: sum M
hipError_t launch_meshmass(const double *phi, const double *m, double *M, int n, Part &p, hipStream_t s);
// t = Sigma + C + E; partials K=2: sum Sigma^2, sum t
hipError_t launch_source(const double *phi, const double *M, double rho_bar, double xi_m, double v_m, double *t, int n,
                         Part &p, hipStream_t s);
// out = c0 f + (1-c0)/6 sum nb - sub
hipError_t launch_smooth(const double *f, double *out, int n, double c0, double sub, hipStream_t s);
// the same three passes with the stencil field streamed through LDS (outer25.hip);
// n a multiple of 64; the same node values, the partial sums grouped per workgroup
bool outer25_supported(int n);
hipError_t launch_meshmass25(const double *phi, const double *m, double *M, int n, Part &p, hipStream_t s);
hipError_t launch_source25(const double *phi, const double *M, double rho_bar, double xi_m, double v_m, double *t,
                           int n, Part &p, hipStream_t s);
hipError_t launch_smooth25(const double *f, double *out, int n, double c0, double sub, hipStream_t s);
// partial K=1 (max): max_a |D_c f|
hipError_t launch_max_shift(const double *f, int n, Part &p, hipStream_t s);
// partial K=ntrial (sum): nodes where I + Hess(phi + 2^-j dphi) is not PD, j = j0..j0+ntrial-1;
// with M and D non-null a node also fails where M + 2^-j D > 0 does not hold
hipError_t launch_pd_trials(const double *phi, const double *dphi, int n, int j0, int ntrial, Part &p,
                            hipStream_t s, const double *M = nullptr, const double *D = nullptr);
// same counts from planes streamed through LDS; n a multiple of 64
bool pd25_supported(int n);
hipError_t launch_pd25(const double *phi, const double *dphi, int n, int j0, int ntrial, Part &p, hipStream_t s,
                       const double *M = nullptr, const double *D = nullptr);
// The exact mass change of a step (massupdate.hip): out = div(K grad f) with
// K = M (I + Hess phi)^{-1}, its six components stored in K's fields.
struct MassTensor {
    double *xx, *yy, *zz, *xy, *xz, *yz;
    double *tr;  // optional: the mean diagonal (xx + yy + zz) / 3
};
hipError_t launch_mass_change(const double *phi, const double *M, const double *f, const MassTensor &K,
                              double *out, int n, hipStream_t s);
// K = M e^-1 at every node; out = L_K f (the exact mass change: no floor);
// q = L_K p with partial K=1 sum p.q; r = b - L_K u (optional FP32 copy r32)
// with partial K=1 sum r^2.  a_min > 0 floors the diagonal face coefficients
// (the exact-Jacobian solve's operator).
hipError_t launch_mass_tensor(const double *phi, const double *M, const MassTensor &K, int n, hipStream_t s);
hipError_t launch_full_apply(const MassTensor &K, const double *f, double *out, int n, hipStream_t s);
hipError_t launch_full_apply_dot(const MassTensor &K, const double *pv, double *q, int n, double a_min, Part &p,
                                 hipStream_t s);
hipError_t launch_full_residual_norm(const MassTensor &K, const double *u, const double *b, double *r, float *r32,
                                     int n, double a_min, Part &p, hipStream_t s);
// Streaming forms of the last two (fullop25.hip; edges that are multiples of
// 64): the residual with its norm, and the Krylov direction p_new = z + beta
// p_old (first: z; beta from ks as in launch_direction25; rounded to P) fused
// with q = L_K p_new and partial K=1 sum p_new.q, and with u += alpha_u p_old
// when u != null (not first).  p_new must not alias p_old, u or q.
bool full25_supported(int n);
// out = L_K f in one streaming pass (out distinct from f)
hipError_t launch_full_apply25(const MassTensor &K, const double *f, double *out, int n, double a_min, hipStream_t s);
hipError_t launch_full_residual_norm25(const MassTensor &K, const double *u, const double *b, double *r, float *r32,
                                       int n, double a_min, Part &p, hipStream_t s);
template <typename Z, typename P>
hipError_t launch_full_direction25(const Z *z, const P *p_old, P *p_new, const MassTensor &K, double *q, double beta,
                                   int n, double a_min, bool first, double *u, double alpha_u, const double *ks,
                                   Part &p, hipStream_t s);
// Particles at their Lagrangian positions (particles.hip): xi = pos n / box;
// Newton for x(xi) = y from the xi given (node shifts of phi into s3, 3 n^3
// doubles;
// partial K=1: particles not within tol); CIC of the particles at xi into M
// (zeroed first), n^3 / np each.
hipError_t launch_init_xi(const float *pos, long long np, int n, double box, double *xi, hipStream_t s);
hipError_t launch_invert_map(const double *phi, const float *pos, long long np, int n, double box, double *xi,
                             double *s3, int max_iter, double tol, Part &p, hipStream_t s);
hipError_t launch_deposit_xi(const double *xi, long long np, int n, double *M, hipStream_t s);
// s = D_c phi, three components per node side by side (3 n^3 doubles); the
// adjoint of the deposit at the Lagrangian positions xi (node shifts s3 of the
// same phi): gpos (3 per particle) +=
// gscale lam, sbar (three fields, x then y then z) -= W lam with atomics
hipError_t launch_node_shifts(const double *phi, double *s3, int n, hipStream_t s);
hipError_t launch_deposit_adj(const double *xi, long long np, int n, const double *s3, const double *Mbar,
                              double *sbar, double *gpos, double gscale, hipStream_t s);
// y += alpha x, X = double or float; with alpha_dev != null alpha is read there
template <typename X>
hipError_t launch_axpy(double *y, const X *x, double alpha, long n3, hipStream_t s,
                       const double *alpha_dev = nullptr);
hipError_t launch_add_scalar(double *y, const double *c_dev, double sign, double scale, long n3, hipStream_t s);
// delta = -L7 phi; phi_out = phi * h2 (if non-null); partials K=3: min det, min lambda0, max delta
hipError_t launch_output(const double *phi, double *delta, double *phi_out, double h2, int n, Part &p,
                         hipStream_t s);
hipError_t launch_sum(const double *f, long n3, Part &p, hipStream_t s);  // K=1 sum

// ------------------------------------------------------------- multigrid
// scale = 4^-l.  T = double or float.
template <typename T>
hipError_t launch_apply(const T *u, const T *a, T *out, int n, T scale, T a_min, hipStream_t s);
template <typename T>
hipError_t launch_rbgs_half(T *u, const T *a, const T *b, int n, T scale, T a_min, int colour, bool zero_init,
                            hipStream_t s, bool fine = false);
// fused two-colour sweep, out of place: u_out = sweep(u_in); colour `first`
// first.  With e (the coarse-grid correction, edge n/2; not with zero_init):
// u_out = sweep(u_in + P e), P the trilinear prolongation.
template <typename T>
hipError_t launch_rbgs_fused(const T *u_in, T *u_out, const T *a, const T *b, int n, T scale, T a_min, int first,
                             bool zero_init, hipStream_t s, const T *e = nullptr);
template <typename T>
bool rbgs_fused_supported(int n);
template <typename T>
hipError_t launch_residual(const T *u, const T *a, const T *b, T *r, int n, T scale, T a_min, hipStream_t s);
template <typename T>
hipError_t launch_restrict(const T *f, T *c, int n, hipStream_t s);
template <typename T>
hipError_t launch_prolong_add(T *u, const T *e, int n, hipStream_t s);
template <typename T>
hipError_t launch_coarse_solve(T *u, const T *a, const T *b, int n, T scale, T a_min, int pairs, hipStream_t s);
hipError_t launch_cast_f32(const double *src, float *dst, long n3, hipStream_t s);
hipError_t launch_cast_f64(const float *src, double *dst, long n3, hipStream_t s);

// ------------------------------------------------------------ Krylov (FP64)
// r = b - A u (FP64) with partial K=1 sum r^2; writes r32 = (float) r if r32 != null
// LDS-streaming variants (stencil25.hip): edge a multiple of 128 (FP32 and
// FP64) and of the j-tile.  launch_direction25 writes p_new = first ? z :
// z + beta p_old (p_new != p_old), q = A p_new and the partial sums of p_new.q;
// with u != null (not first) it also applies u += alpha_u p_old.
template <typename T>
bool stencil25_supported(int n);
template <typename T>
hipError_t launch_residual25(const T *u, const T *a, const T *b, T *r, int n, T scale, T a_min, hipStream_t s);
hipError_t launch_residual_norm25(const double *u, const double *a, const double *b, double *r, float *r32, int n,
                                  double a_min, Part &p, hipStream_t s);
// Streaming grid transfers (transfer25.hip): fine edge a multiple of 256.
template <typename T>
bool transfer25_supported(int n);
template <typename T>
hipError_t launch_restrict25(const T *f, T *c, int n, hipStream_t s);
template <typename T>
hipError_t launch_prolong25(T *u, const T *e, int n, hipStream_t s);
// c = R (b - scale A u) in one streaming pass (resrestrict25.hip): coarse edge
// n/2 a multiple of 32; the same values as the residual and restriction
// kernels one after the other
template <typename T>
bool resrestrict25_supported(int n);
template <typename T>
hipError_t launch_resrestrict25(const T *u, const T *a, const T *b, T *c, int n, T scale, T a_min, hipStream_t s);

// P: storage of p_old and p_new (double, or float with an FP32 z: p_new is
// rounded to FP32 as it is formed and q = A p_new uses the rounded value).
// With ks != null, beta = -ks[KS_ALPHA] ks[KS_ZQ] / ks[KS_RZ_OLD] and alpha_u =
// ks[KS_ALPHA] are read on the device instead of the host values.
template <typename Z, typename P>
hipError_t launch_direction25(const Z *z, const P *p_old, P *p_new, const double *a, double *q, double beta, int n,
                              double a_min, bool first, double *u, double alpha_u, const double *ks, Part &p,
                              hipStream_t s);

hipError_t launch_residual_norm(const double *u, const double *a, const double *b, double *r, float *r32, int n,
                                double a_min, Part &p, hipStream_t s);
// partials K=2: sum z*r, sum z*q (q may be null -> 0).  Z = double or float
template <typename Z>
hipError_t launch_dots_zr_zq(const Z *z, const double *r, const double *q, long n3, Part &p, hipStream_t s);
// p = z + beta p (first: p = z); with ks != null and not first,
// beta = -ks[KS_ALPHA] ks[KS_ZQ] / ks[KS_RZ_OLD]
template <typename Z>
hipError_t launch_update_p(const Z *z, double *pv, double beta, long n3, bool first, const double *ks, hipStream_t s);
// p = z + beta p; q = A z + beta q (first: p = z, q = A z); partial K=1: sum p*q
// beta from ks as for launch_direction25 when ks != null
template <typename Z>
hipError_t launch_update_pq(const Z *z, const double *a, double *pv, double *q, double beta, int n,
                            double a_min, bool first, const double *ks, Part &p, hipStream_t s);
// u += alpha p (if u != null); r -= alpha q; partial K=1: sum r^2; r32 = (float) r if r32 != null.
// With ks != null: alpha = ks[KS_RZ] / ks[KS_PQ], and the kernel stores it in
// ks[KS_ALPHA] and ks[KS_RZ] in ks[KS_RZ_OLD].
hipError_t launch_update_ur(double *u, double *r, const double *pv, const double *q, double alpha,
                            float *r32, long n3, double *ks, Part &p, hipStream_t s);
// u += z (Z = double or float)
template <typename Z>
hipError_t launch_add_correction(double *u, const Z *z, long n3, hipStream_t s);

// ------------------------------------------------------------ adjoint (FP64)
hipError_t launch_out_adj(const double *gd, const double *gp, double h2, double *phibar, int n, hipStream_t s);
hipError_t launch_smooth_scaled(const double *f, double *out, int n, double c0, double scale, hipStream_t s);
hipError_t launch_coefgrad(const double *lam, const double *u, const double *M, double a_min, double *Mbar, int n,
                           hipStream_t s);
// hb: 6 fields (xx, yy, zz, xy, xz, yz); partial K=1: sum of Sigmabar
hipError_t launch_source_adj(const double *phi, const double *M, double rho_bar, const double *tbar, double xi_m,
                             double v_m, double *Mbar, double *hb, int n, Part &p, hipStream_t s);
// xb: 3 fields; mbar accumulated with atomics
hipError_t launch_meshmass_adj(const double *phi, const double *m, const double *Mbar, double *hb, double *xb,
                               double *mbar, int n, hipStream_t s);
hipError_t launch_phibar_update(const double *hb, const double *xb, double *phibar, int n, hipStream_t s);
hipError_t launch_dot(const double *a, const double *b, long n3, Part &p, hipStream_t s);  // K=1
hipError_t launch_rho_grad(const double *mbar, double mm, double mu, double *g, long n3, hipStream_t s);

}  // namespace recon
