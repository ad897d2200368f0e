/*
 * FP64 CPU oracle for the nonlinear reconstruction of Zhu, Yu, Pen, Chen & Yu,
 * "Nonlinear reconstruction" (arXiv:1611.09638).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test suite, by the
 * smoke check and by the benchmark's CPU-baseline leg, and by nothing else.
 * It shares no source, header or generated table with the HIP library; the
 * two meet only through the seeded inputs the tests hand to both.
 *
 * It is written to be read against the paper: plain loops over the periodic
 * lattice, FP64 throughout, no blocking or fusion, sums taken plane by plane
 * in a fixed order.  OpenMP only splits the outer loop of element-wise work.
 *
 * Method (Sec. II and App. A):
 *   mapping   x = xi + grad phi                         (Eq. mapping)
 *   triad     e = dx/dxi = I + Hess phi, sqrt g = det e (App. A)
 *   deviation Sigma = rho_bar - rho sqrt g              (App. A, after Eq. elliptic_diff)
 *   solve     div(rho sqrt g grad phidot) = S(Sigma + C + E), with x ~ xi
 *                                                       (Eq. elliptic, App. A)
 *   increment dphi = S phidot; phi = sum of increments  (App. A, Sec. II)
 *   output    delta_r = -laplacian phi                  (Eq. rec)
 *
 * Readings of points the paper leaves open (all shared with the HIP path by
 * specification, not by code):
 *   - grid: vertex centred, periodic, grid units; value j sits at position j.
 *   - rho sqrt g on the current mesh: M_n = det(e_n) * CIC-interpolant of the
 *     normalised density at x_n = n + D_c phi (central differences).
 *   - Hessian: compact second differences; H_ab uses the 4-point cross stencil.
 *   - rho_bar = mean of M; C = 4 max(0, xi_m/lambda_0 - 1)^2;
 *     E = -2 [sqrt g > v_m] |Sigma|.
 *   - S f = c0 f + (1 - c0)/6 * (sum of the six nearest neighbours), c0 = 1/2.
 *   - operator (x ~ xi): flux form sum_faces c_f (u_nb - u_n) with face
 *     coefficient c_f = max(a_min, (M_n + M_nb)/2), scaled by 4^-l on level l.
 *   - multigrid: symmetric V(n_pre, n_post) cycles with red-black
 *     Gauss-Seidel (red = i+j+k even; pre-smoothing red then black,
 *     post-smoothing black then red), 27-point full-weighting restriction of
 *     residual and coefficient, trilinear prolongation (= 8 R^T), coarsest
 *     grid relaxed from zero on a zero-mean right-hand side by a palindromic
 *     red/black sequence.  The V-cycle preconditions conjugate gradients
 *     (default) or is iterated on its own; stop when ||b - A u||_2 <=
 *     tol ||b||_2; u made mean-free at the end.
 *   - step: alpha = 2^-j, first j with I + Hess(phi + alpha dphi) positive
 *     definite at every node (Sylvester) and max |alpha D_c dphi| <= s_max.
 *   - optional exact-Jacobian solve (full_operator = 1): the linear system is
 *     div(M e^-1 grad u) = b, the operator of Eq. elliptic_diff on the current
 *     mesh instead of the x ~ xi one (diagonal face coefficients floored at
 *     a_min like the x ~ xi operator's), solved by the same Krylov iteration
 *     with an x ~ xi V-cycle as preconditioner, whose coefficient is the
 *     mean diagonal (K^xx + K^yy + K^zz) / 3 of K = M e^-1.
 *   - optional particle deposit (particle_deposit = 1, particle input): each
 *     step, every particle's Lagrangian position xi_p with x(xi_p) = y_p is
 *     found by Newton's method on the continuous map x(xi) = xi + S(xi), S the
 *     trilinear interpolant of the node shifts D_c phi, and M is the CIC
 *     deposit of the particles at xi_p with weight n^3 / N_p (mass exact).
 *   - optional mass update of App. A (mass_update = 1): M is carried from step
 *     to step as M' = M + alpha L_full[dphi], with L_full f = div(M e^-1 grad f)
 *     (Eq. elliptic_diff) discretised in flux form (below), and the step must
 *     also keep M' > 0 at every node.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_INPUT (-2)
#define ORC_E_NOT_PD (-3)
#define ORC_E_NO_CONVERGENCE (-4)
#define ORC_E_NO_TAPE (-5)
#define ORC_E_NOMEM (-7)

#define ORC_MAX_STEPS 256

typedef struct {
    int max_outer;
    int n_pre, n_post;
    int coarse_n;
    int coarse_sweeps;
    int max_vcycles;
    int max_halvings;
    int record_tape;
    int solver;
    int warm_start;
    int mass_update; /* 0: M from the CIC gather each step; 1: M += alpha L_full[dphi] */
    int particle_deposit; /* particle input: 0 CIC onto the grid once, then the gather;
                             1 deposit the particles at their Lagrangian positions each step */
    int full_operator; /* 1: the linear solve uses div(M e^-1 grad .) (no x ~ xi), with an
                          x ~ xi V-cycle (coefficient: mean diagonal of M e^-1) as its
                          preconditioner */
    double tol;
    double outer_tol;
    double xi_m, v_m;
    double smooth_center;
    double s_max;
    double a_min;
} orc_config;

typedef struct {
    int outer_steps;
    int vcycles_total;
    int vcycles[ORC_MAX_STEPS];
    double alpha[ORC_MAX_STEPS];
    double rms_sigma[ORC_MAX_STEPS];
    double kappa[ORC_MAX_STEPS];
    double rel_residual[ORC_MAX_STEPS];
    double min_det, min_lambda0, max_delta_r;
} orc_stats;

/* ------------------------------------------------------------------ lattice */

static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

static inline long at(int n, int i, int j, int k)
{
    return ((long)wrap(i, n) * n + wrap(j, n)) * n + wrap(k, n);
}

static long cube(int n) { return (long)n * n * n; }

/* Sum of a field, plane by plane, planes added in order (fixed order). */
static double field_sum(const double *f, int n)
{
    double *plane = (double *)malloc(sizeof(double) * n);
    #pragma omp parallel for
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (long q = 0; q < (long)n * n; ++q) s += f[(long)i * n * n + q];
        plane[i] = s;
    }
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += plane[i];
    free(plane);
    return s;
}

static double field_dot(const double *f, const double *g, int n)
{
    double *plane = (double *)malloc(sizeof(double) * n);
    #pragma omp parallel for
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (long q = 0; q < (long)n * n; ++q) {
            long p = (long)i * n * n + q;
            s += f[p] * g[p];
        }
        plane[i] = s;
    }
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += plane[i];
    free(plane);
    return s;
}

static double field_mean(const double *f, int n) { return field_sum(f, n) / (double)cube(n); }

/* ------------------------------------------------------ 3x3 symmetric algebra */

static double det3(const double e[3][3])
{
    return e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1])
         - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0])
         + e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
}

/* Smallest eigenvalue of a symmetric 3x3 matrix by cyclic Jacobi rotations
 * (the textbook iteration; converges to working precision in a few sweeps). */
static double lambda_min_jacobi(const double e_in[3][3])
{
    double a[3][3];
    memcpy(a, e_in, sizeof(a));
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-34 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < 3; ++r) { /* columns p, q */
                    double arp = a[r][p], arq = a[r][q];
                    a[r][p] = c * arp - s * arq;
                    a[r][q] = s * arp + c * arq;
                }
                for (int r = 0; r < 3; ++r) { /* rows p, q */
                    double apr = a[p][r], aqr = a[q][r];
                    a[p][r] = c * apr - s * aqr;
                    a[q][r] = s * apr + c * aqr;
                }
            }
    }
    double l = a[0][0];
    if (a[1][1] < l) l = a[1][1];
    if (a[2][2] < l) l = a[2][2];
    return l;
}

double orc_lambda_min(const double *e9) { return lambda_min_jacobi((const double(*)[3])e9); }
double orc_det3(const double *e9) { return det3((const double(*)[3])e9); }

/* Compact Hessian of phi at node (i,j,k): second differences on the diagonal,
 * four-point cross differences off it. */
static void hessian(const double *phi, int n, int i, int j, int k, double H[3][3])
{
    int d[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double c = phi[at(n, i, j, k)];
    for (int a = 0; a < 3; ++a) {
        double p = phi[at(n, i + d[a][0], j + d[a][1], k + d[a][2])];
        double m = phi[at(n, i - d[a][0], j - d[a][1], k - d[a][2])];
        H[a][a] = p - 2.0 * c + m;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b) {
            int pi = d[a][0] + d[b][0], pj = d[a][1] + d[b][1], pk = d[a][2] + d[b][2];
            int qi = d[a][0] - d[b][0], qj = d[a][1] - d[b][1], qk = d[a][2] - d[b][2];
            double pp = phi[at(n, i + pi, j + pj, k + pk)];
            double pm = phi[at(n, i + qi, j + qj, k + qk)];
            double mp = phi[at(n, i - qi, j - qj, k - qk)];
            double mm = phi[at(n, i - pi, j - pj, k - pk)];
            H[a][b] = H[b][a] = 0.25 * (pp - pm - mp + mm);
        }
}

static void triad(const double *phi, int n, int i, int j, int k, double e[3][3])
{
    hessian(phi, n, i, j, k, e);
    for (int a = 0; a < 3; ++a) e[a][a] += 1.0;
}

/* e = I + Hess(phi) at one node, row-major (exposed for the tests). */
void orc_triad_at(const double *phi, int n, int i, int j, int k, double *e9)
{
    double e[3][3];
    triad(phi, n, i, j, k, e);
    memcpy(e9, e, sizeof(e));
}

/* Inverse of a 3x3 matrix by cofactors (transposed cofactors over det). */
static void inverse3(const double e[3][3], double inv[3][3])
{
    double d = det3(e);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            int r0 = (b + 1) % 3, r1 = (b + 2) % 3, c0 = (a + 1) % 3, c1 = (a + 2) % 3;
            /* cofactor of element (b, a) */
            inv[a][b] = (e[r0][c0] * e[r1][c1] - e[r0][c1] * e[r1][c0]) / d;
        }
}

/* The operator of the exact mass change (App. A, Eq. elliptic_diff):
 *   out = d_mu ( K^{mu nu} d_nu f ),  K = M e^{-1},  e = I + Hess phi,
 * where M is the mass per curvilinear cell (rho sqrt g) of the current mesh.
 * Flux form on the periodic lattice, so that the sum of out is zero:
 *   diagonal: sum_mu [ (K^{mumu}_n + K^{mumu}_{n+mu})/2 (f_{n+mu} - f_n)
 *                    - (K^{mumu}_{n-mu} + K^{mumu}_n)/2 (f_n - f_{n-mu}) ]
 *   cross:    sum_{mu != nu} [ K^{munu}_{n+mu} (f_{n+mu+nu} - f_{n+mu-nu})
 *                            - K^{munu}_{n-mu} (f_{n-mu+nu} - f_{n-mu-nu}) ] / 4
 * (central differences of the flux K^{munu} d_nu f in direction mu).  At
 * phi = 0 it is the operator of the solve without the a_min floor.
 * orc_full_operator_floor with a_min > 0 floors the diagonal face
 * coefficients at a_min as the x ~ xi operator does (the operator of the
 * exact-Jacobian solve, equal to the x ~ xi one at phi = 0); the mass update
 * uses the unfloored form (a_min = 0), the exact change. */
void orc_full_operator_floor(const double *phi, const double *M, const double *f, int n, double a_min, double *out)
{
    long N3 = cube(n);
    double *K = (double *)malloc(sizeof(double) * 9 * N3);
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                long p = at(n, i, j, k);
                double e[3][3], inv[3][3];
                triad(phi, n, i, j, k, e);
                inverse3(e, inv);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) K[9 * p + 3 * a + b] = M[p] * inv[a][b];
            }
    int d[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                long p = at(n, i, j, k);
                double s = 0.0;
                for (int a = 0; a < 3; ++a) {
                    long up = at(n, i + d[a][0], j + d[a][1], k + d[a][2]);
                    long dn = at(n, i - d[a][0], j - d[a][1], k - d[a][2]);
                    double kup = 0.5 * (K[9 * p + 4 * a] + K[9 * up + 4 * a]);
                    double kdn = 0.5 * (K[9 * dn + 4 * a] + K[9 * p + 4 * a]);
                    if (a_min > 0.0) {
                        kup = fmax(a_min, kup);
                        kdn = fmax(a_min, kdn);
                    }
                    s += kup * (f[up] - f[p]) - kdn * (f[p] - f[dn]);
                }
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        if (a == b) continue;
                        long up = at(n, i + d[a][0], j + d[a][1], k + d[a][2]);
                        long dn = at(n, i - d[a][0], j - d[a][1], k - d[a][2]);
                        double fu = f[at(n, i + d[a][0] + d[b][0], j + d[a][1] + d[b][1], k + d[a][2] + d[b][2])] -
                                    f[at(n, i + d[a][0] - d[b][0], j + d[a][1] - d[b][1], k + d[a][2] - d[b][2])];
                        double fd = f[at(n, i - d[a][0] + d[b][0], j - d[a][1] + d[b][1], k - d[a][2] + d[b][2])] -
                                    f[at(n, i - d[a][0] - d[b][0], j - d[a][1] - d[b][1], k - d[a][2] - d[b][2])];
                        s += 0.25 * (K[9 * up + 3 * a + b] * fu - K[9 * dn + 3 * a + b] * fd);
                    }
                out[p] = s;
            }
    free(K);
}

void orc_full_operator(const double *phi, const double *M, const double *f, int n, double *out)
{
    orc_full_operator_floor(phi, M, f, n, 0.0, out);
}

/* orc_full_operator at the listed nodes only (flat indices idx[0..count)),
 * with K = M e^-1 formed at each node where it is needed: for checks of
 * large grids at sampled nodes.  Same arithmetic as orc_full_operator. */
static void k_at(const double *phi, const double *M, int n, int i, int j, int k, double K[9])
{
    double e[3][3], inv[3][3];
    long p = at(n, i, j, k);
    triad(phi, n, i, j, k, e);
    inverse3(e, inv);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) K[3 * a + b] = M[p] * inv[a][b];
}

void orc_full_operator_at(const double *phi, const double *M, const double *f, int n, const long *idx, long count,
                          double a_min, double *out)
{
    int d[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    #pragma omp parallel for
    for (long c = 0; c < count; ++c) {
        long q = idx[c];
        int i = (int)(q / ((long)n * n)), j = (int)((q / n) % n), k = (int)(q % n);
        long p = at(n, i, j, k);
        double Kc[9], Kup[3][9], Kdn[3][9];
        k_at(phi, M, n, i, j, k, Kc);
        for (int a = 0; a < 3; ++a) {
            k_at(phi, M, n, i + d[a][0], j + d[a][1], k + d[a][2], Kup[a]);
            k_at(phi, M, n, i - d[a][0], j - d[a][1], k - d[a][2], Kdn[a]);
        }
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            long up = at(n, i + d[a][0], j + d[a][1], k + d[a][2]);
            long dn = at(n, i - d[a][0], j - d[a][1], k - d[a][2]);
            double kup = 0.5 * (Kc[4 * a] + Kup[a][4 * a]);
            double kdn = 0.5 * (Kdn[a][4 * a] + Kc[4 * a]);
            if (a_min > 0.0) {
                kup = fmax(a_min, kup);
                kdn = fmax(a_min, kdn);
            }
            s += kup * (f[up] - f[p]) - kdn * (f[p] - f[dn]);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                if (a == b) continue;
                double fu = f[at(n, i + d[a][0] + d[b][0], j + d[a][1] + d[b][1], k + d[a][2] + d[b][2])] -
                            f[at(n, i + d[a][0] - d[b][0], j + d[a][1] - d[b][1], k + d[a][2] - d[b][2])];
                double fd = f[at(n, i - d[a][0] + d[b][0], j - d[a][1] + d[b][1], k - d[a][2] + d[b][2])] -
                            f[at(n, i - d[a][0] - d[b][0], j - d[a][1] - d[b][1], k - d[a][2] - d[b][2])];
                s += 0.25 * (Kup[a][3 * a + b] * fu - Kdn[a][3 * a + b] * fd);
            }
        out[c] = s;
    }
}

/* Central-difference gradient of phi: the displacement x - xi at a node. */
static void displacement(const double *phi, int n, int i, int j, int k, double s[3])
{
    s[0] = 0.5 * (phi[at(n, i + 1, j, k)] - phi[at(n, i - 1, j, k)]);
    s[1] = 0.5 * (phi[at(n, i, j + 1, k)] - phi[at(n, i, j - 1, k)]);
    s[2] = 0.5 * (phi[at(n, i, j, k + 1)] - phi[at(n, i, j, k - 1)]);
}

/* ----------------------------------------------------------- input (Sec. III) */

/* Cloud-in-cell assignment of particles (positions in box units) onto the
 * n^3 vertex-centred grid: each particle gives weight prod_a (1 - |x_a - j_a|)
 * to the 8 surrounding nodes.  Output is particle count per node. */
int orc_cic_particles(const float *pos, long long np, int n, double box, double *rho)
{
    if (!pos || !rho || n <= 0 || box <= 0) return ORC_E_ARG;
    memset(rho, 0, sizeof(double) * cube(n));
    double toc = (double)n / box;
    for (long long p = 0; p < np; ++p) {
        double x[3];
        int f[3];
        double w1[3];
        for (int a = 0; a < 3; ++a) {
            x[a] = (double)pos[3 * p + a] * toc;
            double fl = floor(x[a]);
            f[a] = (int)fl;
            w1[a] = x[a] - fl;
        }
        for (int c = 0; c < 8; ++c) {
            int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
            double w = (o0 ? w1[0] : 1.0 - w1[0]) * (o1 ? w1[1] : 1.0 - w1[1]) * (o2 ? w1[2] : 1.0 - w1[2]);
            rho[at(n, f[0] + o0, f[1] + o1, f[2] + o2)] += w;
        }
    }
    return ORC_OK;
}

/* Input conditioning: density must be finite, non-negative with positive
 * total; the normalised density m = rho / mean(rho) has mean 1 (Sec. III). */
int orc_normalize(const double *rho, int n, double *m)
{
    long N3 = cube(n);
    for (long p = 0; p < N3; ++p)
        if (!isfinite(rho[p]) || rho[p] < 0.0) return ORC_E_INPUT;
    double mean = field_mean(rho, n);
    if (!(mean > 0.0)) return ORC_E_INPUT;
    for (long p = 0; p < N3; ++p) m[p] = rho[p] / mean;
    return ORC_OK;
}

/* -------------------------------------------- mass on the deformed mesh (App. A) */

/* Trilinear (CIC) interpolant of the grid field m at a point x (grid units). */
static double cic_interp(const double *m, int n, const double x[3])
{
    int f[3];
    double w1[3];
    for (int a = 0; a < 3; ++a) {
        double fl = floor(x[a]);
        f[a] = (int)fl;
        w1[a] = x[a] - fl;
    }
    double s = 0.0;
    for (int c = 0; c < 8; ++c) {
        int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
        double w = (o0 ? w1[0] : 1.0 - w1[0]) * (o1 ? w1[1] : 1.0 - w1[1]) * (o2 ? w1[2] : 1.0 - w1[2]);
        s += w * m[at(n, f[0] + o0, f[1] + o1, f[2] + o2)];
    }
    return s;
}

/* M_n = sqrt g_n * rho(x_n): the mass per curvilinear cell, rho sqrt g. */
void orc_meshmass(const double *phi, const double *m, int n, double *M)
{
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double s[3], e[3][3], x[3];
                displacement(phi, n, i, j, k, s);
                x[0] = i + s[0];
                x[1] = j + s[1];
                x[2] = k + s[2];
                triad(phi, n, i, j, k, e);
                M[at(n, i, j, k)] = det3(e) * cic_interp(m, n, x);
            }
}

/* --------------------------------------------------------- smoothing operator */

void orc_smooth(const double *f, int n, double c0, double *out)
{
    double cn = (1.0 - c0) / 6.0;
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double nb = f[at(n, i + 1, j, k)] + f[at(n, i - 1, j, k)] + f[at(n, i, j + 1, k)]
                          + f[at(n, i, j - 1, k)] + f[at(n, i, j, k + 1)] + f[at(n, i, j, k - 1)];
                out[at(n, i, j, k)] = c0 * f[at(n, i, j, k)] + cn * nb;
            }
}

/* ------------------------------------------------ source of Eq. (elliptic) */

/* --------------------------------- particles at their Lagrangian positions */

/* Node shifts s_n = D_c phi_n (the displacement x_n - n), three per node. */
static void node_shifts(const double *phi, int n, double *s)
{
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) displacement(phi, n, i, j, k, s + 3 * at(n, i, j, k));
}

/* The continuous map x(xi) = xi + S(xi), S the trilinear interpolant of the
 * node shifts (periodic), at one point, with its derivative dx/dxi in the
 * cell of xi (the derivative of the interpolant from the side floor() picks). */
static void map_eval(const double *s, int n, const double xi[3], double x[3], double J[3][3])
{
    int f[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double fl = floor(xi[a]);
        f[a] = (int)fl;
        t[a] = xi[a] - fl;
    }
    for (int a = 0; a < 3; ++a) {
        x[a] = xi[a];
        for (int b = 0; b < 3; ++b) J[a][b] = a == b ? 1.0 : 0.0;
    }
    for (int c = 0; c < 8; ++c) {
        int o[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
        double w[3], dw[3];
        for (int a = 0; a < 3; ++a) {
            w[a] = o[a] ? t[a] : 1.0 - t[a];
            dw[a] = o[a] ? 1.0 : -1.0;
        }
        const double *sc = s + 3 * at(n, f[0] + o[0], f[1] + o[1], f[2] + o[2]);
        double wc = w[0] * w[1] * w[2];
        double g[3] = {dw[0] * w[1] * w[2], w[0] * dw[1] * w[2], w[0] * w[1] * dw[2]};
        for (int b = 0; b < 3; ++b) {
            x[b] += wc * sc[b];
            for (int a = 0; a < 3; ++a) J[b][a] += g[a] * sc[b];
        }
    }
}

/* max_a |x(xi) - y| with each component taken modulo the box (nearest image). */
static double map_residual(const double *s, int n, const double xi[3], const double y[3], double r[3], double J[3][3])
{
    double x[3], mx = 0.0;
    for (int a = 0; a < 3; ++a)
        if (!(fabs(xi[a]) < 1.0e9)) return HUGE_VAL; /* not finite or absurdly far: no descent */
    map_eval(s, n, xi, x, J);
    for (int a = 0; a < 3; ++a) {
        double d = x[a] - y[a];
        d -= n * floor(d / n + 0.5);
        r[a] = d;
        if (fabs(d) > mx) mx = fabs(d);
    }
    return mx;
}

/* Lagrangian positions of particles (the mapping x = xi + grad phi inverted):
 * for each particle at y (grid units) find xi with x(xi) = y modulo the box by
 * Newton steps xi -= t J^-1 (x(xi) - y), t = 1 halved (at most 30 times) while
 * the step does not reduce max |x(xi) - y|.  xi holds the starts on entry and
 * the solutions on exit, wrapped into [0, n).  ORC_E_NO_CONVERGENCE if a
 * particle is not within tol after max_iter steps. */
int orc_invert_map(const double *phi, int n, const double *y, long np, double *xi, int max_iter, double tol)
{
    double *s = (double *)malloc(sizeof(double) * 3 * cube(n));
    node_shifts(phi, n, s);
    int failed = 0;
    #pragma omp parallel for reduction(| : failed)
    for (long p = 0; p < np; ++p) {
        double *q = xi + 3 * p;
        const double *yp = y + 3 * p;
        double r[3], J[3][3], inv[3][3];
        double res = map_residual(s, n, q, yp, r, J);
        int it = 0;
        while (res > tol && it < max_iter) {
            ++it;
            inverse3(J, inv);
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = inv[a][0] * r[0] + inv[a][1] * r[1] + inv[a][2] * r[2];
            double step = 1.0, trial[3], rt[3], Jt[3][3], rest = res;
            for (int h = 0; h <= 30; ++h, step *= 0.5) {
                for (int a = 0; a < 3; ++a) trial[a] = q[a] - step * d[a];
                rest = map_residual(s, n, trial, yp, rt, Jt);
                if (rest < res) break;
            }
            if (!(rest < res)) break; /* no descent: give up on this particle */
            for (int a = 0; a < 3; ++a) {
                q[a] = trial[a];
                r[a] = rt[a];
                for (int b = 0; b < 3; ++b) J[a][b] = Jt[a][b];
            }
            res = rest;
        }
        for (int a = 0; a < 3; ++a) q[a] -= n * floor(q[a] / n);
        if (!(res <= tol)) failed = 1;
    }
    free(s);
    return failed ? ORC_E_NO_CONVERGENCE : ORC_OK;
}

/* Mass per curvilinear cell from particles at Lagrangian positions xi (grid
 * units, [0, n)): CIC deposit in xi-space, n^3 / np per particle (mean 1). */
void orc_deposit_xi(const double *xi, long np, int n, double *M)
{
    memset(M, 0, sizeof(double) * cube(n));
    double wp = (double)cube(n) / (double)np;
    for (long p = 0; p < np; ++p) {
        int f[3];
        double t[3];
        for (int a = 0; a < 3; ++a) {
            double fl = floor(xi[3 * p + a]);
            f[a] = (int)fl;
            t[a] = xi[3 * p + a] - fl;
        }
        for (int c = 0; c < 8; ++c) {
            int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
            double w = (o0 ? t[0] : 1.0 - t[0]) * (o1 ? t[1] : 1.0 - t[1]) * (o2 ? t[2] : 1.0 - t[2]);
            M[at(n, f[0] + o0, f[1] + o1, f[2] + o2)] += wp * w;
        }
    }
}

/* t = Sigma + C + E at every node, Sigma = mean(M) - M (App. A).
 * Returns rho_bar = mean(M). */
double orc_source_terms(const double *phi, const double *M, int n, double xi_m, double v_m, double *t)
{
    double rho_bar = field_mean(M, n);
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double e[3][3];
                triad(phi, n, i, j, k, e);
                double g = det3(e);
                double lam0 = lambda_min_jacobi(e);
                double sigma = rho_bar - M[at(n, i, j, k)];
                double r = xi_m / lam0 - 1.0;
                double C = r > 0.0 ? 4.0 * r * r : 0.0;
                double E = g > v_m ? -2.0 * fabs(sigma) : 0.0;
                t[at(n, i, j, k)] = sigma + C + E;
            }
    return rho_bar;
}

/* b = S(Sigma + C + E) with its mean removed (the periodic operator annihilates
 * constants, so only the mean-free part of the source is solvable). */
void orc_source(const double *phi, const double *M, int n, double xi_m, double v_m, double c0, double *b)
{
    double *t = (double *)malloc(sizeof(double) * cube(n));
    orc_source_terms(phi, M, n, xi_m, v_m, t);
    orc_smooth(t, n, c0, b);
    free(t);
    double mb = field_mean(b, n);
    long N3 = cube(n);
    for (long p = 0; p < N3; ++p) b[p] -= mb;
}

/* ------------------------------------------ operator div(a grad u) and multigrid */

static inline double face(double an, double anb, double a_min)
{
    double c = 0.5 * (an + anb);
    return c > a_min ? c : a_min;
}

/* (A u)_n = scale * sum over the six faces of c_f (u_nb - u_n). */
static double apply_at(const double *u, const double *a, int n, int i, int j, int k, double scale, double a_min)
{
    int off[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    double un = u[at(n, i, j, k)], an = a[at(n, i, j, k)];
    double s = 0.0;
    for (int f = 0; f < 6; ++f) {
        long q = at(n, i + off[f][0], j + off[f][1], k + off[f][2]);
        s += face(an, a[q], a_min) * (u[q] - un);
    }
    return scale * s;
}

void orc_apply(const double *u, const double *a, int n, double scale, double a_min, double *out)
{
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) out[at(n, i, j, k)] = apply_at(u, a, n, i, j, k, scale, a_min);
}

void orc_residual(const double *u, const double *a, const double *b, int n, double scale, double a_min, double *r)
{
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k)
                r[at(n, i, j, k)] = b[at(n, i, j, k)] - apply_at(u, a, n, i, j, k, scale, a_min);
}

/* One Gauss-Seidel relaxation at a node: the value of u_n that makes
 * (A u)_n = b_n with the neighbours held fixed. */
static double relax_at(const double *u, const double *a, const double *b, int n, int i, int j, int k, double scale,
                       double a_min)
{
    int off[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    double an = a[at(n, i, j, k)];
    double num = 0.0, den = 0.0;
    for (int f = 0; f < 6; ++f) {
        long q = at(n, i + off[f][0], j + off[f][1], k + off[f][2]);
        double c = face(an, a[q], a_min);
        num += c * u[q];
        den += c;
    }
    return (num - b[at(n, i, j, k)] / scale) / den;
}

/* Relax every node of one colour (0 = red, i+j+k even; 1 = black). */
void orc_rbgs_half(double *u, const double *a, const double *b, int n, double scale, double a_min, int colour)
{
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k)
                if (((i + j + k) & 1) == colour) u[at(n, i, j, k)] = relax_at(u, a, b, n, i, j, k, scale, a_min);
}

/* One red-black Gauss-Seidel sweep: every node of colour `first`, then every
 * node of the other colour. */
void orc_rbgs_sweep(double *u, const double *a, const double *b, int n, double scale, double a_min, int first)
{
    orc_rbgs_half(u, a, b, n, scale, a_min, first);
    orc_rbgs_half(u, a, b, n, scale, a_min, 1 - first);
}

/* 27-point full weighting onto the coarse lattice (coarse node I = fine 2I). */
void orc_restrict(const double *f, int n, double *c)
{
    int nc = n / 2;
    #pragma omp parallel for
    for (int I = 0; I < nc; ++I)
        for (int J = 0; J < nc; ++J)
            for (int K = 0; K < nc; ++K) {
                double s = 0.0;
                for (int di = -1; di <= 1; ++di)
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int dk = -1; dk <= 1; ++dk) {
                            double w = (di ? 0.25 : 0.5) * (dj ? 0.25 : 0.5) * (dk ? 0.25 : 0.5);
                            s += w * f[at(n, 2 * I + di, 2 * J + dj, 2 * K + dk)];
                        }
                c[at(nc, I, J, K)] = s;
            }
}

/* u += P e, trilinear interpolation from the coarse lattice (n/2)^3. */
void orc_prolong_add(double *u, const double *e, int n)
{
    int nc = n / 2;
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                int lo[3] = {i / 2, j / 2, k / 2};
                int odd[3] = {i & 1, j & 1, k & 1};
                double s = 0.0;
                for (int c = 0; c < 8; ++c) {
                    int o[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
                    double w = 1.0;
                    int skip = 0;
                    for (int d = 0; d < 3; ++d) {
                        if (!odd[d]) {
                            if (o[d]) skip = 1; /* even index: the coarse node itself only */
                        } else {
                            w *= 0.5;
                        }
                    }
                    if (skip) continue;
                    s += w * e[at(nc, lo[0] + o[0], lo[1] + o[1], lo[2] + o[2])];
                }
                u[at(n, i, j, k)] += s;
            }
}

typedef struct {
    int levels;
    int n[32];
    double *a[32]; /* coefficient per level */
    double *u[32], *b[32], *r[32];
    const orc_config *cfg;
} mg_t;

static double level_scale(int l) { return ldexp(1.0, -2 * l); }

/* Coarsest level: zero-mean right-hand side, then from u = 0 the palindromic
 * sequence red, black, red, ..., black, red (2 * coarse_sweeps + 1 colour
 * passes), then the mean of u removed. */
static void coarse_solve(mg_t *mg, int l)
{
    int n = mg->n[l];
    long N3 = cube(n);
    double *b = mg->r[l];
    double mb = field_mean(mg->b[l], n);
    for (long p = 0; p < N3; ++p) b[p] = mg->b[l][p] - mb;
    memset(mg->u[l], 0, sizeof(double) * N3);
    double sc = level_scale(l), amin = mg->cfg->a_min;
    for (int s = 0; s < mg->cfg->coarse_sweeps; ++s) orc_rbgs_sweep(mg->u[l], mg->a[l], b, n, sc, amin, 0);
    orc_rbgs_half(mg->u[l], mg->a[l], b, n, sc, amin, 0);
    double mu = field_mean(mg->u[l], n);
    for (long p = 0; p < N3; ++p) mg->u[l][p] -= mu;
}

/* One V-cycle from u = 0 on level l for right-hand side b[l]: n_pre sweeps
 * red-then-black, residual, full weighting, recursion, trilinear correction,
 * n_post sweeps black-then-red.  With n_pre == n_post this is a symmetric
 * operator b -> u (post-smoother = adjoint of the pre-smoother, P = 8 R^T). */
static void vcycle(mg_t *mg, int l)
{
    int n = mg->n[l];
    memset(mg->u[l], 0, sizeof(double) * cube(n));
    if (l == mg->levels - 1) {
        coarse_solve(mg, l);
        return;
    }
    double sc = level_scale(l), amin = mg->cfg->a_min;
    for (int s = 0; s < mg->cfg->n_pre; ++s) orc_rbgs_sweep(mg->u[l], mg->a[l], mg->b[l], n, sc, amin, 0);
    orc_residual(mg->u[l], mg->a[l], mg->b[l], n, sc, amin, mg->r[l]);
    orc_restrict(mg->r[l], n, mg->b[l + 1]);
    vcycle(mg, l + 1);
    orc_prolong_add(mg->u[l], mg->u[l + 1], n);
    for (int s = 0; s < mg->cfg->n_post; ++s) orc_rbgs_sweep(mg->u[l], mg->a[l], mg->b[l], n, sc, amin, 1);
}

static double norm2(const double *f, int n) { return sqrt(field_dot(f, f, n)); }

int orc_num_levels(int n, int coarse_n)
{
    if (n <= 0 || coarse_n < 2 || (coarse_n & 1)) return -1;
    int L = 1;
    while (n > coarse_n) {
        if (n & 1) return -1;
        n /= 2;
        ++L;
    }
    return n == coarse_n ? L : -1;
}

static int mg_alloc(mg_t *mg, const double *a0, int n, const orc_config *cfg)
{
    memset(mg, 0, sizeof(*mg));
    mg->cfg = cfg;
    mg->levels = orc_num_levels(n, cfg->coarse_n);
    if (mg->levels < 1) return ORC_E_ARG;
    int nl = n;
    for (int l = 0; l < mg->levels; ++l, nl /= 2) {
        mg->n[l] = nl;
        long N3 = cube(nl);
        mg->a[l] = (double *)malloc(sizeof(double) * N3);
        mg->u[l] = (double *)calloc(N3, sizeof(double));
        mg->b[l] = (double *)malloc(sizeof(double) * N3);
        mg->r[l] = (double *)malloc(sizeof(double) * N3);
    }
    memcpy(mg->a[0], a0, sizeof(double) * cube(n));
    /* coefficient hierarchy: full weighting of the fine coefficient */
    for (int l = 1; l < mg->levels; ++l) orc_restrict(mg->a[l - 1], mg->n[l - 1], mg->a[l]);
    return ORC_OK;
}

static void mg_free(mg_t *mg)
{
    for (int l = 0; l < mg->levels; ++l) {
        free(mg->a[l]);
        free(mg->u[l]);
        free(mg->b[l]);
        free(mg->r[l]);
    }
}

/* z = V-cycle applied to r (fine level). */
static void precondition(mg_t *mg, const double *r, double *z)
{
    long N3 = cube(mg->n[0]);
    memcpy(mg->b[0], r, sizeof(double) * N3);
    vcycle(mg, 0);
    memcpy(z, mg->u[0], sizeof(double) * N3);
}

/* Apply one V-cycle to a right-hand side (exposed for the tests). */
int orc_vcycle(const double *a0, const double *r, int n, const orc_config *cfg, double *z)
{
    mg_t mg;
    int rc = mg_alloc(&mg, a0, n, cfg);
    if (rc) return rc;
    precondition(&mg, r, z);
    mg_free(&mg);
    return ORC_OK;
}

/* Solve A(a) u = b on mean-free fields to ||b - A u|| <= tol ||b||, starting
 * from u0 when one is given and ||b - A u0|| < ||b||, else from u = 0.
 * solver 0: conjugate gradients preconditioned by one V-cycle per iteration
 *           (flexible form: beta = z_new.(r_new - r_old) / z_old.r_old);
 * solver 1: plain V-cycle iteration u += V(b - A u).
 * Returns the number of V-cycles (>= 0) or a negative error; *rel receives
 * the final true relative residual. */
/* out = L x: the x ~ xi operator of coefficient a0, or (phi_full given) the
 * full operator div(a0 e^-1 grad x) on the mesh of phi_full, its diagonal
 * face coefficients floored at a_min like the x ~ xi operator's. */
static void krylov_apply(const double *phi_full, const double *a0, const double *x, int n, double a_min, double *out)
{
    if (phi_full) orc_full_operator_floor(phi_full, a0, x, n, a_min, out);
    else orc_apply(x, a0, n, 1.0, a_min, out);
}

/* out = b - L x */
static void krylov_residual(const double *phi_full, const double *a0, const double *b, const double *x, int n,
                            double a_min, double *out)
{
    long N3 = cube(n);
    krylov_apply(phi_full, a0, x, n, a_min, out);
    for (long p = 0; p < N3; ++p) out[p] = b[p] - out[p];
}

/* The linear solve with the operator of krylov_apply (phi_full NULL: x ~ xi),
 * preconditioned by one V-cycle of the x ~ xi operator whose coefficient is
 * a0 (phi_full NULL) or the mean diagonal (K^xx + K^yy + K^zz) / 3 of
 * K = a0 e^-1 (the scalar coefficient closest to the deformed operator's
 * diagonal; it is a0 at phi = 0). */
int orc_mg_solve_full(const double *a0, const double *phi_full, const double *b0, int n, const orc_config *cfg,
                      const double *u0, double *u_out, double *rel)
{
    mg_t mg;
    long N3 = cube(n);
    double *ap = NULL;
    if (phi_full) {
        ap = (double *)malloc(sizeof(double) * N3);
        #pragma omp parallel for
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    long p = at(n, i, j, k);
                    double e[3][3], inv[3][3];
                    triad(phi_full, n, i, j, k, e);
                    inverse3(e, inv);
                    ap[p] = (a0[p] * inv[0][0] + a0[p] * inv[1][1] + a0[p] * inv[2][2]) / 3.0;
                }
    }
    int rc = mg_alloc(&mg, ap ? ap : a0, n, cfg);
    free(ap);
    if (rc) return rc;
    double *u = (double *)calloc(N3, sizeof(double));
    double *r = (double *)malloc(sizeof(double) * N3);
    double *z = (double *)malloc(sizeof(double) * N3);
    double *p = (double *)malloc(sizeof(double) * N3);
    double *q = (double *)malloc(sizeof(double) * N3);
    double *r_old = (double *)malloc(sizeof(double) * N3);

    int status = ORC_E_NO_CONVERGENCE;
    double bn = norm2(b0, n);
    int cycles = 0;
    memcpy(r, b0, sizeof(double) * N3);
    if (u0 && bn > 0.0) {
        krylov_residual(phi_full, a0, b0, u0, n, cfg->a_min, z);
        if (norm2(z, n) < bn) {
            memcpy(u, u0, sizeof(double) * N3);
            memcpy(r, z, sizeof(double) * N3);
        }
    }
    if (bn == 0.0) {
        status = 0;
    } else if (cfg->solver == 1) {
        for (cycles = 1; cycles <= cfg->max_vcycles; ++cycles) {
            krylov_residual(phi_full, a0, b0, u, n, cfg->a_min, r);
            precondition(&mg, r, z);
            for (long i = 0; i < N3; ++i) u[i] += z[i];
            krylov_residual(phi_full, a0, b0, u, n, cfg->a_min, r);
            double rn = norm2(r, n);
            if (!isfinite(rn)) break;
            if (rn <= cfg->tol * bn) {
                status = cycles;
                break;
            }
        }
    } else {
        precondition(&mg, r, z);
        cycles = 1;
        memcpy(p, z, sizeof(double) * N3);
        double rz = field_dot(r, z, n);
        while (cycles <= cfg->max_vcycles) {
            krylov_apply(phi_full, a0, p, n, cfg->a_min, q);
            double pq = field_dot(p, q, n);
            double alpha = rz / pq;
            memcpy(r_old, r, sizeof(double) * N3);
            for (long i = 0; i < N3; ++i) {
                u[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            double rn = norm2(r, n);
            if (!isfinite(rn)) break;
            if (rn <= cfg->tol * bn) {
                status = cycles;
                break;
            }
            if (cycles == cfg->max_vcycles) break;
            precondition(&mg, r, z);
            ++cycles;
            double rz_new = field_dot(z, r, n);
            double beta = (rz_new - field_dot(z, r_old, n)) / rz;
            rz = rz_new;
            for (long i = 0; i < N3; ++i) p[i] = z[i] + beta * p[i];
        }
    }
    double mu = field_mean(u, n);
    for (long i = 0; i < N3; ++i) u_out[i] = u[i] - mu;
    krylov_residual(phi_full, a0, b0, u_out, n, cfg->a_min, r);
    *rel = bn > 0.0 ? norm2(r, n) / bn : 0.0;
    free(u);
    free(r);
    free(z);
    free(p);
    free(q);
    free(r_old);
    mg_free(&mg);
    return status;
}

int orc_mg_solve_from(const double *a0, const double *b0, int n, const orc_config *cfg, const double *u0,
                      double *u_out, double *rel)
{
    return orc_mg_solve_full(a0, NULL, b0, n, cfg, u0, u_out, rel);
}

int orc_mg_solve(const double *a0, const double *b0, int n, const orc_config *cfg, double *u_out, double *rel)
{
    return orc_mg_solve_from(a0, b0, n, cfg, NULL, u_out, rel);
}

/* ------------------------------------------------ positive-definite step control */

/* Number of nodes where I + Hess(phi) is not positive definite: some leading
 * principal minor (e11, e11 e22 - e12^2, det) is not positive (Sec. II: the
 * map x = xi + grad phi must stay positive definite). */
long orc_count_not_pd(const double *phi, int n)
{
    long bad = 0;
    #pragma omp parallel for reduction(+ : bad)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double e[3][3];
                triad(phi, n, i, j, k, e);
                double m1 = e[0][0];
                double m2 = e[0][0] * e[1][1] - e[0][1] * e[1][0];
                double m3 = det3(e);
                if (!(m1 > 0.0 && m2 > 0.0 && m3 > 0.0)) ++bad;
            }
    return bad;
}

/* 1 if I + Hess(phi) is positive definite at every node. */
int orc_is_pd(const double *phi, int n)
{
    return orc_count_not_pd(phi, n) == 0;
}

double orc_max_shift(const double *f, int n)
{
    double mx = 0.0;
    #pragma omp parallel for reduction(max : mx)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double s[3];
                displacement(f, n, i, j, k, s);
                for (int a = 0; a < 3; ++a)
                    if (fabs(s[a]) > mx) mx = fabs(s[a]);
            }
    return mx;
}

/* First alpha = 2^-j (j = 0..max_halvings) for which phi + alpha dphi keeps the
 * map positive definite everywhere and no node moves more than s_max cells;
 * with M and D given (the mass update), also M + alpha D > 0 at every node.
 * Returns j, or -1 when every trial fails. */
int orc_choose_step_mass(const double *phi, const double *dphi, const double *M, const double *D, int n,
                         const orc_config *cfg, double *alpha_out)
{
    long N3 = cube(n);
    double *trial = (double *)malloc(sizeof(double) * N3);
    double shift = orc_max_shift(dphi, n);
    int found = -1;
    for (int j = 0; j <= cfg->max_halvings; ++j) {
        double alpha = ldexp(1.0, -j);
        if (alpha * shift > cfg->s_max) continue;
        if (M && D) {
            int positive = 1;
            for (long p = 0; p < N3; ++p)
                if (!(M[p] + alpha * D[p] > 0.0)) positive = 0;
            if (!positive) continue;
        }
        for (long p = 0; p < N3; ++p) trial[p] = phi[p] + alpha * dphi[p];
        if (orc_is_pd(trial, n)) {
            found = j;
            *alpha_out = alpha;
            break;
        }
    }
    free(trial);
    return found;
}

int orc_choose_step(const double *phi, const double *dphi, int n, const orc_config *cfg, double *alpha_out)
{
    return orc_choose_step_mass(phi, dphi, NULL, NULL, n, cfg, alpha_out);
}

/* -------------------------------------------------------- the outer iteration */

void orc_config_default(orc_config *c)
{
    c->max_outer = 10;
    c->n_pre = 2;
    c->n_post = 2;
    c->coarse_n = 8;
    c->coarse_sweeps = 64;
    c->max_vcycles = 100;
    c->max_halvings = 30;
    c->record_tape = 0;
    c->solver = 0;
    c->warm_start = 1;
    c->mass_update = 0;
    c->particle_deposit = 0;
    c->full_operator = 0;
    c->tol = 1e-10;
    c->outer_tol = 0.0;
    c->xi_m = 0.1;
    c->v_m = 10.0;
    c->smooth_center = 0.5;
    c->s_max = 1.0;
    c->a_min = 1e-3;
}

/* Reconstructed density delta_r = -(discrete Laplacian of phi), Eq. (rec). */
void orc_delta_r(const double *phi, int n, double *delta)
{
    #pragma omp parallel for
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double c = phi[at(n, i, j, k)];
                double lap = phi[at(n, i + 1, j, k)] + phi[at(n, i - 1, j, k)] + phi[at(n, i, j + 1, k)]
                           + phi[at(n, i, j - 1, k)] + phi[at(n, i, j, k + 1)] + phi[at(n, i, j, k - 1)] - 6.0 * c;
                delta[at(n, i, j, k)] = -lap;
            }
}

static void invariants(const double *phi, int n, orc_stats *st)
{
    double mind = INFINITY, minl = INFINITY, maxd = -INFINITY;
    #pragma omp parallel for reduction(min : mind, minl) reduction(max : maxd)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double e[3][3];
                triad(phi, n, i, j, k, e);
                double g = det3(e), l = lambda_min_jacobi(e);
                double d = 3.0 - (e[0][0] + e[1][1] + e[2][2]);
                if (g < mind) mind = g;
                if (l < minl) minl = l;
                if (d > maxd) maxd = d;
            }
    st->min_det = mind;
    st->min_lambda0 = minl;
    st->max_delta_r = maxd;
}

/* Tape of the forward iteration: the solution u of every outer step and its
 * accepted alpha (phi_{i+1} = phi_i + alpha_i S u_i). */
typedef struct {
    int n, steps;
    double *u[ORC_MAX_STEPS];
    double alpha[ORC_MAX_STEPS];
    double *m;   /* normalised input density */
    double mean; /* mean of the raw input density */
    double *y;   /* particle deposit: the particle positions in grid units (3 per particle) */
    long np;
} orc_tape;

static orc_tape g_tape;

void orc_tape_clear(void)
{
    for (int s = 0; s < g_tape.steps; ++s) free(g_tape.u[s]);
    free(g_tape.m);
    free(g_tape.y);
    memset(&g_tape, 0, sizeof(g_tape));
}

/* Full forward reconstruction, from a density grid (rho) or, with
 * particle_deposit, from particles (pos, np: float positions in [0, box)).
 * phi_out in (box/n)^2 units (length^2), delta_out dimensionless.  Either
 * output may be NULL. */
static int solve_core(const double *rho, const float *pos, long long np, int n, double box, const orc_config *cfg,
                      double *phi_out, double *delta_out, orc_stats *st)
{
    if ((!rho && !pos) || n <= 0 || box <= 0 || !cfg || cfg->tol <= 0) return ORC_E_ARG;
    if (pos && (np <= 0 || cfg->mass_update)) return ORC_E_ARG;
    if (orc_num_levels(n, cfg->coarse_n) < 1) return ORC_E_ARG;
    if (cfg->max_outer > ORC_MAX_STEPS) return ORC_E_ARG;
    if (cfg->mass_update && cfg->record_tape) return ORC_E_ARG; /* no reverse mode for the mass update */
    long N3 = cube(n);
    double *m = (double *)malloc(sizeof(double) * N3);
    double *phi = (double *)calloc(N3, sizeof(double));
    double *M = (double *)malloc(sizeof(double) * N3);
    double *b = (double *)malloc(sizeof(double) * N3);
    double *u = (double *)malloc(sizeof(double) * N3);
    double *dphi = (double *)malloc(sizeof(double) * N3);
    double *D = cfg->mass_update ? (double *)malloc(sizeof(double) * N3) : NULL;
    /* particle deposit: positions in grid units and their Lagrangian positions
     * (at phi = 0 the map is the identity) */
    double *y = NULL, *xi = NULL;
    if (pos) {
        y = (double *)malloc(sizeof(double) * 3 * np);
        xi = (double *)malloc(sizeof(double) * 3 * np);
        for (long long p = 0; p < 3 * np; ++p) y[p] = xi[p] = (double)pos[p] * ((double)n / box);
    }
    orc_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    if (cfg->record_tape) orc_tape_clear();

    int status = pos ? ORC_OK : orc_normalize(rho, n, m);
    if (status == ORC_OK) {
        for (int it = 0; it < cfg->max_outer; ++it) {
            /* the CIC gather each step, or (mass update) only at phi = 0, where it
             * gives M = m, after which M is carried by the update below */
            if (pos) {
                /* the particles at their Lagrangian positions, warm-started from
                 * the previous step's */
                status = orc_invert_map(phi, n, y, np, xi, 100, 1e-12);
                if (status != ORC_OK) break;
                orc_deposit_xi(xi, np, n, M);
            } else if (!cfg->mass_update || it == 0) {
                orc_meshmass(phi, m, n, M);
            }
            double rho_bar = field_mean(M, n);
            double ss = 0.0;
            {
                /* rms of Sigma = rho_bar - M */
                double *sig = b;
                for (long p = 0; p < N3; ++p) sig[p] = rho_bar - M[p];
                ss = field_dot(sig, sig, n);
            }
            double rms = sqrt(ss / (double)N3);
            st->rms_sigma[it] = rms;
            st->kappa[it] = rho_bar;
            if (rms <= cfg->outer_tol) break;
            orc_source(phi, M, n, cfg->xi_m, cfg->v_m, cfg->smooth_center, b);
            double rel = 0.0;
            /* warm start: the previous step's solution (the steps are small) */
            int cyc = orc_mg_solve_full(M, cfg->full_operator ? phi : NULL, b, n, cfg,
                                        (cfg->warm_start && it > 0) ? u : NULL, u, &rel);
            st->rel_residual[it] = rel;
            if (cyc < 0) {
                status = cyc;
                break;
            }
            st->vcycles[it] = cyc;
            st->vcycles_total += cyc;
            orc_smooth(u, n, cfg->smooth_center, dphi);
            /* mass update: the exact change per unit step on the current mesh */
            if (cfg->mass_update) orc_full_operator(phi, M, dphi, n, D);
            double alpha = 0.0;
            if (orc_choose_step_mass(phi, dphi, D ? M : NULL, D, n, cfg, &alpha) < 0) {
                status = ORC_E_NOT_PD;
                break;
            }
            if (D)
                for (long p = 0; p < N3; ++p) M[p] += alpha * D[p];
            for (long p = 0; p < N3; ++p) phi[p] += alpha * dphi[p];
            st->alpha[it] = alpha;
            st->outer_steps = it + 1;
            if (cfg->record_tape) {
                g_tape.u[it] = (double *)malloc(sizeof(double) * N3);
                memcpy(g_tape.u[it], u, sizeof(double) * N3);
                g_tape.alpha[it] = alpha;
                g_tape.steps = it + 1;
            }
        }
    }
    if (status == ORC_OK && st->outer_steps == cfg->max_outer) {
        /* mass deviation left after the last step (the carried M under the
         * mass update) */
        if (pos) {
            status = orc_invert_map(phi, n, y, np, xi, 100, 1e-12);
            if (status == ORC_OK) orc_deposit_xi(xi, np, n, M);
        } else if (!cfg->mass_update) {
            orc_meshmass(phi, m, n, M);
        }
        double rho_bar = field_mean(M, n);
        for (long p = 0; p < N3; ++p) b[p] = rho_bar - M[p];
        st->rms_sigma[cfg->max_outer] = sqrt(field_dot(b, b, n) / (double)N3);
        st->kappa[cfg->max_outer] = rho_bar;
    }
    if (status == ORC_OK) {
        invariants(phi, n, st);
        if (delta_out) orc_delta_r(phi, n, delta_out);
        double h = box / n;
        if (phi_out)
            for (long p = 0; p < N3; ++p) phi_out[p] = phi[p] * h * h;
        if (cfg->record_tape) {
            g_tape.n = n;
            if (pos) {
                g_tape.y = y;
                g_tape.np = (long)np;
                y = NULL;
            } else {
                g_tape.m = m;
                g_tape.mean = field_mean(rho, n);
                m = NULL;
            }
        }
    } else if (cfg->record_tape) {
        orc_tape_clear();
    }
    free(m);
    free(phi);
    free(M);
    free(b);
    free(u);
    free(dphi);
    free(D);
    free(y);
    free(xi);
    return status;
}

int orc_solve(const double *rho, int n, double box, const orc_config *cfg, double *phi_out, double *delta_out,
              orc_stats *st)
{
    if (!rho || (cfg && cfg->particle_deposit)) return ORC_E_ARG;
    return solve_core(rho, NULL, 0, n, box, cfg, phi_out, delta_out, st);
}

/* Forward reconstruction from particles: CIC onto the grid once, or, with
 * particle_deposit, the particles deposited at their Lagrangian positions
 * every step. */
int orc_solve_particles(const float *pos, long long np, int n, double box, const orc_config *cfg, double *phi_out,
                        double *delta_out, orc_stats *st)
{
    if (!pos || np <= 0 || n <= 0 || box <= 0 || !cfg) return ORC_E_ARG;
    if (cfg->particle_deposit) return solve_core(NULL, pos, np, n, box, cfg, phi_out, delta_out, st);
    double *rho = (double *)malloc(sizeof(double) * cube(n));
    int rc = orc_cic_particles(pos, np, n, box, rho);
    if (rc == ORC_OK) rc = solve_core(rho, NULL, 0, n, box, cfg, phi_out, delta_out, st);
    free(rho);
    return rc;
}

int orc_tape_steps(void) { return g_tape.steps; }

/* ======================================================================
 * Reverse mode (adjoint) of orc_solve for a recorded tape.
 *
 * The forward step i maps phi_i to phi_{i+1} through
 *   M = det(e) * CIC(m)(xi + D_c phi),  e = I + Hess(phi)
 *   Sigma = mean(M) - M;  t = Sigma + C(lambda_0(e)) - 2 [det e > v_m] |Sigma|
 *   b = S t - mean(S t);  u = A(M)^+ b;  phi_{i+1} = phi_i + alpha_i S u
 * with alpha_i and the limiter masks held fixed (piecewise constant), and
 * the linear solve differentiated as exact: for u = A^+ b with A symmetric,
 * lambda = A^+ ubar gives bbar = lambda and, per face f of coefficient
 * c_f = max(a_min, (M_n + M_nb)/2), cbar_f = (lambda_nb - lambda_n)(u_nb - u_n).
 * With particles deposited at their Lagrangian positions, M = CIC_xi(xi) with
 * xi = X^-1(y; D_c phi) instead, and the gradient is taken with respect to
 * the particle positions y (deposit_adjoint).
 * ====================================================================== */

/* Smallest eigenvalue and its unit eigenvector, cyclic Jacobi with the
 * rotations accumulated. */
static double eig_min_vec(const double e_in[3][3], double v[3])
{
    double a[3][3], V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    memcpy(a, e_in, sizeof(a));
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-34 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < 3; ++r) {
                    double arp = a[r][p], arq = a[r][q];
                    a[r][p] = c * arp - s * arq;
                    a[r][q] = s * arp + c * arq;
                }
                for (int r = 0; r < 3; ++r) {
                    double apr = a[p][r], aqr = a[q][r];
                    a[p][r] = c * apr - s * aqr;
                    a[q][r] = s * apr + c * aqr;
                }
                for (int r = 0; r < 3; ++r) {
                    double vrp = V[r][p], vrq = V[r][q];
                    V[r][p] = c * vrp - s * vrq;
                    V[r][q] = s * vrp + c * vrq;
                }
            }
    }
    int k = 0;
    if (a[1][1] < a[k][k]) k = 1;
    if (a[2][2] < a[k][k]) k = 2;
    for (int r = 0; r < 3; ++r) v[r] = V[r][k];
    return a[k][k];
}

void orc_eig_min_vec(const double *e9, double *lam, double *v)
{
    *lam = eig_min_vec((const double(*)[3])e9, v);
}

/* cofactor matrix: d det(e) / d e_ab */
static void cofactor(const double e[3][3], double c[3][3])
{
    c[0][0] = e[1][1] * e[2][2] - e[1][2] * e[2][1];
    c[0][1] = -(e[1][0] * e[2][2] - e[1][2] * e[2][0]);
    c[0][2] = e[1][0] * e[2][1] - e[1][1] * e[2][0];
    c[1][0] = -(e[0][1] * e[2][2] - e[0][2] * e[2][1]);
    c[1][1] = e[0][0] * e[2][2] - e[0][2] * e[2][0];
    c[1][2] = -(e[0][0] * e[2][1] - e[0][1] * e[2][0]);
    c[2][0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
    c[2][1] = -(e[0][0] * e[1][2] - e[0][2] * e[1][0]);
    c[2][2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
}

/* phibar += Hess^T applied to the per-node partials hb[n][a][b] with respect
 * to the entries of e (a symmetric matrix whose off-diagonal pair is the
 * single quantity H_ab, hence the factor hb_ab + hb_ba). */
static void hess_transpose_add(const double *hb, int n, double *phibar)
{
    int d[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                const double *h = hb + at(n, i, j, k) * 9;
                for (int a = 0; a < 3; ++a) {
                    /* H_aa = phi(+a) - 2 phi + phi(-a) */
                    phibar[at(n, i + d[a][0], j + d[a][1], k + d[a][2])] += h[a * 3 + a];
                    phibar[at(n, i, j, k)] -= 2.0 * h[a * 3 + a];
                    phibar[at(n, i - d[a][0], j - d[a][1], k - d[a][2])] += h[a * 3 + a];
                }
                for (int a = 0; a < 3; ++a)
                    for (int b = a + 1; b < 3; ++b) {
                        double w = 0.25 * (h[a * 3 + b] + h[b * 3 + a]);
                        int pi = d[a][0] + d[b][0], pj = d[a][1] + d[b][1], pk = d[a][2] + d[b][2];
                        int qi = d[a][0] - d[b][0], qj = d[a][1] - d[b][1], qk = d[a][2] - d[b][2];
                        phibar[at(n, i + pi, j + pj, k + pk)] += w;
                        phibar[at(n, i + qi, j + qj, k + qk)] -= w;
                        phibar[at(n, i - qi, j - qj, k - qk)] -= w;
                        phibar[at(n, i - pi, j - pj, k - pk)] += w;
                    }
            }
}

/* Adjoint of the particle deposit M = orc_deposit_xi(xi) with xi = X^-1(y; s)
 * on the mesh of node shifts s = D_c phi.  The deposit gives
 *   xibar_p = wp sum_c Mbar(q_c) grad W_c(xi_p),
 * and the implicit function theorem on x(xi; s) = y (x = xi + sum_c W_c(xi) s_c)
 * turns it into lam_p = J^-T xibar_p with J = dx/dxi, so that
 *   ybar_p += lam_p,  sbar(q_c) -= W_c(xi_p) lam_p  (each component). */
static void deposit_adjoint(const double *s, int n, const double *xi, long np, const double *Mbar, double *sbar,
                            double *ybar)
{
    const double wp = (double)cube(n) / (double)np;
    for (long p = 0; p < np; ++p) {
        const double *q = xi + 3 * p;
        int f[3];
        double t[3];
        for (int a = 0; a < 3; ++a) {
            double fl = floor(q[a]);
            f[a] = (int)fl;
            t[a] = q[a] - fl;
        }
        double xib[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 8; ++c) {
            int o[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
            double w[3], dw[3];
            for (int a = 0; a < 3; ++a) {
                w[a] = o[a] ? t[a] : 1.0 - t[a];
                dw[a] = o[a] ? 1.0 : -1.0;
            }
            double mb = wp * Mbar[at(n, f[0] + o[0], f[1] + o[1], f[2] + o[2])];
            xib[0] += mb * dw[0] * w[1] * w[2];
            xib[1] += mb * w[0] * dw[1] * w[2];
            xib[2] += mb * w[0] * w[1] * dw[2];
        }
        double x[3], J[3][3], inv[3][3], lam[3];
        map_eval(s, n, q, x, J);
        inverse3(J, inv);
        for (int a = 0; a < 3; ++a) {
            lam[a] = inv[0][a] * xib[0] + inv[1][a] * xib[1] + inv[2][a] * xib[2];
            ybar[3 * p + a] += lam[a];
        }
        for (int c = 0; c < 8; ++c) {
            int o[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
            double wc = (o[0] ? t[0] : 1.0 - t[0]) * (o[1] ? t[1] : 1.0 - t[1]) * (o[2] ? t[2] : 1.0 - t[2]);
            double *sb = sbar + 3 * at(n, f[0] + o[0], f[1] + o[1], f[2] + o[2]);
            for (int a = 0; a < 3; ++a) sb[a] -= wc * lam[a];
        }
    }
}

/* Gradient of the loss L(delta_r, phi_out) with respect to the input of the
 * last recorded forward: the density of orc_solve (grad_rho, n^3), or the
 * particle positions of orc_solve_particles with particle_deposit (grad_pos,
 * np x 3, in the units of the positions).  grad_delta = dL/d delta_r,
 * grad_phi = dL/d phi_out (may be NULL).  box as in the forward. */
static int backward_core(const double *grad_delta, const double *grad_phi, double box, const orc_config *cfg,
                         double *grad_rho, double *grad_pos)
{
    const int n = g_tape.n, K = g_tape.steps;
    const long N3 = cube(n);
    const double h = box / n;
    double *phis = (double *)malloc(sizeof(double) * N3 * (K + 1));
    double *tmp = (double *)malloc(sizeof(double) * N3);
    double *phibar = (double *)malloc(sizeof(double) * N3);
    double *mbar = (double *)calloc(N3, sizeof(double));
    double *M = (double *)malloc(sizeof(double) * N3);
    double *ubar = (double *)malloc(sizeof(double) * N3);
    double *lam = (double *)malloc(sizeof(double) * N3);
    double *Mbar = (double *)malloc(sizeof(double) * N3);
    double *tbar = (double *)malloc(sizeof(double) * N3);
    double *hb = (double *)malloc(sizeof(double) * N3 * 9);
    double *xb = (double *)malloc(sizeof(double) * N3 * 3);
    int status = ORC_OK;
    const long np = g_tape.np;
    double *xis = grad_pos ? (double *)malloc(sizeof(double) * 3 * np * (K > 0 ? K : 1)) : NULL;
    double *ybar = grad_pos ? (double *)calloc(3 * np, sizeof(double)) : NULL;

    /* replay the potentials phi_0 .. phi_K exactly as the forward formed them,
     * and (particles) the Lagrangian positions of each step by the forward's
     * own sequence of warm-started inversions */
    memset(phis, 0, sizeof(double) * N3);
    for (int s = 0; s < K; ++s) {
        orc_smooth(g_tape.u[s], n, cfg->smooth_center, tmp);
        for (long p = 0; p < N3; ++p) phis[(s + 1) * N3 + p] = phis[s * N3 + p] + g_tape.alpha[s] * tmp[p];
    }
    for (int s = 0; s < K && grad_pos && status == ORC_OK; ++s) {
        double *xi = xis + (size_t)3 * np * s;
        memcpy(xi, s ? xi - 3 * np : g_tape.y, sizeof(double) * 3 * np);
        status = orc_invert_map(phis + (size_t)s * N3, n, g_tape.y, np, xi, 100, 1e-12);
    }
    /* output: delta_r = -L7 phi_K (L7 symmetric), phi_out = h^2 phi_K */
    orc_delta_r(grad_delta, n, phibar);
    if (grad_phi)
        for (long p = 0; p < N3; ++p) phibar[p] += h * h * grad_phi[p];

    for (int s = K - 1; s >= 0 && status == ORC_OK; --s) {
        const double *phi = phis + s * N3;
        const double *u = g_tape.u[s];
        if (grad_pos) orc_deposit_xi(xis + (size_t)3 * np * s, np, n, M);
        else orc_meshmass(phi, g_tape.m, n, M);
        double rho_bar = field_mean(M, n);
        /* phi_{s+1} = phi_s + alpha S u  ->  ubar = alpha S phibar */
        orc_smooth(phibar, n, cfg->smooth_center, ubar);
        for (long p = 0; p < N3; ++p) ubar[p] *= g_tape.alpha[s];
        /* u = A^+ b (mean-free)  ->  lambda = A^+ (ubar - mean ubar), bbar = lambda */
        double mu = field_mean(ubar, n);
        for (long p = 0; p < N3; ++p) ubar[p] -= mu;
        double rel = 0.0;
        int cyc = orc_mg_solve(M, ubar, n, cfg, lam, &rel);
        if (cyc < 0) {
            status = cyc;
            break;
        }
        /* coefficient gradient, fine level: Mbar_n = 1/2 sum over the unfloored
         * faces of n of (lambda_nb - lambda_n)(u_nb - u_n) */
        int off[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    long c = at(n, i, j, k);
                    double acc = 0.0;
                    for (int f = 0; f < 6; ++f) {
                        long q = at(n, i + off[f][0], j + off[f][1], k + off[f][2]);
                        if (0.5 * (M[c] + M[q]) > cfg->a_min) acc += (lam[q] - lam[c]) * (u[q] - u[c]);
                    }
                    Mbar[c] = 0.5 * acc;
                }
        /* b = S t - mean(S t)  ->  tbar = S (lambda - mean lambda) */
        double ml = field_mean(lam, n);
        for (long p = 0; p < N3; ++p) lam[p] -= ml;
        orc_smooth(lam, n, cfg->smooth_center, tbar);
        /* source: Sigma = rho_bar - M, E = -2 [g > v_m] |Sigma|, C(lambda_0) */
        double sum_sigbar = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    long c = at(n, i, j, k);
                    double e[3][3], v[3];
                    triad(phi, n, i, j, k, e);
                    double g = det3(e);
                    double l0 = eig_min_vec(e, v);
                    double sigma = rho_bar - M[c];
                    double sgn = sigma > 0 ? 1.0 : (sigma < 0 ? -1.0 : 0.0);
                    double sigbar = tbar[c] * (1.0 - (g > cfg->v_m ? 2.0 * sgn : 0.0));
                    /* Sigma = rho_bar - M: Mbar -= sigbar, and every M_k gets mean(sigbar) */
                    Mbar[c] -= sigbar;
                    sum_sigbar += sigbar;
                    double r = cfg->xi_m / l0 - 1.0;
                    double lbar = r > 0.0 ? tbar[c] * 8.0 * r * (-cfg->xi_m / (l0 * l0)) : 0.0;
                    double *hh = hb + c * 9;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) hh[a * 3 + b] = lbar * v[a] * v[b];
                }
        double msb = sum_sigbar / (double)N3;
        for (long p = 0; p < N3; ++p) Mbar[p] += msb;
        /* particles: M from the deposit at xi = X^-1(y; D_c phi); xbar holds
         * the adjoint of the node shifts D_c phi */
        if (grad_pos) {
            double *sh = (double *)malloc(sizeof(double) * 3 * N3);
            node_shifts(phi, n, sh);
            memset(xb, 0, sizeof(double) * N3 * 3);
            deposit_adjoint(sh, n, xis + (size_t)3 * np * s, np, Mbar, xb, ybar);
            free(sh);
        }
        /* M = det(e) * rho~(x):  gbar = Mbar rho~,  xbar = Mbar det(e) grad rho~,
         * mbar += Mbar det(e) W(x - j)  (the transposed CIC deposit) */
        for (int i = 0; i < n && !grad_pos; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    long c = at(n, i, j, k);
                    double e[3][3], cof[3][3], s3[3], x[3];
                    triad(phi, n, i, j, k, e);
                    double g = det3(e);
                    cofactor(e, cof);
                    displacement(phi, n, i, j, k, s3);
                    x[0] = i + s3[0];
                    x[1] = j + s3[1];
                    x[2] = k + s3[2];
                    int f[3];
                    double w1[3];
                    for (int a = 0; a < 3; ++a) {
                        double fl = floor(x[a]);
                        f[a] = (int)fl;
                        w1[a] = x[a] - fl;
                    }
                    double rho_t = 0.0, grad[3] = {0, 0, 0};
                    for (int cc = 0; cc < 8; ++cc) {
                        int o[3] = {(cc >> 2) & 1, (cc >> 1) & 1, cc & 1};
                        double w[3], dw[3];
                        for (int a = 0; a < 3; ++a) {
                            w[a] = o[a] ? w1[a] : 1.0 - w1[a];
                            dw[a] = o[a] ? 1.0 : -1.0;
                        }
                        long q = at(n, f[0] + o[0], f[1] + o[1], f[2] + o[2]);
                        double mv = g_tape.m[q];
                        rho_t += w[0] * w[1] * w[2] * mv;
                        grad[0] += dw[0] * w[1] * w[2] * mv;
                        grad[1] += w[0] * dw[1] * w[2] * mv;
                        grad[2] += w[0] * w[1] * dw[2] * mv;
                        mbar[q] += Mbar[c] * g * w[0] * w[1] * w[2];
                    }
                    double gbar = Mbar[c] * rho_t;
                    double *hh = hb + c * 9;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) hh[a * 3 + b] += gbar * cof[a][b];
                    for (int a = 0; a < 3; ++a) xb[c * 3 + a] = Mbar[c] * g * grad[a];
                }
        /* phi enters through e (Hessian) and x (central differences) */
        hess_transpose_add(hb, n, phibar);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    long c = at(n, i, j, k);
                    /* x_a(n) = n_a + (phi(n+a) - phi(n-a)) / 2 */
                    phibar[at(n, i + 1, j, k)] += 0.5 * xb[c * 3 + 0];
                    phibar[at(n, i - 1, j, k)] -= 0.5 * xb[c * 3 + 0];
                    phibar[at(n, i, j + 1, k)] += 0.5 * xb[c * 3 + 1];
                    phibar[at(n, i, j - 1, k)] -= 0.5 * xb[c * 3 + 1];
                    phibar[at(n, i, j, k + 1)] += 0.5 * xb[c * 3 + 2];
                    phibar[at(n, i, j, k - 1)] -= 0.5 * xb[c * 3 + 2];
                }
    }
    if (status == ORC_OK && grad_pos) {
        /* y = pos n / box */
        for (long p = 0; p < 3 * np; ++p) grad_pos[p] = ybar[p] * ((double)n / box);
    } else if (status == ORC_OK) {
        /* m = rho / mean(rho):  rhobar = (mbar - mean(mbar m)) / mean(rho) */
        double mm = field_dot(mbar, g_tape.m, n) / (double)N3;
        for (long p = 0; p < N3; ++p) grad_rho[p] = (mbar[p] - mm) / g_tape.mean;
    }
    free(xis);
    free(ybar);
    free(phis);
    free(tmp);
    free(phibar);
    free(mbar);
    free(M);
    free(ubar);
    free(lam);
    free(Mbar);
    free(tbar);
    free(hb);
    free(xb);
    return status;
}

int orc_backward(const double *grad_delta, const double *grad_phi, double box, const orc_config *cfg,
                 double *grad_rho)
{
    if (!g_tape.m || g_tape.steps < 0 || !grad_delta || !grad_rho) return ORC_E_NO_TAPE;
    return backward_core(grad_delta, grad_phi, box, cfg, grad_rho, NULL);
}

/* dL/d pos for the last orc_solve_particles run with particle_deposit and
 * record_tape (np x 3, FP64). */
int orc_backward_particles(const double *grad_delta, const double *grad_phi, double box, const orc_config *cfg,
                           double *grad_pos)
{
    if (!g_tape.y || g_tape.steps < 0 || !grad_delta || !grad_pos) return ORC_E_NO_TAPE;
    return backward_core(grad_delta, grad_phi, box, cfg, NULL, grad_pos);
}

long orc_tape_particles(void) { return g_tape.y ? g_tape.np : 0; }
