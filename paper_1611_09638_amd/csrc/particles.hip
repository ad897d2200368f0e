// Particles deposited on the deformed mesh at their Lagrangian positions: for
// a particle at y, the position xi with x(xi) = y under the moving-mesh map
// x = xi + grad phi (Sec. II), taken continuous as xi + S(xi) with S the
// trilinear interpolant of the node shifts s_n = D_c phi_n; then its mass is
// assigned to the xi-grid by CIC.  The mass per curvilinear cell is then
// exactly the particles' (no interpolation of an Eulerian density).
//
// xi is found by Newton's method, xi <- xi - t J^-1 (x(xi) - y) with J the
// derivative of the map in the cell of xi, t = 1 halved (at most 30 times)
// until max |x(xi) - y| (nearest periodic image) decreases; it starts from the
// previous outer step's xi, which is close because the steps are small.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

namespace {

// s_n = D_c phi_n, the three components of a node side by side (s3[3 n + a]),
// so that one corner of a particle's cell is one cache line in the gathers
__global__ void k_node_shifts(const double *__restrict__ phi, double *__restrict__ s3, int n, int ipb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        const size_t c = lin(i, j, k, n);
        s3[3 * c] = 0.5 * (phi[lin(wrapc(i + 1, n), j, k, n)] - phi[lin(wrapc(i - 1, n), j, k, n)]);
        s3[3 * c + 1] = 0.5 * (phi[lin(i, jp, k, n)] - phi[lin(i, jm, k, n)]);
        s3[3 * c + 2] = 0.5 * (phi[lin(i, j, kp, n)] - phi[lin(i, j, km, n)]);
    }
}

struct Shifts {
    const double *s;  // node shifts, three per node
};

// x(xi) - y (nearest image) and its derivative; returns max |x(xi) - y|, or
// +inf (r and J untouched) for a point that is not finite or absurdly far out,
// so that no cell index is ever formed from it
__device__ double map_residual(const Shifts &s, int n, const double xi[3], const double y[3], double r[3],
                               double J[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!(fabs(xi[a]) < 1.0e9)) return INFINITY;
    int f[3];
    double t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double fl = floor(xi[a]);
        t[a] = xi[a] - fl;
        int fi = (int)fl % n;
        f[a] = fi < 0 ? fi + n : fi;
    }
    double x[3] = {xi[0], xi[1], xi[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) J[a][b] = a == b ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
        const double w0 = o0 ? t[0] : 1.0 - t[0], w1 = o1 ? t[1] : 1.0 - t[1], w2 = o2 ? t[2] : 1.0 - t[2];
        const double d0 = o0 ? 1.0 : -1.0, d1 = o1 ? 1.0 : -1.0, d2 = o2 ? 1.0 : -1.0;
        const size_t q = lin(o0 ? wrapc(f[0] + 1, n) : f[0], o1 ? wrapc(f[1] + 1, n) : f[1],
                             o2 ? wrapc(f[2] + 1, n) : f[2], n);
        const double sc[3] = {s.s[3 * q], s.s[3 * q + 1], s.s[3 * q + 2]};
        const double wc = w0 * w1 * w2;
        const double g[3] = {d0 * w1 * w2, w0 * d1 * w2, w0 * w1 * d2};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            x[b] += wc * sc[b];
#pragma unroll
            for (int a = 0; a < 3; ++a) J[b][a] += g[a] * sc[b];
        }
    }
    double mx = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double d = x[a] - y[a];
        d -= n * floor(d / n + 0.5);
        r[a] = d;
        mx = fmax(mx, fabs(d));
    }
    return mx;
}

__global__ void k_init_xi(const float *__restrict__ pos, long long np, double toc, double *__restrict__ xi)
{
    for (long long p = blockIdx.x * 256LL + threadIdx.x; p < 3 * np; p += 256LL * gridDim.x)
        xi[p] = (double)pos[p] * toc;
}

__global__ void k_invert(const float *__restrict__ pos, long long np, double toc, Shifts s, int n,
                         double *__restrict__ xi, int max_iter, double tol, double *part)
{
    double bad[1] = {0.0};
    for (long long p = blockIdx.x * 256LL + threadIdx.x; p < np; p += 256LL * gridDim.x) {
        double y[3], q[3], r[3], J[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            y[a] = (double)pos[3 * p + a] * toc;
            q[a] = xi[3 * p + a];
        }
        double res = map_residual(s, n, q, y, r, J);
        for (int it = 0; res > tol && it < max_iter; ++it) {
            // d = J^-1 r by the adjugate
            const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
            const double a00 = c00, a01 = J[0][2] * J[2][1] - J[0][1] * J[2][2], a02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
            const double a10 = c01, a11 = J[0][0] * J[2][2] - J[0][2] * J[2][0], a12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
            const double a20 = c02, a21 = J[0][1] * J[2][0] - J[0][0] * J[2][1], a22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double d[3] = {(a00 * r[0] + a01 * r[1] + a02 * r[2]) / det,
                                 (a10 * r[0] + a11 * r[1] + a12 * r[2]) / det,
                                 (a20 * r[0] + a21 * r[1] + a22 * r[2]) / det};
            double step = 1.0, trial[3], rt[3], Jt[3][3], rest = res;
            for (int h = 0; h <= 30; ++h, step *= 0.5) {
#pragma unroll
                for (int a = 0; a < 3; ++a) trial[a] = q[a] - step * d[a];
                rest = map_residual(s, n, trial, y, rt, Jt);
                if (rest < res) break;
            }
            if (!(rest < res)) break;  // no descent: left as a failure
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                q[a] = trial[a];
                r[a] = rt[a];
#pragma unroll
                for (int b = 0; b < 3; ++b) J[a][b] = Jt[a][b];
            }
            res = rest;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) xi[3 * p + a] = q[a] - n * floor(q[a] / n);
        if (!(res <= tol)) bad[0] += 1.0;
    }
    block_reduce_store<1, RED_SUM>(bad, part, blockIdx.x);
}

// CIC of the particles at xi (grid units, periodic), weight wp each; a
// particle with a coordinate that is not finite or beyond 1e9 cells is skipped
__global__ void k_deposit_xi(const double *__restrict__ xi, long long np, int n, double wp, double *__restrict__ M)
{
    for (long long p = blockIdx.x * 256LL + threadIdx.x; p < np; p += 256LL * gridDim.x) {
        if (!(fabs(xi[3 * p]) < 1.0e9 && fabs(xi[3 * p + 1]) < 1.0e9 && fabs(xi[3 * p + 2]) < 1.0e9)) continue;
        int f[3];
        double t[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double x = xi[3 * p + a];
            const double fl = floor(x);
            t[a] = x - fl;
            int fi = (int)fl % n;
            f[a] = fi < 0 ? fi + n : fi;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
            const double w = (o0 ? t[0] : 1.0 - t[0]) * (o1 ? t[1] : 1.0 - t[1]) * (o2 ? t[2] : 1.0 - t[2]);
            atomicAdd(&M[lin(o0 ? wrapc(f[0] + 1, n) : f[0], o1 ? wrapc(f[1] + 1, n) : f[1],
                             o2 ? wrapc(f[2] + 1, n) : f[2], n)],
                      wp * w);
        }
    }
}

// The same deposit for n^3 particles stored in lattice order (particle
// (i, j, k) at index (i n + j) n + k): a workgroup takes a DBI x DBJ x DBK
// block of the lattice and sums its particles' CIC weights in an LDS window
// of the nodes around the block (two cells below it to three above), then
// adds the window's non-zero entries to M, one atomic each, instead of eight
// per particle.  A particle with a corner outside the window (displaced by
// two cells or more from its lattice site, or particles not in lattice
// order) adds to M directly, so the result is the same sum in any case.
constexpr int DBI = 2, DBJ = 8, DBK = 16;  // 256 particles per workgroup
constexpr int DEI = DBI + 5, DEJ = DBJ + 5, DEK = DBK + 5;
constexpr int DWIN = DEI * DEJ * DEK;

__global__ void __launch_bounds__(256) k_deposit_block(const double *__restrict__ xi, int n, double wp,
                                                       double *__restrict__ M)
{
    __shared__ double win[DWIN];
    const int tid = threadIdx.x;
    for (int q = tid; q < DWIN; q += 256) win[q] = 0.0;
    const int bk = n / DBK, bj = n / DBJ;
    const int b = blockIdx.x;
    const int i0 = (b / (bj * bk)) * DBI, j0 = ((b / bk) % bj) * DBJ, k0 = (b % bk) * DBK;
    const int li = tid / (DBJ * DBK), lj = (tid / DBK) % DBJ, lk = tid % DBK;
    const long long p = ((long long)(i0 + li) * n + (j0 + lj)) * n + (k0 + lk);
    const int org[3] = {wrapc(i0 - 2, n), wrapc(j0 - 2, n), wrapc(k0 - 2, n)};
    const int ext[3] = {DEI, DEJ, DEK};
    __syncthreads();
    if (fabs(xi[3 * p]) < 1.0e9 && fabs(xi[3 * p + 1]) < 1.0e9 && fabs(xi[3 * p + 2]) < 1.0e9) {
        int f[3], r[3];
        double t[3];
        bool inwin = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double x = xi[3 * p + a];
            const double fl = floor(x);
            t[a] = x - fl;
            int fi = (int)fl % n;
            f[a] = fi < 0 ? fi + n : fi;
            int ra = f[a] - org[a];
            r[a] = ra < 0 ? ra + n : ra;  // in [0, n)
            inwin = inwin && r[a] <= ext[a] - 2;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
            const double w = (o0 ? t[0] : 1.0 - t[0]) * (o1 ? t[1] : 1.0 - t[1]) * (o2 ? t[2] : 1.0 - t[2]);
            if (inwin)
                atomicAdd(&win[((r[0] + o0) * DEJ + (r[1] + o1)) * DEK + (r[2] + o2)], wp * w);
            else
                atomicAdd(&M[lin(o0 ? wrapc(f[0] + 1, n) : f[0], o1 ? wrapc(f[1] + 1, n) : f[1],
                                 o2 ? wrapc(f[2] + 1, n) : f[2], n)],
                          wp * w);
        }
    }
    __syncthreads();
    for (int q = tid; q < DWIN; q += 256) {
        const double v = win[q];
        if (v != 0.0) {
            const int wi = q / (DEJ * DEK), wj = (q / DEK) % DEJ, wk = q % DEK;
            atomicAdd(&M[lin(wrapc(org[0] + wi, n), wrapc(org[1] + wj, n), wrapc(org[2] + wk, n), n)], v);
        }
    }
}

bool deposit_block_fits(long long np, int n)
{
    return n >= 32 && n % DBK == 0 && n % DBJ == 0 && n % DBI == 0 && np == (long long)n * n * n;
}

// Adjoint of the deposit at xi = X^-1(y; s) (s = D_c phi): per particle,
//   xibar = wp sum_c Mbar(q_c) grad W_c(xi),  lam = J^-T xibar,
// with J = dx/dxi in the cell of xi (implicit function theorem on
// x(xi; s) = y); then gpos += gscale lam (the particle's own entry) and
// sbar(q_c) -= W_c(xi) lam, component by component, with FP64 atomics.
// One particle of the deposit's adjoint: its cell f and offsets t, the eight
// corner nodes q and weights wc, and lam = J^-T xibar; gpos gets gscale lam.
// Returns false (nothing done) for a position that is not finite or beyond
// 1e9 cells.
__device__ __forceinline__ bool deposit_adj_particle(const double *__restrict__ xi, long long p, const Shifts &s,
                                                     int n, double wp, const double *__restrict__ Mbar,
                                                     double *__restrict__ gpos, double gscale, int f[3],
                                                     size_t q[8], double wc[8], double lam[3])
{
    if (!(fabs(xi[3 * p]) < 1.0e9 && fabs(xi[3 * p + 1]) < 1.0e9 && fabs(xi[3 * p + 2]) < 1.0e9)) return false;
    double t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double x = xi[3 * p + a];
        const double fl = floor(x);
        t[a] = x - fl;
        int fi = (int)fl % n;
        f[a] = fi < 0 ? fi + n : fi;
    }
    double xb[3] = {0.0, 0.0, 0.0};
    double J[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
        const double w0 = o0 ? t[0] : 1.0 - t[0], w1 = o1 ? t[1] : 1.0 - t[1], w2 = o2 ? t[2] : 1.0 - t[2];
        const double d0 = o0 ? 1.0 : -1.0, d1 = o1 ? 1.0 : -1.0, d2 = o2 ? 1.0 : -1.0;
        q[c] = lin(o0 ? wrapc(f[0] + 1, n) : f[0], o1 ? wrapc(f[1] + 1, n) : f[1], o2 ? wrapc(f[2] + 1, n) : f[2], n);
        wc[c] = w0 * w1 * w2;
        const double g[3] = {d0 * w1 * w2, w0 * d1 * w2, w0 * w1 * d2};
        const double mb = wp * Mbar[q[c]];
        const double sc[3] = {s.s[3 * q[c]], s.s[3 * q[c] + 1], s.s[3 * q[c] + 2]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xb[a] += mb * g[a];
#pragma unroll
            for (int b = 0; b < 3; ++b) J[b][a] += g[a] * sc[b];
        }
    }
    // lam = J^-T xibar by the adjugate: (J^-1)_{ba} = adj_{ba} / det
    const double a00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], a01 = J[0][2] * J[2][1] - J[0][1] * J[2][2],
                 a02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    const double a10 = J[1][2] * J[2][0] - J[1][0] * J[2][2], a11 = J[0][0] * J[2][2] - J[0][2] * J[2][0],
                 a12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    const double a20 = J[1][0] * J[2][1] - J[1][1] * J[2][0], a21 = J[0][1] * J[2][0] - J[0][0] * J[2][1],
                 a22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * a00 + J[0][1] * a10 + J[0][2] * a20;
    lam[0] = (a00 * xb[0] + a10 * xb[1] + a20 * xb[2]) / det;
    lam[1] = (a01 * xb[0] + a11 * xb[1] + a21 * xb[2]) / det;
    lam[2] = (a02 * xb[0] + a12 * xb[1] + a22 * xb[2]) / det;
#pragma unroll
    for (int a = 0; a < 3; ++a) gpos[3 * p + a] += gscale * lam[a];
    return true;
}

__global__ void k_deposit_adj(const double *__restrict__ xi, long long np, Shifts s, int n, double wp,
                              const double *__restrict__ Mbar, double *__restrict__ sbx, double *__restrict__ sby,
                              double *__restrict__ sbz, double *__restrict__ gpos, double gscale)
{
    for (long long p = blockIdx.x * 256LL + threadIdx.x; p < np; p += 256LL * gridDim.x) {
        int f[3];
        size_t q[8];
        double wc[8], lam[3];
        if (!deposit_adj_particle(xi, p, s, n, wp, Mbar, gpos, gscale, f, q, wc, lam)) continue;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            atomicAdd(&sbx[q[c]], -wc[c] * lam[0]);
            atomicAdd(&sby[q[c]], -wc[c] * lam[1]);
            atomicAdd(&sbz[q[c]], -wc[c] * lam[2]);
        }
    }
}

// The same for n^3 particles in lattice order, with the scatter of sbar summed
// in three LDS windows around the workgroup's lattice block as in
// k_deposit_block (particles with a corner outside go straight to sbar).
__global__ void __launch_bounds__(256) k_deposit_adj_block(const double *__restrict__ xi, Shifts s, int n,
                                                           double wp, const double *__restrict__ Mbar,
                                                           double *__restrict__ sbx, double *__restrict__ sby,
                                                           double *__restrict__ sbz, double *__restrict__ gpos,
                                                           double gscale)
{
    __shared__ double win[3][DWIN];
    const int tid = threadIdx.x;
    for (int q = tid; q < DWIN; q += 256) win[0][q] = win[1][q] = win[2][q] = 0.0;
    const int bk = n / DBK, bj = n / DBJ;
    const int b = blockIdx.x;
    const int i0 = (b / (bj * bk)) * DBI, j0 = ((b / bk) % bj) * DBJ, k0 = (b % bk) * DBK;
    const int li = tid / (DBJ * DBK), lj = (tid / DBK) % DBJ, lk = tid % DBK;
    const long long p = ((long long)(i0 + li) * n + (j0 + lj)) * n + (k0 + lk);
    const int org[3] = {wrapc(i0 - 2, n), wrapc(j0 - 2, n), wrapc(k0 - 2, n)};
    const int ext[3] = {DEI, DEJ, DEK};
    __syncthreads();
    int f[3];
    size_t q[8];
    double wc[8], lam[3];
    if (deposit_adj_particle(xi, p, s, n, wp, Mbar, gpos, gscale, f, q, wc, lam)) {
        int r[3];
        bool inwin = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int ra = f[a] - org[a];
            r[a] = ra < 0 ? ra + n : ra;  // in [0, n)
            inwin = inwin && r[a] <= ext[a] - 2;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
            if (inwin) {
                const int w = ((r[0] + o0) * DEJ + (r[1] + o1)) * DEK + (r[2] + o2);
                atomicAdd(&win[0][w], -wc[c] * lam[0]);
                atomicAdd(&win[1][w], -wc[c] * lam[1]);
                atomicAdd(&win[2][w], -wc[c] * lam[2]);
            } else {
                atomicAdd(&sbx[q[c]], -wc[c] * lam[0]);
                atomicAdd(&sby[q[c]], -wc[c] * lam[1]);
                atomicAdd(&sbz[q[c]], -wc[c] * lam[2]);
            }
        }
    }
    __syncthreads();
    for (int w = tid; w < DWIN; w += 256) {
        const int wi = w / (DEJ * DEK), wj = (w / DEK) % DEJ, wk = w % DEK;
        const size_t g = lin(wrapc(org[0] + wi, n), wrapc(org[1] + wj, n), wrapc(org[2] + wk, n), n);
        if (win[0][w] != 0.0) atomicAdd(&sbx[g], win[0][w]);
        if (win[1][w] != 0.0) atomicAdd(&sby[g], win[1][w]);
        if (win[2][w] != 0.0) atomicAdd(&sbz[g], win[2][w]);
    }
}

int particle_blocks(long long np)
{
    long long b = (np + 255) / 256;
    int nb = (int)(b < 8192 ? b : 8192);
    return nb < 1 ? 1 : nb;
}

}  // namespace

hipError_t launch_init_xi(const float *pos, long long np, int n, double box, double *xi, hipStream_t s)
{
    k_init_xi<<<particle_blocks(3 * np), 256, 0, s>>>(pos, np, (double)n / box, xi);
    return hipGetLastError();
}

hipError_t launch_invert_map(const double *phi, const float *pos, long long np, int n, double box, double *xi,
                             double *s3, int max_iter, double tol, Part &p, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_node_shifts<<<sh.grid, sh.block, 0, s>>>(phi, s3, n, sh.ipb);
    const int nb = particle_blocks(np);
    if (nb > kPartCap) return hipErrorInvalidValue;
    k_invert<<<nb, 256, 0, s>>>(pos, np, (double)n / box, Shifts{s3}, n, xi, max_iter, tol, p.part);
    p.blocks = nb;
    p.k = 1;
    return hipGetLastError();
}

hipError_t launch_deposit_xi(const double *xi, long long np, int n, double *M, hipStream_t s)
{
    hipError_t e = launch_zero(M, (long)n * n * n * 8, s);
    if (e != hipSuccess) return e;
    const double wp = (double)n * n * n / (double)np;
    if (deposit_block_fits(np, n))
        k_deposit_block<<<(unsigned)(np / 256), 256, 0, s>>>(xi, n, wp, M);
    else
        k_deposit_xi<<<particle_blocks(np), 256, 0, s>>>(xi, np, n, wp, M);
    return hipGetLastError();
}

hipError_t launch_node_shifts(const double *phi, double *s3, int n, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_node_shifts<<<sh.grid, sh.block, 0, s>>>(phi, s3, n, sh.ipb);
    return hipGetLastError();
}

hipError_t launch_deposit_adj(const double *xi, long long np, int n, const double *s3, const double *Mbar,
                              double *sbar, double *gpos, double gscale, hipStream_t s)
{
    const size_t n3 = (size_t)n * n * n;
    const double wp = (double)n3 / (double)np;
    if (deposit_block_fits(np, n))
        k_deposit_adj_block<<<(unsigned)(np / 256), 256, 0, s>>>(xi, Shifts{s3}, n, wp, Mbar, sbar,
                                                                 sbar + n3, sbar + 2 * n3, gpos, gscale);
    else
        k_deposit_adj<<<particle_blocks(np), 256, 0, s>>>(xi, np, Shifts{s3}, n, wp, Mbar, sbar, sbar + n3,
                                                          sbar + 2 * n3, gpos, gscale);
    return hipGetLastError();
}

}  // namespace recon
