// gfx950 kernels of the reverse mode (adjoint) of the reconstruction.
//
// Forward step (grid units): M = det(e) rho~(xi + D_c phi), e = I + Hess phi;
// Sigma = mean(M) - M; t = Sigma + C(lambda_0(e)) - 2 [det e > v_m] |Sigma|;
// b = S t - mean; u = A(M)^+ b; phi' = phi + alpha S u.  With alpha and the
// limiter masks held fixed, each kernel below is the transpose of one of
// these maps, evaluated at the recomputed forward state.  Partials with
// respect to e are kept per node as six fields (xx, yy, zz, xy, xz, yz),
// derivatives with respect to the matrix entries; an off-diagonal pair
// e_ab = e_ba is one Hessian entry, hence the factor 2 in the transpose.
#include "device_common.h"

namespace recon {

// phibar = -L7 g_delta + h^2 g_phi   (delta_r = -L7 phi, phi_out = h^2 phi)
__global__ void k_out_adj(const double *__restrict__ gd, const double *__restrict__ gp, double h2,
                          double *__restrict__ phibar, int n, int ipb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
        const size_t p = lin(i, j, k, n);
        const double lap = gd[lin(ip, j, k, n)] + gd[lin(im, j, k, n)] + gd[lin(i, jp, k, n)] + gd[lin(i, jm, k, n)]
                         + gd[lin(i, j, kp, n)] + gd[lin(i, j, km, n)] - 6.0 * gd[p];
        phibar[p] = -lap + (gp ? h2 * gp[p] : 0.0);
    }
}

hipError_t launch_out_adj(const double *gd, const double *gp, double h2, double *phibar, int n, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_out_adj<<<sh.grid, sh.block, 0, s>>>(gd, gp, h2, phibar, n, sh.ipb);
    return hipGetLastError();
}

// out = scale * S f  (S symmetric, so this is also its transpose)
__global__ void k_smooth_scaled(const double *__restrict__ f, double *__restrict__ out, int n, int ipb, double c0,
                                double cn, double scale)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
        const double nb = f[lin(ip, j, k, n)] + f[lin(im, j, k, n)] + f[lin(i, jp, k, n)] + f[lin(i, jm, k, n)]
                        + f[lin(i, j, kp, n)] + f[lin(i, j, km, n)];
        out[lin(i, j, k, n)] = scale * (c0 * f[lin(i, j, k, n)] + cn * nb);
    }
}

hipError_t launch_smooth_scaled(const double *f, double *out, int n, double c0, double scale, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_smooth_scaled<<<sh.grid, sh.block, 0, s>>>(f, out, n, sh.ipb, c0, (1.0 - c0) / 6.0, scale);
    return hipGetLastError();
}

// Coefficient gradient of u = A(M)^+ b on the fine level: with lambda =
// A^+ ubar, du = -A^+ (dA) u gives cbar_f = (lambda_nb - lambda_n)(u_nb - u_n)
// for each face whose coefficient (M_n + M_nb)/2 is above the floor, shared
// equally by its two nodes.
__global__ void k_coefgrad(const double *__restrict__ lam, const double *__restrict__ u, const double *__restrict__ M,
                           double a_min, double *__restrict__ Mbar, int n, int ipb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
        const size_t p = lin(i, j, k, n);
        const size_t q[6] = {lin(ip, j, k, n), lin(im, j, k, n), lin(i, jp, k, n),
                             lin(i, jm, k, n), lin(i, j, kp, n), lin(i, j, km, n)};
        const double ln = lam[p], un = u[p], mn = M[p];
        double acc = 0.0;
#pragma unroll
        for (int f = 0; f < 6; ++f)
            if (0.5 * (mn + M[q[f]]) > a_min) acc += (lam[q[f]] - ln) * (u[q[f]] - un);
        Mbar[p] = 0.5 * acc;
    }
}

hipError_t launch_coefgrad(const double *lam, const double *u, const double *M, double a_min, double *Mbar, int n,
                           hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_coefgrad<<<sh.grid, sh.block, 0, s>>>(lam, u, M, a_min, Mbar, n, sh.ipb);
    return hipGetLastError();
}

// Unit eigenvector of a symmetric 3x3 matrix for the eigenvalue lam: the
// largest cross product of two rows of e - lam I (the rows span the
// orthogonal complement of the eigenvector when lam is simple).
__device__ void eigvec_sym(const Sym3 &e, double lam, double v[3])
{
    const double r0[3] = {e.xx - lam, e.xy, e.xz};
    const double r1[3] = {e.xy, e.yy - lam, e.yz};
    const double r2[3] = {e.xz, e.yz, e.zz - lam};
    double c[3][3];
    const double *ra[3] = {r0, r0, r1}, *rb[3] = {r1, r2, r2};
    int best = 0;
    double bn = -1.0;
    for (int t = 0; t < 3; ++t) {
        c[t][0] = ra[t][1] * rb[t][2] - ra[t][2] * rb[t][1];
        c[t][1] = ra[t][2] * rb[t][0] - ra[t][0] * rb[t][2];
        c[t][2] = ra[t][0] * rb[t][1] - ra[t][1] * rb[t][0];
        const double nn = c[t][0] * c[t][0] + c[t][1] * c[t][1] + c[t][2] * c[t][2];
        if (nn > bn) {
            bn = nn;
            best = t;
        }
    }
    if (bn > 0.0) {
        const double s = 1.0 / sqrt(bn);
        v[0] = c[best][0] * s;
        v[1] = c[best][1] * s;
        v[2] = c[best][2] * s;
    } else {
        // repeated eigenvalue: any unit vector orthogonal to the largest row
        const double *rows[3] = {r0, r1, r2};
        int rm = 0;
        double mn = -1.0;
        for (int t = 0; t < 3; ++t) {
            const double nn = rows[t][0] * rows[t][0] + rows[t][1] * rows[t][1] + rows[t][2] * rows[t][2];
            if (nn > mn) {
                mn = nn;
                rm = t;
            }
        }
        const double *r = rows[rm];
        double w[3] = {r[1], -r[0], 0.0};
        double nn = w[0] * w[0] + w[1] * w[1];
        if (nn <= 0.0) {
            w[0] = 0.0;
            w[1] = r[2];
            w[2] = -r[1];
            nn = w[1] * w[1] + w[2] * w[2];
        }
        if (nn <= 0.0) {
            v[0] = 1.0;
            v[1] = v[2] = 0.0;
        } else {
            const double s = 1.0 / sqrt(nn);
            v[0] = w[0] * s;
            v[1] = w[1] * s;
            v[2] = w[2] * s;
        }
    }
}

// Source adjoint.  tbar -> Sigmabar = tbar (1 - 2 [det e > v_m] sign Sigma),
// Mbar -= Sigmabar (the mean(M) part is added afterwards from the partial
// sums), lambda_0bar = tbar dC/dlambda_0 -> ebar = lambda_0bar v v^T.
__global__ void k_source_adj(const double *__restrict__ phi, const double *__restrict__ M, double rho_bar,
                             const double *__restrict__ tbar, double xi_m, double v_m, double *__restrict__ Mbar,
                             double *__restrict__ hb, int n, int ipb, double *part)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const size_t n3 = (size_t)n * n * n;
    double v1[1] = {0.0};
    if (k < n && j < n) {
        const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
        for (int i = i0; i < i1; ++i) {
            Stencil19 s;
            load19(phi, i, j, k, n, s);
            const Sym3 e = triad19(s);
            const double g = det_sym(e);
            const size_t p = lin(i, j, k, n);
            const double tb = tbar[p];
            const double sigma = rho_bar - M[p];
            const double sgn = sigma > 0.0 ? 1.0 : (sigma < 0.0 ? -1.0 : 0.0);
            const double sigbar = tb * (1.0 - (g > v_m ? 2.0 * sgn : 0.0));
            Mbar[p] -= sigbar;
            v1[0] += sigbar;
            const double l0 = lambda_min_sym(e);
            const double r = xi_m / l0 - 1.0;
            double h6[6] = {0, 0, 0, 0, 0, 0};
            if (r > 0.0) {
                const double lbar = tb * 8.0 * r * (-xi_m / (l0 * l0));
                double v[3];
                eigvec_sym(e, l0, v);
                h6[0] = lbar * v[0] * v[0];
                h6[1] = lbar * v[1] * v[1];
                h6[2] = lbar * v[2] * v[2];
                h6[3] = lbar * v[0] * v[1];
                h6[4] = lbar * v[0] * v[2];
                h6[5] = lbar * v[1] * v[2];
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) hb[c * n3 + p] = h6[c];
        }
    }
    block_reduce_store<1, RED_SUM>(v1, part, block_row());
}

hipError_t launch_source_adj(const double *phi, const double *M, double rho_bar, const double *tbar, double xi_m,
                             double v_m, double *Mbar, double *hb, int n, Part &p, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_source_adj<<<sh.grid, sh.block, 0, s>>>(phi, M, rho_bar, tbar, xi_m, v_m, Mbar, hb, n, sh.ipb, p.part);
    p.blocks = rows_of(sh);
    p.k = 1;
    return hipGetLastError();
}

// Deformed-mesh mass adjoint, M = det(e) rho~(x):
//   ebar += Mbar rho~(x) cof(e);  xbar = Mbar det(e) grad rho~(x);
//   mbar_j += Mbar det(e) W(x - j)   (the transposed CIC deposit: an FP64
//   atomic scatter, the one order-dependent sum of the adjoint).
__global__ void k_meshmass_adj(const double *__restrict__ phi, const double *__restrict__ m,
                               const double *__restrict__ Mbar, double *__restrict__ hb, double *__restrict__ xb,
                               double *__restrict__ mbar, int n, int ipb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const size_t n3 = (size_t)n * n * n;
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        Stencil19 s;
        load19(phi, i, j, k, n, s);
        const Sym3 e = triad19(s);
        const double g = det_sym(e);
        const double x[3] = {i + 0.5 * (s.xp - s.xm), j + 0.5 * (s.yp - s.ym), k + 0.5 * (s.zp - s.zm)};
        int f0[3], f1[3];
        double w1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double fl = floor(x[a]);
            w1[a] = x[a] - fl;
            int fi = (int)fl % n;
            fi = fi < 0 ? fi + n : fi;
            f0[a] = fi;
            f1[a] = fi + 1 == n ? 0 : fi + 1;
        }
        const size_t p = lin(i, j, k, n);
        const double mb = Mbar[p];
        const double mg = mb * g;
        double rho_t = 0.0, gr0 = 0.0, gr1 = 0.0, gr2 = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
            const double wa = o0 ? w1[0] : 1.0 - w1[0], wb = o1 ? w1[1] : 1.0 - w1[1], wc = o2 ? w1[2] : 1.0 - w1[2];
            const size_t q = lin(o0 ? f1[0] : f0[0], o1 ? f1[1] : f0[1], o2 ? f1[2] : f0[2], n);
            const double mv = m[q];
            rho_t += wa * wb * wc * mv;
            gr0 += (o0 ? 1.0 : -1.0) * wb * wc * mv;
            gr1 += wa * (o1 ? 1.0 : -1.0) * wc * mv;
            gr2 += wa * wb * (o2 ? 1.0 : -1.0) * mv;
            if (mg != 0.0) atomicAdd(&mbar[q], mg * wa * wb * wc);
        }
        const double gb = mb * rho_t;
        // cofactors of the symmetric e
        const double cxx = e.yy * e.zz - e.yz * e.yz, cyy = e.xx * e.zz - e.xz * e.xz, czz = e.xx * e.yy - e.xy * e.xy;
        const double cxy = -(e.xy * e.zz - e.yz * e.xz), cxz = e.xy * e.yz - e.yy * e.xz;
        const double cyz = -(e.xx * e.yz - e.xy * e.xz);
        hb[0 * n3 + p] += gb * cxx;
        hb[1 * n3 + p] += gb * cyy;
        hb[2 * n3 + p] += gb * czz;
        hb[3 * n3 + p] += gb * cxy;
        hb[4 * n3 + p] += gb * cxz;
        hb[5 * n3 + p] += gb * cyz;
        xb[0 * n3 + p] = mg * gr0;
        xb[1 * n3 + p] = mg * gr1;
        xb[2 * n3 + p] = mg * gr2;
    }
}

hipError_t launch_meshmass_adj(const double *phi, const double *m, const double *Mbar, double *hb, double *xb,
                               double *mbar, int n, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_meshmass_adj<<<sh.grid, sh.block, 0, s>>>(phi, m, Mbar, hb, xb, mbar, n, sh.ipb);
    return hipGetLastError();
}

// phibar += Hess^T ebar + D_c^T xbar, gathered at each node:
//   diagonal  H_aa(n) = phi(n+a) - 2 phi(n) + phi(n-a)
//   cross     H_ab(n) = (phi(n+a+b) - phi(n+a-b) - phi(n-a+b) + phi(n-a-b)) / 4, weight 2 ebar_ab
//   shift     x_a(n)  = n_a + (phi(n+a) - phi(n-a)) / 2
__global__ void k_phibar_update(const double *__restrict__ hb, const double *__restrict__ xb,
                                double *__restrict__ phibar, int n, int ipb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const size_t n3 = (size_t)n * n * n;
    const double *hxx = hb, *hyy = hb + n3, *hzz = hb + 2 * n3, *hxy = hb + 3 * n3, *hxz = hb + 4 * n3,
                 *hyz = hb + 5 * n3;
    const double *xx = xb, *xy = xb + n3, *xz = xb + 2 * n3;
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
        const size_t p = lin(i, j, k, n);
        double acc = 0.0;
        acc += hxx[lin(im, j, k, n)] - 2.0 * hxx[p] + hxx[lin(ip, j, k, n)];
        acc += hyy[lin(i, jm, k, n)] - 2.0 * hyy[p] + hyy[lin(i, jp, k, n)];
        acc += hzz[lin(i, j, km, n)] - 2.0 * hzz[p] + hzz[lin(i, j, kp, n)];
        acc += 0.5 * (hxy[lin(im, jm, k, n)] - hxy[lin(im, jp, k, n)] - hxy[lin(ip, jm, k, n)] + hxy[lin(ip, jp, k, n)]);
        acc += 0.5 * (hxz[lin(im, j, km, n)] - hxz[lin(im, j, kp, n)] - hxz[lin(ip, j, km, n)] + hxz[lin(ip, j, kp, n)]);
        acc += 0.5 * (hyz[lin(i, jm, km, n)] - hyz[lin(i, jm, kp, n)] - hyz[lin(i, jp, km, n)] + hyz[lin(i, jp, kp, n)]);
        acc += 0.5 * (xx[lin(im, j, k, n)] - xx[lin(ip, j, k, n)]);
        acc += 0.5 * (xy[lin(i, jm, k, n)] - xy[lin(i, jp, k, n)]);
        acc += 0.5 * (xz[lin(i, j, km, n)] - xz[lin(i, j, kp, n)]);
        phibar[p] += acc;
    }
}

hipError_t launch_phibar_update(const double *hb, const double *xb, double *phibar, int n, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_phibar_update<<<sh.grid, sh.block, 0, s>>>(hb, xb, phibar, n, sh.ipb);
    return hipGetLastError();
}

// partial sums of a . b
__global__ void k_dot(const double *__restrict__ a, const double *__restrict__ b, long n3, double *part)
{
    double v[1] = {0.0};
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) v[0] += a[p] * b[p];
    block_reduce_store<1, RED_SUM>(v, part, blockIdx.x);
}

hipError_t launch_dot(const double *a, const double *b, long n3, Part &p, hipStream_t s)
{
    const int nb = flat_blocks(n3);
    k_dot<<<nb, 256, 0, s>>>(a, b, n3, p.part);
    p.blocks = nb;
    p.k = 1;
    return hipGetLastError();
}

// m = rho / mu:  rhobar = (mbar - mm) / mu  with mm = mean(mbar m)
__global__ void k_rho_grad(const double *__restrict__ mbar, double mm, double inv_mu, double *__restrict__ g,
                           long n3)
{
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) g[p] = (mbar[p] - mm) * inv_mu;
}

hipError_t launch_rho_grad(const double *mbar, double mm, double mu, double *g, long n3, hipStream_t s)
{
    k_rho_grad<<<flat_blocks(n3), 256, 0, s>>>(mbar, mm, 1.0 / mu, g, n3);
    return hipGetLastError();
}

}  // namespace recon
