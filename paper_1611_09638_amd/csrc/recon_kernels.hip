// gfx950 kernels of the nonlinear reconstruction (Zhu, Yu, Pen, Chen & Yu,
// arXiv:1611.09638): deformed-mesh mass, limited source, smoothing, the
// multigrid pieces of the elliptic solve, Krylov vector updates, step
// control and output.  Every kernel is a nearest-neighbour stencil or a
// stream over HBM (<= 0.5 flop/byte), so none uses MFMA; they are written for
// coalesced 64-wide wavefront access along the fastest (k) axis.
//
// Lattice: n^3, C-order [i][j][k] (k fastest), periodic, grid units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "kernels.h"

namespace recon {

struct OpsK {
    int op[8];
};

__global__ void k_finalize(const double *__restrict__ part, int rows, int K, OpsK ops, double *__restrict__ out)
{
    __shared__ double sm[256];
    const int t = threadIdx.x;
    for (int c = 0; c < K; ++c) {
        const int op = ops.op[c];
        auto fold = [op](double x, double y) {
            return op == RED_SUM ? x + y : (op == RED_MAX ? (x > y ? x : y) : (x < y ? x : y));
        };
        double x = op == RED_SUM ? 0.0 : (op == RED_MAX ? -INFINITY : INFINITY);
        // rows t, t + 256, ... in order; eight loads in flight at a time
        int r = t;
        for (; r + 7 * 256 < rows; r += 8 * 256) {
            double y[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) y[v] = part[(size_t)(r + v * 256) * K + c];
#pragma unroll
            for (int v = 0; v < 8; ++v) x = fold(x, y[v]);
        }
        for (; r < rows; r += 256) x = fold(x, part[(size_t)r * K + c]);
        sm[t] = x;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w) sm[t] = fold(sm[t], sm[t + w]);
            __syncthreads();
        }
        if (t == 0) out[c] = sm[0];
        __syncthreads();
    }
}

hipError_t reduce_finalize(const Part &p, const int *ops, double *out, hipStream_t s)
{
    OpsK o;
    for (int c = 0; c < 8; ++c) o.op[c] = c < p.k ? ops[c] : RED_SUM;
    k_finalize<<<1, 256, 0, s>>>(p.part, p.blocks, p.k, o, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------- input

__global__ void k_check_input(const double *__restrict__ rho, long n3, double *part)
{
    double v[2] = {0.0, 0.0};
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) {
        double x = rho[p];
        if (!(x >= 0.0) || !isfinite(x)) v[1] += 1.0;
        else v[0] += x;
    }
    block_reduce_store<2, RED_SUM>(v, part, blockIdx.x);
}

hipError_t launch_check_input(const double *rho, long n3, Part &p, hipStream_t s)
{
    int nb = flat_blocks(n3);
    k_check_input<<<nb, 256, 0, s>>>(rho, n3, p.part);
    p.blocks = nb;
    p.k = 2;
    return hipGetLastError();
}

__global__ void k_scale(const double *__restrict__ rho, double *__restrict__ m, long n3, const double *mean)
{
    const double mu = *mean;
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) m[p] = rho[p] / mu;
}

hipError_t launch_scale(const double *rho, double *m, long n3, const double *mean_dev, hipStream_t s)
{
    k_scale<<<flat_blocks(n3), 256, 0, s>>>(rho, m, n3, mean_dev);
    return hipGetLastError();
}

__global__ void k_fill(double *__restrict__ f, long n3, double v)
{
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) f[p] = v;
}

hipError_t launch_fill(double *f, long n3, double v, hipStream_t s)
{
    k_fill<<<flat_blocks(n3), 256, 0, s>>>(f, n3, v);
    return hipGetLastError();
}

__global__ void k_zero_words(unsigned *__restrict__ f, long words)
{
    for (long p = blockIdx.x * 256L + threadIdx.x; p < words; p += 256L * gridDim.x) f[p] = 0u;
}

hipError_t launch_zero(void *f, long bytes, hipStream_t s)
{
    long words = bytes / 4;
    k_zero_words<<<flat_blocks(words), 256, 0, s>>>((unsigned *)f, words);
    return hipGetLastError();
}

__global__ void k_copy(double *__restrict__ d, const double *__restrict__ src, long n3)
{
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) d[p] = src[p];
}

hipError_t launch_copy(double *dst, const double *src, long n3, hipStream_t s)
{
    k_copy<<<flat_blocks(n3), 256, 0, s>>>(dst, src, n3);
    return hipGetLastError();
}

// Cloud-in-cell assignment of particles to the vertex-centred lattice
// (Sec. III gridding).  FP64 atomics: the only order-dependent sum here.
__global__ void k_cic(const float *__restrict__ pos, long long np, int n, double toc, double *__restrict__ rho)
{
    for (long long p = blockIdx.x * 256LL + threadIdx.x; p < np; p += 256LL * gridDim.x) {
        double x[3], w1[3];
        int f[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x[a] = (double)pos[3 * p + a] * toc;
            double fl = floor(x[a]);
            w1[a] = x[a] - fl;
            int fi = (int)fl % n;
            f[a] = fi < 0 ? fi + n : fi;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
            const double w = (o0 ? w1[0] : 1.0 - w1[0]) * (o1 ? w1[1] : 1.0 - w1[1]) * (o2 ? w1[2] : 1.0 - w1[2]);
            const int i = o0 ? wrapc(f[0] + 1, n) : f[0];
            const int j = o1 ? wrapc(f[1] + 1, n) : f[1];
            const int k = o2 ? wrapc(f[2] + 1, n) : f[2];
            atomicAdd(&rho[lin(i, j, k, n)], w);
        }
    }
}

hipError_t launch_cic(const float *pos, long long np, int n, double box, double *rho, hipStream_t s)
{
    long long b = (np + 255) / 256;
    int nb = (int)(b < 65536 ? b : 65536);
    if (nb < 1) nb = 1;
    k_cic<<<nb, 256, 0, s>>>(pos, np, n, (double)n / box, rho);
    return hipGetLastError();
}

// ---------------------------------------------- mass on the deformed mesh

// M_n = det(I + H_n) * trilinear interpolant of m at x_n = n + D_c phi_n
// (rho sqrt g of App. A evaluated on the current curvilinear mesh).
__global__ void k_meshmass(const double *__restrict__ phi, const double *__restrict__ m, double *__restrict__ M,
                           int n, int ipb, double *part)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double v[1] = {0.0};
    if (k < n && j < n) {
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
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int o0 = (c >> 2) & 1, o1 = (c >> 1) & 1, o2 = c & 1;
                const double w = (o0 ? w1[0] : 1.0 - w1[0]) * (o1 ? w1[1] : 1.0 - w1[1]) * (o2 ? w1[2] : 1.0 - w1[2]);
                acc += w * m[lin(o0 ? f1[0] : f0[0], o1 ? f1[1] : f0[1], o2 ? f1[2] : f0[2], n)];
            }
            const double Mv = g * acc;
            M[lin(i, j, k, n)] = Mv;
            v[0] += Mv;
        }
    }
    block_reduce_store<1, RED_SUM>(v, part, block_row());
}

hipError_t launch_meshmass(const double *phi, const double *m, double *M, int n, Part &p, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_meshmass<<<sh.grid, sh.block, 0, s>>>(phi, m, M, n, sh.ipb, p.part);
    p.blocks = rows_of(sh);
    p.k = 1;
    return hipGetLastError();
}

// ------------------------------------------------------------------ source

// t = Sigma + C + E with Sigma = rho_bar - M, C = 4 max(0, xi_m/lambda_0 - 1)^2,
// E = -2 [sqrt g > v_m] |Sigma|  (App. A, Eq. elliptic and the limiters).
__global__ void k_source(const double *__restrict__ phi, const double *__restrict__ M, double rho_bar, double xi_m,
                         double v_m, double *__restrict__ t, int n, int ipb, double *part)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double v[2] = {0.0, 0.0};
    if (k < n && j < n) {
        const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
        for (int i = i0; i < i1; ++i) {
            Stencil19 s;
            load19(phi, i, j, k, n, s);
            const Sym3 e = triad19(s);
            const double g = det_sym(e);
            const size_t p = lin(i, j, k, n);
            const double sigma = rho_bar - M[p];
            const double C = compression_limiter(e, xi_m);
            const double E = g > v_m ? -2.0 * fabs(sigma) : 0.0;
            const double tv = sigma + C + E;
            t[p] = tv;
            v[0] += sigma * sigma;
            v[1] += tv;
        }
    }
    block_reduce_store<2, RED_SUM>(v, part, block_row());
}

hipError_t launch_source(const double *phi, const double *M, double rho_bar, double xi_m, double v_m, double *t, int n,
                         Part &p, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_source<<<sh.grid, sh.block, 0, s>>>(phi, M, rho_bar, xi_m, v_m, t, n, sh.ipb, p.part);
    p.blocks = rows_of(sh);
    p.k = 2;
    return hipGetLastError();
}

// S f = c0 f + (1 - c0)/6 * (six nearest neighbours), minus a constant (the
// mean, so that the smoothed source is mean-free).
__global__ void k_smooth(const double *__restrict__ f, double *__restrict__ out, int n, int ipb, double c0, double cn,
                         double sv)
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
        out[lin(i, j, k, n)] = c0 * f[lin(i, j, k, n)] + cn * nb - sv;
    }
}

hipError_t launch_smooth(const double *f, double *out, int n, double c0, double sub, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_smooth<<<sh.grid, sh.block, 0, s>>>(f, out, n, sh.ipb, c0, (1.0 - c0) / 6.0, sub);
    return hipGetLastError();
}

// --------------------------------------------------------------- step control

__global__ void k_max_shift(const double *__restrict__ f, int n, int ipb, double *part)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double v[1] = {0.0};
    if (k < n && j < n) {
        const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
        const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
        for (int i = i0; i < i1; ++i) {
            const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
            const double sx = fabs(0.5 * (f[lin(ip, j, k, n)] - f[lin(im, j, k, n)]));
            const double sy = fabs(0.5 * (f[lin(i, jp, k, n)] - f[lin(i, jm, k, n)]));
            const double sz = fabs(0.5 * (f[lin(i, j, kp, n)] - f[lin(i, j, km, n)]));
            v[0] = fmax(v[0], fmax(sx, fmax(sy, sz)));
        }
    }
    block_reduce_store<1, RED_MAX>(v, part, block_row());
}

hipError_t launch_max_shift(const double *f, int n, Part &p, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_max_shift<<<sh.grid, sh.block, 0, s>>>(f, n, sh.ipb, p.part);
    p.blocks = rows_of(sh);
    p.k = 1;
    return hipGetLastError();
}

// Count nodes where I + Hess(phi + 2^-j dphi) fails Sylvester's criterion
// (e11 > 0, e11 e22 - e12^2 > 0, det > 0) for NT consecutive j, or (mass update,
// Mm and Dm given) where Mm + 2^-j Dm > 0 fails.  The trial potential is formed
// per stencil point exactly as phi + alpha * dphi.
template <int NT>
__global__ void k_pd_trials(const double *__restrict__ phi, const double *__restrict__ dphi, int n, int ipb, int j0,
                            double *part, const double *__restrict__ Mm, const double *__restrict__ Dm)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double v[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) v[t] = 0.0;
    if (k < n && j < n) {
        const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
        for (int i = i0; i < i1; ++i) {
            Stencil19 a, d;
            load19(phi, i, j, k, n, a);
            load19(dphi, i, j, k, n, d);
            // the mass update's positivity test: M + alpha D > 0
            const double mv = Mm ? Mm[lin(i, j, k, n)] : 1.0, dv = Mm ? Dm[lin(i, j, k, n)] : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double al = ldexp(1.0, -(j0 + t));
                Stencil19 s;
                s.c = a.c + al * d.c;
                s.xp = a.xp + al * d.xp;
                s.xm = a.xm + al * d.xm;
                s.yp = a.yp + al * d.yp;
                s.ym = a.ym + al * d.ym;
                s.zp = a.zp + al * d.zp;
                s.zm = a.zm + al * d.zm;
                s.xpyp = a.xpyp + al * d.xpyp;
                s.xpym = a.xpym + al * d.xpym;
                s.xmyp = a.xmyp + al * d.xmyp;
                s.xmym = a.xmym + al * d.xmym;
                s.xpzp = a.xpzp + al * d.xpzp;
                s.xpzm = a.xpzm + al * d.xpzm;
                s.xmzp = a.xmzp + al * d.xmzp;
                s.xmzm = a.xmzm + al * d.xmzm;
                s.ypzp = a.ypzp + al * d.ypzp;
                s.ypzm = a.ypzm + al * d.ypzm;
                s.ymzp = a.ymzp + al * d.ymzp;
                s.ymzm = a.ymzm + al * d.ymzm;
                const Sym3 e = triad19(s);
                const double m2 = e.xx * e.yy - e.xy * e.xy;
                const bool ok = e.xx > 0.0 && m2 > 0.0 && det_sym(e) > 0.0 && mv + al * dv > 0.0;
                v[t] += ok ? 0.0 : 1.0;
            }
        }
    }
    block_reduce_store<NT, RED_SUM>(v, part, block_row());
}

hipError_t launch_pd_trials(const double *phi, const double *dphi, int n, int j0, int ntrial, Part &p, hipStream_t s,
                            const double *M, const double *D)
{
    if ((M == nullptr) != (D == nullptr)) return hipErrorInvalidValue;
    Shape3 sh = shape3(n);
    if (ntrial == 1) k_pd_trials<1><<<sh.grid, sh.block, 0, s>>>(phi, dphi, n, sh.ipb, j0, p.part, M, D);
    else k_pd_trials<4><<<sh.grid, sh.block, 0, s>>>(phi, dphi, n, sh.ipb, j0, p.part, M, D);
    p.blocks = rows_of(sh);
    p.k = ntrial == 1 ? 1 : 4;
    return hipGetLastError();
}

template <typename X>
__global__ void k_axpy(double *__restrict__ y, const X *__restrict__ x, double alpha, long n3,
                       const double *__restrict__ alpha_dev)
{
    if (alpha_dev) alpha = *alpha_dev;
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) y[p] += alpha * (double)x[p];
}

template <typename X>
hipError_t launch_axpy(double *y, const X *x, double alpha, long n3, hipStream_t s, const double *alpha_dev)
{
    k_axpy<X><<<flat_blocks(n3), 256, 0, s>>>(y, x, alpha, n3, alpha_dev);
    return hipGetLastError();
}
template hipError_t launch_axpy<double>(double *, const double *, double, long, hipStream_t, const double *);
template hipError_t launch_axpy<float>(double *, const float *, double, long, hipStream_t, const double *);

// y += sign * (*c) * scale
__global__ void k_add_scalar(double *__restrict__ y, const double *c, double sign, double scale, long n3)
{
    const double v = sign * (*c) * scale;
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) y[p] += v;
}

hipError_t launch_add_scalar(double *y, const double *c_dev, double sign, double scale, long n3, hipStream_t s)
{
    k_add_scalar<<<flat_blocks(n3), 256, 0, s>>>(y, c_dev, sign, scale, n3);
    return hipGetLastError();
}

__global__ void k_sum(const double *__restrict__ f, long n3, double *part)
{
    double v[1] = {0.0};
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) v[0] += f[p];
    block_reduce_store<1, RED_SUM>(v, part, blockIdx.x);
}

hipError_t launch_sum(const double *f, long n3, Part &p, hipStream_t s)
{
    int nb = flat_blocks(n3);
    k_sum<<<nb, 256, 0, s>>>(f, n3, p.part);
    p.blocks = nb;
    p.k = 1;
    return hipGetLastError();
}

// ------------------------------------------------------------------ output

// delta_r = -(7-point Laplacian of phi) (Sec. II, Eq. rec), phi_out = phi h^2,
// and the invariants min det(I+H), min lambda_0, max delta_r (stored negated
// so that all three reduce by min).
__global__ void k_output(const double *__restrict__ phi, double *__restrict__ delta, double *__restrict__ phi_out,
                         double h2, int n, int ipb, double *part)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double v[3] = {INFINITY, INFINITY, INFINITY};
    if (k < n && j < n) {
        const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
        for (int i = i0; i < i1; ++i) {
            Stencil19 s;
            load19(phi, i, j, k, n, s);
            const Sym3 e = triad19(s);
            const double lap = s.xp + s.xm + s.yp + s.ym + s.zp + s.zm - 6.0 * s.c;
            const size_t p = lin(i, j, k, n);
            if (delta) delta[p] = -lap;
            if (phi_out) phi_out[p] = s.c * h2;
            v[0] = fmin(v[0], det_sym(e));
            v[1] = fmin(v[1], lambda_min_sym(e));
            v[2] = fmin(v[2], -(3.0 - (e.xx + e.yy + e.zz)));
        }
    }
    block_reduce_store<3, RED_MIN>(v, part, block_row());
}

hipError_t launch_output(const double *phi, double *delta, double *phi_out, double h2, int n, Part &p, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_output<<<sh.grid, sh.block, 0, s>>>(phi, delta, phi_out, h2, n, sh.ipb, p.part);
    p.blocks = rows_of(sh);
    p.k = 3;
    return hipGetLastError();
}

// --------------------------------------------------------------- multigrid
//
// Operator of Eq. (elliptic) with x ~ xi: (A u)_n = scale * sum over the six
// faces of c_f (u_nb - u_n), c_f = max(a_min, (a_n + a_nb) / 2), scale = 4^-l.

template <typename T>
__global__ void k_apply(const T *__restrict__ u, const T *__restrict__ a, T *__restrict__ out, int n, int ipb, T scale,
                        T a_min, const T *__restrict__ b)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
        const size_t p = lin(i, j, k, n);
        const T un = u[p], an = a[p];
        const size_t q[6] = {lin(ip, j, k, n), lin(im, j, k, n), lin(i, jp, k, n),
                             lin(i, jm, k, n), lin(i, j, kp, n), lin(i, j, km, n)};
        T acc = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) acc += facec(an, a[q[f]], a_min) * (u[q[f]] - un);
        const T Au = scale * acc;
        out[p] = b ? b[p] - Au : Au;
    }
}

template <typename T>
hipError_t launch_apply(const T *u, const T *a, T *out, int n, T scale, T a_min, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_apply<T><<<sh.grid, sh.block, 0, s>>>(u, a, out, n, sh.ipb, scale, a_min, nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(const T *u, const T *a, const T *b, T *r, int n, T scale, T a_min, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_apply<T><<<sh.grid, sh.block, 0, s>>>(u, a, r, n, sh.ipb, scale, a_min, b);
    return hipGetLastError();
}

// Gauss-Seidel relaxation of one colour, in place: u_n <- (sum c_f u_nb -
// b_n / scale) / sum c_f at nodes with (i+j+k) % 2 == colour.  With zero_init
// every neighbour is taken as 0 (the first half-sweep from u = 0).
// (FINE only separates the finest-level launches by name in kernel traces.)
template <typename T, int FINE>
__global__ void k_rbgs_half(T *__restrict__ u, const T *__restrict__ a, const T *__restrict__ b, int n, int ipb,
                            T inv_scale, T a_min, int colour, int zero_init)
{
    const int kk = blockIdx.x * blockDim.x + threadIdx.x;  // pair index along k
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int half = n >> 1;
    if (kk >= half || j >= n) return;
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n);
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        const int k = 2 * kk + ((i + j + colour) & 1);
        const int kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
        const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
        const size_t p = lin(i, j, k, n);
        const size_t q[6] = {lin(ip, j, k, n), lin(im, j, k, n), lin(i, jp, k, n),
                             lin(i, jm, k, n), lin(i, j, kp, n), lin(i, j, km, n)};
        const T an = a[p];
        T num = 0, den = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const T c = facec(an, a[q[f]], a_min);
            if (!zero_init) num += c * u[q[f]];
            den += c;
        }
        u[p] = qdiv(num - b[p] * inv_scale, den);
    }
}

template <typename T>
hipError_t launch_rbgs_half(T *u, const T *a, const T *b, int n, T scale, T a_min, int colour, bool zero_init,
                            hipStream_t s, bool fine)
{
    const int half = n / 2;
    int bx = half < 64 ? half : 64;
    int by = 256 / bx;
    if (by > n) by = n;
    int gz = n < 64 ? n : 64;
    int ipb = (n + gz - 1) / gz;
    gz = (n + ipb - 1) / ipb;
    dim3 grid((half + bx - 1) / bx, (n + by - 1) / by, gz), block(bx, by, 1);
    if (fine)
        k_rbgs_half<T, 1><<<grid, block, 0, s>>>(u, a, b, n, ipb, (T)1 / scale, a_min, colour, zero_init ? 1 : 0);
    else
        k_rbgs_half<T, 0><<<grid, block, 0, s>>>(u, a, b, n, ipb, (T)1 / scale, a_min, colour, zero_init ? 1 : 0);
    return hipGetLastError();
}

// 27-point full weighting: coarse node I <- sum_d w(d) f(2I + d), w = prod
// over axes of 1/2 (d = 0) or 1/4 (d = +-1).
template <typename T>
__global__ void k_restrict(const T *__restrict__ f, T *__restrict__ c, int n)
{
    const int nc = n >> 1;
    const int K = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int I = blockIdx.z;
    if (K >= nc || J >= nc) return;
    const int ii[3] = {wrapc(2 * I - 1, n), 2 * I, wrapc(2 * I + 1, n)};
    const int jj[3] = {wrapc(2 * J - 1, n), 2 * J, wrapc(2 * J + 1, n)};
    const int kk[3] = {wrapc(2 * K - 1, n), 2 * K, wrapc(2 * K + 1, n)};
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    T acc = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T pa = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T *row = f + ((size_t)ii[a] * n + jj[b]) * (size_t)n;
            const T pb = w[0] * row[kk[0]] + w[1] * row[kk[1]] + w[2] * row[kk[2]];
            pa += w[b] * pb;
        }
        acc += w[a] * pa;
    }
    c[lin(I, J, K, nc)] = acc;
}

template <typename T>
hipError_t launch_restrict(const T *f, T *c, int n, hipStream_t s)
{
    const int nc = n / 2;
    int bx = nc < 64 ? nc : 64;
    int by = 256 / bx;
    if (by > nc) by = nc;
    dim3 grid((nc + bx - 1) / bx, (nc + by - 1) / by, nc), block(bx, by, 1);
    k_restrict<T><<<grid, block, 0, s>>>(f, c, n);
    return hipGetLastError();
}

// u += P e, trilinear interpolation from (n/2)^3 (= 8 R^T).
template <typename T>
__global__ void k_prolong_add(T *__restrict__ u, const T *__restrict__ e, int n, int ipb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const int nc = n >> 1;
    const int k0 = k >> 1, k1 = (k & 1) ? (k0 + 1 == nc ? 0 : k0 + 1) : k0;
    const int j0 = j >> 1, j1 = (j & 1) ? (j0 + 1 == nc ? 0 : j0 + 1) : j0;
    const T wk = (k & 1) ? (T)0.5 : (T)1, wj = (j & 1) ? (T)0.5 : (T)1;
    const int i0b = blockIdx.z * ipb, i1b = min(n, i0b + ipb);
    for (int i = i0b; i < i1b; ++i) {
        const int i0 = i >> 1, i1 = (i & 1) ? (i0 + 1 == nc ? 0 : i0 + 1) : i0;
        const T wi = (i & 1) ? (T)0.5 : (T)1;
        // planes i0 and i1 (the same plane when i is even: weight 1 = 0.5 + 0.5
        // would double count, so even indices use a single term)
        T acc;
        {
            const T a00 = e[lin(i0, j0, k0, nc)], a01 = e[lin(i0, j0, k1, nc)];
            const T a10 = e[lin(i0, j1, k0, nc)], a11 = e[lin(i0, j1, k1, nc)];
            T r0 = (k & 1) ? wk * (a00 + a01) : a00;
            T r1 = (k & 1) ? wk * (a10 + a11) : a10;
            acc = (j & 1) ? wj * (r0 + r1) : r0;
        }
        if (i & 1) {
            const T a00 = e[lin(i1, j0, k0, nc)], a01 = e[lin(i1, j0, k1, nc)];
            const T a10 = e[lin(i1, j1, k0, nc)], a11 = e[lin(i1, j1, k1, nc)];
            T r0 = (k & 1) ? wk * (a00 + a01) : a00;
            T r1 = (k & 1) ? wk * (a10 + a11) : a10;
            const T acc1 = (j & 1) ? wj * (r0 + r1) : r0;
            acc = wi * (acc + acc1);
        }
        u[lin(i, j, k, n)] += acc;
    }
}

template <typename T>
hipError_t launch_prolong_add(T *u, const T *e, int n, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_prolong_add<T><<<sh.grid, sh.block, 0, s>>>(u, e, n, sh.ipb);
    return hipGetLastError();
}

// Coarsest level in one workgroup, LDS resident: b made mean-free, u = 0,
// then the palindromic red/black sequence (pairs of red, black, then a final
// red), then the mean of u removed.  n^3 <= 4096.
template <typename T>
__global__ void __launch_bounds__(1024) k_coarse_solve(T *__restrict__ ug, const T *__restrict__ ag,
                                                       const T *__restrict__ bg, int n, T inv_scale, T a_min,
                                                       int pairs)
{
    __shared__ T u[4096], a[4096], b[4096];
    __shared__ double red[1024];
    const int n3 = n * n * n, t = threadIdx.x;
    double sb = 0.0;
    for (int p = t; p < n3; p += blockDim.x) {
        a[p] = ag[p];
        b[p] = bg[p];
        u[p] = 0;
        sb += (double)bg[p];
    }
    red[t] = sb;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const T mb = (T)(red[0] / n3);
    __syncthreads();
    for (int p = t; p < n3; p += blockDim.x) b[p] -= mb;
    __syncthreads();
    // Each thread keeps its nodes' neighbour offsets, face coefficients, their
    // sum and b in registers: only u changes between passes.  The arithmetic
    // per relaxation is unchanged (faces in the order +i, -i, +j, -j, +k, -k).
    constexpr int NPT = 4096 / 1024;
    int q[NPT][6], col[NPT];
    T cf[NPT][6], den[NPT], bv[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int p = t + r * 1024;
        const int pp = p < n3 ? p : 0;
        const int i = pp / (n * n), j = (pp / n) % n, k = pp % n;
        col[r] = p < n3 ? ((i + j + k) & 1) : -1;
        q[r][0] = (wrapc(i + 1, n) * n + j) * n + k;
        q[r][1] = (wrapc(i - 1, n) * n + j) * n + k;
        q[r][2] = (i * n + wrapc(j + 1, n)) * n + k;
        q[r][3] = (i * n + wrapc(j - 1, n)) * n + k;
        q[r][4] = (i * n + j) * n + wrapc(k + 1, n);
        q[r][5] = (i * n + j) * n + wrapc(k - 1, n);
        const T an = a[pp];
        T d = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            cf[r][f] = facec(an, a[q[r][f]], a_min);
            d += cf[r][f];
        }
        den[r] = d;
        bv[r] = b[pp];
    }
    const int passes = 2 * pairs + 1;
    for (int ps = 0; ps < passes; ++ps) {
        const int colour = ps & 1;
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            if (col[r] != colour) continue;
            T num = 0;
#pragma unroll
            for (int f = 0; f < 6; ++f) num += cf[r][f] * u[q[r][f]];
            u[t + r * 1024] = (num - bv[r] * inv_scale) / den[r];
        }
        __syncthreads();
    }
    double su = 0.0;
    for (int p = t; p < n3; p += blockDim.x) su += (double)u[p];
    red[t] = su;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const T mu = (T)(red[0] / n3);
    for (int p = t; p < n3; p += blockDim.x) ug[p] = u[p] - mu;
}

template <typename T>
hipError_t launch_coarse_solve(T *u, const T *a, const T *b, int n, T scale, T a_min, int pairs, hipStream_t s)
{
    if (n * n * n > 4096) return hipErrorInvalidValue;
    k_coarse_solve<T><<<1, 1024, 0, s>>>(u, a, b, n, (T)1 / scale, a_min, pairs);
    return hipGetLastError();
}

__global__ void k_cast_f32(const double *__restrict__ s, float *__restrict__ d, long n3)
{
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) d[p] = (float)s[p];
}

hipError_t launch_cast_f32(const double *src, float *dst, long n3, hipStream_t s)
{
    k_cast_f32<<<flat_blocks(n3), 256, 0, s>>>(src, dst, n3);
    return hipGetLastError();
}

__global__ void k_cast_f64(const float *__restrict__ s, double *__restrict__ d, long n3)
{
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) d[p] = (double)s[p];
}

hipError_t launch_cast_f64(const float *src, double *dst, long n3, hipStream_t s)
{
    k_cast_f64<<<flat_blocks(n3), 256, 0, s>>>(src, dst, n3);
    return hipGetLastError();
}

// ------------------------------------------------------------ Krylov (FP64)

// r = b - A u on the fine level (scale 1) with sum r^2; optional FP32 copy of r.
__global__ void k_residual_norm(const double *__restrict__ u, const double *__restrict__ a,
                                const double *__restrict__ b, double *__restrict__ r, float *__restrict__ r32, int n,
                                int ipb, double a_min, double *part)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double v[1] = {0.0};
    if (k < n && j < n) {
        const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
        const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
        for (int i = i0; i < i1; ++i) {
            const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
            const size_t p = lin(i, j, k, n);
            const double un = u[p], an = a[p];
            const size_t q[6] = {lin(ip, j, k, n), lin(im, j, k, n), lin(i, jp, k, n),
                                 lin(i, jm, k, n), lin(i, j, kp, n), lin(i, j, km, n)};
            double acc = 0.0;
#pragma unroll
            for (int f = 0; f < 6; ++f) acc += facec(an, a[q[f]], a_min) * (u[q[f]] - un);
            const double rv = b[p] - acc;
            r[p] = rv;
            if (r32) r32[p] = (float)rv;
            v[0] += rv * rv;
        }
    }
    block_reduce_store<1, RED_SUM>(v, part, block_row());
}

hipError_t launch_residual_norm(const double *u, const double *a, const double *b, double *r, float *r32, int n,
                                double a_min, Part &p, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_residual_norm<<<sh.grid, sh.block, 0, s>>>(u, a, b, r, r32, n, sh.ipb, a_min, p.part);
    p.blocks = rows_of(sh);
    p.k = 1;
    return hipGetLastError();
}

template <typename Z>
__global__ void k_dots_zr_zq(const Z *__restrict__ z, const double *__restrict__ r, const double *__restrict__ q,
                             long n3, double *part)
{
    double v[2] = {0.0, 0.0};
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) {
        const double zv = (double)z[p];
        v[0] += zv * r[p];
        if (q) v[1] += zv * q[p];
    }
    block_reduce_store<2, RED_SUM>(v, part, blockIdx.x);
}

template <typename Z>
hipError_t launch_dots_zr_zq(const Z *z, const double *r, const double *q, long n3, Part &p, hipStream_t s)
{
    int nb = flat_blocks(n3);
    k_dots_zr_zq<Z><<<nb, 256, 0, s>>>(z, r, q, n3, p.part);
    p.blocks = nb;
    p.k = 2;
    return hipGetLastError();
}

// p = z + beta p (first: p = z)
template <typename Z>
__global__ void k_update_p(const Z *__restrict__ z, double *__restrict__ pv, double beta, int first, long n3,
                           const double *__restrict__ ks)
{
    if (ks && !first) beta = -ks[KS_ALPHA] * ks[KS_ZQ] / ks[KS_RZ_OLD];
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x)
        pv[p] = first ? (double)z[p] : (double)z[p] + beta * pv[p];
}

// q = A p (scale 1) with sum p*q
__global__ void k_apply_dot(const double *__restrict__ pv, const double *__restrict__ a, double *__restrict__ q,
                            int n, int ipb, double a_min, double *part)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double v[1] = {0.0};
    if (k < n && j < n) {
        const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
        const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
        for (int i = i0; i < i1; ++i) {
            const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
            const size_t p = lin(i, j, k, n);
            const double un = pv[p], an = a[p];
            const size_t qq[6] = {lin(ip, j, k, n), lin(im, j, k, n), lin(i, jp, k, n),
                                  lin(i, jm, k, n), lin(i, j, kp, n), lin(i, j, km, n)};
            double acc = 0.0;
#pragma unroll
            for (int f = 0; f < 6; ++f) acc += facec(an, a[qq[f]], a_min) * (pv[qq[f]] - un);
            q[p] = acc;
            v[0] += un * acc;
        }
    }
    block_reduce_store<1, RED_SUM>(v, part, block_row());
}

template <typename Z>
hipError_t launch_update_pq(const Z *z, const double *a, double *pv, double *q, double beta, int n, double a_min,
                            bool first, const double *ks, Part &p, hipStream_t s)
{
    const long n3 = (long)n * n * n;
    k_update_p<Z><<<flat_blocks(n3), 256, 0, s>>>(z, pv, beta, first ? 1 : 0, n3, ks);
    Shape3 sh = shape3(n);
    k_apply_dot<<<sh.grid, sh.block, 0, s>>>(pv, a, q, n, sh.ipb, a_min, p.part);
    p.blocks = rows_of(sh);
    p.k = 1;
    return hipGetLastError();
}

template <typename Z>
hipError_t launch_update_p(const Z *z, double *pv, double beta, long n3, bool first, const double *ks, hipStream_t s)
{
    k_update_p<Z><<<flat_blocks(n3), 256, 0, s>>>(z, pv, beta, first ? 1 : 0, n3, ks);
    return hipGetLastError();
}

// Vector types that the nontemporal store builtins accept.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

// r and its FP32 copy are stored nontemporally: the next kernels that read
// them stream fields far larger than the caches, and keeping the stores out
// of L2 measured faster at 256^3 and 512^3.
template <bool U>
__global__ void k_update_ur(double *__restrict__ u, double *__restrict__ r, const double *__restrict__ pv,
                            const double *__restrict__ q, double alpha, float *__restrict__ r32, long n3, double *part,
                            double *ks)
{
    if (ks) {
        const double rz = ks[KS_RZ];
        alpha = rz / ks[KS_PQ];
        // only this kernel's other lanes read ks, and only KS_RZ and KS_PQ
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ks[KS_ALPHA] = alpha;
            ks[KS_RZ_OLD] = rz;
        }
    }
    // two consecutive elements per thread (16-byte accesses; every field is
    // 256-byte aligned), the last element of an odd count by thread 0.  A
    // thread visits its pairs p, p + stride, ... in order; the loads of eight
    // of them are issued together, which keeps the same order of the sum.
    double v[1] = {0.0};
    const long h = n3 >> 1, stride = 256L * gridDim.x;
    auto pair = [&](long e, const v2d rr, const v2d qq) {
        if (U) {
            const v2d pp = *reinterpret_cast<const v2d *>(pv + e);
            v2d uu = *reinterpret_cast<v2d *>(u + e);
            uu.x += alpha * pp.x;
            uu.y += alpha * pp.y;
            *reinterpret_cast<v2d *>(u + e) = uu;
        }
        const double r0 = rr.x - alpha * qq.x, r1 = rr.y - alpha * qq.y;
        v2d rv;
        rv.x = r0;
        rv.y = r1;
        __builtin_nontemporal_store(rv, reinterpret_cast<v2d *>(r + e));
        if (r32) {
            v2f fv;
            fv.x = (float)r0;
            fv.y = (float)r1;
            __builtin_nontemporal_store(fv, reinterpret_cast<v2f *>(r32 + e));
        }
        v[0] += r0 * r0;
        v[0] += r1 * r1;
    };
    constexpr int UN = 8;
    long p = blockIdx.x * 256L + threadIdx.x;
    for (; p + (UN - 1) * stride < h; p += UN * stride) {
        v2d rr[UN], qq[UN];
#pragma unroll
        for (int k = 0; k < UN; ++k) {
            rr[k] = *reinterpret_cast<const v2d *>(r + 2 * (p + k * stride));
            qq[k] = *reinterpret_cast<const v2d *>(q + 2 * (p + k * stride));
        }
#pragma unroll
        for (int k = 0; k < UN; ++k) pair(2 * (p + k * stride), rr[k], qq[k]);
    }
    for (; p < h; p += stride)
        pair(2 * p, *reinterpret_cast<const v2d *>(r + 2 * p), *reinterpret_cast<const v2d *>(q + 2 * p));
    if ((n3 & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const long e = n3 - 1;
        if (U) u[e] += alpha * pv[e];
        const double rv = r[e] - alpha * q[e];
        r[e] = rv;
        if (r32) r32[e] = (float)rv;
        v[0] += rv * rv;
    }
    block_reduce_store<1, RED_SUM>(v, part, blockIdx.x);
}

hipError_t launch_update_ur(double *u, double *r, const double *pv, const double *q, double alpha, float *r32, long n3,
                            double *ks, Part &p, hipStream_t s)
{
    // the paired accesses need 16-byte aligned fields
    if ((reinterpret_cast<uintptr_t>(r) | reinterpret_cast<uintptr_t>(q) | reinterpret_cast<uintptr_t>(u) |
         reinterpret_cast<uintptr_t>(pv)) % 16 ||
        reinterpret_cast<uintptr_t>(r32) % 8)
        return hipErrorInvalidValue;
    // up to 16384 workgroups (measured 755 against 813 us at 512^3 with 8192)
    const long pairs = (n3 + 1) / 2;
    const int nb = (int)std::min<long>((pairs + 255) / 256, 16384);
    if (u) k_update_ur<true><<<nb, 256, 0, s>>>(u, r, pv, q, alpha, r32, n3, p.part, ks);
    else k_update_ur<false><<<nb, 256, 0, s>>>(u, r, pv, q, alpha, r32, n3, p.part, ks);
    p.blocks = nb;
    p.k = 1;
    return hipGetLastError();
}

template <typename Z>
__global__ void k_add_correction(double *__restrict__ u, const Z *__restrict__ z, long n3)
{
    for (long p = blockIdx.x * 256L + threadIdx.x; p < n3; p += 256L * gridDim.x) u[p] += (double)z[p];
}

template <typename Z>
hipError_t launch_add_correction(double *u, const Z *z, long n3, hipStream_t s)
{
    k_add_correction<Z><<<flat_blocks(n3), 256, 0, s>>>(u, z, n3);
    return hipGetLastError();
}

// ------------------------------------------------------ explicit instances

#define RECON_INSTANTIATE(T)                                                                                       \
    template hipError_t launch_apply<T>(const T *, const T *, T *, int, T, T, hipStream_t);                        \
    template hipError_t launch_rbgs_half<T>(T *, const T *, const T *, int, T, T, int, bool, hipStream_t, bool);   \
    template hipError_t launch_residual<T>(const T *, const T *, const T *, T *, int, T, T, hipStream_t);          \
    template hipError_t launch_restrict<T>(const T *, T *, int, hipStream_t);                                      \
    template hipError_t launch_prolong_add<T>(T *, const T *, int, hipStream_t);                                   \
    template hipError_t launch_coarse_solve<T>(T *, const T *, const T *, int, T, T, int, hipStream_t);            \
    template hipError_t launch_dots_zr_zq<T>(const T *, const double *, const double *, long, Part &, hipStream_t); \
    template hipError_t launch_update_pq<T>(const T *, const double *, double *, double *, double, int, double,     \
                                            bool, const double *, Part &, hipStream_t);                           \
    template hipError_t launch_update_p<T>(const T *, double *, double, long, bool, const double *, hipStream_t);  \
    template hipError_t launch_add_correction<T>(double *, const T *, long, hipStream_t);                        \

RECON_INSTANTIATE(double)
RECON_INSTANTIATE(float)

}  // namespace recon
