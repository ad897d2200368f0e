// Device helpers shared by the kernel files (internal, not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace recon {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ size_t lin(int i, int j, int k, int n)
{
    return ((size_t)i * n + j) * (size_t)n + k;
}

template <int OP>
__device__ __forceinline__ double red_op(double a, double b)
{
    if (OP == RED_SUM) return a + b;
    if (OP == RED_MAX) return a > b ? a : b;
    return a < b ? a : b;
}

template <int OP>
__device__ __forceinline__ double red_identity()
{
    if (OP == RED_SUM) return 0.0;
    if (OP == RED_MAX) return -INFINITY;
    return INFINITY;
}

// Block reduction of K values per thread into one row of partials.  Fixed
// order: wavefront butterfly (64 lanes), then waves in index order.
// Blocks must have at most 256 threads; blocks that are not a whole number of
// 64-lane waves (grids below 8^3) take an LDS tree instead of the shuffles.
template <int K, int OP>
__device__ void block_reduce_store(double (&v)[K], double *part, int row)
{
    __shared__ double sm[16][K];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    if (nthreads & 63) {
        __shared__ double lds[256][K];
        for (int s = tid; s < 256; s += nthreads)
#pragma unroll
            for (int c = 0; c < K; ++c) lds[s][c] = s == tid ? v[c] : red_identity<OP>();
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            for (int s = tid; s < w; s += nthreads)
#pragma unroll
                for (int c = 0; c < K; ++c) lds[s][c] = red_op<OP>(lds[s][c], lds[s + w][c]);
            __syncthreads();
        }
        if (tid == 0)
#pragma unroll
            for (int c = 0; c < K; ++c) part[(size_t)row * K + c] = lds[0][c];
        return;
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        double x = v[c];
        for (int off = 32; off > 0; off >>= 1) x = red_op<OP>(x, __shfl_down(x, off, 64));
        v[c] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < K; ++c) sm[wave][c] = v[c];
    }
    __syncthreads();
    if (tid == 0) {
        const int nw = (nthreads + 63) >> 6;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            double x = sm[0][c];
            for (int w = 1; w < nw; ++w) x = red_op<OP>(x, sm[w][c]);
            part[(size_t)row * K + c] = x;
        }
    }
}

__device__ __forceinline__ int block_row()
{
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// Launch shape for n^3 stencil kernels: blocks of (bx, by) threads over
// (k, j), each thread walking `ipb` consecutive i-planes.
struct Shape3 {
    dim3 grid, block;
    int ipb;
};

static inline Shape3 shape3(int n)
{
    Shape3 sh;
    // power-of-two block edges: whole 64-lane waves for every n >= 8
    int bx = 1;
    while (bx < n && bx < 64) bx <<= 1;
    int by = 1;
    while (by < n && by < 256 / bx) by <<= 1;
    int gz = n < 64 ? n : 64;
    int ipb = (n + gz - 1) / gz;
    gz = (n + ipb - 1) / ipb;
    sh.block = dim3(bx, by, 1);
    sh.grid = dim3((n + bx - 1) / bx, (n + by - 1) / by, gz);
    sh.ipb = ipb;
    return sh;
}

static inline int rows_of(const Shape3 &sh) { return sh.grid.x * sh.grid.y * sh.grid.z; }

// Launch shape for flat streams over n3 elements (grid-stride, fixed grid).
static inline int flat_blocks(long n3)
{
    long b = (n3 + 255) / 256;
    return (int)(b < 8192 ? b : 8192);
}

// ------------------------------------------------------------ symmetric 3x3

struct Sym3 {
    double xx, yy, zz, xy, xz, yz;
};

__device__ __forceinline__ double det_sym(const Sym3 &e)
{
    return e.xx * (e.yy * e.zz - e.yz * e.yz) - e.xy * (e.xy * e.zz - e.yz * e.xz) + e.xz * (e.xy * e.yz - e.yy * e.xz);
}

// Smallest eigenvalue of a symmetric 3x3 matrix, trigonometric closed form of
// the characteristic cubic (O. K. Smith, CACM 4 (1961) 168).
__device__ double lambda_min_sym(const Sym3 &e)
{
    const double p1 = e.xy * e.xy + e.xz * e.xz + e.yz * e.yz;
    const double q = (e.xx + e.yy + e.zz) * (1.0 / 3.0);
    const double dx = e.xx - q, dy = e.yy - q, dz = e.zz - q;
    const double p2 = dx * dx + dy * dy + dz * dz + 2.0 * p1;
    if (p2 <= 0.0) return q;
    const double p = sqrt(p2 * (1.0 / 6.0));
    const double ip = 1.0 / p;
    Sym3 b{dx * ip, dy * ip, dz * ip, e.xy * ip, e.xz * ip, e.yz * ip};
    double r = 0.5 * det_sym(b);
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double ang = acos(r) * (1.0 / 3.0);
    return q + 2.0 * p * cos(ang + 2.0943951023931954923);  // + 2 pi / 3
}

// The compression limiter C = 4 max(0, xi_m / lambda_0 - 1)^2 (App. A).  It
// vanishes wherever lambda_0 >= xi_m, that is wherever e - xi_m I is positive
// semidefinite; where Sylvester's leading minors of e - xi_m I are all
// positive the eigenvalue is not formed (most nodes of a mildly deformed
// mesh, and the trigonometric closed form is the costliest step of a node).
__device__ __forceinline__ double compression_limiter(const Sym3 &e, double xi_m)
{
    const Sym3 d{e.xx - xi_m, e.yy - xi_m, e.zz - xi_m, e.xy, e.xz, e.yz};
    if (d.xx > 0.0 && d.xx * d.yy - d.xy * d.xy > 0.0 && det_sym(d) > 0.0) return 0.0;
    const double r = xi_m / lambda_min_sym(e) - 1.0;
    return r > 0.0 ? 4.0 * r * r : 0.0;
}

// 19-point neighbourhood of a node (centre, 6 faces, 12 edges), periodic.
struct Stencil19 {
    double c, xp, xm, yp, ym, zp, zm;
    double xpyp, xpym, xmyp, xmym, xpzp, xpzm, xmzp, xmzm, ypzp, ypzm, ymzp, ymzm;
};

__device__ __forceinline__ void load19(const double *__restrict__ f, int i, int j, int k, int n, Stencil19 &s)
{
    const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n);
    const int kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
    s.c = f[lin(i, j, k, n)];
    s.xp = f[lin(ip, j, k, n)];
    s.xm = f[lin(im, j, k, n)];
    s.yp = f[lin(i, jp, k, n)];
    s.ym = f[lin(i, jm, k, n)];
    s.zp = f[lin(i, j, kp, n)];
    s.zm = f[lin(i, j, km, n)];
    s.xpyp = f[lin(ip, jp, k, n)];
    s.xpym = f[lin(ip, jm, k, n)];
    s.xmyp = f[lin(im, jp, k, n)];
    s.xmym = f[lin(im, jm, k, n)];
    s.xpzp = f[lin(ip, j, kp, n)];
    s.xpzm = f[lin(ip, j, km, n)];
    s.xmzp = f[lin(im, j, kp, n)];
    s.xmzm = f[lin(im, j, km, n)];
    s.ypzp = f[lin(i, jp, kp, n)];
    s.ypzm = f[lin(i, jp, km, n)];
    s.ymzp = f[lin(i, jm, kp, n)];
    s.ymzm = f[lin(i, jm, km, n)];
}

// The coefficients K = M e^-1 that the flux form of div(K grad f) reads around
// one node: each diagonal component at the node and its two neighbours along
// its own axis, each off-diagonal one at the four face neighbours across which
// it couples.
struct FluxK {
    double xx_c, xx_p, xx_m, yy_c, yy_p, yy_m, zz_c, zz_p, zz_m;
    double xy_xp, xy_xm, xy_yp, xy_ym, xz_xp, xz_xm, xz_zp, xz_zm, yz_yp, yz_ym, yz_zp, yz_zm;
};

// div(K grad f) at a node in flux form on the periodic lattice: diagonal
// fluxes with face-averaged coefficients (floored at a_min when a_min > 0,
// as the x ~ xi operator's), cross fluxes as central differences of
// K^{mu nu} d_nu f taken at the two neighbours along mu (sums to zero over
// the lattice; at K = a I it is the x ~ xi operator, with its floor when
// a_min > 0).
__device__ __forceinline__ double face_floor(double k, double a_min) { return a_min > 0.0 ? fmax(a_min, k) : k; }

__device__ __forceinline__ double full_flux(const Stencil19 &s, const FluxK &K, double a_min)
{
    double acc = 0.0;
    // diagonal fluxes, directions x, y, z
    acc += face_floor(0.5 * (K.xx_c + K.xx_p), a_min) * (s.xp - s.c) -
           face_floor(0.5 * (K.xx_m + K.xx_c), a_min) * (s.c - s.xm);
    acc += face_floor(0.5 * (K.yy_c + K.yy_p), a_min) * (s.yp - s.c) -
           face_floor(0.5 * (K.yy_m + K.yy_c), a_min) * (s.c - s.ym);
    acc += face_floor(0.5 * (K.zz_c + K.zz_p), a_min) * (s.zp - s.c) -
           face_floor(0.5 * (K.zz_m + K.zz_c), a_min) * (s.c - s.zm);
    // cross fluxes: direction mu of the difference, nu of the gradient
    acc += 0.25 * (K.xy_xp * (s.xpyp - s.xpym) - K.xy_xm * (s.xmyp - s.xmym));  // mu = x, nu = y
    acc += 0.25 * (K.xz_xp * (s.xpzp - s.xpzm) - K.xz_xm * (s.xmzp - s.xmzm));  // mu = x, nu = z
    acc += 0.25 * (K.xy_yp * (s.xpyp - s.xmyp) - K.xy_ym * (s.xpym - s.xmym));  // mu = y, nu = x
    acc += 0.25 * (K.yz_yp * (s.ypzp - s.ypzm) - K.yz_ym * (s.ymzp - s.ymzm));  // mu = y, nu = z
    acc += 0.25 * (K.xz_zp * (s.xpzp - s.xmzp) - K.xz_zm * (s.xpzm - s.xmzm));  // mu = z, nu = x
    acc += 0.25 * (K.yz_zp * (s.ypzp - s.ymzp) - K.yz_zm * (s.ypzm - s.ymzm));  // mu = z, nu = y
    return acc;
}

// e = I + compact Hessian of the 19-point neighbourhood.
__device__ __forceinline__ Sym3 triad19(const Stencil19 &s)
{
    Sym3 e;
    e.xx = 1.0 + (s.xp - 2.0 * s.c + s.xm);
    e.yy = 1.0 + (s.yp - 2.0 * s.c + s.ym);
    e.zz = 1.0 + (s.zp - 2.0 * s.c + s.zm);
    e.xy = 0.25 * (s.xpyp - s.xpym - s.xmyp + s.xmym);
    e.xz = 0.25 * (s.xpzp - s.xpzm - s.xmzp + s.xmzm);
    e.yz = 0.25 * (s.ypzp - s.ypzm - s.ymzp + s.ymzm);
    return e;
}

template <typename T>
__device__ __forceinline__ T facec(T an, T anb, T a_min)
{
    const T c = (T)0.5 * (an + anb);
    return c > a_min ? c : a_min;
}

// Quotient x / d for d > 0 (a sum of floored face coefficients) without the
// IEEE division sequence: hardware reciprocal, Newton refinement of the
// reciprocal (FP64), then one residual correction of the quotient
// (Markstein's method); within an ulp of the rounded quotient.  Every
// Gauss-Seidel kernel of the smoother uses it, so they round identically.
__device__ __forceinline__ float qdiv(float x, float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    const float q = x * r;
    return fmaf(fmaf(-d, q, x), r, q);
}

__device__ __forceinline__ double qdiv(double x, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    const double q = x * r;
    return fma(fma(-d, q, x), r, q);
}


}  // namespace recon
