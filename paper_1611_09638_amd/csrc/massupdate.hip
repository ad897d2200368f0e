// The paper's own mass update (App. A): after a step, the mass per curvilinear
// cell changes by the operator of Eq. elliptic_diff applied to the increment,
//   D = d_mu ( K^{mu nu} d_nu f ),  K = M e^{-1},  e = I + Hess phi,
// taken on the mesh before the step (M is rho sqrt g there).  Flux form on
// the periodic lattice, so that D sums to zero and the update conserves mass:
//   diagonal: sum_mu [ (K^{mumu}_n + K^{mumu}_{n+mu})/2 (f_{n+mu} - f_n)
//                    - (K^{mumu}_{n-mu} + K^{mumu}_n)/2 (f_n - f_{n-mu}) ]
//   cross:    sum_{mu != nu} [ K^{munu}_{n+mu} (f_{n+mu+nu} - f_{n+mu-nu})
//                            - K^{munu}_{n-mu} (f_{n-mu+nu} - f_{n-mu-nu}) ] / 4
// Two passes: K at every node (six fields, since e is symmetric), then the
// 19-point application.  The same application, with a dot product or as a
// residual, is the operator of the exact-Jacobian linear solve, where it runs
// once per Krylov iteration; it gathers from L2.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

namespace {

// K = M e^{-1} from the transposed cofactors of the symmetric triad, and
// optionally its mean diagonal (the coefficient of the exact-Jacobian solve's
// x ~ xi preconditioner).
__global__ void k_mass_tensor(const double *__restrict__ phi, const double *__restrict__ M, MassTensor K, int n,
                              int ipb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= n || j >= n) return;
    const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
    for (int i = i0; i < i1; ++i) {
        Stencil19 s;
        load19(phi, i, j, k, n, s);
        const Sym3 e = triad19(s);
        const double w = M[lin(i, j, k, n)] / det_sym(e);
        const size_t p = lin(i, j, k, n);
        K.xx[p] = w * (e.yy * e.zz - e.yz * e.yz);
        K.yy[p] = w * (e.xx * e.zz - e.xz * e.xz);
        K.zz[p] = w * (e.xx * e.yy - e.xy * e.xy);
        K.xy[p] = w * (e.xz * e.yz - e.xy * e.zz);
        K.xz[p] = w * (e.xy * e.yz - e.xz * e.yy);
        K.yz[p] = w * (e.xy * e.xz - e.xx * e.yz);
        if (K.tr) K.tr[p] = (K.xx[p] + K.yy[p] + K.zz[p]) / 3.0;
    }
}

// L_K f at one node, in the flux form above; fc receives f at the node
__device__ inline double full_node(const MassTensor &K, const double *__restrict__ f, int i, int j, int k, int n,
                                   double a_min, double &fc)
{
    const int ip = wrapc(i + 1, n), im = wrapc(i - 1, n);
    const int jp = wrapc(j + 1, n), jm = wrapc(j - 1, n), kp = wrapc(k + 1, n), km = wrapc(k - 1, n);
    Stencil19 s;
    load19(f, i, j, k, n, s);
    fc = s.c;
    const size_t c = lin(i, j, k, n);
    const size_t xp = lin(ip, j, k, n), xm = lin(im, j, k, n);
    const size_t yp = lin(i, jp, k, n), ym = lin(i, jm, k, n);
    const size_t zp = lin(i, j, kp, n), zm = lin(i, j, km, n);
    const FluxK q{K.xx[c],  K.xx[xp], K.xx[xm], K.yy[c],  K.yy[yp], K.yy[ym], K.zz[c],
                  K.zz[zp], K.zz[zm], K.xy[xp], K.xy[xm], K.xy[yp], K.xy[ym], K.xz[xp],
                  K.xz[xm], K.xz[zp], K.xz[zm], K.yz[yp], K.yz[ym], K.yz[zp], K.yz[zm]};
    return full_flux(s, q, a_min);
}

enum FullMode { FULL_APPLY = 0, FULL_DOT = 1, FULL_RESID = 2 };

// FULL_APPLY: out = L_K f.  FULL_DOT: out = L_K f with sum f (L_K f) (the
// conjugate-gradient product q = A p with p.q).  FULL_RESID: out = b - L_K f
// with sum out^2 and an optional FP32 copy (the Krylov residual).
template <int MODE>
__global__ void k_full_apply(MassTensor K, const double *__restrict__ f, const double *__restrict__ b,
                             double *__restrict__ out, float *__restrict__ out32, int n, int ipb, double a_min,
                             double *part)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double v[1] = {0.0};
    if (k < n && j < n) {
        const int i0 = blockIdx.z * ipb, i1 = min(n, i0 + ipb);
        for (int i = i0; i < i1; ++i) {
            const size_t c = lin(i, j, k, n);
            double fc;
            const double acc = full_node(K, f, i, j, k, n, a_min, fc);
            if (MODE == FULL_RESID) {
                const double rv = b[c] - acc;
                out[c] = rv;
                if (out32) out32[c] = (float)rv;
                v[0] += rv * rv;
            } else {
                out[c] = acc;
                if (MODE == FULL_DOT) v[0] += fc * acc;
            }
        }
    }
    if (MODE != FULL_APPLY) block_reduce_store<1, RED_SUM>(v, part, block_row());
}

}  // namespace

hipError_t launch_mass_tensor(const double *phi, const double *M, const MassTensor &K, int n, hipStream_t s)
{
    Shape3 sh = shape3(n);
    k_mass_tensor<<<sh.grid, sh.block, 0, s>>>(phi, M, K, n, sh.ipb);
    return hipGetLastError();
}

hipError_t launch_full_apply(const MassTensor &K, const double *f, double *out, int n, hipStream_t s)
{
    // the exact mass change: no floor; one streaming pass where it applies
    if (n >= 256 && full25_supported(n) && out != f) return launch_full_apply25(K, f, out, n, 0.0, s);
    Shape3 sh = shape3(n);
    k_full_apply<FULL_APPLY><<<sh.grid, sh.block, 0, s>>>(K, f, nullptr, out, nullptr, n, sh.ipb, 0.0, nullptr);
    return hipGetLastError();
}

hipError_t launch_mass_change(const double *phi, const double *M, const double *f, const MassTensor &K,
                              double *out, int n, hipStream_t s)
{
    hipError_t e = launch_mass_tensor(phi, M, K, n, s);
    return e != hipSuccess ? e : launch_full_apply(K, f, out, n, s);
}

hipError_t launch_full_apply_dot(const MassTensor &K, const double *pv, double *q, int n, double a_min, Part &p,
                                 hipStream_t s)
{
    Shape3 sh = shape3(n);
    if (rows_of(sh) > kPartCap) return hipErrorInvalidValue;
    k_full_apply<FULL_DOT><<<sh.grid, sh.block, 0, s>>>(K, pv, nullptr, q, nullptr, n, sh.ipb, a_min, p.part);
    p.blocks = rows_of(sh);
    p.k = 1;
    return hipGetLastError();
}

hipError_t launch_full_residual_norm(const MassTensor &K, const double *u, const double *b, double *r, float *r32,
                                     int n, double a_min, Part &p, hipStream_t s)
{
    Shape3 sh = shape3(n);
    if (rows_of(sh) > kPartCap) return hipErrorInvalidValue;
    k_full_apply<FULL_RESID><<<sh.grid, sh.block, 0, s>>>(K, u, b, r, r32, n, sh.ipb, a_min, p.part);
    p.blocks = rows_of(sh);
    p.k = 1;
    return hipGetLastError();
}

}  // namespace recon
