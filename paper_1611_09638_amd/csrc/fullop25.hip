// Streaming applications of the exact-Jacobian operator L_K f = div(K grad f),
// K = M e^-1 (App. A, Eq. elliptic_diff without x ~ xi), in the flux form of
// full_flux: the Krylov residual with its norm, and the Krylov direction
// update fused with its operator product (and with the deferred solution
// update of the previous step).
//
// A workgroup owns a TJ x TK tile of (j, k) and a chunk of consecutive
// i-planes.  The operand is needed with its in-plane neighbours on planes
// i - 1, i and i + 1 (the 19-point cross terms), so its planes sit in a ring
// of four LDS slots with a one-cell halo in j and k, corners included; the
// components K.xy, K.xz, K.yy, K.zz and K.yz are needed with in-plane
// neighbours on plane i only and sit in rings of two slots.  K.xx, and K.xy,
// K.xz one plane above and below, are needed at the node's own column only and
// are kept in per-thread register queues.  Each field is read from HBM once
// per launch plus the halo lines; a plane is staged in registers one plane
// ahead of its deposit, and one barrier per plane orders deposits and reads.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

namespace {

enum { F25_RESNORM = 0, F25_DIRECTION = 1, F25_APPLY = 2 };

template <int TJ, int TK, int NT>
struct F25 {
    static constexpr int H = TJ + 2, W = TK + 2, PLANE = H * W;
    static constexpr int LU = (PLANE + NT - 1) / NT;
    // every thread loads and deposits LU values unconditionally: spare lanes
    // load a valid address and write one spare word past the plane
    static constexpr int SL = PLANE + 1;
    static constexpr int RS = TJ * TK / NT;  // nodes per thread per plane
};

__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// MODE F25_RESNORM:   out = b - L_K x, out32 = (float) out, sum out^2   (x = xin, P = double)
// MODE F25_DIRECTION: x = first ? z : z + beta xin (rounded to P, written to pout),
//                     out = L_K x, sum x out
// MODE F25_APPLY:     out = L_K x (x = xin, P = double; no reduction)
// FIRST: the first Krylov step (p = z, p_old not read).  UPD (not FIRST):
// also ug += alpha_u xin, the previous step's solution update.  With ks,
// beta and alpha_u come from the device scalars of the Krylov loop.
template <typename Z, typename P, int MODE, int TJ, int TK, int NT, int FIRST = 0, int UPD = 0>
__global__ void __launch_bounds__(NT)
    k_full25(const P *__restrict__ xin, const Z *__restrict__ zg, const double *__restrict__ bg, MassTensor K,
             double *__restrict__ out, float *__restrict__ out32, P *__restrict__ pout, int n, int ci, double beta,
             double a_min, double *part, double *__restrict__ ug, double alpha_u, const double *__restrict__ ks)
{
    if constexpr (MODE == F25_DIRECTION && !FIRST) {
        if (ks) {
            beta = -ks[KS_ALPHA] * ks[KS_ZQ] / ks[KS_RZ_OLD];
            alpha_u = ks[KS_ALPHA];
        }
    }
    static_assert(!UPD || (MODE == F25_DIRECTION && !FIRST), "the deferred update needs p_old");
    static_assert(MODE == F25_DIRECTION || sizeof(P) == 8, "the residual's and the product's operand is FP64");
    using F = F25<TJ, TK, NT>;
    static_assert(TJ * TK % NT == 0, "every thread owns whole rounds of the tile");
    constexpr int W = F::W, PLANE = F::PLANE, LU = F::LU, RS = F::RS, SL = F::SL;
    constexpr bool HAS_B = MODE == F25_RESNORM;
    __shared__ double sF[4][SL];
    __shared__ double sK[5][2][SL];  // xy, xz, yy, zz, yz

    const int tid = threadIdx.x;
    const int tiles_k = n / TK, tiles_j = n / TJ, chunks = n / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int j0 = tj * TJ, k0 = tk * TK, i0 = ch * ci;
    const size_t n2 = (size_t)n * n;

    int offL[LU], dL[LU];
#pragma unroll
    for (int r = 0; r < LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / W, col = q % W;
        offL[r] = q < PLANE ? wrapc(j0 - 1 + row, n) * n + wrapc(k0 - 1 + col, n) : 0;
        dL[r] = q < PLANE ? q : PLANE;
    }
    int oN[RS], gN[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int q = tid + r * NT;
        const int row = q / TK, col = q % TK;
        oN[r] = (row + 1) * W + (col + 1);
        gN[r] = (j0 + row) * n + (k0 + col);
    }
    auto plane = [&](int p) -> size_t { return (size_t)wrapc(p, n) * n2; };

    auto operand = [&](size_t g) -> double {
        if constexpr (MODE == F25_DIRECTION) {
            const double zv = (double)zg[g];
            double x;
            if constexpr (FIRST)
                x = zv;
            else
                x = zv + beta * (double)xin[g];
            if constexpr (sizeof(P) < 8) x = (double)(P)x;
            return x;
        } else {
            return xin[g];
        }
    };
    const double *Kin[5] = {K.xy, K.xz, K.yy, K.zz, K.yz};

    // register stage: operand halo of plane p + 2, K halos of plane p + 1, the
    // column values K.xx, K.xy, K.xz of plane p + 2, and b (or u, p_old) of
    // plane p + 1 at this thread's nodes
    double rf[LU], rk[5][LU], rcx[RS], rcy[RS], rcz[RS];
    double rb[HAS_B ? RS : 1], ru[UPD ? RS : 1], rq[UPD ? RS : 1];
    auto fetch = [&](int p) {  // p: the plane computed next
        const size_t bf = plane(p + 2), bk = plane(p + 1);
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            rf[r] = operand(bf + offL[r]);
#pragma unroll
            for (int f = 0; f < 5; ++f) rk[f][r] = Kin[f][bk + offL[r]];
        }
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            rcx[r] = K.xx[bf + gN[r]];
            rcy[r] = K.xy[bf + gN[r]];
            rcz[r] = K.xz[bf + gN[r]];
        }
        if constexpr (HAS_B) {
#pragma unroll
            for (int r = 0; r < RS; ++r) rb[r] = bg[bk + gN[r]];
        }
        if constexpr (UPD) {
#pragma unroll
            for (int r = 0; r < RS; ++r) {
                ru[r] = ug[bk + gN[r]];
                rq[r] = (double)xin[bk + gN[r]];
            }
        }
    };

    // column queues at this thread's nodes: K.xx at p - 1, p, p + 1; K.xy and
    // K.xz at p - 1 and p + 1; b (or u, p_old) at p
    double qxx0[RS], qxx1[RS], qxx2[RS], qxym[RS], qxyp[RS], qxzm[RS], qxzp[RS];
    double cb[HAS_B ? RS : 1], cu[UPD ? RS : 1], cq[UPD ? RS : 1];
    double v = 0.0;

    // prologue: operand planes i0 - 1, i0, i0 + 1 and K plane i0 resident
    {
        const size_t bm = plane(i0 - 1), b0 = plane(i0), b1 = plane(i0 + 1);
        const size_t bs[3] = {bm, b0, b1};
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int r = 0; r < LU; ++r) sF[(s + 3) & 3][dL[r]] = operand(bs[s] + offL[r]);
#pragma unroll
        for (int r = 0; r < LU; ++r)
#pragma unroll
            for (int f = 0; f < 5; ++f) sK[f][0][dL[r]] = Kin[f][b0 + offL[r]];
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            qxx0[r] = K.xx[bm + gN[r]];
            qxx1[r] = K.xx[b0 + gN[r]];
            qxx2[r] = K.xx[b1 + gN[r]];
            qxym[r] = K.xy[bm + gN[r]];
            qxyp[r] = K.xy[b1 + gN[r]];
            qxzm[r] = K.xz[bm + gN[r]];
            qxzp[r] = K.xz[b1 + gN[r]];
            if constexpr (HAS_B) cb[r] = bg[b0 + gN[r]];
            if constexpr (UPD) {
                cu[r] = ug[b0 + gN[r]];
                cq[r] = (double)xin[b0 + gN[r]];
            }
        }
    }
    fetch(i0);
    lds_barrier();

    for (int p = i0; p < i0 + ci; ++p) {
        const int s0 = (p - i0 + 3) & 3, s1 = (p - i0) & 3, s2 = (p - i0 + 1) & 3, kc = (p - i0) & 1;
        const double *F0 = sF[s0], *F1 = sF[s1], *F2 = sF[s2];
        const double *Sxy = sK[0][kc], *Sxz = sK[1][kc], *Syy = sK[2][kc], *Szz = sK[3][kc], *Syz = sK[4][kc];
        const size_t base = (size_t)p * n2;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            const int c = oN[r];
            Stencil19 s;
            s.c = F1[c];
            s.xp = F2[c];
            s.xm = F0[c];
            s.yp = F1[c + W];
            s.ym = F1[c - W];
            s.zp = F1[c + 1];
            s.zm = F1[c - 1];
            s.xpyp = F2[c + W];
            s.xpym = F2[c - W];
            s.xmyp = F0[c + W];
            s.xmym = F0[c - W];
            s.xpzp = F2[c + 1];
            s.xpzm = F2[c - 1];
            s.xmzp = F0[c + 1];
            s.xmzm = F0[c - 1];
            s.ypzp = F1[c + W + 1];
            s.ypzm = F1[c + W - 1];
            s.ymzp = F1[c - W + 1];
            s.ymzm = F1[c - W - 1];
            const FluxK q{qxx1[r],     qxx2[r],     qxx0[r],     Syy[c],      Syy[c + W],  Syy[c - W], Szz[c],
                          Szz[c + 1],  Szz[c - 1],  qxyp[r],     qxym[r],     Sxy[c + W],  Sxy[c - W], qxzp[r],
                          qxzm[r],     Sxz[c + 1],  Sxz[c - 1],  Syz[c + W],  Syz[c - W],  Syz[c + 1], Syz[c - 1]};
            const double acc = full_flux(s, q, a_min);
            const size_t g = base + gN[r];
            if constexpr (MODE == F25_RESNORM) {
                const double rv = cb[r] - acc;
                out[g] = rv;
                if (out32) out32[g] = (float)rv;
                v += rv * rv;
            } else if constexpr (MODE == F25_APPLY) {
                out[g] = acc;
            } else {
                pout[g] = (P)s.c;
                out[g] = acc;
                v += s.c * acc;
                if constexpr (UPD) ug[g] = cu[r] + alpha_u * cq[r];
            }
            // advance the column queues to plane p + 1
            qxx0[r] = qxx1[r];
            qxx1[r] = qxx2[r];
            qxx2[r] = rcx[r];
            qxym[r] = Sxy[c];
            qxyp[r] = rcy[r];
            qxzm[r] = Sxz[c];
            qxzp[r] = rcz[r];
            if constexpr (HAS_B) cb[r] = rb[r];
            if constexpr (UPD) {
                cu[r] = ru[r];
                cq[r] = rq[r];
            }
        }
        // operand plane p + 2 into the slot of p - 2, K plane p + 1 into the
        // slot of p - 1: both last read before the previous barrier
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            sF[(p - i0 + 2) & 3][dL[r]] = rf[r];
#pragma unroll
            for (int f = 0; f < 5; ++f) sK[f][kc ^ 1][dL[r]] = rk[f][r];
        }
        lds_barrier();
        fetch(p + 1);
    }
    if constexpr (MODE != F25_APPLY) {
        double vv[1] = {v};
        block_reduce_store<1, RED_SUM>(vv, part, blockIdx.x);
    }
}

// 8 x 64 tiles, 256 threads: 14 LDS slots of 10 x 66 doubles (74 KB, two
// workgroups per CU); the i-chunk is halved from n until the launch has
// MIN_BLOCKS workgroups (each chunk reads three extra operand planes).
struct F25Launch {
    static constexpr int TJ = 8, TK = 64, NT = 256, MIN_BLOCKS = 1024;
};

bool f25_fits(int n) { return n >= F25Launch::TK && n % F25Launch::TK == 0 && n % F25Launch::TJ == 0; }

int f25_chunk(int n)
{
    using C = F25Launch;
    int ci = n;
    while (ci % 2 == 0 && ci > 8 && (n / C::TK) * (n / C::TJ) * (n / ci) < C::MIN_BLOCKS) ci /= 2;
    return ci;
}

int f25_blocks(int n, int ci) { return (n / F25Launch::TK) * (n / F25Launch::TJ) * (n / ci); }

}  // namespace

bool full25_supported(int n) { return f25_fits(n); }

hipError_t launch_full_residual_norm25(const MassTensor &K, const double *u, const double *b, double *r, float *r32,
                                       int n, double a_min, Part &p, hipStream_t s)
{
    using C = F25Launch;
    if (!f25_fits(n)) return hipErrorInvalidValue;
    const int ci = f25_chunk(n), nb = f25_blocks(n, ci);
    if ((long)nb > kPartCap) return hipErrorInvalidValue;
    k_full25<double, double, F25_RESNORM, C::TJ, C::TK, C::NT><<<nb, C::NT, 0, s>>>(
        u, nullptr, b, K, r, r32, nullptr, n, ci, 0.0, a_min, p.part, nullptr, 0.0, nullptr);
    p.blocks = nb;
    p.k = 1;
    return hipGetLastError();
}

hipError_t launch_full_apply25(const MassTensor &K, const double *f, double *out, int n, double a_min, hipStream_t s)
{
    using C = F25Launch;
    if (!f25_fits(n) || out == f) return hipErrorInvalidValue;
    const int ci = f25_chunk(n), nb = f25_blocks(n, ci);
    k_full25<double, double, F25_APPLY, C::TJ, C::TK, C::NT><<<nb, C::NT, 0, s>>>(
        f, nullptr, nullptr, K, out, nullptr, nullptr, n, ci, 0.0, a_min, nullptr, nullptr, 0.0, nullptr);
    return hipGetLastError();
}

template <typename Z, typename P>
hipError_t launch_full_direction25(const Z *z, const P *p_old, P *p_new, const MassTensor &K, double *q, double beta,
                                   int n, double a_min, bool first, double *u, double alpha_u, const double *ks,
                                   Part &p, hipStream_t s)
{
    using C = F25Launch;
    const void *po = p_old;
    if (!f25_fits(n) || po == p_new || (u && (first || po == u || (void *)p_new == u || u == q)))
        return hipErrorInvalidValue;
    const int ci = f25_chunk(n), nb = f25_blocks(n, ci);
    if ((long)nb > kPartCap) return hipErrorInvalidValue;
    if (first)
        k_full25<Z, P, F25_DIRECTION, C::TJ, C::TK, C::NT, 1, 0><<<nb, C::NT, 0, s>>>(
            p_old, z, nullptr, K, q, nullptr, p_new, n, ci, beta, a_min, p.part, nullptr, 0.0, nullptr);
    else if (u)
        k_full25<Z, P, F25_DIRECTION, C::TJ, C::TK, C::NT, 0, 1><<<nb, C::NT, 0, s>>>(
            p_old, z, nullptr, K, q, nullptr, p_new, n, ci, beta, a_min, p.part, u, alpha_u, ks);
    else
        k_full25<Z, P, F25_DIRECTION, C::TJ, C::TK, C::NT, 0, 0><<<nb, C::NT, 0, s>>>(
            p_old, z, nullptr, K, q, nullptr, p_new, n, ci, beta, a_min, p.part, nullptr, 0.0, ks);
    p.blocks = nb;
    p.k = 1;
    return hipGetLastError();
}

template hipError_t launch_full_direction25<float, float>(const float *, const float *, float *, const MassTensor &,
                                                          double *, double, int, double, bool, double *, double,
                                                          const double *, Part &, hipStream_t);
template hipError_t launch_full_direction25<float, double>(const float *, const double *, double *,
                                                           const MassTensor &, double *, double, int, double, bool, double *,
                                                           double, const double *, Part &, hipStream_t);
template hipError_t launch_full_direction25<double, double>(const double *, const double *, double *,
                                                            const MassTensor &, double *, double, int, double, bool, double *,
                                                            double, const double *, Part &, hipStream_t);

}  // namespace recon
