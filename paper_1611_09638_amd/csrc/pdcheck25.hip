// Step-size trials of the moving mesh (Sec. II: the map x = xi + grad phi
// must stay positive definite; App. A: small steps): for NTR consecutive
// alpha = 2^-j, count the nodes where I + Hess(phi + alpha dphi) fails
// Sylvester's criterion (e11 > 0, e11 e22 - e12^2 > 0, det > 0), or, under the
// mass update of App. A, where the updated mass M + alpha D is not positive.
//
// The compact Hessian reads a 19-point neighbourhood of two fields.  Here a
// workgroup owns a TJ x TK tile and a chunk of i-planes; planes of phi and
// dphi stream through a 4-slot LDS ring with a 1-cell halo in j and k, so
// each value is read from HBM once instead of 38 gathers per node.  The trial
// potential is formed per stencil point exactly as phi + alpha dphi (alpha is
// a power of two), as in the per-node kernel, so the counts are the same.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

namespace {

__device__ __forceinline__ void lds_fence_barrier_pd()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int TJ, int TK, int NT>
struct PdTile {
    static constexpr int W = TK + 2, PLANE = (TJ + 2) * W;
    static constexpr int LU = (PLANE + NT - 1) / NT;
    static constexpr int PU = PLANE + 1;  // + one spare word for lanes past the plane
    static constexpr int RS = TJ * TK / NT;
};

template <int NTR, int TJ, int TK, int NT>
__global__ void __launch_bounds__(NT) k_pd25(const double *__restrict__ phi, const double *__restrict__ dphi, int n,
                                            int ci, int j0, double *part, const double *__restrict__ massM,
                                            const double *__restrict__ massD)
{
    using F = PdTile<TJ, TK, NT>;
    static_assert(TJ * TK % NT == 0, "every thread owns whole rounds of the tile");
    constexpr int W = F::W, PLANE = F::PLANE, LU = F::LU, RS = F::RS;
    __shared__ double sP[4][F::PU];
    __shared__ double sD[4][F::PU];

    const int tid = threadIdx.x;
    const int tiles_k = n / TK, tiles_j = n / TJ, chunks = n / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int jb = tj * TJ, kb = tk * TK, i0 = ch * ci;
    const size_t n2 = (size_t)n * n;

    int offL[LU], dstL[LU];
#pragma unroll
    for (int r = 0; r < LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / W, col = q % W;
        offL[r] = q < PLANE ? wrapc(jb - 1 + row, n) * n + wrapc(kb - 1 + col, n) : 0;
        dstL[r] = q < PLANE ? q : PLANE;
    }
    int oN[RS], gN[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int q = tid + r * NT;
        oN[r] = (q / TK + 1) * W + (q % TK + 1);
        gN[r] = (jb + q / TK) * n + (kb + q % TK);
    }

    double rp[2][LU], rd[2][LU];
    auto fetch = [&](int set, int p) {
        const size_t base = (size_t)wrapc(p, n) * n2;
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            rp[set][r] = phi[base + offL[r]];
            rd[set][r] = dphi[base + offL[r]];
        }
    };
    auto deposit = [&](int set, int p) {
        double *P = sP[(p - i0 + 4) & 3], *D = sD[(p - i0 + 4) & 3];
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            P[dstL[r]] = rp[set][r];
            D[dstL[r]] = rd[set][r];
        }
    };

    double cnt[NTR];
#pragma unroll
    for (int m = 0; m < NTR; ++m) cnt[m] = 0.0;
    // trials on plane p (slots of p - 1, p, p + 1 resident)
    auto trials = [&](int p) {
        const double *Pm = sP[(p - i0 + 3) & 3], *Pc = sP[(p - i0 + 4) & 3], *Pp = sP[(p - i0 + 5) & 3];
        const double *Dm = sD[(p - i0 + 3) & 3], *Dc = sD[(p - i0 + 4) & 3], *Dp = sD[(p - i0 + 5) & 3];
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            const int c = oN[r];
            // the mass update's positivity test: M + alpha D > 0
            double mv = 1.0, dv = 0.0;
            if (massM) {
                mv = massM[(size_t)p * n2 + gN[r]];
                dv = massD[(size_t)p * n2 + gN[r]];
            }
            Stencil19 a, d;
            a.c = Pc[c]; d.c = Dc[c];
            a.xp = Pp[c]; d.xp = Dp[c];
            a.xm = Pm[c]; d.xm = Dm[c];
            a.yp = Pc[c + W]; d.yp = Dc[c + W];
            a.ym = Pc[c - W]; d.ym = Dc[c - W];
            a.zp = Pc[c + 1]; d.zp = Dc[c + 1];
            a.zm = Pc[c - 1]; d.zm = Dc[c - 1];
            a.xpyp = Pp[c + W]; d.xpyp = Dp[c + W];
            a.xpym = Pp[c - W]; d.xpym = Dp[c - W];
            a.xmyp = Pm[c + W]; d.xmyp = Dm[c + W];
            a.xmym = Pm[c - W]; d.xmym = Dm[c - W];
            a.xpzp = Pp[c + 1]; d.xpzp = Dp[c + 1];
            a.xpzm = Pp[c - 1]; d.xpzm = Dp[c - 1];
            a.xmzp = Pm[c + 1]; d.xmzp = Dm[c + 1];
            a.xmzm = Pm[c - 1]; d.xmzm = Dm[c - 1];
            a.ypzp = Pc[c + W + 1]; d.ypzp = Dc[c + W + 1];
            a.ypzm = Pc[c + W - 1]; d.ypzm = Dc[c + W - 1];
            a.ymzp = Pc[c - W + 1]; d.ymzp = Dc[c - W + 1];
            a.ymzm = Pc[c - W - 1]; d.ymzm = Dc[c - W - 1];
#pragma unroll
            for (int m = 0; m < NTR; ++m) {
                const double al = ldexp(1.0, -(j0 + m));
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
                cnt[m] += ok ? 0.0 : 1.0;
            }
        }
    };

    // prologue: planes i0-1, i0, i0+1 resident; i0+2 and i0+3 staged
    fetch(0, i0 - 1);
    deposit(0, i0 - 1);
    fetch(0, i0);
    deposit(0, i0);
    fetch(0, i0 + 1);
    deposit(0, i0 + 1);
    fetch(0, i0 + 2);
    fetch(1, i0 + 3);
    lds_fence_barrier_pd();
    // Plane p: trials, then plane p + 2 into the slot of plane p - 2 (last read
    // by the trials on p - 1, before the previous barrier).  ci is even; the
    // last steps stage and deposit planes past the chunk into unread slots.
    for (int s = i0; s < i0 + ci; s += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = s + h;
            trials(p);
            deposit(h, p + 2);
            fetch(h, p + 4);
            lds_fence_barrier_pd();
        }
    }
    block_reduce_store<NTR, RED_SUM>(cnt, part, blockIdx.x);
}

constexpr int kPdTJ = 8, kPdTK = 64, kPdNT = 256, kPdMinBlocks = 2048;

}  // namespace

bool pd25_supported(int n)
{
    return n >= kPdTK && n % kPdTK == 0 && n % kPdTJ == 0;
}

hipError_t launch_pd25(const double *phi, const double *dphi, int n, int j0, int ntrial, Part &p, hipStream_t s,
                       const double *M, const double *D)
{
    if ((M == nullptr) != (D == nullptr)) return hipErrorInvalidValue;
    if (!pd25_supported(n) || (ntrial != 1 && ntrial != 4)) return hipErrorInvalidValue;
    int ci = n;
    while (ci % 4 == 0 && (n / kPdTK) * (n / kPdTJ) * (n / ci) < kPdMinBlocks) ci /= 2;  // ci stays even
    const int nb = (n / kPdTK) * (n / kPdTJ) * (n / ci);
    if ((long)nb * ntrial > kPartCap) return hipErrorInvalidValue;
    if (ntrial == 1)
        k_pd25<1, kPdTJ, kPdTK, kPdNT><<<nb, kPdNT, 0, s>>>(phi, dphi, n, ci, j0, p.part, M, D);
    else
        k_pd25<4, kPdTJ, kPdTK, kPdNT><<<nb, kPdNT, 0, s>>>(phi, dphi, n, ci, j0, p.part, M, D);
    p.blocks = nb;
    p.k = ntrial;
    return hipGetLastError();
}

}  // namespace recon
