// Streaming forms of the outer step's per-node passes (App. A):
//   * the mass on the deformed mesh, M_n = det(I + H_n) * (trilinear
//     interpolant of m at x_n = n + D_c phi_n), and its sum;
//   * the limited source t = Sigma + C + E (Eq. elliptic and the limiters),
//     with the sums of Sigma^2 and t;
//   * the nearest-neighbour smoothing S f = c0 f + cn (six neighbours) - sv.
//
// The gather kernels read a 19-point (or 7-point) neighbourhood per node from
// global memory.  Here a workgroup owns a TJ x TK tile and a chunk of
// i-planes; planes of the one stencil field (phi, or f for the smoothing)
// stream through a 4-slot LDS ring with a 1-cell halo in j and k, as the step
// trials do, so each value is read from HBM once.  The node arithmetic is the
// gather kernels' own, in the same order.  m is still gathered at the
// displaced positions (they move with phi).

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

namespace {

__device__ __forceinline__ void ring_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

enum { OUT_MESHMASS = 0, OUT_SOURCE = 1, OUT_SMOOTH = 2 };

template <int TJ, int TK, int NT>
struct RingTile {
    static constexpr int W = TK + 2, PLANE = (TJ + 2) * W;
    static constexpr int LU = (PLANE + NT - 1) / NT;
    static constexpr int PU = PLANE + 1;  // + one spare word for lanes past the plane
    static constexpr int RS = TJ * TK / NT;
};

struct OuterArgs {
    const double *m;     // meshmass: the normalised density
    const double *M;     // source: the mass per cell
    double *out;         // M, t or the smoothed field
    double rho_bar, xi_m, v_m;
    double c0, cn, sv;   // smoothing: centre weight, neighbour weight, subtracted constant
};

template <int MODE, int TJ, int TK, int NT>
__global__ void __launch_bounds__(NT) k_outer25(const double *__restrict__ f, int n, int ci, OuterArgs A, double *part)
{
    using F = RingTile<TJ, TK, NT>;
    static_assert(TJ * TK % NT == 0, "every thread owns whole rounds of the tile");
    constexpr int W = F::W, PLANE = F::PLANE, LU = F::LU, RS = F::RS;
    constexpr int K = MODE == OUT_SOURCE ? 2 : 1;
    __shared__ double sF[4][F::PU];

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
    int oN[RS], gN[RS], jN[RS], kN[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int q = tid + r * NT;
        oN[r] = (q / TK + 1) * W + (q % TK + 1);
        jN[r] = jb + q / TK;
        kN[r] = kb + q % TK;
        gN[r] = jN[r] * n + kN[r];
    }

    double rf[2][LU];
    auto fetch = [&](int set, int p) {
        const size_t base = (size_t)wrapc(p, n) * n2;
#pragma unroll
        for (int r = 0; r < LU; ++r) rf[set][r] = f[base + offL[r]];
    };
    auto deposit = [&](int set, int p) {
        double *P = sF[(p - i0 + 4) & 3];
#pragma unroll
        for (int r = 0; r < LU; ++r) P[dstL[r]] = rf[set][r];
    };

    double v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) v[c] = 0.0;
    // plane p (slots of p - 1, p, p + 1 resident)
    auto nodes = [&](int p) {
        const double *Pm = sF[(p - i0 + 3) & 3], *Pc = sF[(p - i0 + 4) & 3], *Pp = sF[(p - i0 + 5) & 3];
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            const int c = oN[r];
            const size_t g = (size_t)p * n2 + gN[r];
            if constexpr (MODE == OUT_SMOOTH) {
                const double nb = Pp[c] + Pm[c] + Pc[c + W] + Pc[c - W] + Pc[c + 1] + Pc[c - 1];
                __builtin_nontemporal_store(A.c0 * Pc[c] + A.cn * nb - A.sv, &A.out[g]);
            } else {
                Stencil19 s;
                s.c = Pc[c];
                s.xp = Pp[c];
                s.xm = Pm[c];
                s.yp = Pc[c + W];
                s.ym = Pc[c - W];
                s.zp = Pc[c + 1];
                s.zm = Pc[c - 1];
                s.xpyp = Pp[c + W];
                s.xpym = Pp[c - W];
                s.xmyp = Pm[c + W];
                s.xmym = Pm[c - W];
                s.xpzp = Pp[c + 1];
                s.xpzm = Pp[c - 1];
                s.xmzp = Pm[c + 1];
                s.xmzm = Pm[c - 1];
                s.ypzp = Pc[c + W + 1];
                s.ypzm = Pc[c + W - 1];
                s.ymzp = Pc[c - W + 1];
                s.ymzm = Pc[c - W - 1];
                const Sym3 e = triad19(s);
                const double gdet = det_sym(e);
                if constexpr (MODE == OUT_MESHMASS) {
                    const double x[3] = {p + 0.5 * (s.xp - s.xm), jN[r] + 0.5 * (s.yp - s.ym),
                                         kN[r] + 0.5 * (s.zp - s.zm)};
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
                    for (int cc = 0; cc < 8; ++cc) {
                        const int o0 = (cc >> 2) & 1, o1 = (cc >> 1) & 1, o2 = cc & 1;
                        const double w = (o0 ? w1[0] : 1.0 - w1[0]) * (o1 ? w1[1] : 1.0 - w1[1]) *
                                         (o2 ? w1[2] : 1.0 - w1[2]);
                        acc += w * A.m[lin(o0 ? f1[0] : f0[0], o1 ? f1[1] : f0[1], o2 ? f1[2] : f0[2], n)];
                    }
                    const double Mv = gdet * acc;
                    A.out[g] = Mv;
                    v[0] += Mv;
                } else {
                    const double sigma = A.rho_bar - A.M[g];
                    const double C = compression_limiter(e, A.xi_m);
                    const double E = gdet > A.v_m ? -2.0 * fabs(sigma) : 0.0;
                    const double tv = sigma + C + E;
                    A.out[g] = tv;
                    v[0] += sigma * sigma;
                    v[1] += tv;
                }
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
    ring_barrier();
    // Plane p: its nodes, then plane p + 2 into the slot of plane p - 2 (last
    // read by the nodes of p - 1, before the previous barrier).  ci is even;
    // the last steps stage and deposit planes past the chunk into unread slots.
    for (int s = i0; s < i0 + ci; s += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = s + h;
            nodes(p);
            deposit(h, p + 2);
            fetch(h, p + 4);
            ring_barrier();
        }
    }
    if constexpr (MODE != OUT_SMOOTH) block_reduce_store<K, RED_SUM>(v, part, blockIdx.x);
}

constexpr int kOutTJ = 8, kOutTK = 64, kOutNT = 256, kOutMinBlocks = 2048;

template <int MODE>
hipError_t launch_outer25(const double *f, int n, const OuterArgs &A, Part *p, hipStream_t s)
{
    if (!outer25_supported(n)) return hipErrorInvalidValue;
    int ci = n;
    while (ci % 4 == 0 && (n / kOutTK) * (n / kOutTJ) * (n / ci) < kOutMinBlocks) ci /= 2;  // ci stays even
    const int nb = (n / kOutTK) * (n / kOutTJ) * (n / ci);
    constexpr int K = MODE == OUT_SOURCE ? 2 : 1;
    if (p && (long)nb * K > kPartCap) return hipErrorInvalidValue;
    k_outer25<MODE, kOutTJ, kOutTK, kOutNT><<<nb, kOutNT, 0, s>>>(f, n, ci, A, p ? p->part : nullptr);
    if (p) {
        p->blocks = nb;
        p->k = K;
    }
    return hipGetLastError();
}

}  // namespace

bool outer25_supported(int n)
{
    return n >= kOutTK && n % kOutTK == 0 && n % kOutTJ == 0;
}

hipError_t launch_meshmass25(const double *phi, const double *m, double *M, int n, Part &p, hipStream_t s)
{
    OuterArgs A{};
    A.m = m;
    A.out = M;
    return launch_outer25<OUT_MESHMASS>(phi, n, A, &p, s);
}

hipError_t launch_source25(const double *phi, const double *M, double rho_bar, double xi_m, double v_m, double *t,
                           int n, Part &p, hipStream_t s)
{
    OuterArgs A{};
    A.M = M;
    A.out = t;
    A.rho_bar = rho_bar;
    A.xi_m = xi_m;
    A.v_m = v_m;
    return launch_outer25<OUT_SOURCE>(phi, n, A, &p, s);
}

hipError_t launch_smooth25(const double *f, double *out, int n, double c0, double sub, hipStream_t s)
{
    OuterArgs A{};
    A.out = out;
    A.c0 = c0;
    A.cn = (1.0 - c0) / 6.0;
    A.sv = sub;
    return launch_outer25<OUT_SMOOTH>(f, n, A, nullptr, s);
}

}  // namespace recon
