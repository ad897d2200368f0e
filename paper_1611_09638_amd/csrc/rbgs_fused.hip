// Fused two-colour red-black Gauss-Seidel sweep (the smoother of the
// multigrid solves, App. A), in a translation unit of its own so that its
// source can be tied to the hardware counters measured on it.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace recon {

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for every
// outstanding global load, which would drain the register prefetch at each
// barrier; here the loads stay in flight until their registers are used.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------- fused two-colour RB-GS sweep
//
// u_out = one full red-black sweep of u_in (colour `first` relaxed first),
// streaming every field through HBM once.  A workgroup owns a TJ x TK tile of
// (j, k) and a chunk of CI consecutive i-planes.  Planes of u_in and a enter a
// 4-plane LDS ring with a 2-cell halo in j and k, two planes ahead of use
// (register-staged prefetch); b is fetched straight into registers at each
// thread's relaxation nodes, also two planes ahead.  Iteration s relaxes the
// first colour on plane s+1 over the tile plus a 1-cell ring (the ring values
// are recomputed here rather than exchanged with neighbouring tiles), then
// the second colour on plane s over the tile, writes plane s and deposits
// plane s+3 into the slot of plane s-1 (three barriers per plane).  The old
// first-colour values are never read (Gauss-Seidel overwrites them), so the
// new ones are stored in place in the ring.  Out of place because the
// neighbouring tiles read this tile's halo from u_in.  Load lanes past the
// halo plane write one spare word per slot, so every thread loads and
// deposits unconditionally and the load queue stays countable.
//
// SLOTS = 6 keeps six planes in the ring instead of four: plane s+3 then goes
// into the slot of plane s-3, dead since the step before, at the start of
// step s, so the barrier after the first colour also publishes it and a
// step needs two barriers instead of three (76 KB of LDS in FP32, still two
// workgroups per CU).  The steady loop is unrolled by six; a chunk whose
// length is not a multiple of six runs up to five extra steps past its end,
// which relax planes that are not stored.  Both forms give the same sweep
// bit for bit.
//
// Face order in the relaxation: +i, -i, +j, -j, +k, -k (as in k_rbgs_half),
// so the fused and per-colour sweeps round identically; a is stored halved
// (the face coefficient max(a_min, (a_n + a_nb) / 2) is max(a_min, h_n + h_nb)).
// ZERO: u_in is taken as 0 and not read (the first sweep from a zero guess).
// The first colour then has only zero neighbours: its weighted sum is +0, so
// only the face coefficients are summed, and the zero planes of u are never
// staged in LDS (every value the second colour and the plane store read is
// written by a relaxation first).  The result is the same bit for bit.
template <typename T, int TJ, int TK_, int NT_>
struct Ring4 {
    static constexpr int TK = TK_, NT = NT_;
    static constexpr int H = TJ + 4, W = TK + 4, PLANE = H * W;  // u, a: halo 2
    static constexpr int LU = (PLANE + NT - 1) / NT;
    static constexpr int PU = PLANE + 1;                          // + one spare word
    static constexpr int N1 = (TJ + 2) * (TK / 2 + 1);           // first colour: tile + ring
    static constexpr int N2 = TJ * (TK / 2);                     // second colour: tile
    static constexpr int R1 = (N1 + NT - 1) / NT, R2 = (N2 + NT - 1) / NT;
    static constexpr int RS = TJ * TK / NT;
};

template <int X>
using IC = std::integral_constant<int, X>;

// FIRST: the colour relaxed first (a template parameter: chunks start on
// planes that are multiples of 4, so with the steady loop unrolled by the
// ring depth every ring slot and every plane parity is a compile-time
// constant, and each LDS access is one per-thread offset plus an immediate).
// NTS = 1 stores the swept planes nontemporally: on fields far larger than
// the caches nothing reads them back soon, and keeping them out of L2 leaves
// it to the halo rows that neighbouring tiles share (5-8% faster at 512^3).
// PRO = 1 folds the multigrid's coarse correction into the sweep (the first
// post-smoothing sweep of a V-cycle): every plane of u_in enters the ring as
// u_in + P e, with P the trilinear prolongation of the coarse-grid correction
// e (edge n/2), formed exactly as the prolongation kernels form it (weights
// 1/2 along k, then j, then between coarse planes).  The coarse planes a
// plane needs pass through a 4-slot LDS ring of their own ((TJ/2 + 3) x
// (TK/2 + 3) nodes, one coarse node beyond the fine halo); the coarse plane
// c + 1 is staged with fine plane 2c and stored with it.  u_out is then
// exactly the sweep of the prolonged field, without the prolongation's own
// pass over u.
template <int TJ, int TK, int NT>
struct CoarseTile {
    static constexpr int CH = TJ / 2 + 3, CW = TK / 2 + 3, PLANE = CH * CW;
    static constexpr int LU = (PLANE + NT - 1) / NT, PU = PLANE + 1;
};

template <typename T, int TJ, int ZERO, int FIRST, int TK_ = 64, int NT_ = 512, int MINW = 1, int SLOTS = 4,
          int PRO = 0, int NTS = 0>
__global__ void __launch_bounds__(NT_, MINW) k_rbgs_fused(const T *__restrict__ uin, T *__restrict__ uout,
                                                    const T *__restrict__ ag, const T *__restrict__ bg, int n,
                                                    int ci, T inv_scale, T a_min, const T *__restrict__ eg)
{
    using F = Ring4<T, TJ, TK_, NT_>;
    using CT = CoarseTile<TJ, TK_, NT_>;
    static_assert(TJ * TK_ % NT_ == 0, "every thread stores whole rounds of the tile");
    static_assert(SLOTS == 4 || SLOTS == 6, "a ring of four or six planes");
    static_assert(!(PRO && ZERO), "the coarse correction is added to a sweep's input");
    __shared__ T sE[PRO ? 4 : 1][PRO ? CT::PU : 1];
    constexpr int W = F::W, HW = W / 2, PLANE = F::PLANE, NT = F::NT, LU = F::LU, R1 = F::R1, R2 = F::R2;
    constexpr int RS = F::RS, C1 = FIRST, C2 = 1 - FIRST;
    static_assert(W % 2 == 0, "rows split into equal even and odd halves");
    __shared__ T sU[SLOTS][F::PU];
    __shared__ T sA[SLOTS][F::PU];

    const int tid = threadIdx.x;
    const int tiles_k = n / F::TK, tiles_j = n / TJ, chunks = n / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int j0 = tj * TJ, k0 = tk * F::TK, i0 = ch * ci;
    const size_t plane_bytes = (size_t)n * n * sizeof(T);
    // LDS position of halo-plane row `row`, column `col`: the even and odd
    // columns of each row sit in separate halves, so that the nodes of one
    // colour and each of their neighbours are contiguous across a wavefront
    auto lidx = [](int row, int col) { return row * W + (col & 1) * HW + (col >> 1); };

    // halo load slots: in-plane byte offset and LDS destination
    unsigned offU[LU];
    int dstU[LU];
#pragma unroll
    for (int r = 0; r < LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / W, col = q % W;
        const int gj = wrapc(j0 - 2 + row, n), gk = wrapc(k0 - 2 + col, n);
        offU[r] = q < PLANE ? (unsigned)(gj * n + gk) * (unsigned)sizeof(T) : 0u;
        dstU[r] = q < PLANE ? lidx(row, col) : PLANE;
    }
    // relaxation nodes for both plane parities P: LDS offsets of the node and
    // of its +k neighbour (the -k neighbour is the next word down in the other
    // half), and the in-plane byte offset of b.  First colour: tile + 1-cell
    // ring, node q at row jj = q / (TK/2 + 1) - 1, column kk = 2 (q % (TK/2 + 1))
    // - 1 + e; second colour: tile, jj = q / (TK/2), kk = 2 (q % (TK/2)) + e; e
    // makes (i + j + k) % 2 the colour.  Lanes past the node count use a valid
    // node and skip the relaxation.
    int c1[R1][2], p1[R1][2], c2[R2][2], p2[R2][2];
    unsigned g1[R1][2], g2[R2][2];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        const int q = tid + r * NT;
        const bool on = q < F::N1;
        const int jj = on ? q / (F::TK / 2 + 1) - 1 : 0, pr = on ? q % (F::TK / 2 + 1) : 1;
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            const int kk = 2 * pr - 1 + ((P + jj + 1) & 1);
            c1[r][P] = lidx(jj + 2, kk + 2);
            p1[r][P] = lidx(jj + 2, kk + 3);
            g1[r][P] = (unsigned)(wrapc(j0 + jj, n) * n + wrapc(k0 + kk, n)) * (unsigned)sizeof(T);
        }
    }
#pragma unroll
    for (int r = 0; r < R2; ++r) {
        const int q = tid + r * NT;
        const bool on = q < F::N2;
        const int jj = on ? q / (F::TK / 2) : 0, pr = on ? q % (F::TK / 2) : 0;
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            const int kk = 2 * pr + ((P + jj) & 1);
            c2[r][P] = lidx(jj + 2, kk + 2);
            p2[r][P] = lidx(jj + 2, kk + 3);
            g2[r][P] = (unsigned)((j0 + jj) * n + (k0 + kk)) * (unsigned)sizeof(T);
        }
    }
    // this thread's nodes of the tile for the plane store
    int sN[RS];
    unsigned gS[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int q = tid + r * NT;
        const int row = q / F::TK, col = q % F::TK;
        sN[r] = lidx(row + 2, col + 2);
        gS[r] = (unsigned)((j0 + row) * n + (k0 + col)) * (unsigned)sizeof(T);
    }

    auto plane = [&](const T *f, int p) {
        return reinterpret_cast<const char *>(f) + (size_t)wrapc(p, n) * plane_bytes;
    };
    auto at = [](const char *base, unsigned off) { return *reinterpret_cast<const T *>(base + off); };

    // PRO: the coarse tile's loads (offsets into a coarse plane, LDS words)
    // and, per halo-load slot, the coarse LDS word of its (j, k) corner with
    // the node's parities (bit 0: k odd, bit 1: j odd)
    constexpr int CLU = PRO ? CT::LU : 1;
    const int nc = n >> 1;
    const size_t cplane = (size_t)nc * nc;
    unsigned offC[CLU];
    int dstC[CLU], cor[PRO ? LU : 1];
    unsigned par = 0;
    if constexpr (PRO) {
#pragma unroll
        for (int r = 0; r < CLU; ++r) {
            const int q = tid + r * NT;
            const int row = q / CT::CW, col = q % CT::CW;
            const int gj = (j0 >> 1) - 1 + row, gk = (k0 >> 1) - 1 + col;
            offC[r] = q < CT::PLANE ? (unsigned)(wrapc(gj, nc) * nc + wrapc(gk, nc)) : 0u;
            dstC[r] = q < CT::PLANE ? q : CT::PLANE;
        }
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            const int q = tid + r * NT;
            const int row = q < PLANE ? q / W : 0, col = q < PLANE ? q % W : 0;
            cor[r] = (row >> 1) * CT::CW + (col >> 1);
            par |= (unsigned)((col & 1) | ((row & 1) << 1)) << (2 * r);
        }
    }
    T rcs[2][CLU];
    auto coarse_load = [&](int c, T (&dst)[CLU]) {
        const T *pl = eg + (size_t)wrapc(c, nc) * cplane;
#pragma unroll
        for (int r = 0; r < CLU; ++r) dst[r] = pl[offC[r]];
    };
    auto coarse_store = [&](int c, const T (&src)[CLU]) {
        T *E = sE[c & 3];
#pragma unroll
        for (int r = 0; r < CLU; ++r) E[dstC[r]] = src[r];
    };
    // the coarse correction at halo-load slot r from coarse plane c: the
    // in-plane interpolation of the prolongation kernels
    auto inplane = [&](int c, int r) {
        const T *E = sE[c & 3];
        const int kod = (par >> (2 * r)) & 1, jod = (par >> (2 * r + 1)) & 1;
        const int a00 = cor[r], a01 = a00 + kod, a10 = a00 + jod * CT::CW, a11 = a10 + kod;
        const T v00 = E[a00], v01 = E[a01], v10 = E[a10], v11 = E[a11];
        const T wk = (T)0.5, wj = (T)0.5;
        const T r0 = kod ? wk * (v00 + v01) : v00;
        const T r1 = kod ? wk * (v10 + v11) : v10;
        return jod ? wj * (r0 + r1) : r0;
    };

    // PRO: each halo-load slot's in-plane interpolation of the coarse plane
    // above the last odd plane deposited (deposits run through consecutive
    // planes, so every coarse plane is interpolated once per slot and serves
    // the fine planes 2c - 1, 2c and 2c + 1 from registers).  The FP64 sweep
    // on the six-plane ring recomputes them instead, which measured faster
    // there (0.93 against 0.95 ms at 512^3; elsewhere keeping them saves 8-15%).
    constexpr bool KEEP = PRO && !(sizeof(T) == 8 && SLOTS == 6);
    T ic[KEEP ? LU : 1];
    T ru[2][LU], ra[2][LU];
    auto fetch = [&](auto SETc, int p) {
        constexpr int SET = decltype(SETc)::value;
        const char *ub = plane(uin, p), *ab = plane(ag, p);
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            if constexpr (!ZERO) ru[SET][r] = at(ub, offU[r]);
            ra[SET][r] = at(ab, offU[r]);
        }
        // PRO: an even plane 2c brings coarse plane c + 1 along
        if constexpr (PRO)
            if (!(p & 1)) coarse_load((p >> 1) + 1, rcs[SET]);
    };
    // the interpolation of coarse plane c at slot r, kept or recomputed
    auto held = [&](int c, int r) {
        if constexpr (KEEP) return ic[r];
        else return inplane(c, r);
    };
    // store the staged plane p (PRO: plus its coarse correction; with cw,
    // an even plane also stores the coarse plane staged with it)
    auto deposit = [&](auto SETc, auto SLOTc, int p = 0, bool cw = false) {
        constexpr int SET = decltype(SETc)::value, SLOT = decltype(SLOTc)::value;
        if constexpr (PRO) {
            const int c = p >> 1;
            const T wi = (T)0.5;
            if (p & 1) {
#pragma unroll
                for (int r = 0; r < LU; ++r) {
                    const T lo = held(c, r);
                    const T up = inplane(c + 1, r);
                    if constexpr (KEEP) ic[r] = up;
                    sU[SLOT][dstU[r]] = ru[SET][r] + wi * (lo + up);
                }
            } else {
#pragma unroll
                for (int r = 0; r < LU; ++r) sU[SLOT][dstU[r]] = ru[SET][r] + held(c, r);
                if (cw) coarse_store(c + 1, rcs[SET]);
            }
        } else if constexpr (!ZERO) {
#pragma unroll
            for (int r = 0; r < LU; ++r) sU[SLOT][dstU[r]] = ru[SET][r];
        }
#pragma unroll
        for (int r = 0; r < LU; ++r) sA[SLOT][dstU[r]] = (T)0.5 * ra[SET][r];
    };
    // PRO: the coarse planes the prologue's deposits read, c0 - 1 .. c0 + K
    // with c0 = i0 / 2, stored before them, and (when kept) the interpolation
    // of c0 - 1 for the first deposit (plane i0 - 2)
    auto coarse_preload = [&](int K) {
        if constexpr (PRO) {
            for (int c = (i0 >> 1) - 1; c <= (i0 >> 1) + K; ++c) {
                T tmp[CLU];
                coarse_load(c, tmp);
                coarse_store(c, tmp);
            }
            lds_barrier();
            if constexpr (KEEP)
#pragma unroll
                for (int r = 0; r < LU; ++r) ic[r] = inplane((i0 >> 1) - 1, r);
        }
    };
    // b at the first-colour nodes of plane q1 (parity P1) and at the
    // second-colour nodes of plane q2 (parity P2)
    T rb1[2][R1], rb2[2][R2];
    auto fetch_b = [&](auto SETc, int q1, auto P1c, int q2, auto P2c) {
        constexpr int SET = decltype(SETc)::value, P1 = decltype(P1c)::value, P2 = decltype(P2c)::value;
        const char *b1 = plane(bg, q1), *b2 = plane(bg, q2);
#pragma unroll
        for (int r = 0; r < R1; ++r) rb1[SET][r] = at(b1, g1[r][P1]);
#pragma unroll
        for (int r = 0; r < R2; ++r) rb2[SET][r] = at(b2, g2[r][P2]);
    };

    // one Gauss-Seidel relaxation from ring slots SC (the node's plane), SU
    // (+i) and SD (-i); c: node, pk: its +k neighbour, pk - 1: its -k neighbour
    auto relax = [&](auto SCc, auto SUc, auto SDc, int c, int pk, T bval) {
        constexpr int SC = decltype(SCc)::value, SU = decltype(SUc)::value, SD = decltype(SDc)::value;
        const T hn = sA[SC][c];
        T num = 0, den = 0, cf;
        cf = fmax(hn + sA[SU][c], a_min); num += cf * sU[SU][c]; den += cf;
        cf = fmax(hn + sA[SD][c], a_min); num += cf * sU[SD][c]; den += cf;
        cf = fmax(hn + sA[SC][c + W], a_min); num += cf * sU[SC][c + W]; den += cf;
        cf = fmax(hn + sA[SC][c - W], a_min); num += cf * sU[SC][c - W]; den += cf;
        cf = fmax(hn + sA[SC][pk], a_min); num += cf * sU[SC][pk]; den += cf;
        cf = fmax(hn + sA[SC][pk - 1], a_min); num += cf * sU[SC][pk - 1]; den += cf;
        return qdiv(num - bval * inv_scale, den);
    };
    // the same relaxation with every neighbour zero (ZERO's first colour):
    // the weighted sum stays +0 and the face coefficients add up in order
    auto relax_zero = [&](auto SCc, auto SUc, auto SDc, int c, int pk, T bval) {
        constexpr int SC = decltype(SCc)::value, SU = decltype(SUc)::value, SD = decltype(SDc)::value;
        const T hn = sA[SC][c];
        T den = 0;
        den += fmax(hn + sA[SU][c], a_min);
        den += fmax(hn + sA[SD][c], a_min);
        den += fmax(hn + sA[SC][c + W], a_min);
        den += fmax(hn + sA[SC][c - W], a_min);
        den += fmax(hn + sA[SC][pk], a_min);
        den += fmax(hn + sA[SC][pk - 1], a_min);
        const T num = 0;
        return qdiv(num - bval * inv_scale, den);
    };
    // first colour over the tile and its ring (reads only second-colour values)
    auto relax_first = [&](auto SCc, auto SUc, auto SDc, auto Pc, const T (&bv)[R1]) {
        constexpr int SC = decltype(SCc)::value, P = decltype(Pc)::value;
#pragma unroll
        for (int r = 0; r < R1; ++r)
            if (tid + r * NT < F::N1) {
                if constexpr (ZERO) sU[SC][c1[r][P]] = relax_zero(SCc, SUc, SDc, c1[r][P], p1[r][P], bv[r]);
                else sU[SC][c1[r][P]] = relax(SCc, SUc, SDc, c1[r][P], p1[r][P], bv[r]);
            }
    };
    // second colour over the tile (reads only new first-colour values)
    auto relax_second = [&](auto SCc, auto SUc, auto SDc, auto Pc, const T (&bv)[R2]) {
        constexpr int SC = decltype(SCc)::value, P = decltype(Pc)::value;
#pragma unroll
        for (int r = 0; r < R2; ++r)
            if (tid + r * NT < F::N2) sU[SC][c2[r][P]] = relax(SCc, SUc, SDc, c2[r][P], p2[r][P], bv[r]);
    };
    auto store_plane = [&](auto SLOTc, int p) {
        constexpr int SLOT = decltype(SLOTc)::value;
        char *ob = reinterpret_cast<char *>(uout) + (size_t)wrapc(p, n) * plane_bytes;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            T *dst = reinterpret_cast<T *>(ob + gS[r]);
            if constexpr (NTS) __builtin_nontemporal_store(sU[SLOT][sN[r]], dst);
            else *dst = sU[SLOT][sN[r]];
        }
    };

    if constexpr (SLOTS == 6) {
    // Ring slot of plane i0 + d is (d + 60) % 6.  Prologue: planes i0-2 ..
    // i0+2 resident, i0+3 (set 0) and i0+4 (set 1) staged, b of the first
    // two steps staged; warm-up: first colour on planes i0-1 and i0 (they
    // read only second-colour values, so no barrier between them).
    coarse_preload(2);
    fetch(IC<0>{}, i0 - 2);
    deposit(IC<0>{}, IC<4>{}, i0 - 2);
    fetch(IC<0>{}, i0 - 1);
    deposit(IC<0>{}, IC<5>{}, i0 - 1);
    fetch(IC<0>{}, i0);
    deposit(IC<0>{}, IC<0>{}, i0);
    fetch(IC<0>{}, i0 + 1);
    deposit(IC<0>{}, IC<1>{}, i0 + 1);
    fetch(IC<0>{}, i0 + 2);
    deposit(IC<0>{}, IC<2>{}, i0 + 2);
    fetch(IC<0>{}, i0 + 3);
    fetch(IC<1>{}, i0 + 4);
    fetch_b(IC<0>{}, i0 + 1, IC<(C1 + 1) & 1>{}, i0, IC<C2 & 1>{});
    fetch_b(IC<1>{}, i0 + 2, IC<C1 & 1>{}, i0 + 1, IC<(C2 + 1) & 1>{});
    lds_barrier();
    {
        T bw[R1], bx[R1];
        const char *bb = plane(bg, i0 - 1), *bc = plane(bg, i0);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            bw[r] = at(bb, g1[r][(C1 + 1) & 1]);
            bx[r] = at(bc, g1[r][C1 & 1]);
        }
        relax_first(IC<5>{}, IC<0>{}, IC<4>{}, IC<(C1 + 1) & 1>{}, bw);
        relax_first(IC<0>{}, IC<1>{}, IC<5>{}, IC<C1 & 1>{}, bx);
    }
    lds_barrier();
    const int iend = i0 + ci;
    // Step H (plane ss): deposit ss+3 into the slot of ss-3, stage ss+5;
    // first colour on ss+1; second colour on ss; store ss unless past the
    // chunk; stage the b values of the step after next.
    auto step6 = [&](auto Hc, int ss) {
        constexpr int H = decltype(Hc)::value, h = H & 1;
        deposit(IC<h>{}, IC<(H + 3) % 6>{}, ss + 3, true);
        fetch(IC<h>{}, ss + 5);
        relax_first(IC<(H + 1) % 6>{}, IC<(H + 2) % 6>{}, IC<H % 6>{}, IC<(C1 + H + 1) & 1>{}, rb1[h]);
        lds_barrier();
        relax_second(IC<H % 6>{}, IC<(H + 1) % 6>{}, IC<(H + 5) % 6>{}, IC<(C2 + H) & 1>{}, rb2[h]);
        lds_barrier();
        if (ss < iend) store_plane(IC<H % 6>{}, ss);
        fetch_b(IC<h>{}, ss + 3, IC<(C1 + H + 3) & 1>{}, ss + 2, IC<(C2 + H + 2) & 1>{});
    };
    for (int s = i0; s < iend; s += 6) {
        step6(IC<0>{}, s);
        step6(IC<1>{}, s + 1);
        step6(IC<2>{}, s + 2);
        step6(IC<3>{}, s + 3);
        step6(IC<4>{}, s + 4);
        step6(IC<5>{}, s + 5);
    }
    } else {
    // Ring slot of plane i0 + d is d & 3 (d >= -2: slot (d + 4) & 3); the
    // first colour's parity on plane i0 + d is (C1 + d) & 1, the second's
    // (C2 + d) & 1 (i0 is even).
    // prologue: planes i0-2 .. i0+1 resident, i0+2 (set 1) and i0+3 (set 0)
    // staged, b for the first two steady steps staged
    coarse_preload(1);
    fetch(IC<0>{}, i0 - 2);
    deposit(IC<0>{}, IC<2>{}, i0 - 2);
    fetch(IC<0>{}, i0 - 1);
    deposit(IC<0>{}, IC<3>{}, i0 - 1);
    fetch(IC<0>{}, i0);
    deposit(IC<0>{}, IC<0>{}, i0);
    fetch(IC<0>{}, i0 + 1);
    deposit(IC<0>{}, IC<1>{}, i0 + 1);
    fetch(IC<1>{}, i0 + 2);
    fetch(IC<0>{}, i0 + 3);
    fetch_b(IC<0>{}, i0 + 1, IC<(C1 + 1) & 1>{}, i0, IC<C2 & 1>{});
    fetch_b(IC<1>{}, i0 + 2, IC<C1 & 1>{}, i0 + 1, IC<(C2 + 1) & 1>{});
    lds_barrier();
    // warm-up: first colour on planes i0-1 and i0
    {
        T bw[R1];
        const char *bb = plane(bg, i0 - 1);
#pragma unroll
        for (int r = 0; r < R1; ++r) bw[r] = at(bb, g1[r][(C1 + 1) & 1]);
        relax_first(IC<3>{}, IC<0>{}, IC<2>{}, IC<(C1 + 1) & 1>{}, bw);
    }
    lds_barrier();
    deposit(IC<1>{}, IC<2>{}, i0 + 2, true);  // plane i0+2 into the slot of plane i0-2, read last just above
    fetch(IC<1>{}, i0 + 4);
    lds_barrier();
    {
        T bw[R1];
        const char *bb = plane(bg, i0);
#pragma unroll
        for (int r = 0; r < R1; ++r) bw[r] = at(bb, g1[r][C1 & 1]);
        relax_first(IC<0>{}, IC<1>{}, IC<3>{}, IC<C1 & 1>{}, bw);
    }
    // Steady state, branch-free, four planes per trip (ci is a multiple of 4).
    // Step H (plane ss = i0 + 4m + H): first colour on ss+1, second colour on
    // ss, store ss, deposit ss+3 into the slot of ss-1, stage ss+5 and the b
    // values of the step after next.  The last steps fetch and deposit planes
    // past the chunk: they wrap to valid addresses and land in ring slots that
    // are no longer read.
    auto step = [&](auto Hc, int ss) {
        constexpr int H = decltype(Hc)::value, h = H & 1;
        relax_first(IC<(H + 1) & 3>{}, IC<(H + 2) & 3>{}, IC<H & 3>{}, IC<(C1 + H + 1) & 1>{}, rb1[h]);
        lds_barrier();
        relax_second(IC<H & 3>{}, IC<(H + 1) & 3>{}, IC<(H + 3) & 3>{}, IC<(C2 + H) & 1>{}, rb2[h]);
        lds_barrier();
        deposit(IC<h>{}, IC<(H + 3) & 3>{}, ss + 3, true);
        store_plane(IC<H & 3>{}, ss);
        fetch(IC<h>{}, ss + 5);
        fetch_b(IC<h>{}, ss + 3, IC<(C1 + H + 3) & 1>{}, ss + 2, IC<(C2 + H + 2) & 1>{});
        lds_barrier();
    };
    for (int s = i0; s < i0 + ci; s += 4) {
        step(IC<0>{}, s);
        step(IC<1>{}, s + 1);
        step(IC<2>{}, s + 2);
        step(IC<3>{}, s + 3);
    }
    }
}

// Launch shapes, as measured best inside the solve (and in standalone
// timings of every shape and ring on fixed fields, each bitwise equal to
// the others):
//   FP32: 8 x 128 tiles, 256 threads, 4-plane ring (50 KB of LDS, two
//     workgroups per CU; rows of 512 B, so the k-halo columns cost fewer
//     partly used cache lines than 64-wide rows); from 512^3 the sweep that
//     starts from zero takes the 6-plane ring (76 KB, still two per CU), and
//     from 1024^3 the others take 16 x 128 tiles with 512 threads on the
//     6-plane ring (127 KB, one per CU; half the j-halo rows per node);
//   FP64: 16 x 64 tiles, 512 threads (one per CU), 4-plane ring below 512^3,
//     6-plane ring from 512^3 (131 KB).
// These launches keep at least 512 workgroups, each streaming the longest
// i-chunk that allows (every chunk re-reads four planes), and store their
// planes nontemporally.  Levels below 256^3 (L2-resident) take narrow tiles
// with short chunks instead: 8 x 32 tiles of 256 threads with 8-plane chunks
// from 128^3 and 4-plane chunks at 64^3, 8 x 16 tiles of 128 threads below.
// FOLD = 0: a shape only the zero-start sweep uses, built without the
// folded coarse correction.  CI > 0 fixes the i-chunk length (the small
// levels, where a launch costs more than its bytes and short chunks keep
// every CU busy); CI = 0 takes the longest chunk that keeps MIN_BLOCKS
// workgroups.
template <typename T, int TJ_, int TK_, int NT_, int MINW_, int SLOTS_, int FOLD_ = 1, int CI_ = 0>
struct FusedShape {
    static constexpr int TJ = TJ_, TK = TK_, NT = NT_, MINW = MINW_, SLOTS = SLOTS_, MIN_BLOCKS = 512;
    static constexpr bool FOLD = FOLD_;
    static constexpr int CI = CI_;
    static constexpr int NTS = CI_ == 0;  // the streaming shapes store nontemporally
};

template <typename C, typename T>
hipError_t launch_fused_shape(const T *u_in, T *u_out, const T *a, const T *b, int n, T inv, T a_min, int first,
                              bool zero_init, hipStream_t s, const T *e = nullptr)
{
    if (e && (zero_init || n % 2)) return hipErrorInvalidValue;
    if (n < C::TK || n % C::TK || n % C::TJ) return hipErrorInvalidValue;
    int ci = C::CI ? C::CI : n;
    if (!C::CI)
        while (ci > 16 && (n / C::TK) * (n / C::TJ) * (n / ci) < C::MIN_BLOCKS) ci /= 2;
    if (n % ci || (C::SLOTS == 4 && ci % 4)) return hipErrorInvalidValue;  // the 4-slot loop takes planes in fours
    const int nblk = (n / C::TK) * (n / C::TJ) * (n / ci);
#define RECON_FUSED(Z, F1)                                                                                \
    k_rbgs_fused<T, C::TJ, Z, F1, C::TK, C::NT, C::MINW, C::SLOTS, 0, C::NTS><<<nblk, C::NT, 0, s>>>(         \
        u_in, u_out, a, b, n, ci, inv, a_min, nullptr)
#define RECON_FUSED_PRO(F1)                                                                                   \
    k_rbgs_fused<T, C::TJ, 0, F1, C::TK, C::NT, C::MINW, C::SLOTS, 1, C::NTS><<<nblk, C::NT, 0, s>>>(         \
        u_in, u_out, a, b, n, ci, inv, a_min, e)
    if (e) {
        if constexpr (C::FOLD) {
            if (first) RECON_FUSED_PRO(1);
            else RECON_FUSED_PRO(0);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (zero_init) {
        if (first) RECON_FUSED(1, 1);
        else RECON_FUSED(1, 0);
    } else {
        if (first) RECON_FUSED(0, 1);
        else RECON_FUSED(0, 0);
    }
#undef RECON_FUSED
#undef RECON_FUSED_PRO
    return hipGetLastError();
}

// The shapes of levels from 256^3 whose edge they divide.
template <typename T>
bool fused_large(int n)
{
    const int tk = sizeof(T) == 4 ? 128 : 64, tj = sizeof(T) == 4 ? (n >= 1024 ? 16 : 8) : 16;
    return n >= 256 && n % tk == 0 && n % tj == 0;
}

// Every shape divides the edges it is used for: the large ones above, the
// small ones (8 x 32 and 8 x 16 tiles, 8- and 4-plane chunks) edges that are
// multiples of 16.
template <typename T>
bool rbgs_fused_supported(int n)
{
    return fused_large<T>(n) || (n >= 16 && n % 16 == 0);
}

template <typename T>
hipError_t launch_rbgs_fused(const T *u_in, T *u_out, const T *a, const T *b, int n, T scale, T a_min, int first,
                             bool zero_init, hipStream_t s, const T *e)
{
    if (!rbgs_fused_supported<T>(n)) return hipErrorInvalidValue;
    const T inv = (T)1 / scale;
    if (!fused_large<T>(n)) {
        // levels below 256^3 (L2-resident): narrow tiles and 4- or 8-plane
        // chunks, so that even 16^3 spreads over several workgroups
        if (n % 32 == 0 && n >= 64) {
            if (n >= 128)
                return launch_fused_shape<FusedShape<T, 8, 32, 256, 2, 4, 1, 8>>(u_in, u_out, a, b, n, inv, a_min,
                                                                                first, zero_init, s, e);
            return launch_fused_shape<FusedShape<T, 8, 32, 256, 2, 4, 1, 4>>(u_in, u_out, a, b, n, inv, a_min, first,
                                                                            zero_init, s, e);
        }
        return launch_fused_shape<FusedShape<T, 8, 16, 128, 2, 4, 1, 4>>(u_in, u_out, a, b, n, inv, a_min, first,
                                                                        zero_init, s, e);
    }
    if constexpr (sizeof(T) == 4) {
        if (n >= 1024 && !zero_init)
            return launch_fused_shape<FusedShape<T, 16, 128, 512, 1, 6>>(u_in, u_out, a, b, n, inv, a_min, first,
                                                                        zero_init, s, e);
        if (n >= 512 && n < 1024 && zero_init)
            return launch_fused_shape<FusedShape<T, 8, 128, 256, 2, 6, 0>>(u_in, u_out, a, b, n, inv, a_min, first,
                                                                          zero_init, s);
        return launch_fused_shape<FusedShape<T, 8, 128, 256, 2, 4>>(u_in, u_out, a, b, n, inv, a_min, first,
                                                                   zero_init, s, e);
    } else {
        if (n >= 512)
            return launch_fused_shape<FusedShape<T, 16, 64, 512, 2, 6>>(u_in, u_out, a, b, n, inv, a_min, first,
                                                                       zero_init, s, e);
        return launch_fused_shape<FusedShape<T, 16, 64, 512, 2, 4>>(u_in, u_out, a, b, n, inv, a_min, first,
                                                                   zero_init, s, e);
    }
}

template hipError_t launch_rbgs_fused<float>(const float *, float *, const float *, const float *, int, float,
                                              float, int, bool, hipStream_t, const float *);
template hipError_t launch_rbgs_fused<double>(const double *, double *, const double *, const double *, int, double,
                                               double, int, bool, hipStream_t, const double *);
template bool rbgs_fused_supported<float>(int);
template bool rbgs_fused_supported<double>(int);

}  // namespace recon
