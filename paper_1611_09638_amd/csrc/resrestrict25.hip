// The V-cycle's coarse right-hand side in one streaming pass (App. A: the
// residual of the fine level, restricted by 27-point full weighting):
// c = R (b - scale A u), without writing the fine residual to HBM and reading
// it back.
//
// A workgroup owns a CJ x CK tile of coarse (J, K) and a chunk of ci coarse
// planes.  Fine planes of u and a stream through a 4-slot LDS ring as blocks
// with a 2-cell halo around the fine rows 2 J0 - 1 .. 2 (J0 + CJ) - 1 and
// columns 2 K0 - 1 .. 2 (K0 + CK) - 1; b comes straight into registers at
// the residual nodes, two planes ahead.  For each fine plane q the residual
// of that (2 CJ + 1) x (2 CK + 1) block goes into an LDS slot, and each
// thread adds the weighted in-plane sum at its coarse nodes into the coarse
// plane q belongs to.  The residual (face order +i, -i, +j, -j, +k, -k, a
// stored halved) and the restriction (weights 1/4, 1/2, 1/4, k innermost,
// then j, then i) are formed exactly as the separate streaming kernels form
// them, so the result is the same.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

namespace {

// LDS-only barrier.  In FP64 a scheduling barrier follows it: without one
// the compiler moves the halving of staged a values across it, so that a
// wave waits for loads issued just before the barrier (4% slower at 512^3).
// The FP32 kernel measured 5% faster without it.
template <typename T>
__device__ __forceinline__ void lds_fence_barrier_rr()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    if constexpr (sizeof(T) == 8) __builtin_amdgcn_sched_barrier(0);
}

template <int CJ, int CK, int NT>
struct ResRestrictTile {
    static constexpr int FH = 2 * CJ + 1, FW = 2 * CK + 1, RPLANE = FH * FW;  // residual block
    static constexpr int UW = FW + 2, UPLANE = (FH + 2) * UW;                 // u and a block
    static constexpr int LU = (UPLANE + NT - 1) / NT;
    static constexpr int RR = (RPLANE + NT - 1) / NT;
    static constexpr int RS = CJ * CK / NT;
};

template <typename T, int CJ, int CK, int NT>
__global__ void __launch_bounds__(NT) k_resrestrict25(const T *__restrict__ ug, const T *__restrict__ ag,
                                                     const T *__restrict__ bg, T *__restrict__ c, int n, int ci,
                                                     T scale, T a_min)
{
    using F = ResRestrictTile<CJ, CK, NT>;
    static_assert(CJ * CK % NT == 0, "every thread owns whole rounds of the coarse tile");
    constexpr int FW = F::FW, UW = F::UW, UPLANE = F::UPLANE, RPLANE = F::RPLANE;
    constexpr int LU = F::LU, RR = F::RR, RS = F::RS;
    __shared__ T sU[4][UPLANE + 1];  // + one spare word for lanes past the block
    __shared__ T sA[4][UPLANE + 1];
    __shared__ T sR[2][RPLANE + 1];

    const int nc = n >> 1;
    const int tid = threadIdx.x;
    const int tiles_k = nc / CK, tiles_j = nc / CJ, chunks = nc / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int J0 = tj * CJ, K0 = tk * CK, I0 = ch * ci;
    const size_t n2 = (size_t)n * n;

    // u and a load slots: in-plane offset and LDS destination
    int offL[LU], dstL[LU];
#pragma unroll
    for (int r = 0; r < LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / UW, col = q % UW;
        offL[r] = q < UPLANE ? wrapc(2 * J0 - 2 + row, n) * n + wrapc(2 * K0 - 2 + col, n) : 0;
        dstL[r] = q < UPLANE ? q : UPLANE;
    }
    // residual nodes: LDS position in the u/a block and in the residual block,
    // and the in-plane offset of b (lanes past the block take node 0 and
    // write the spare word)
    int oU[RR], oR[RR], gB[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int m = tid + r * NT;
        const bool on = m < RPLANE;
        const int mm = on ? m : 0;
        const int row = mm / FW, col = mm % FW;
        oU[r] = (row + 1) * UW + (col + 1);
        oR[r] = on ? m : RPLANE;
        gB[r] = wrapc(2 * J0 - 1 + row, n) * n + wrapc(2 * K0 - 1 + col, n);
    }
    // this thread's coarse nodes: position of their (2J-1, 2K-1) corner in the
    // residual block, and their in-plane offset on the coarse grid
    int oN[RS];
    size_t gN[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int q = tid + r * NT;
        const int jj = q / CK, kk = q % CK;
        oN[r] = 2 * jj * FW + 2 * kk;
        gN[r] = (size_t)(J0 + jj) * nc + (K0 + kk);
    }

    const int q0 = 2 * I0 - 1;  // first fine plane of the chunk
    auto slot = [&](int p) { return (p - q0 + 1) & 3; };

    T ru[2][LU], ra[2][LU], rb[2][RR];
    auto fetch_ua = [&](int set, int p) {
        const size_t base = (size_t)wrapc(p, n) * n2;
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            ru[set][r] = ug[base + offL[r]];
            ra[set][r] = ag[base + offL[r]];
        }
    };
    auto fetch_b = [&](int set, int p) {
        const size_t base = (size_t)wrapc(p, n) * n2;
#pragma unroll
        for (int r = 0; r < RR; ++r) rb[set][r] = bg[base + gB[r]];
    };
    auto deposit = [&](int set, int p) {
        T *U = sU[slot(p)], *A = sA[slot(p)];
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            U[dstL[r]] = ru[set][r];
            A[dstL[r]] = (T)0.5 * ra[set][r];
        }
    };
    // residual of plane p (b in rb[set]) into sR[rs]; planes p - 1, p, p + 1 resident
    auto residual = [&](int p, int set, int rs) {
        const T *Uc = sU[slot(p)], *Ac = sA[slot(p)];
        const T *Uu = sU[slot(p + 1)], *Au = sA[slot(p + 1)];
        const T *Ud = sU[slot(p - 1)], *Ad = sA[slot(p - 1)];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int o = oU[r];
            const T xc = Uc[o], hc = Ac[o];
            T acc = 0;
            acc += fmax(hc + Au[o], a_min) * (Uu[o] - xc);
            acc += fmax(hc + Ad[o], a_min) * (Ud[o] - xc);
            acc += fmax(hc + Ac[o + UW], a_min) * (Uc[o + UW] - xc);
            acc += fmax(hc + Ac[o - UW], a_min) * (Uc[o - UW] - xc);
            acc += fmax(hc + Ac[o + 1], a_min) * (Uc[o + 1] - xc);
            acc += fmax(hc + Ac[o - 1], a_min) * (Uc[o - 1] - xc);
            sR[rs][oR[r]] = rb[set][r] - scale * acc;
        }
    };
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    // in-plane 9-point weighted sum of residual slot rs at coarse node r
    auto inplane = [&](int rs, int r) {
        const T *P = sR[rs] + oN[r];
        T pa = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T *row = P + b * FW;
            const T pb = w[0] * row[0] + w[1] * row[1] + w[2] * row[2];
            pa += w[b] * pb;
        }
        return pa;
    };
    // one fine plane: its residual, the ring advanced by one plane, then (after
    // the barrier) its contribution to the coarse sums.  Plane q + 2 goes into
    // the slot of plane q - 2, last read by the previous plane's residual.
    auto advance = [&](int q, int h) {
        residual(q, h, h);
        deposit(h, q + 2);
        fetch_ua(h, q + 4);
        fetch_b(h, q + 2);
        lds_fence_barrier_rr<T>();
    };

    // prologue: planes q0 - 1 .. q0 + 1 resident, u and a of q0 + 2 and
    // q0 + 3 and b of q0 and q0 + 1 staged
    fetch_ua(0, q0 - 1);
    deposit(0, q0 - 1);
    fetch_ua(0, q0);
    deposit(0, q0);
    fetch_ua(0, q0 + 1);
    deposit(0, q0 + 1);
    fetch_ua(0, q0 + 2);
    fetch_b(0, q0);
    fetch_ua(1, q0 + 3);
    fetch_b(1, q0 + 1);
    lds_fence_barrier_rr<T>();

    T acc[RS];
    // plane 2 I0 - 1 opens coarse plane I0 (weight 1/4)
    advance(q0, 0);
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        acc[r] = 0;
        acc[r] += w[0] * inplane(0, r);
    }
    // coarse plane I: fine plane 2I (weight 1/2), then 2I + 1, which closes I
    // (1/4) and opens I + 1 (1/4).  The last step stages planes past the chunk:
    // they wrap to valid addresses and land in slots that are no longer read.
    for (int I = I0; I < I0 + ci; ++I) {
        const int q = 2 * I;
        advance(q, 1);
#pragma unroll
        for (int r = 0; r < RS; ++r) acc[r] += w[1] * inplane(1, r);
        advance(q + 1, 0);
        T *out = c + (size_t)I * nc * nc;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            const T pa = inplane(0, r);
            T a2 = acc[r];
            a2 += w[2] * pa;
            out[gN[r]] = a2;
            acc[r] = 0;
            acc[r] += w[0] * pa;
        }
    }
}

// Coarse tile, threads and smallest launch per precision (the coarse chunk
// is halved until the launch has that many workgroups), as measured at 256^3
// and 512^3: 4 x 32 coarse tiles (9 x 65 fine residuals, 11 x 67 u and a)
// with 128 threads; 1024 workgroups in FP32, 512 in FP64, whose longer chunks
// re-read fewer halo planes (3% faster there).
template <typename T>
struct ResRestrictLaunch {
    static constexpr int CJ = 4, CK = 32, NT = 128, MIN_BLOCKS = sizeof(T) == 8 ? 512 : 1024;
};

}  // namespace

template <typename T>
bool resrestrict25_supported(int n)
{
    using C = ResRestrictLaunch<T>;
    const int nc = n / 2;
    return n % 2 == 0 && nc >= C::CK && nc % C::CK == 0 && nc % C::CJ == 0;
}

template <typename T>
hipError_t launch_resrestrict25(const T *u, const T *a, const T *b, T *c, int n, T scale, T a_min, hipStream_t s)
{
    using C = ResRestrictLaunch<T>;
    if (!resrestrict25_supported<T>(n)) return hipErrorInvalidValue;
    const int nc = n / 2;
    int ci = nc;
    while (ci > 1 && (nc / C::CK) * (nc / C::CJ) * (nc / ci) < C::MIN_BLOCKS) ci /= 2;
    const int nb = (nc / C::CK) * (nc / C::CJ) * (nc / ci);
    k_resrestrict25<T, C::CJ, C::CK, C::NT><<<nb, C::NT, 0, s>>>(u, a, b, c, n, ci, scale, a_min);
    return hipGetLastError();
}

template bool resrestrict25_supported<float>(int);
template bool resrestrict25_supported<double>(int);
template hipError_t launch_resrestrict25<float>(const float *, const float *, const float *, float *, int, float, float,
                                                hipStream_t);
template hipError_t launch_resrestrict25<double>(const double *, const double *, const double *, double *, int,
                                                 double, double, hipStream_t);

}  // namespace recon
