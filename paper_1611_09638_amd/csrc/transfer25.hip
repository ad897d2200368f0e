// Streaming grid transfers of the multigrid V-cycle (App. A): 27-point full
// weighting R onto the coarse grid and u += P e with trilinear P = 8 R^T.
//
// Both walk i-planes through LDS so that every fine value is read from HBM
// once (plus halo lines) and every fine node of u is read and written once;
// the per-node gather kernels they replace issue 27 (restriction) or up to 8
// (prolongation) global loads per node.  The arithmetic and its order are the
// gather kernels' (weights 1/4, 1/2, 1/4 per axis, k innermost, then j, then
// i), so both produce the same values.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

namespace {

__device__ __forceinline__ void lds_fence_barrier25()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- restriction
//
// A workgroup owns a CJ x CK tile of coarse (J, K) and a chunk of CI coarse
// planes.  Fine plane q (from 2 I0 - 1 to 2 (I0 + CI) - 1) enters an LDS slot
// as the (2 CJ + 1) x (2 CK + 1) block of fine rows 2 J0 - 1 .. and columns
// 2 K0 - 1 ..; each thread forms, for its coarse node, the in-plane weighted
// sum pa(q) and adds w(a) pa(q) into the coarse plane that q belongs to
// (q = 2I - 1, 2I, 2I + 1 for a = 0, 1, 2).
template <int CJ, int CK, int NT>
struct RestrictTile {
    static constexpr int FH = 2 * CJ + 1, FW = 2 * CK + 1, PLANE = FH * FW;
    static constexpr int LU = (PLANE + NT - 1) / NT;
    static constexpr int PU = PLANE + 1;  // + one spare word for lanes past the plane
    static constexpr int RS = CJ * CK / NT;
};

template <typename T, int CJ, int CK, int NT>
__global__ void __launch_bounds__(NT) k_restrict25(const T *__restrict__ f, T *__restrict__ c, int n, int ci)
{
    using F = RestrictTile<CJ, CK, NT>;
    static_assert(CJ * CK % NT == 0, "every thread owns whole rounds of the coarse tile");
    constexpr int FW = F::FW, PLANE = F::PLANE, LU = F::LU, RS = F::RS;
    __shared__ T sF[2][F::PU];

    const int nc = n >> 1;
    const int tid = threadIdx.x;
    const int tiles_k = nc / CK, tiles_j = nc / CJ, chunks = nc / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int J0 = tj * CJ, K0 = tk * CK, I0 = ch * ci;
    const size_t n2 = (size_t)n * n;

    int offL[LU], dstL[LU];
#pragma unroll
    for (int r = 0; r < LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / FW, col = q % FW;
        offL[r] = q < PLANE ? wrapc(2 * J0 - 1 + row, n) * n + wrapc(2 * K0 - 1 + col, n) : 0;
        dstL[r] = q < PLANE ? q : PLANE;
    }
    // this thread's coarse nodes: LDS position of their (2J-1, 2K-1) corner
    int oN[RS];
    size_t gN[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int q = tid + r * NT;
        const int jj = q / CK, kk = q % CK;
        oN[r] = 2 * jj * FW + 2 * kk;
        gN[r] = (size_t)(J0 + jj) * nc + (K0 + kk);
    }

    T rf[2][LU];
    auto fetch = [&](int set, int q) {
        const T *pl = f + (size_t)wrapc(q, n) * n2;
#pragma unroll
        for (int r = 0; r < LU; ++r) rf[set][r] = pl[offL[r]];
    };
    auto deposit = [&](int set, int slot) {
#pragma unroll
        for (int r = 0; r < LU; ++r) sF[slot][dstL[r]] = rf[set][r];
    };
    const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
    // in-plane 9-point weighted sum at this thread's coarse node r
    auto inplane = [&](int slot, int r) {
        const T *P = sF[slot] + oN[r];
        T pa = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T *row = P + b * FW;
            const T pb = w[0] * row[0] + w[1] * row[1] + w[2] * row[2];
            pa += w[b] * pb;
        }
        return pa;
    };

    T acc[RS];
    // Fine planes q0 + s (q0 = 2 I0 - 1, s = 0 .. 2 ci) alternate between
    // slot 0 (s even) and slot 1 (s odd); register set 0 stages the next even
    // plane, set 1 the next odd one.
    const int q0 = 2 * I0 - 1;
    fetch(0, q0);
    deposit(0, 0);
    fetch(0, q0 + 1);
    deposit(0, 1);
    fetch(0, q0 + 2);
    fetch(1, q0 + 3);
    lds_fence_barrier25();
    // plane 2 I0 - 1 opens coarse plane I0 (a = 0)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        acc[r] = 0;
        acc[r] += w[0] * inplane(0, r);
    }
    lds_fence_barrier25();
    // Coarse plane I: plane 2I (slot 1, a = 1), then plane 2I + 1 (slot 0),
    // which closes I (a = 2) and opens I + 1 (a = 0).
    for (int I = I0; I < I0 + ci; ++I) {
        const int s = 2 * (I - I0) + 1;
#pragma unroll
        for (int r = 0; r < RS; ++r) acc[r] += w[1] * inplane(1, r);
        deposit(0, 0);  // plane s + 1 into slot 0, last read before the previous barrier
        fetch(0, q0 + s + 3);
        lds_fence_barrier25();
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
        lds_fence_barrier25();
        deposit(1, 1);  // plane s + 2 into slot 1, read at the top of this iteration
        fetch(1, q0 + s + 4);
        lds_fence_barrier25();
    }
}

// -------------------------------------------------------------- prolongation
//
// A workgroup owns an FJ x FK tile of fine (j, k) and a chunk of ci fine
// planes (ci even, starting on an even plane).  Coarse planes enter a 2-slot
// LDS ring as (FJ/2 + 1) x (FK/2 + 1) blocks; fine plane 2c uses coarse plane
// c, fine plane 2c + 1 uses c and c + 1.
template <int FJ, int FK, int NT>
struct ProlongTile {
    static constexpr int CH = FJ / 2 + 1, CW = FK / 2 + 1, PLANE = CH * CW;
    static constexpr int LU = (PLANE + NT - 1) / NT;
    static constexpr int PU = PLANE + 1;
    static constexpr int RS = FJ * FK / NT;
};

template <typename T, int FJ, int FK, int NT>
__global__ void __launch_bounds__(NT) k_prolong25(T *__restrict__ u, const T *__restrict__ e, int n, int ci)
{
    using F = ProlongTile<FJ, FK, NT>;
    static_assert(FJ * FK % NT == 0 && FJ % 2 == 0 && FK % 2 == 0, "whole rounds of even tiles");
    constexpr int CW = F::CW, PLANE = F::PLANE, LU = F::LU, RS = F::RS;
    __shared__ T sE[2][F::PU];

    const int nc = n >> 1;
    const int tid = threadIdx.x;
    const int tiles_k = n / FK, tiles_j = n / FJ, chunks = n / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int j0 = tj * FJ, k0 = tk * FK, i0 = ch * ci;
    const int cj0 = j0 >> 1, ck0 = k0 >> 1, c0 = i0 >> 1;
    const size_t n2 = (size_t)n * n, nc2 = (size_t)nc * nc;

    int offL[LU], dstL[LU];
#pragma unroll
    for (int r = 0; r < LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / CW, col = q % CW;
        offL[r] = q < PLANE ? wrapc(cj0 + row, nc) * nc + wrapc(ck0 + col, nc) : 0;
        dstL[r] = q < PLANE ? q : PLANE;
    }
    // this thread's fine nodes: the LDS positions of the coarse corners
    // (j0c, k0c), (j0c, k1c), (j1c, k0c), (j1c, k1c), the parities and the
    // in-plane fine offset
    int a00[RS], a01[RS], a10[RS], a11[RS], kod[RS], jod[RS];
    size_t gN[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int q = tid + r * NT;
        const int jj = q / FK, kk = q % FK;
        const int jc = jj >> 1, kc = kk >> 1;
        const int jc1 = (jj & 1) ? jc + 1 : jc, kc1 = (kk & 1) ? kc + 1 : kc;
        a00[r] = jc * CW + kc;
        a01[r] = jc * CW + kc1;
        a10[r] = jc1 * CW + kc;
        a11[r] = jc1 * CW + kc1;
        kod[r] = kk & 1;
        jod[r] = jj & 1;
        gN[r] = (size_t)(j0 + jj) * n + (k0 + kk);
    }

    T re[2][LU];
    auto fetch = [&](int set, int cp) {
        const T *pl = e + (size_t)wrapc(cp, nc) * nc2;
#pragma unroll
        for (int r = 0; r < LU; ++r) re[set][r] = pl[offL[r]];
    };
    auto deposit = [&](int set, int slot) {
#pragma unroll
        for (int r = 0; r < LU; ++r) sE[slot][dstL[r]] = re[set][r];
    };
    const T wk = (T)0.5, wj = (T)0.5, wi = (T)0.5;
    // the in-plane interpolation of coarse slot `slot` at fine node r
    auto inplane = [&](int slot, int r) {
        const T *E = sE[slot];
        const T v00 = E[a00[r]], v01 = E[a01[r]], v10 = E[a10[r]], v11 = E[a11[r]];
        const T r0 = kod[r] ? wk * (v00 + v01) : v00;
        const T r1 = kod[r] ? wk * (v10 + v11) : v10;
        return jod[r] ? wj * (r0 + r1) : r0;
    };
    // u at this thread's nodes, staged one plane pair ahead
    T ru[2][RS];
    auto fetch_u = [&](int set, int i) {
        const T *pl = u + (size_t)i * n2;
#pragma unroll
        for (int r = 0; r < RS; ++r) ru[set][r] = pl[gN[r]];
    };

    // coarse planes c0 + m in slot m & 1; staged two coarse planes ahead
    fetch(0, c0);
    deposit(0, 0);
    fetch(0, c0 + 1);
    deposit(0, 1);
    fetch(0, c0 + 2);
    fetch(1, c0 + 3);
    fetch_u(0, i0);
    fetch_u(1, i0 + 1);
    lds_fence_barrier25();
    for (int m = 0; m < ci / 2; ++m) {
        const int i = i0 + 2 * m, sc = m & 1;
        // fine plane i = 2c: coarse plane c only
        T *pe = u + (size_t)i * n2;
#pragma unroll
        for (int r = 0; r < RS; ++r) pe[gN[r]] = ru[0][r] + inplane(sc, r);
        fetch_u(0, wrapc(i + 2, n));  // past the last plane: a valid plane, not used
        // fine plane i + 1: coarse planes c and c + 1
        T *po = u + (size_t)(i + 1) * n2;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            T acc = inplane(sc, r);
            const T acc1 = inplane(sc ^ 1, r);
            acc = wi * (acc + acc1);
            po[gN[r]] = ru[1][r] + acc;
        }
        fetch_u(1, wrapc(i + 3, n));
        lds_fence_barrier25();
        deposit(m & 1, sc);  // coarse plane c + 2 into the slot of plane c
        fetch(m & 1, c0 + m + 4);
        lds_fence_barrier25();
    }
}

template <typename T>
struct TransferLaunch {
    // restriction: coarse tile CJ x CK; prolongation: fine tile FJ x FK
    static constexpr int CJ = 4, CK = 64, FJ = 4, FK = 256, NT = 256, MIN_BLOCKS = 2048;
};

}  // namespace

template <typename T>
bool transfer25_supported(int n)
{
    using C = TransferLaunch<T>;
    const int nc = n / 2;
    return n % 2 == 0 && nc >= C::CK && nc % C::CK == 0 && nc % C::CJ == 0 && n >= C::FK && n % C::FK == 0 &&
           n % C::FJ == 0;
}

template <typename T>
hipError_t launch_restrict25(const T *f, T *c, int n, hipStream_t s)
{
    using C = TransferLaunch<T>;
    if (!transfer25_supported<T>(n)) return hipErrorInvalidValue;
    const int nc = n / 2;
    int ci = nc;
    while (ci > 1 && (nc / C::CK) * (nc / C::CJ) * (nc / ci) < C::MIN_BLOCKS) ci /= 2;
    const int nb = (nc / C::CK) * (nc / C::CJ) * (nc / ci);
    k_restrict25<T, C::CJ, C::CK, C::NT><<<nb, C::NT, 0, s>>>(f, c, n, ci);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong25(T *u, const T *e, int n, hipStream_t s)
{
    using C = TransferLaunch<T>;
    if (!transfer25_supported<T>(n)) return hipErrorInvalidValue;
    int ci = n;
    while (ci > 2 && (n / C::FK) * (n / C::FJ) * (n / ci) < C::MIN_BLOCKS) ci /= 2;
    const int nb = (n / C::FK) * (n / C::FJ) * (n / ci);
    k_prolong25<T, C::FJ, C::FK, C::NT><<<nb, C::NT, 0, s>>>(u, e, n, ci);
    return hipGetLastError();
}

template bool transfer25_supported<float>(int);
template bool transfer25_supported<double>(int);
template hipError_t launch_restrict25<float>(const float *, float *, int, hipStream_t);
template hipError_t launch_restrict25<double>(const double *, double *, int, hipStream_t);
template hipError_t launch_prolong25<float>(float *, const float *, int, hipStream_t);
template hipError_t launch_prolong25<double>(double *, const double *, int, hipStream_t);

}  // namespace recon
