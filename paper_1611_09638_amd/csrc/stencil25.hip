// Streaming applications of the flux-form operator A u = div(a grad u)
// (App. A, Eq. elliptic with x ~ xi): the residual inside the V-cycle, the
// FP64 residual of the Krylov loop, and the Krylov direction update fused
// with its operator product.
//
// A workgroup owns a TJ x TK tile of (j, k) and a chunk of consecutive
// i-planes.  Each plane of the operand and of the coefficient enters an LDS
// slot with a 1-cell halo in j and k (two slots: the plane being computed
// and the next one), staged two planes ahead in registers; the value one
// plane below each node is kept in registers from the previous plane.  So
// every field is read from HBM once per launch, plus the halo lines, and
// the six neighbours come from LDS instead of from 14 global loads per node.
//
// Face order +i, -i, +j, -j, +k, -k and the face coefficient
// max(a_min, (a_n + a_nb) / 2) = max(a_min, a_n/2 + a_nb/2) (a is stored
// halved; halving is exact) match the per-node kernels, so both round alike.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

namespace {

enum { S25_RESID = 0, S25_RESNORM = 1, S25_DIRECTION = 2 };

template <int TJ, int NT, int TK_ = 64>
struct S25 {
    static constexpr int TK = TK_, H = TJ + 2, W = TK + 2, PLANE = H * W;
    static constexpr int LU = (PLANE + NT - 1) / NT;
    // slots padded to whole rounds of NT loads: every thread loads and
    // deposits unconditionally (spare lanes load a valid address and write
    // into the padding), which keeps the load queue countable
    static constexpr int PU = LU * NT;
    static constexpr int RS = TJ * TK / NT;  // nodes per thread per plane
};

// LDS-only barrier.  The scheduling barrier keeps the compiler from moving
// arithmetic on staged registers across it: that would make a wave wait for
// loads issued just before the barrier instead of two planes earlier.
__device__ __forceinline__ void lds_fence_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    __builtin_amdgcn_sched_barrier(0);
}

// MODE S25_RESID:     out = b - scale A x                    (x = xin, type T)
// MODE S25_RESNORM:   out = b - A x, out32 = (float) out, sum out^2   (T = double)
// MODE S25_DIRECTION: x = first ? z : z + beta xin (written to pout),
//                     out = A x, sum x out                   (T = double, z of type Z)
// The Krylov modes store their outputs nontemporally (nothing reads them
// back before they have left the caches; 512^3 solves 0.7-1% faster).
// FIRST (direction only): the first Krylov step, p = z, p_old not read.
// UPD (direction only, not FIRST): also ug += alpha_u xin, the solution update
// of the previous Krylov step, deferred to this pass, which reads p_old anyway.
// P (direction only): storage type of p_old and p_new.  With P = float the new
// direction is rounded to FP32 as it is formed, so the stored p_new is exactly
// the operand of A and of the later solution update.
template <typename T, typename Z, int MODE, int TJ, int NT, int TK = 64, int FIRST = 0, int UPD = 0,
          typename P = T>
__global__ void __launch_bounds__(NT)
    k_flux25(const P *__restrict__ xin, const Z *__restrict__ zg, const T *__restrict__ ag,
             const T *__restrict__ bg, T *__restrict__ out, float *__restrict__ out32, P *__restrict__ pout, int n,
             int ci, T scale, T a_min, T beta, double *part, double *__restrict__ ug, double alpha_u,
             const double *__restrict__ ks)
{
    if constexpr (MODE == S25_DIRECTION && !FIRST) {
        // the step sizes of the conjugate-gradient loop, formed on the device
        if (ks) {
            beta = -ks[KS_ALPHA] * ks[KS_ZQ] / ks[KS_RZ_OLD];
            alpha_u = ks[KS_ALPHA];
        }
    }
    static_assert(!UPD || (MODE == S25_DIRECTION && !FIRST), "the deferred update needs p_old");
    static_assert(MODE == S25_DIRECTION || sizeof(P) == sizeof(T), "P differs from T only for directions");
    using F = S25<TJ, NT, TK>;
    static_assert(TJ * F::TK % NT == 0, "every thread owns whole rounds of the tile");
    constexpr int W = F::W, PLANE = F::PLANE, LU = F::LU, RS = F::RS;
    constexpr bool HAS_B = MODE != S25_DIRECTION;
    __shared__ T sX[2][F::PU];
    __shared__ T sA[2][F::PU];

    const int tid = threadIdx.x;
    const int tiles_k = n / F::TK, tiles_j = n / TJ, chunks = n / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int j0 = tj * TJ, k0 = tk * F::TK, i0 = ch * ci;
    const size_t n2 = (size_t)n * n;

    // in-plane offsets of this thread's halo load slots
    int offL[LU];
#pragma unroll
    for (int r = 0; r < LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / W, col = q % W;
        const int gj = wrapc(j0 - 1 + row, n), gk = wrapc(k0 - 1 + col, n);
        offL[r] = q < PLANE ? gj * n + gk : 0;
    }
    // this thread's nodes: LDS offset and in-plane global offset
    int oN[RS], gN[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int q = tid + r * NT;
        const int row = q / F::TK, col = q % F::TK;
        oN[r] = (row + 1) * W + (col + 1);
        gN[r] = (j0 + row) * n + (k0 + col);
    }

    // the operand from its loaded parts: x itself, or the direction
    // z + beta p_old (z alone on the first step)
    auto combine = [&](Z zv, P xv) -> T {
        if constexpr (MODE == S25_DIRECTION) {
            T x;
            if constexpr (FIRST)
                x = (T)zv;
            else
                x = (T)zv + beta * (T)xv;
            if constexpr (sizeof(P) < sizeof(T)) x = (T)(P)x;
            return x;
        } else {
            return xv;
        }
    };
    constexpr bool HAS_Z = MODE == S25_DIRECTION, HAS_X = !(MODE == S25_DIRECTION && FIRST);
    auto operand = [&](size_t g) -> T { return combine(HAS_Z ? zg[g] : Z(0), HAS_X ? xin[g] : P(0)); };

    // register stage, as loaded: halo plane p of x (or of z and p_old) and a,
    // and b (or u and p_old) at this thread's nodes of plane p - 2.  The
    // operand is formed when the plane is deposited, so a wave waits for
    // these loads only there, two planes after issuing them.
    Z rz[2][HAS_Z ? LU : 1];
    P rx[2][HAS_X ? LU : 1], rq[2][UPD ? RS : 1];
    T ra[2][LU], rb[2][HAS_B ? RS : 1];
    double ru[2][UPD ? RS : 1];
    auto fetch = [&](int set, int p) {
        const size_t base = (size_t)wrapc(p, n) * n2;
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            if constexpr (HAS_Z) rz[set][r] = zg[base + offL[r]];
            if constexpr (HAS_X) rx[set][r] = xin[base + offL[r]];
            ra[set][r] = ag[base + offL[r]];
        }
        if constexpr (HAS_B) {
            const size_t bb = (size_t)wrapc(p - 2, n) * n2;
#pragma unroll
            for (int r = 0; r < RS; ++r) rb[set][r] = bg[bb + gN[r]];
        }
        if constexpr (UPD) {
            const size_t bb = (size_t)wrapc(p - 2, n) * n2;
#pragma unroll
            for (int r = 0; r < RS; ++r) {
                ru[set][r] = ug[bb + gN[r]];
                rq[set][r] = xin[bb + gN[r]];
            }
        }
    };
    auto deposit = [&](int set, int slot) {
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            sX[slot][tid + r * NT] = combine(HAS_Z ? rz[set][r] : Z(0), HAS_X ? rx[set][r] : P(0));
            sA[slot][tid + r * NT] = (T)0.5 * ra[set][r];
        }
    };

    // the plane below the first one, at this thread's nodes
    T xd[RS], hd[RS];
    {
        const size_t base = (size_t)wrapc(i0 - 1, n) * n2;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            xd[r] = operand(base + gN[r]);
            hd[r] = (T)0.5 * ag[base + gN[r]];
        }
    }
    double v = 0.0;

    auto compute = [&](int p, int set) {
        const int sc = (p - i0) & 1, su = sc ^ 1;
        const T *Xc = sX[sc], *Ac = sA[sc], *Xu = sX[su], *Au = sA[su];
        const size_t base = (size_t)p * n2;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            const int c = oN[r];
            const T xc = Xc[c], hc = Ac[c];
            T acc = 0;
            acc += fmax(hc + Au[c], a_min) * (Xu[c] - xc);
            acc += fmax(hc + hd[r], a_min) * (xd[r] - xc);
            acc += fmax(hc + Ac[c + W], a_min) * (Xc[c + W] - xc);
            acc += fmax(hc + Ac[c - W], a_min) * (Xc[c - W] - xc);
            acc += fmax(hc + Ac[c + 1], a_min) * (Xc[c + 1] - xc);
            acc += fmax(hc + Ac[c - 1], a_min) * (Xc[c - 1] - xc);
            const size_t g = base + gN[r];
            if constexpr (MODE == S25_RESID) {
                out[g] = rb[set][r] - scale * acc;
            } else if constexpr (MODE == S25_RESNORM) {
                const T rv = rb[set][r] - acc;
                __builtin_nontemporal_store(rv, &out[g]);
                if (out32) __builtin_nontemporal_store((float)rv, &out32[g]);
                v += rv * rv;
            } else {
                __builtin_nontemporal_store((P)xc, &pout[g]);
                __builtin_nontemporal_store(acc, &out[g]);
                v += xc * acc;
                if constexpr (UPD) __builtin_nontemporal_store(ru[set][r] + alpha_u * (double)rq[set][r], &ug[g]);
            }
            xd[r] = xc;
            hd[r] = hc;
        }
    };

    // prologue: planes i0 and i0+1 resident, i0+2 and i0+3 staged
    fetch(0, i0);
    deposit(0, 0);
    fetch(0, i0 + 1);
    deposit(0, 1);
    fetch(0, i0 + 2);
    fetch(1, i0 + 3);
    lds_fence_barrier();
    // Branch-free steady state (ci is even).  The last two iterations fetch and
    // deposit planes past the chunk: they wrap to valid addresses and land in
    // slots that are no longer read.
    for (int s = i0; s < i0 + ci; s += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = s + h;
            compute(p, h);
            lds_fence_barrier();
            deposit(h, (p - i0) & 1);  // plane p + 2 into the slot of plane p
            lds_fence_barrier();
            fetch(h, p + 4);
        }
    }
    if constexpr (MODE != S25_RESID) {
        double vv[1] = {v};
        block_reduce_store<1, RED_SUM>(vv, part, blockIdx.x);
    }
}

// Launch shape per operation: tile rows TJ, tile width TK (a multiple of 64),
// threads, and the smallest launch (the i-chunk is halved from n until the
// launch has that many workgroups; each chunk reads one extra plane of every
// field).  As measured best at 512^3 (and 256^3 for the residual): 128-wide
// tiles, whose rows span whole cache lines with few partly used halo lines,
// 512 threads, and long i-chunks (two workgroups per CU for the residuals,
// one for the direction pass, which streams more fields).
template <typename T, int MODE>
struct S25Launch;
template <>
struct S25Launch<float, S25_RESID> {
    static constexpr int TJ = 8, TK = 128, NT = 512, MIN_BLOCKS = 512;
};
template <>
struct S25Launch<double, S25_RESID> {
    static constexpr int TJ = 8, TK = 128, NT = 512, MIN_BLOCKS = 512;
};
template <>
struct S25Launch<double, S25_RESNORM> {
    static constexpr int TJ = 8, TK = 128, NT = 512, MIN_BLOCKS = 512;
};
template <>
struct S25Launch<double, S25_DIRECTION> {
    static constexpr int TJ = 16, TK = 128, NT = 512, MIN_BLOCKS = 256;
};

template <typename C>
bool s25_fits(int n)
{
    return n >= C::TK && n % C::TK == 0 && n % C::TJ == 0;
}

template <typename C>
int s25_chunk(int n)
{
    int ci = n;
    while (ci % 4 == 0 && (n / C::TK) * (n / C::TJ) * (n / ci) < C::MIN_BLOCKS) ci /= 2;  // ci stays even
    return ci;
}

template <typename C>
int s25_blocks(int n, int ci)
{
    return (n / C::TK) * (n / C::TJ) * (n / ci);
}

}  // namespace

template <typename T>
bool stencil25_supported(int n)
{
    if constexpr (sizeof(T) == 4)
        return s25_fits<S25Launch<float, S25_RESID>>(n);
    else
        return s25_fits<S25Launch<double, S25_RESID>>(n) && s25_fits<S25Launch<double, S25_RESNORM>>(n) &&
               s25_fits<S25Launch<double, S25_DIRECTION>>(n);
}

template <typename T>
hipError_t launch_residual25(const T *u, const T *a, const T *b, T *r, int n, T scale, T a_min, hipStream_t s)
{
    using C = S25Launch<T, S25_RESID>;
    if (!s25_fits<C>(n)) return hipErrorInvalidValue;
    const int ci = s25_chunk<C>(n), nb = s25_blocks<C>(n, ci);
    k_flux25<T, T, S25_RESID, C::TJ, C::NT, C::TK, 0, 0, T><<<nb, C::NT, 0, s>>>(u, nullptr, a, b, r, nullptr, nullptr, n, ci,
                                                                       scale, a_min, (T)0, nullptr, nullptr, 0.0,
                                                                       nullptr);
    return hipGetLastError();
}

hipError_t launch_residual_norm25(const double *u, const double *a, const double *b, double *r, float *r32, int n,
                                  double a_min, Part &p, hipStream_t s)
{
    using C = S25Launch<double, S25_RESNORM>;
    if (!s25_fits<C>(n)) return hipErrorInvalidValue;
    const int ci = s25_chunk<C>(n), nb = s25_blocks<C>(n, ci);
    if ((long)nb > kPartCap) return hipErrorInvalidValue;
    k_flux25<double, double, S25_RESNORM, C::TJ, C::NT, C::TK, 0, 0, double><<<nb, C::NT, 0, s>>>(
        u, nullptr, a, b, r, r32, nullptr, n, ci, 1.0, a_min, 0.0, p.part, nullptr, 0.0, nullptr);
    p.blocks = nb;
    p.k = 1;
    return hipGetLastError();
}

template <typename Z, typename P>
hipError_t launch_direction25(const Z *z, const P *p_old, P *p_new, const double *a, double *q, double beta, int n,
                              double a_min, bool first, double *u, double alpha_u, const double *ks, Part &p,
                              hipStream_t s)
{
    using C = S25Launch<double, S25_DIRECTION>;
    const void *po = p_old;
    if (!s25_fits<C>(n) || po == p_new || (u && (first || po == u || (void *)p_new == u || u == q)))
        return hipErrorInvalidValue;
    const int ci = s25_chunk<C>(n), nb = s25_blocks<C>(n, ci);
    if ((long)nb > kPartCap) return hipErrorInvalidValue;
    if (first)
        k_flux25<double, Z, S25_DIRECTION, C::TJ, C::NT, C::TK, 1, 0, P><<<nb, C::NT, 0, s>>>(
            p_old, z, a, nullptr, q, nullptr, p_new, n, ci, 1.0, a_min, beta, p.part, nullptr, 0.0, nullptr);
    else if (u)
        k_flux25<double, Z, S25_DIRECTION, C::TJ, C::NT, C::TK, 0, 1, P><<<nb, C::NT, 0, s>>>(
            p_old, z, a, nullptr, q, nullptr, p_new, n, ci, 1.0, a_min, beta, p.part, u, alpha_u, ks);
    else
        k_flux25<double, Z, S25_DIRECTION, C::TJ, C::NT, C::TK, 0, 0, P><<<nb, C::NT, 0, s>>>(
            p_old, z, a, nullptr, q, nullptr, p_new, n, ci, 1.0, a_min, beta, p.part, nullptr, 0.0, ks);
    p.blocks = nb;
    p.k = 1;
    return hipGetLastError();
}

template bool stencil25_supported<float>(int);
template bool stencil25_supported<double>(int);
template hipError_t launch_residual25<float>(const float *, const float *, const float *, float *, int, float, float,
                                             hipStream_t);
template hipError_t launch_residual25<double>(const double *, const double *, const double *, double *, int, double,
                                              double, hipStream_t);
template hipError_t launch_direction25<float, double>(const float *, const double *, double *, const double *,
                                                      double *, double, int, double, bool, double *, double,
                                                      const double *, Part &, hipStream_t);
template hipError_t launch_direction25<float, float>(const float *, const float *, float *, const double *, double *,
                                                     double, int, double, bool, double *, double, const double *,
                                                     Part &, hipStream_t);
template hipError_t launch_direction25<double, double>(const double *, const double *, double *, const double *,
                                                       double *, double, int, double, bool, double *, double,
                                                       const double *, Part &, hipStream_t);

}  // namespace recon
