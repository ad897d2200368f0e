// Fused two-colour red-black Gauss-Seidel sweep (the smoother of the
// multigrid solves, App. A), in a translation unit of its own so that its
// source can be tied to the hardware counters measured on it.

#include <hip/hip_runtime.h>

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
// streaming every field through HBM once.  A workgroup owns a TJ x 64 tile of
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
// Face order in the relaxation: +i, -i, +j, -j, +k, -k (as in k_rbgs_half),
// so the fused and per-colour sweeps round identically; a is stored halved
// (the face coefficient max(a_min, (a_n + a_nb) / 2) is max(a_min, h_n + h_nb)).
// ZERO: u_in is taken as 0 and not read (the first sweep from a zero guess).
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

template <typename T, int TJ, int ZERO, int TK_ = 64, int NT_ = 512>
__global__ void __launch_bounds__(NT_) k_rbgs_fused(const T *__restrict__ uin, T *__restrict__ uout,
                                                    const T *__restrict__ ag, const T *__restrict__ bg, int n,
                                                    int ci, T inv_scale, T a_min, int first)
{
    using F = Ring4<T, TJ, TK_, NT_>;
    static_assert(TJ * TK_ % NT_ == 0, "every thread stores whole rounds of the tile");
    constexpr int W = F::W, PLANE = F::PLANE, NT = F::NT, LU = F::LU, R1 = F::R1, R2 = F::R2;
    __shared__ T sU[4][F::PU];
    __shared__ T sA[4][F::PU];

    const int tid = threadIdx.x;
    const int tiles_k = n / F::TK, tiles_j = n / TJ, chunks = n / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int j0 = tj * TJ, k0 = tk * F::TK, i0 = ch * ci;
    const size_t n2 = (size_t)n * n;

    // halo load slots: global in-plane offset and LDS destination
    int offU[LU], dstU[LU];
#pragma unroll
    for (int r = 0; r < LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / W, col = q % W;
        const int gj = wrapc(j0 - 2 + row, n), gk = wrapc(k0 - 2 + col, n);
        offU[r] = q < PLANE ? gj * n + gk : 0;
        dstU[r] = q < PLANE ? q : PLANE;
    }

    const int c1 = first, c2 = 1 - first;
    // relaxation nodes for both plane parities: LDS offset and global in-plane
    // offset (for b).  First colour: tile + 1-cell ring, node q at row
    // jj = q / (TK/2 + 1) - 1, column kk = 2 (q % (TK/2 + 1)) - 1 + e; second
    // colour: tile, jj = q / (TK/2), kk = 2 (q % (TK/2)) + e; e makes
    // (i + j + k) % 2 the colour.  Lanes past the node count use slot 0 and skip.
    int o1[R1][2], g1[R1][2], o2[R2][2], g2[R2][2];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        const int q = tid + r * NT;
        const int jj = q / (F::TK / 2 + 1) - 1, pr = q % (F::TK / 2 + 1);
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            const int kk = 2 * pr - 1 + ((P + jj + 1) & 1);
            const bool on = q < F::N1;
            o1[r][P] = on ? (jj + 2) * W + (kk + 2) : 2 * W + 2;
            g1[r][P] = on ? wrapc(j0 + jj, n) * n + wrapc(k0 + kk, n) : 0;
        }
    }
#pragma unroll
    for (int r = 0; r < R2; ++r) {
        const int q = tid + r * NT;
        const int jj = q / (F::TK / 2), pr = q % (F::TK / 2);
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            const int kk = 2 * pr + ((P + jj) & 1);
            const bool on = q < F::N2;
            o2[r][P] = on ? (jj + 2) * W + (kk + 2) : 2 * W + 2;
            g2[r][P] = on ? (j0 + jj) * n + (k0 + kk) : 0;
        }
    }
    auto slot = [&](int p) { return (p - i0 + 8) & 3; };
    auto par1 = [&](int p) { return (c1 + wrapc(p, n)) & 1; };
    auto par2 = [&](int p) { return (c2 + wrapc(p, n)) & 1; };

    T ru[2][LU], ra[2][LU];
    auto fetch = [&](int set, int p) {
        const size_t bu = (size_t)wrapc(p, n) * n2;
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            ru[set][r] = ZERO ? (T)0 : uin[bu + offU[r]];
            ra[set][r] = ag[bu + offU[r]];
        }
    };
    auto deposit = [&](int set, int p) {
        T *U = sU[slot(p)], *A = sA[slot(p)];
#pragma unroll
        for (int r = 0; r < LU; ++r) {
            U[dstU[r]] = ru[set][r];
            A[dstU[r]] = (T)0.5 * ra[set][r];
        }
    };
    // b at the first-colour nodes of plane p1 and the second-colour nodes of plane p2
    T rb1[2][R1], rb2[2][R2];
    auto fetch_b = [&](int set, int p1, int p2) {
        const size_t b1 = (size_t)wrapc(p1, n) * n2, b2 = (size_t)wrapc(p2, n) * n2;
        const int P1 = par1(p1), P2 = par2(p2);
#pragma unroll
        for (int r = 0; r < R1; ++r) rb1[set][r] = bg[b1 + g1[r][P1]];
#pragma unroll
        for (int r = 0; r < R2; ++r) rb2[set][r] = bg[b2 + g2[r][P2]];
    };

    // one Gauss-Seidel relaxation from the LDS planes (a stored halved)
    auto relax = [&](const T *Uc, const T *Uu, const T *Ud, const T *Ac, const T *Au, const T *Ad, int c,
                     T bval) {
        const T hn = Ac[c];
        T num = 0, den = 0, cf;
        cf = fmax(hn + Au[c], a_min); num += cf * Uu[c]; den += cf;
        cf = fmax(hn + Ad[c], a_min); num += cf * Ud[c]; den += cf;
        cf = fmax(hn + Ac[c + W], a_min); num += cf * Uc[c + W]; den += cf;
        cf = fmax(hn + Ac[c - W], a_min); num += cf * Uc[c - W]; den += cf;
        cf = fmax(hn + Ac[c + 1], a_min); num += cf * Uc[c + 1]; den += cf;
        cf = fmax(hn + Ac[c - 1], a_min); num += cf * Uc[c - 1]; den += cf;
        return qdiv(num - bval * inv_scale, den);
    };
    auto relax_first = [&](int p, const T (&bv)[R1]) {
        const int P = par1(p);
        const T *Uc = sU[slot(p)], *Ac = sA[slot(p)];
        const T *Uu = sU[slot(p + 1)], *Au = sA[slot(p + 1)];
        const T *Ud = sU[slot(p - 1)], *Ad = sA[slot(p - 1)];
        T *Uw = sU[slot(p)];
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            if (tid + r * NT < F::N1) {
                const int c = o1[r][P];
                Uw[c] = relax(Uc, Uu, Ud, Ac, Au, Ad, c, bv[r]);
            }
        }
    };
    auto relax_second = [&](int p, const T (&bv)[R2]) {
        const int P = par2(p);
        const T *Uc = sU[slot(p)], *Ac = sA[slot(p)];
        const T *Uu = sU[slot(p + 1)], *Au = sA[slot(p + 1)];
        const T *Ud = sU[slot(p - 1)], *Ad = sA[slot(p - 1)];
        T *Uw = sU[slot(p)];
#pragma unroll
        for (int r = 0; r < R2; ++r) {
            if (tid + r * NT < F::N2) {
                const int c = o2[r][P];
                Uw[c] = relax(Uc, Uu, Ud, Ac, Au, Ad, c, bv[r]);
            }
        }
    };
    auto store_plane = [&](int p) {
        const size_t base = (size_t)wrapc(p, n) * n2;
        const T *Uc = sU[slot(p)];
#pragma unroll
        for (int r = 0; r < F::RS; ++r) {
            const int q = tid + r * NT;
            const int row = q / F::TK, col = q % F::TK;
            uout[base + (size_t)(j0 + row) * n + (k0 + col)] = Uc[(row + 2) * W + (col + 2)];
        }
    };

    // prologue: u, a planes i0-2 .. i0+1 resident; i0+2 (set 1) and i0+3 (set 0)
    // staged; b for the first two steady iterations staged
    fetch(0, i0 - 2);
    deposit(0, i0 - 2);
    fetch(0, i0 - 1);
    deposit(0, i0 - 1);
    fetch(0, i0);
    deposit(0, i0);
    fetch(0, i0 + 1);
    deposit(0, i0 + 1);
    fetch(1, i0 + 2);
    fetch(0, i0 + 3);
    fetch_b(0, i0 + 1, i0);
    fetch_b(1, i0 + 2, i0 + 1);
    lds_barrier();
    // warm-up: first colour on planes i0-1 and i0
    {
        T bw[R1];
        const size_t bb = (size_t)wrapc(i0 - 1, n) * n2;
#pragma unroll
        for (int r = 0; r < R1; ++r) bw[r] = bg[bb + g1[r][par1(i0 - 1)]];
        relax_first(i0 - 1, bw);
    }
    lds_barrier();
    deposit(1, i0 + 2);  // into the slot of plane i0-2, read last just above
    fetch(1, i0 + 4);
    lds_barrier();
    {
        T bw[R1];
        const size_t bb = (size_t)wrapc(i0, n) * n2;
#pragma unroll
        for (int r = 0; r < R1; ++r) bw[r] = bg[bb + g1[r][par1(i0)]];
        relax_first(i0, bw);
    }
    // Steady state, branch-free (ci is even).  The last two iterations fetch and
    // deposit planes past the chunk: they wrap to valid addresses and land in
    // ring slots that are no longer read.
    for (int s = i0; s < i0 + ci; s += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ss = s + h;
            relax_first(ss + 1, rb1[h]);
            lds_barrier();
            relax_second(ss, rb2[h]);
            lds_barrier();
            deposit(h, ss + 3);  // into the slot of plane ss-1
            store_plane(ss);
            fetch(h, ss + 5);
            fetch_b(h, ss + 3, ss + 2);
            lds_barrier();
        }
    }
}

// Tile rows, workgroup size and the smallest launch, per precision: FP32 takes
// 32 x 64 tiles (78 KB of LDS, two workgroups per CU), FP64 8 x 64 tiles with
// 256 threads (52 KB, three per CU), sizes measured best at 512^3.
template <typename T>
struct FusedLaunch;
template <>
struct FusedLaunch<float> {
    static constexpr int TJ = 32, NT = 512, MIN_BLOCKS = 512;
};
template <>
struct FusedLaunch<double> {
    static constexpr int TJ = 8, NT = 256, MIN_BLOCKS = 2048;
};

template <typename T>
bool rbgs_fused_supported(int n)
{
    return n >= 64 && n % 64 == 0 && n % FusedLaunch<T>::TJ == 0;
}

template <typename T>
hipError_t launch_rbgs_fused(const T *u_in, T *u_out, const T *a, const T *b, int n, T scale, T a_min, int first,
                             bool zero_init, hipStream_t s)
{
    using C = FusedLaunch<T>;
    if (!rbgs_fused_supported<T>(n)) return hipErrorInvalidValue;
    // i-chunk: as long as possible while the launch still has MIN_BLOCKS
    // workgroups (each chunk re-reads 4 planes of u and a)
    int ci = n;
    while (ci > 16 && (n / 64) * (n / C::TJ) * (n / ci) < C::MIN_BLOCKS) ci /= 2;
    if (ci & 1) return hipErrorInvalidValue;  // the kernel's steady-state loop takes planes in pairs
    const int nblk = (n / 64) * (n / C::TJ) * (n / ci);
    if (zero_init)
        k_rbgs_fused<T, C::TJ, 1, 64, C::NT><<<nblk, C::NT, 0, s>>>(u_in, u_out, a, b, n, ci, (T)1 / scale, a_min,
                                                                    first);
    else
        k_rbgs_fused<T, C::TJ, 0, 64, C::NT><<<nblk, C::NT, 0, s>>>(u_in, u_out, a, b, n, ci, (T)1 / scale, a_min,
                                                                    first);
    return hipGetLastError();
}

template hipError_t launch_rbgs_fused<float>(const float *, float *, const float *, const float *, int, float,
                                              float, int, bool, hipStream_t);
template hipError_t launch_rbgs_fused<double>(const double *, double *, const double *, const double *, int, double,
                                               double, int, bool, hipStream_t);
template bool rbgs_fused_supported<float>(int);
template bool rbgs_fused_supported<double>(int);

}  // namespace recon
