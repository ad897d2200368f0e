// Fused two-colour red-black Gauss-Seidel sweep (the smoother of the
// multigrid solves, App. A), in a translation unit of its own so that its
// source can be tied to the hardware counters measured on it.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace recon {

// ---------------------------------------------- fused two-colour RB-GS sweep
//
// u_out = one full red-black sweep of u_in (colour `first` relaxed first),
// streaming every field through HBM once.  A workgroup owns a TJ x 64 tile of
// (j, k) and a chunk of CI consecutive i-planes.  Planes of u_in and a enter
// LDS ring buffers with a 2-cell halo in j and k, b with a 1-cell halo, two
// planes ahead of use (register-staged prefetch).  Iteration s relaxes the
// first colour on plane s+1 over the tile plus a 1-cell ring (the ring values
// are recomputed here rather than exchanged with neighbouring tiles), then
// the second colour on plane s over the tile, and writes plane s.  The old
// first-colour values are never read (Gauss-Seidel overwrites them), so the
// new ones are stored in place in the u ring.  Out of place because the
// neighbouring tiles read this tile's halo from u_in.
template <typename T, int TJ, int TK_ = 64, int NT_ = 256>
struct Fused {
    static constexpr int TK = TK_, NT = NT_;
    static constexpr int H = TJ + 4, W = TK + 4, PLANE = H * W;     // u, a: halo 2
    static constexpr int HB = TJ + 2, WB = TK + 2, PLANEB = HB * WB;  // b: halo 1
    static constexpr int LU = (PLANE + NT - 1) / NT;
    static constexpr int LB = (PLANEB + NT - 1) / NT;
    // LDS planes padded to whole rounds of NT loads: every thread loads and
    // deposits unconditionally (lanes past the plane load a valid address and
    // write into the padding), which keeps the load queue countable.
    static constexpr int PU = LU * NT, PB = LB * NT;
    static constexpr int N1 = (TJ + 2) * (TK / 2 + 1);  // first-colour nodes on tile + ring
    static constexpr int N2 = TJ * (TK / 2);            // second-colour nodes on the tile
    static constexpr int R1 = (N1 + NT - 1) / NT, R2 = (N2 + NT - 1) / NT;
    static constexpr int RS = TJ * TK / NT;             // stores per thread
    static constexpr int US = 5, BS = 3;                // ring depths
};

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for every
// outstanding global load, which would drain the register prefetch at each
// barrier; here the loads stay in flight until their registers are used.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Face order in both relaxations: +i, -i, +j, -j, +k, -k (as in k_rbgs_half),
// so the fused and per-colour sweeps round identically.
// ZERO: u_in is taken as 0 and not read (the first sweep from a zero guess).
template <typename T, int TJ, int ZERO, int TK_ = 64, int NT_ = 256>
__global__ void __launch_bounds__(NT_) k_rbgs_fused(const T *__restrict__ uin, T *__restrict__ uout,
                                                    const T *__restrict__ ag, const T *__restrict__ bg, int n,
                                                    int ci, T inv_scale, T a_min, int first)
{
    using F = Fused<T, TJ, TK_, NT_>;
    static_assert(TJ * TK_ % NT_ == 0, "every thread stores whole rounds of the tile");
    constexpr int W = F::W, PLANE = F::PLANE, WB = F::WB, PLANEB = F::PLANEB, NT = F::NT;
    __shared__ T sU[F::US][F::PU];
    __shared__ T sA[F::US][F::PU];
    __shared__ T sB[F::BS][F::PB];

    const int tid = threadIdx.x;
    const int tiles_k = n / F::TK, tiles_j = n / TJ, chunks = n / ci;
    const int nblk = tiles_k * tiles_j * chunks;
    int t = blockIdx.x;
    if ((nblk & 7) == 0) t = (t & 7) * (nblk >> 3) + (t >> 3);  // one contiguous tile range per XCD
    const int tk = t % tiles_k, tj = (t / tiles_k) % tiles_j, ch = t / (tiles_k * tiles_j);
    const int j0 = tj * TJ, k0 = tk * F::TK, i0 = ch * ci;
    const size_t n2 = (size_t)n * n;

    // in-plane global offsets of this thread's halo-2 and halo-1 load slots
    int offU[F::LU], offB[F::LB];
#pragma unroll
    for (int r = 0; r < F::LU; ++r) {
        const int q = tid + r * NT;
        const int row = q / W, col = q % W;
        const int gj = wrapc(j0 - 2 + row, n), gk = wrapc(k0 - 2 + col, n);
        offU[r] = q < PLANE ? gj * n + gk : 0;
    }
#pragma unroll
    for (int r = 0; r < F::LB; ++r) {
        const int q = tid + r * NT;
        const int row = q / WB, col = q % WB;
        const int gj = wrapc(j0 - 1 + row, n), gk = wrapc(k0 - 1 + col, n);
        offB[r] = q < PLANEB ? gj * n + gk : 0;
    }

    T ru[2][F::LU], ra[2][F::LU], rb[2][F::LB];
    auto fetch = [&](int set, int pu, int pb) {
        const size_t bu = (size_t)wrapc(pu, n) * n2, bb = (size_t)wrapc(pb, n) * n2;
#pragma unroll
        for (int r = 0; r < F::LU; ++r) {
            ru[set][r] = ZERO ? (T)0 : uin[bu + offU[r]];
            ra[set][r] = ag[bu + offU[r]];
        }
#pragma unroll
        for (int r = 0; r < F::LB; ++r) rb[set][r] = bg[bb + offB[r]];
    };
    auto deposit = [&](int set, int pu, int pb) {
        const int su = (pu - i0 + 10) % F::US, sb = (pb - i0 + 9) % F::BS;
#pragma unroll
        for (int r = 0; r < F::LU; ++r) {
            sU[su][tid + r * NT] = ru[set][r];
            sA[su][tid + r * NT] = (T)0.5 * ra[set][r];
        }
#pragma unroll
        for (int r = 0; r < F::LB; ++r) sB[sb][tid + r * NT] = rb[set][r];
    };
    auto slotU = [&](int p) { return (p - i0 + 10) % F::US; };
    auto slotB = [&](int p) { return (p - i0 + 9) % F::BS; };

    const int c1 = first, c2 = 1 - first;
    // LDS offsets (u/a plane, b plane) of this thread's relaxation nodes, for
    // both plane parities.  First colour: tile + 1-cell ring, node q at row
    // jj = q / 33 - 1 and column kk = 2 (q % 33) - 1 + e; second colour: tile,
    // jj = q / 32, kk = 2 (q % 32) + e; e makes (i + j + k) % 2 the colour.
    int o1[F::R1][2], b1[F::R1][2], o2[F::R2][2], b2[F::R2][2];
#pragma unroll
    for (int r = 0; r < F::R1; ++r) {
        const int q = tid + r * NT;
        const int jj = q / (F::TK / 2 + 1) - 1, pr = q % (F::TK / 2 + 1);
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            const int kk = 2 * pr - 1 + ((P + jj + 1) & 1);
            o1[r][P] = q < F::N1 ? (jj + 2) * W + (kk + 2) : 2 * W + 2;
            b1[r][P] = q < F::N1 ? (jj + 1) * WB + (kk + 1) : 0;
        }
    }
#pragma unroll
    for (int r = 0; r < F::R2; ++r) {
        const int q = tid + r * NT;
        const int jj = q / (F::TK / 2), pr = q % (F::TK / 2);
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            const int kk = 2 * pr + ((P + jj) & 1);
            o2[r][P] = q < F::N2 ? (jj + 2) * W + (kk + 2) : 2 * W + 2;
            b2[r][P] = q < F::N2 ? (jj + 1) * WB + (kk + 1) : 0;
        }
    }
    // one Gauss-Seidel relaxation from the LDS planes (a is stored halved:
    // the face coefficient max(a_min, (a_n + a_nb) / 2) is max(a_min, h_n + h_nb))
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
    // relax colour c1 on plane p over the tile plus a 1-cell ring (reads only
    // second-colour values, writes first-colour slots)
    auto relax_first = [&](int p) {
        const int P = (c1 + wrapc(p, n)) & 1;
        const T *Uc = sU[slotU(p)], *Ac = sA[slotU(p)];
        const T *Uu = sU[slotU(p + 1)], *Au = sA[slotU(p + 1)];
        const T *Ud = sU[slotU(p - 1)], *Ad = sA[slotU(p - 1)];
        const T *Bc = sB[slotB(p)];
        T *Uw = sU[slotU(p)];
#pragma unroll
        for (int r = 0; r < F::R1; ++r) {
            if (tid + r * NT < F::N1) {
                const int c = o1[r][P];
                Uw[c] = relax(Uc, Uu, Ud, Ac, Au, Ad, c, Bc[b1[r][P]]);
            }
        }
    };
    // relax colour c2 on plane p over the tile (reads only the new first-colour
    // values, writes second-colour slots that no other thread reads here)
    auto relax_second = [&](int p) {
        const int P = (c2 + wrapc(p, n)) & 1;
        const T *Uc = sU[slotU(p)], *Ac = sA[slotU(p)];
        const T *Uu = sU[slotU(p + 1)], *Au = sA[slotU(p + 1)];
        const T *Ud = sU[slotU(p - 1)], *Ad = sA[slotU(p - 1)];
        const T *Bc = sB[slotB(p)];
        T *Uw = sU[slotU(p)];
#pragma unroll
        for (int r = 0; r < F::R2; ++r) {
            if (tid + r * NT < F::N2) {
                const int c = o2[r][P];
                Uw[c] = relax(Uc, Uu, Ud, Ac, Au, Ad, c, Bc[b2[r][P]]);
            }
        }
    };
    auto store_plane = [&](int p) {
        const size_t base = (size_t)wrapc(p, n) * n2;
        const T *Uc = sU[slotU(p)];
#pragma unroll
        for (int r = 0; r < F::RS; ++r) {
            const int q = tid + r * NT;
            const int row = q / F::TK, col = q % F::TK;
            uout[base + (size_t)(j0 + row) * n + (k0 + col)] = Uc[(row + 2) * W + (col + 2)];
        }
    };

    // prologue: u, a planes i0-2 .. i0 and b plane i0-1 resident; planes
    // i0+1 (u, a) / i0 (b) and i0+2 / i0+1 staged in registers
    fetch(0, i0 - 2, i0 - 1);
    deposit(0, i0 - 2, i0 - 1);
    fetch(0, i0 - 1, i0 - 1);
    deposit(0, i0 - 1, i0 - 1);
    fetch(0, i0, i0 - 1);
    deposit(0, i0, i0 - 1);
    fetch(0, i0 + 1, i0);
    fetch(1, i0 + 2, i0 + 1);
    lds_barrier();

    // warm-up: first colour on planes i0-1 and i0 only
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int ss = i0 - 2 + h;
        relax_first(ss + 1);
        lds_barrier();
        deposit(h, ss + 3, ss + 2);
        lds_barrier();
        fetch(h, ss + 5, ss + 4);
    }
    // Steady state, branch-free so that the compiler can count the loads in
    // flight and wait only for the register set being deposited (ci is even).
    // The last two iterations fetch and deposit planes past the chunk: they
    // wrap to valid addresses and land in ring slots that are no longer read.
    for (int s = i0; s < i0 + ci; s += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ss = s + h;
            relax_first(ss + 1);
            lds_barrier();
            relax_second(ss);
            deposit(h, ss + 3, ss + 2);
            lds_barrier();
            store_plane(ss);
            fetch(h, ss + 5, ss + 4);
        }
    }
}

template <typename T>
static constexpr int fused_tj()
{
    return sizeof(T) == 4 ? 16 : 8;
}

template <typename T>
bool rbgs_fused_supported(int n)
{
    return n >= 64 && n % 64 == 0 && n % fused_tj<T>() == 0;
}

template <typename T>
hipError_t launch_rbgs_fused(const T *u_in, T *u_out, const T *a, const T *b, int n, T scale, T a_min, int first,
                             bool zero_init, hipStream_t s)
{
    if (!rbgs_fused_supported<T>(n)) return hipErrorInvalidValue;
    constexpr int TJ = fused_tj<T>();
    // i-chunk: as long as possible while the launch still has >= 1024
    // workgroups (each chunk re-reads 4 planes of u and a)
    int ci = n;
    while (ci > 16 && (n / 64) * (n / TJ) * (n / ci) < 1024) ci /= 2;
    if (ci & 1) return hipErrorInvalidValue;  // the kernel's steady-state loop takes planes in pairs
    const int nblk = (n / 64) * (n / TJ) * (n / ci);
    if (zero_init)
        k_rbgs_fused<T, TJ, 1, 64, 512><<<nblk, 512, 0, s>>>(u_in, u_out, a, b, n, ci, (T)1 / scale, a_min, first);
    else
        k_rbgs_fused<T, TJ, 0, 64, 512><<<nblk, 512, 0, s>>>(u_in, u_out, a, b, n, ci, (T)1 / scale, a_min, first);
    return hipGetLastError();
}

template hipError_t launch_rbgs_fused<float>(const float *, float *, const float *, const float *, int, float,
                                              float, int, bool, hipStream_t);
template hipError_t launch_rbgs_fused<double>(const double *, double *, const double *, const double *, int, double,
                                               double, int, bool, hipStream_t);
template bool rbgs_fused_supported<float>(int);
template bool rbgs_fused_supported<double>(int);

}  // namespace recon
