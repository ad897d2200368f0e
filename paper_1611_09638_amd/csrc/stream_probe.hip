// Streaming-bandwidth probes: the HBM ceilings against which the library's
// stencil kernels are measured (include/stream_probe.h).  Plain grid-stride
// loops over 16-byte vectors, four independent vectors in flight per thread
// per iteration, no LDS, no reuse: every byte is moved once.  The
// nontemporal variants load and store with the streaming cache policy.
#include <hip/hip_runtime.h>

#include "../../include/stream_probe.h"

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;

typedef float v4f __attribute__((ext_vector_type(4)));

template <int NT>
__device__ __forceinline__ v4f ld(const v4f *p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <int NT>
__device__ __forceinline__ void st(v4f *p, v4f v)
{
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// read: sum of every element, one partial per block (so the loads are live)
template <int NT>
__global__ __launch_bounds__(kThreads) void k_read(const v4f *__restrict__ a, long nv, float *__restrict__ part)
{
    const long stride = (long)gridDim.x * kThreads;
    long i = (long)blockIdx.x * kThreads + threadIdx.x;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
        v4f v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = ld<NT>(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += v[u];
    }
    for (; i < nv; i += stride) acc += ld<NT>(a + i);
    float s = acc.x + acc.y + acc.z + acc.w;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ float ws[kThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < kThreads / 64; ++w) t += ws[w];
        part[blockIdx.x] = t;
    }
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_write(v4f *__restrict__ d, long nv, float val)
{
    const long stride = (long)gridDim.x * kThreads;
    const v4f v = {val, val, val, val};
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < nv; i += stride) st<NT>(d + i, v);
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_copy(v4f *__restrict__ d, const v4f *__restrict__ a, long nv)
{
    const long stride = (long)gridDim.x * kThreads;
    long i = (long)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
        v4f v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = ld<NT>(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) st<NT>(d + i + u * stride, v[u]);
    }
    for (; i < nv; i += stride) st<NT>(d + i, ld<NT>(a + i));
}

// d = a + b * c: three reads and one write, the mix of a smoother sweep
template <int NT>
__global__ __launch_bounds__(kThreads) void k_triad(v4f *__restrict__ d, const v4f *__restrict__ a,
                                                    const v4f *__restrict__ b, const v4f *__restrict__ c, long nv)
{
    const long stride = (long)gridDim.x * kThreads;
    long i = (long)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
        v4f x[kUnroll], y[kUnroll], z[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            x[u] = ld<NT>(a + i + u * stride);
            y[u] = ld<NT>(b + i + u * stride);
            z[u] = ld<NT>(c + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) st<NT>(d + i + u * stride, x[u] + y[u] * z[u]);
    }
    for (; i < nv; i += stride) st<NT>(d + i, ld<NT>(a + i) + ld<NT>(b + i) * ld<NT>(c + i));
}

template <int NT>
hipError_t launch_nt(int kind, void *d, const void *a, const void *b, const void *c, long nv, int blocks, float *part,
                     hipStream_t s)
{
    switch (kind) {
    case STREAM_PROBE_READ:
        k_read<NT><<<blocks, kThreads, 0, s>>>((const v4f *)a, nv, part);
        break;
    case STREAM_PROBE_WRITE:
        k_write<NT><<<blocks, kThreads, 0, s>>>((v4f *)d, nv, 1.0f);
        break;
    case STREAM_PROBE_COPY:
        k_copy<NT><<<blocks, kThreads, 0, s>>>((v4f *)d, (const v4f *)a, nv);
        break;
    case STREAM_PROBE_TRIAD:
        k_triad<NT><<<blocks, kThreads, 0, s>>>((v4f *)d, (const v4f *)a, (const v4f *)b, (const v4f *)c, nv);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch(int kind, void *d, const void *a, const void *b, const void *c, long nv, int blocks, float *part,
                  hipStream_t s)
{
    if (kind & STREAM_PROBE_NONTEMPORAL) return launch_nt<1>(kind & ~STREAM_PROBE_NONTEMPORAL, d, a, b, c, nv, blocks, part, s);
    return launch_nt<0>(kind, d, a, b, c, nv, blocks, part, s);
}

}  // namespace

extern "C" {

int stream_probe_run(int kind, void *d, const void *a, const void *b, const void *c, size_t bytes, int blocks,
                     float *part, int reps, void *hip_stream, float *ms_out)
{
    if (!ms_out || reps < 1 || blocks < 1 || blocks > STREAM_PROBE_MAX_BLOCKS || bytes == 0 || bytes % 16)
        return -1;
    const int base = kind & ~STREAM_PROBE_NONTEMPORAL;
    if (base < STREAM_PROBE_READ || base > STREAM_PROBE_TRIAD) return -1;
    const bool needs_d = base != STREAM_PROBE_READ, needs_a = base != STREAM_PROBE_WRITE;
    const bool needs_bc = base == STREAM_PROBE_TRIAD;
    if ((needs_d && !d) || (needs_a && !a) || (needs_bc && (!b || !c)) || (base == STREAM_PROBE_READ && !part))
        return -1;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const long nv = (long)(bytes / 16);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -2;
    // one untimed launch, then reps timed back to back
    if (!rc && launch(kind, d, a, b, c, nv, blocks, part, s) != hipSuccess) rc = -2;
    if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = -2;
    for (int r = 0; !rc && r < reps; ++r)
        if (launch(kind, d, a, b, c, nv, blocks, part, s) != hipSuccess) rc = -2;
    if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)) rc = -2;
    float ms = 0.0f;
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -2;
    if (!rc) *ms_out = ms / (float)reps;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
