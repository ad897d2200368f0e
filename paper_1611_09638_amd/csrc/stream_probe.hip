// Streaming-bandwidth probes: the HBM ceilings against which the library's
// stencil kernels are measured (include/stream_probe.h).  Plain grid-stride
// loops over 16-byte vectors, four independent vectors in flight per thread
// per iteration, no LDS, no reuse: every byte is moved once.
#include <hip/hip_runtime.h>

#include "../../include/stream_probe.h"

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;

// read: sum of every element, one partial per block (so the loads are live)
__global__ __launch_bounds__(kThreads) void k_read(const float4 *__restrict__ a, long nv, float *__restrict__ part)
{
    const long stride = (long)gridDim.x * kThreads;
    long i = (long)blockIdx.x * kThreads + threadIdx.x;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
        float4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = a[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    for (; i < nv; i += stride) {
        float4 v = a[i];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
    }
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

__global__ __launch_bounds__(kThreads) void k_write(float4 *__restrict__ d, long nv, float val)
{
    const long stride = (long)gridDim.x * kThreads;
    const float4 v = make_float4(val, val, val, val);
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < nv; i += stride) d[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_copy(float4 *__restrict__ d, const float4 *__restrict__ a, long nv)
{
    const long stride = (long)gridDim.x * kThreads;
    long i = (long)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
        float4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = a[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) d[i + u * stride] = v[u];
    }
    for (; i < nv; i += stride) d[i] = a[i];
}

// d = a + b * c: three reads and one write, the mix of a smoother sweep
__global__ __launch_bounds__(kThreads) void k_triad(float4 *__restrict__ d, const float4 *__restrict__ a,
                                                    const float4 *__restrict__ b, const float4 *__restrict__ c,
                                                    long nv)
{
    const long stride = (long)gridDim.x * kThreads;
    long i = (long)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
        float4 x[kUnroll], y[kUnroll], z[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            x[u] = a[i + u * stride];
            y[u] = b[i + u * stride];
            z[u] = c[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            float4 r;
            r.x = x[u].x + y[u].x * z[u].x;
            r.y = x[u].y + y[u].y * z[u].y;
            r.z = x[u].z + y[u].z * z[u].z;
            r.w = x[u].w + y[u].w * z[u].w;
            d[i + u * stride] = r;
        }
    }
    for (; i < nv; i += stride) {
        float4 x = a[i], y = b[i], z = c[i], r;
        r.x = x.x + y.x * z.x;
        r.y = x.y + y.y * z.y;
        r.z = x.z + y.z * z.z;
        r.w = x.w + y.w * z.w;
        d[i] = r;
    }
}

hipError_t launch(int kind, void *d, const void *a, const void *b, const void *c, long nv, int blocks, float *part,
                  hipStream_t s)
{
    switch (kind) {
    case STREAM_PROBE_READ:
        k_read<<<blocks, kThreads, 0, s>>>((const float4 *)a, nv, part);
        break;
    case STREAM_PROBE_WRITE:
        k_write<<<blocks, kThreads, 0, s>>>((float4 *)d, nv, 1.0f);
        break;
    case STREAM_PROBE_COPY:
        k_copy<<<blocks, kThreads, 0, s>>>((float4 *)d, (const float4 *)a, nv);
        break;
    case STREAM_PROBE_TRIAD:
        k_triad<<<blocks, kThreads, 0, s>>>((float4 *)d, (const float4 *)a, (const float4 *)b, (const float4 *)c, nv);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" {

int stream_probe_run(int kind, void *d, const void *a, const void *b, const void *c, size_t bytes, int blocks,
                     float *part, int reps, void *hip_stream, float *ms_out)
{
    if (!ms_out || reps < 1 || blocks < 1 || blocks > STREAM_PROBE_MAX_BLOCKS || bytes == 0 || bytes % 16)
        return -1;
    const bool needs_d = kind != STREAM_PROBE_READ, needs_a = kind != STREAM_PROBE_WRITE;
    const bool needs_bc = kind == STREAM_PROBE_TRIAD;
    if ((needs_d && !d) || (needs_a && !a) || (needs_bc && (!b || !c)) || (kind == STREAM_PROBE_READ && !part))
        return -1;
    if (kind < STREAM_PROBE_READ || kind > STREAM_PROBE_TRIAD) return -1;
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
