/*
 * stream_probe.h -- streaming-bandwidth probes of one MI355X (gfx950), built
 * as libstream_probe.so beside the reconstruction library.
 *
 * Not part of the method: these kernels measure the HBM ceilings against
 * which the reconstruction's stencil kernels (all bound by HBM bandwidth,
 * none a dense contraction) are reported, and give the plain kernels of known
 * traffic that calibrate the FETCH_SIZE and WRITE_SIZE counters.  Each moves
 * every byte exactly once with 16-byte vector accesses.
 */
#ifndef STREAM_PROBE_H
#define STREAM_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STREAM_PROBE_READ 0  /* sum a (bytes read)                           */
#define STREAM_PROBE_WRITE 1 /* fill d (bytes written)                        */
#define STREAM_PROBE_COPY 2  /* d = a (bytes read + bytes written)            */
#define STREAM_PROBE_TRIAD 3 /* d = a + b * c (3 x bytes read + bytes written) */
#define STREAM_PROBE_NONTEMPORAL 16 /* or-ed into a kind: streaming (nontemporal) loads and stores */

#define STREAM_PROBE_MAX_BLOCKS (1 << 22)

/* Launch probe `kind` (optionally | STREAM_PROBE_NONTEMPORAL) once untimed, then `reps` times back to back on
 * hip_stream (a hipStream_t, NULL = default stream), and write the mean
 * duration of one launch in milliseconds (hipEvents) to *ms_out (host).
 * d, a, b, c: device buffers of `bytes` bytes each (a multiple of 16), float32
 * data; the kind reads a (and b, c for the triad) and writes d; unused ones
 * may be NULL.  blocks: workgroups of 256 threads (1..STREAM_PROBE_MAX_BLOCKS),
 * each striding over the arrays (blocks * 256 * 16 >= bytes: one vector per
 * thread).  part: device float[blocks], the read
 * probe's per-block sums (NULL for the others).  Returns 0, -1 for a bad
 * argument (nothing launched) or -2 for a HIP error. */
int stream_probe_run(int kind, void *d, const void *a, const void *b, const void *c, size_t bytes, int blocks,
                     float *part, int reps, void *hip_stream, float *ms_out);

#ifdef __cplusplus
}
#endif

#endif /* STREAM_PROBE_H */
