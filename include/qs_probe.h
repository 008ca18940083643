/*
 * qs_probe.h -- memory-bandwidth probes of the device that libqs runs on.
 *
 * These kernels move data and do no simulation work.  They measure what the
 * HBM of the current device sustains for the access mixes and the tile
 * geometries that the simulator's passes use, so that a pass's measured rate
 * can be set against the device's own ceiling for the same mix as well as
 * against the published peak.  Not needed to run a circuit.
 */
#ifndef QS_PROBE_H
#define QS_PROBE_H

#include <stddef.h>

#include "qs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QS_PROBE_READ = 0,   /* read every 16-byte element of b; a receives 16 B per workgroup */
    QS_PROBE_WRITE = 1,  /* write every 16-byte element of a */
    QS_PROBE_COPY = 2,   /* a = b */
    QS_PROBE_UPDATE = 3, /* a = s * a in place: one read and one write of each element */
    QS_PROBE_PHASE = 4,  /* complex64 a[x] *= unit phase of int32 b[x] in place: the byte mix of a cost
                            layer (8 B read + 4 B read + 8 B written per amplitude); bytes counts a */
    QS_PROBE_TILE = 5,   /* complex64 state a of 2^n amplitudes read and written back in place, tile by
                            tile, in the geometry of a mixer pass (fields c and q0); no arithmetic */
    QS_PROBE_WINDOW_VALU = 6, /* mixer window, butterflies: two complex64 vectors a and b of 2^n amplitudes
                            (the two vectors of a reverse pass), each group of 16 consecutive amplitudes
                            multiplied `windows` times per load by K = (x)^4 [[1, -iu], [-iu, 1]], u = 1/4
                            (the tangent-form RX of eq. (3) on four qubits), as 4 x 8 two-FMA pair updates
                            per vector; a thread holds one group of each vector */
    QS_PROBE_WINDOW_MFMA = 7  /* the same product as WINDOW_VALU on FP32 matrix cores: with D = diag(i^|r|)
                            the matrix D K D^-1 is real, so each application is a real 16 x 16 matrix times
                            the real and the imaginary parts of 16 groups (v_mfma_f32_16x16x4f32, eight per
                            vector); D is applied once before and undone once after the repeats */
} qs_probe_kind;

#define QS_PROBE_NT_LOAD 1  /* nontemporal loads (streamed past the caches) */
#define QS_PROBE_NT_STORE 2 /* nontemporal stores */

typedef struct qs_probe {
    int kind;       /* qs_probe_kind */
    int flags;      /* QS_PROBE_NT_LOAD | QS_PROBE_NT_STORE */
    int wg_per_cu;  /* 0: one workgroup per chunk of 16 KiB (or per tile); k > 0: k persistent workgroups
                       per compute unit walking the chunks */
    int unroll;     /* 16-byte elements per thread per chunk: 1, 2, 4 or 8 (0 = 4); ignored for tiles */
    int n;          /* QS_PROBE_TILE: 2^n complex64 amplitudes in a, 14 <= n <= 34 */
    int c;          /* QS_PROBE_TILE: carrier bits (contiguous runs of 2^c amplitudes), 0..8 */
    int q0;         /* QS_PROBE_TILE: global bit of the first strided tile bit; a tile holds 2^13
                       amplitudes at indices base | (e & (2^c - 1)) | (e >> c) << q0, e < 2^13 */
    int swizzle;    /* QS_PROBE_TILE: 1 = the library's state layout (qs_layout_index), 0 = plain */
    int windows;    /* QS_PROBE_WINDOW_*: applications of K per load, 1..64; 12 <= n <= 34 */
} qs_probe;

/*
 * Run the probe reps times (reps >= 1) on hip_stream and return the mean
 * duration of one launch from HIP events (ms_per_launch) and the bytes one
 * launch reads plus writes (bytes_per_launch; both nullable).  Synchronises.
 * a, b: device buffers of `bytes` bytes each (b unused by WRITE, UPDATE and
 * TILE; for PHASE, b holds bytes / 2 bytes of int32), 256-byte aligned; bytes
 * a multiple of 16 KiB (for TILE and WINDOW_*, bytes = 2^n * 8).  The contents
 * of a are overwritten (TILE and UPDATE with s = 1 leave the values
 * unchanged); WINDOW_* overwrite a and b with K^(windows (reps + 1)) applied
 * to each group, and bytes_per_launch counts both vectors.
 * Errors: QS_ERR_ARG (bad kind, flags, sizes, alignment or geometry),
 * QS_ERR_HIP.
 */
qs_status qs_bandwidth_probe(const qs_probe *probe, void *a, const void *b, size_t bytes, int reps, void *hip_stream,
                             double *ms_per_launch, double *bytes_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* QS_PROBE_H */
