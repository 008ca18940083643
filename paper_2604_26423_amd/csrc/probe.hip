// Bandwidth probes (declared in include/qs_probe.h): kernels that only move
// data, for the device's own ceilings under the access mixes of the
// simulator's passes.  Streaming kinds work on chunks of 256 threads x U
// 16-byte elements: every thread issues its U loads before any store.  The
// tile kind walks a complex64 state exactly as the forward tile passes do
// (same tile bases, XCD order, register windows and memory layout) but keeps
// the tile in registers with no butterflies and no LDS.
#include "../../include/qs_probe.h"
#include "tiles.h"

namespace qs {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kProbeThreads = 256;

template <bool NT>
__device__ __forceinline__ f4 ld(const f4 *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ i2 ld(const i2 *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st(f4 *p, f4 v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// One chunk: elements base + u * 256 + tid, u < U.
template <int KIND, int U, bool NTL, bool NTS>
__device__ __forceinline__ void probe_chunk(f4 *a, const f4 *b, const i2 *ph, int64_t base, float s, f4 &acc)
{
    const int tid = threadIdx.x;
    f4 v[U];
    if constexpr (KIND == QS_PROBE_READ || KIND == QS_PROBE_COPY) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld<NTL>(b + base + u * kProbeThreads + tid);
    } else if constexpr (KIND == QS_PROBE_UPDATE || KIND == QS_PROBE_PHASE) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld<NTL>(a + base + u * kProbeThreads + tid);
    }
    if constexpr (KIND == QS_PROBE_READ) {
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    } else if constexpr (KIND == QS_PROBE_WRITE) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = f4{s, s, s, s};
    } else if constexpr (KIND == QS_PROBE_UPDATE) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] *= s;
    } else if constexpr (KIND == QS_PROBE_PHASE) {
        // two amplitudes per element, each multiplied by a unit complex number
        // drawn from its int32 (a cheap stand-in for the phase table)
        i2 c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = ld<NTL>(ph + base + u * kProbeThreads + tid);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float t0 = (float)(c[u].x & 1023) * s, t1 = (float)(c[u].y & 1023) * s;
            const float c0 = 1.0f - t0 * t0, c1 = 1.0f - t1 * t1;
            const f4 x = v[u];
            v[u] = f4{c0 * x.x - t0 * x.y, c0 * x.y + t0 * x.x, c1 * x.z - t1 * x.w, c1 * x.w + t1 * x.z};
        }
    }
    if constexpr (KIND != QS_PROBE_READ) {
#pragma unroll
        for (int u = 0; u < U; ++u) st<NTS>(a + base + u * kProbeThreads + tid, v[u]);
    }
}

template <int KIND, int U, bool NTL, bool NTS>
__global__ void __launch_bounds__(kProbeThreads) stream_kernel(f4 *a, const f4 *b, const i2 *ph, int64_t nchunks,
                                                               float s, int persistent)
{
    f4 acc{0.f, 0.f, 0.f, 0.f};
    constexpr int64_t CH = (int64_t)U * kProbeThreads;
    if (persistent) {
        for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) probe_chunk<KIND, U, NTL, NTS>(a, b, ph, c * CH, s, acc);
    } else {
        probe_chunk<KIND, U, NTL, NTS>(a, b, ph, (int64_t)blockIdx.x * CH, s, acc);
    }
    if constexpr (KIND == QS_PROBE_READ) {
        if (threadIdx.x == 0) a[blockIdx.x] = acc;  // keeps the loads live: 16 B per workgroup
    }
}

// Tile geometry of a forward pass, data movement only.
template <bool NTL, bool NTS>
__device__ __forceinline__ f2 ld2(const f2 *p)
{
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NTS>
__device__ __forceinline__ void st2(f2 *p, f2 v)
{
    if constexpr (NTS) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <bool NTL, bool NTS>
__global__ void __launch_bounds__(1 << kFwdThreadBits) tile_probe_kernel(f2 *psi, int64_t ntiles, int c, int q0,
                                                                         int swizzle, int xcd, float s)
{
    constexpr int T = kTileBitsC64, TB = kFwdThreadBits, RB = T - TB, NR = 1 << RB;
    const int tid = threadIdx.x;
    const int m = T - c;
    const int64_t tile = xcd_tile(xcd);
    if (tile >= ntiles) return;
    const int64_t base = tile_base(tile, c, q0, m);
    const Addr ad = win_addr(tid, TB, RB, base, c, q0);
    f2 v[NR];
    if (swizzle) {
        for_each_reg<NR>(ad, [&](int r, int64_t x) { v[r] = ld2<NTL, NTS>(psi + x); });
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = ld2<NTL, NTS>(psi + ad.fast_idx(r));
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] *= s;
    if (swizzle) {
        for_each_reg<NR>(ad, [&](int r, int64_t x) { st2<NTS>(psi + x, v[r]); });
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) st2<NTS>(psi + ad.fast_idx(r), v[r]);
    }
}

// ---- mixer-window microbenchmark: butterflies against FP32 matrix cores ----
// Both kernels multiply every group of 16 consecutive amplitudes of two
// complex64 vectors by K = (x)^4 [[1, -iu], [-iu, 1]] (the tangent-form RX of
// one four-qubit register window), `windows` times per load.
constexpr float kWinU = 0.25f;

__global__ void __launch_bounds__(256) window_valu_kernel(float2 *a, float2 *b, int windows)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;  // one group per thread
    f4 *pa = reinterpret_cast<f4 *>(a + g * 16), *pb = reinterpret_cast<f4 *>(b + g * 16);
    float2 x[16], y[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const f4 u = pa[i], v = pb[i];
        x[2 * i] = float2{u.x, u.y};
        x[2 * i + 1] = float2{u.z, u.w};
        y[2 * i] = float2{v.x, v.y};
        y[2 * i + 1] = float2{v.z, v.w};
    }
#pragma unroll 1
    for (int w = 0; w < windows; ++w) {
        rxt_reg_bit<0>(x, kWinU);
        rxt_reg_bit<1>(x, kWinU);
        rxt_reg_bit<2>(x, kWinU);
        rxt_reg_bit<3>(x, kWinU);
        rxt_reg_bit<0>(y, kWinU);
        rxt_reg_bit<1>(y, kWinU);
        rxt_reg_bit<2>(y, kWinU);
        rxt_reg_bit<3>(y, kWinU);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        pa[i] = f4{x[2 * i].x, x[2 * i].y, x[2 * i + 1].x, x[2 * i + 1].y};
        pb[i] = f4{y[2 * i].x, y[2 * i].y, y[2 * i + 1].x, y[2 * i + 1].y};
    }
}

// Multiply by i^k (k mod 4).
__device__ __forceinline__ float2 rot_i(float2 v, int k)
{
    switch (k & 3) {
    case 0: return v;
    case 1: return float2{-v.y, v.x};
    case 2: return float2{-v.x, -v.y};
    default: return float2{v.y, -v.x};
    }
}

// v_mfma_f32_16x16x4f32 (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[4 (l / 16) + i][l % 16], i = 0..3.  A wave
// takes 16 groups as the columns of a 16 x 16 matrix X; lane (j = l / 16,
// c = l % 16) holds rows 4j .. 4j + 3 of column c, the layout of D, so the
// product can be fed back.  The K = 16 sum runs as four slices s, in which
// lane (j, c) supplies B = X[4j + s][c] (its own s-th row) and A = M[c][4j + s],
// with M = D K D^-1, M[r][q] = (-1)^|q & ~r| u^|r ^ q|, D = diag(i^|r|).
__global__ void __launch_bounds__(256) window_mfma_kernel(float2 *a, float2 *b, int windows)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane >> 4, c = lane & 15;
    const int64_t g = ((int64_t)blockIdx.x * 4 + wave) * 16 + c;  // this lane's group
    f4 *pa = reinterpret_cast<f4 *>(a + g * 16 + 4 * j), *pb = reinterpret_cast<f4 *>(b + g * 16 + 4 * j);
    float am[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int q = 4 * j + s;
        float m = 1.0f;
        for (int t = __builtin_popcount(c ^ q); t > 0; --t) m *= kWinU;
        am[s] = (__builtin_popcount(q & ~c) & 1) ? -m : m;
    }
    float2 x[4], y[4];
    {
        const f4 u0 = pa[0], u1 = pa[1], v0 = pb[0], v1 = pb[1];
        x[0] = float2{u0.x, u0.y};
        x[1] = float2{u0.z, u0.w};
        x[2] = float2{u1.x, u1.y};
        x[3] = float2{u1.z, u1.w};
        y[0] = float2{v0.x, v0.y};
        y[1] = float2{v0.z, v0.w};
        y[2] = float2{v1.x, v1.y};
        y[3] = float2{v1.z, v1.w};
    }
    f4 xr, xi, yr, yi;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = __builtin_popcount(4 * j + i);
        const float2 p = rot_i(x[i], k), q = rot_i(y[i], k);
        xr[i] = p.x;
        xi[i] = p.y;
        yr[i] = q.x;
        yi[i] = q.y;
    }
#pragma unroll 1
    for (int w = 0; w < windows; ++w) {
        f4 nxr{0.f, 0.f, 0.f, 0.f}, nxi = nxr, nyr = nxr, nyi = nxr;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            nxr = __builtin_amdgcn_mfma_f32_16x16x4f32(am[s], xr[s], nxr, 0, 0, 0);
            nxi = __builtin_amdgcn_mfma_f32_16x16x4f32(am[s], xi[s], nxi, 0, 0, 0);
            nyr = __builtin_amdgcn_mfma_f32_16x16x4f32(am[s], yr[s], nyr, 0, 0, 0);
            nyi = __builtin_amdgcn_mfma_f32_16x16x4f32(am[s], yi[s], nyi, 0, 0, 0);
        }
        xr = nxr;
        xi = nxi;
        yr = nyr;
        yi = nyi;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 - __builtin_popcount(4 * j + i);
        x[i] = rot_i(float2{xr[i], xi[i]}, k);
        y[i] = rot_i(float2{yr[i], yi[i]}, k);
    }
    pa[0] = f4{x[0].x, x[0].y, x[1].x, x[1].y};
    pa[1] = f4{x[2].x, x[2].y, x[3].x, x[3].y};
    pb[0] = f4{y[0].x, y[0].y, y[1].x, y[1].y};
    pb[1] = f4{y[2].x, y[2].y, y[3].x, y[3].y};
}

template <int KIND, int U, bool NTL, bool NTS>
void launch_stream_u(f4 *a, const f4 *b, const i2 *ph, int64_t nchunks, int64_t grid, float s, hipStream_t st)
{
    hipLaunchKernelGGL((stream_kernel<KIND, U, NTL, NTS>), dim3((unsigned)grid), dim3(kProbeThreads), 0, st, a, b,
                       ph, nchunks, s, grid < nchunks ? 1 : 0);
}

template <int KIND, bool NTL, bool NTS>
void launch_stream_k(int U, f4 *a, const f4 *b, const i2 *ph, int64_t nchunks, int64_t grid, float s, hipStream_t st)
{
    switch (U) {
    case 1: launch_stream_u<KIND, 1, NTL, NTS>(a, b, ph, nchunks, grid, s, st); break;
    case 2: launch_stream_u<KIND, 2, NTL, NTS>(a, b, ph, nchunks, grid, s, st); break;
    case 8: launch_stream_u<KIND, 8, NTL, NTS>(a, b, ph, nchunks, grid, s, st); break;
    default: launch_stream_u<KIND, 4, NTL, NTS>(a, b, ph, nchunks, grid, s, st); break;
    }
}

template <bool NTL, bool NTS>
void launch_stream_f(int kind, int U, f4 *a, const f4 *b, const i2 *ph, int64_t nchunks, int64_t grid, float s,
                     hipStream_t st)
{
    switch (kind) {
    case QS_PROBE_READ: launch_stream_k<QS_PROBE_READ, NTL, NTS>(U, a, b, ph, nchunks, grid, s, st); break;
    case QS_PROBE_WRITE: launch_stream_k<QS_PROBE_WRITE, NTL, NTS>(U, a, b, ph, nchunks, grid, s, st); break;
    case QS_PROBE_COPY: launch_stream_k<QS_PROBE_COPY, NTL, NTS>(U, a, b, ph, nchunks, grid, s, st); break;
    case QS_PROBE_UPDATE: launch_stream_k<QS_PROBE_UPDATE, NTL, NTS>(U, a, b, ph, nchunks, grid, s, st); break;
    default: launch_stream_k<QS_PROBE_PHASE, NTL, NTS>(U, a, b, ph, nchunks, grid, s, st); break;
    }
}

void launch_probe(const qs_probe &pr, void *a, const void *b, size_t bytes, int64_t cus, float s, hipStream_t st)
{
    const bool ntl = (pr.flags & QS_PROBE_NT_LOAD) != 0, nts = (pr.flags & QS_PROBE_NT_STORE) != 0;
    if (pr.kind == QS_PROBE_WINDOW_VALU) {  // 256 groups of 16 amplitudes per workgroup
        hipLaunchKernelGGL(window_valu_kernel, dim3((unsigned)((int64_t)1 << (pr.n - 12))), dim3(256), 0, st,
                           (float2 *)a, (float2 *)b, pr.windows);
        return;
    }
    if (pr.kind == QS_PROBE_WINDOW_MFMA) {  // 64 groups per workgroup
        hipLaunchKernelGGL(window_mfma_kernel, dim3((unsigned)((int64_t)1 << (pr.n - 10))), dim3(256), 0, st,
                           (float2 *)a, (float2 *)b, pr.windows);
        return;
    }
    if (pr.kind == QS_PROBE_TILE) {
        const int64_t ntiles = (int64_t)1 << (pr.n - kTileBitsC64);
        const int xcd = ntiles % 8 == 0 ? 1 : 0;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)ntiles), dim3(1 << kFwdThreadBits), 0, st, (f2 *)a, ntiles,
                               pr.c, pr.q0, pr.swizzle, xcd, s);
        };
        if (ntl && nts) go(tile_probe_kernel<true, true>);
        else if (ntl) go(tile_probe_kernel<true, false>);
        else if (nts) go(tile_probe_kernel<false, true>);
        else go(tile_probe_kernel<false, false>);
        return;
    }
    const int U = pr.unroll ? pr.unroll : 4;
    const int64_t nchunks = (int64_t)(bytes / 16) / ((int64_t)U * kProbeThreads);
    const int64_t grid = pr.wg_per_cu > 0 ? std::min<int64_t>(nchunks, cus * pr.wg_per_cu) : nchunks;
    f4 *fa = (f4 *)a;
    const f4 *fb = (const f4 *)b;
    const i2 *ph = (const i2 *)b;
    if (ntl && nts) launch_stream_f<true, true>(pr.kind, U, fa, fb, ph, nchunks, grid, s, st);
    else if (ntl) launch_stream_f<true, false>(pr.kind, U, fa, fb, ph, nchunks, grid, s, st);
    else if (nts) launch_stream_f<false, true>(pr.kind, U, fa, fb, ph, nchunks, grid, s, st);
    else launch_stream_f<false, false>(pr.kind, U, fa, fb, ph, nchunks, grid, s, st);
}

}  // namespace

// Records a message for qs_last_error (defined with the other entry points).
qs_status set_error(qs_status st, const char *fmt, ...);

}  // namespace qs

using namespace qs;

extern "C" qs_status qs_bandwidth_probe(const qs_probe *pr, void *a, const void *b, size_t bytes, int reps,
                                        void *hip_stream, double *ms_per_launch, double *bytes_per_launch)
{
    if (!pr) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: null probe");
    if (pr->kind < QS_PROBE_READ || pr->kind > QS_PROBE_WINDOW_MFMA)
        return set_error(QS_ERR_ARG, "qs_bandwidth_probe: bad kind");
    if (pr->flags & ~(QS_PROBE_NT_LOAD | QS_PROBE_NT_STORE)) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: bad flags");
    if (pr->wg_per_cu < 0 || pr->wg_per_cu > 64) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: wg_per_cu outside 0..64");
    if (reps < 1 || reps > 1000) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: reps outside 1..1000");
    if (!a || ((uintptr_t)a & 255)) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: a must be a 256-byte aligned buffer");
    double moved = 0.0;
    if (pr->kind == QS_PROBE_WINDOW_VALU || pr->kind == QS_PROBE_WINDOW_MFMA) {
        if (pr->n < 12 || pr->n > QS_MAX_QUBITS_C64)
            return set_error(QS_ERR_ARG, "qs_bandwidth_probe: window probe needs 12 <= n <= 34");
        if (pr->windows < 1 || pr->windows > 64)
            return set_error(QS_ERR_ARG, "qs_bandwidth_probe: windows outside 1..64");
        if (bytes != ((size_t)8 << pr->n)) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: window probe needs bytes = 2^n * 8");
        if (!b || ((uintptr_t)b & 255)) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: b must be a 256-byte aligned buffer");
        if (pr->flags) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: window probes take no flags");
        moved = 4.0 * (double)bytes;
    } else if (pr->kind == QS_PROBE_TILE) {
        if (pr->n < kTileBitsC64 + 1 || pr->n > QS_MAX_QUBITS_C64)
            return set_error(QS_ERR_ARG, "qs_bandwidth_probe: tile probe needs 14 <= n <= 34");
        const int m = kTileBitsC64 - pr->c;
        if (pr->c < 0 || pr->c > 8 || pr->q0 < pr->c || pr->q0 + m > pr->n)
            return set_error(QS_ERR_ARG, "qs_bandwidth_probe: tile geometry c = %d, q0 = %d outside n = %d", pr->c,
                             pr->q0, pr->n);
        if (pr->swizzle != 0 && pr->swizzle != 1) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: swizzle is 0 or 1");
        if (bytes != ((size_t)8 << pr->n)) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: tile probe needs bytes = 2^n * 8");
        moved = 2.0 * (double)bytes;
    } else {
        const int U = pr->unroll ? pr->unroll : 4;
        if (U != 1 && U != 2 && U != 4 && U != 8) return set_error(QS_ERR_ARG, "qs_bandwidth_probe: unroll is 1, 2, 4 or 8");
        if (bytes == 0 || bytes % (16 << 10) != 0 || bytes % ((size_t)16 * U * kProbeThreads) != 0)
            return set_error(QS_ERR_ARG, "qs_bandwidth_probe: bytes must be a positive multiple of 16 KiB");
        if (pr->kind != QS_PROBE_WRITE && pr->kind != QS_PROBE_UPDATE && (!b || ((uintptr_t)b & 255)))
            return set_error(QS_ERR_ARG, "qs_bandwidth_probe: b must be a 256-byte aligned buffer");
        if ((bytes / 16) / ((size_t)U * kProbeThreads) > 0xffffffffull)
            return set_error(QS_ERR_ARG, "qs_bandwidth_probe: too many chunks");
        const double B = (double)bytes;
        moved = pr->kind == QS_PROBE_READ || pr->kind == QS_PROBE_WRITE ? B : pr->kind == QS_PROBE_PHASE ? 2.5 * B : 2.0 * B;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0, cus = 256;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        launch_probe(*pr, a, b, bytes, cus, 1.0f, st);  // untimed first launch
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; e == hipSuccess && i < reps; ++i) {
        launch_probe(*pr, a, b, bytes, cus, 1.0f, st);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return set_error(QS_ERR_HIP, "qs_bandwidth_probe: %s", hipGetErrorString(e));
    if (ms_per_launch) *ms_per_launch = ms / reps;
    if (bytes_per_launch) *bytes_per_launch = moved;
    return QS_OK;
}
