// Cost diagonal C_t[x] = sum_{i<j} w_ij (x_i XOR x_j) in tenths (the cut
// function of arXiv:2604.26423, eq. 6), its maximum C(x*) (eq. 5), for all
// 2^n basis states.
//
// Split the vertices into L = {0..12} (the low 13 index bits) and H = the
// rest.  For a fixed high part x_H:
//   C(x) = C_HH(x_H) + sum_{i in L} A_i + C_LL(x_L) + sum_{i in L} x_i e_i,
//   A_i = sum_{j in H} w_ij x_j,  D_i = sum_{j in H} w_ij,  e_i = D_i - 2 A_i,
// because a cross edge contributes w_ij (x_i + x_j - 2 x_i x_j), which is
// linear in x_i once x_j is fixed.  C_LL is a 2^13-entry table shared by all
// workgroups; each workgroup owns one x_H (8192 consecutive states), sets up
// e_i and the constant part once, and then each state costs a table load and
// a few adds.  The kernel is bound by the 4-byte store per state.
#include "device.h"

namespace qs {

namespace {

constexpr int kLowBits = kDiagLowBits;
constexpr int kDiagThreads = 256;

// Cut value restricted to vertices [0, L), by the double loop.  When L == n
// this is the full diagonal; the per-workgroup maximum goes to wg_max.
__global__ void __launch_bounds__(kDiagThreads) diag_low_kernel(const int32_t *wm, int n, int L, int32_t *out,
                                                                int32_t *wg_max)
{
    __shared__ int red[kDiagThreads / 64];
    const int x = blockIdx.x * kDiagThreads + threadIdx.x;
    int best = 0;
    if (x < (1 << L)) {
        int s = 0;
        for (int i = 0; i < L; ++i)
            for (int j = i + 1; j < L; ++j) s += wm[i * n + j] * (((x >> i) ^ (x >> j)) & 1);
        out[x] = s;
        best = s;
    }
    if (wg_max) {
        for (int off = 32; off >= 1; off >>= 1) best = max(best, __shfl_xor(best, off, 64));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            int m = red[0];
            for (int w = 1; w < kDiagThreads / 64; ++w) m = max(m, red[w]);
            wg_max[blockIdx.x] = m;
        }
    }
}

__global__ void __launch_bounds__(kDiagThreads) diag_main_kernel(const int32_t *wm, int n, const int32_t *low,
                                                                 int32_t *diag, int32_t *wg_max)
{
    __shared__ int e[kLowBits];
    __shared__ int red[kDiagThreads / 64];
    __shared__ int part[kDiagThreads / 64];
    const int tid = threadIdx.x;
    const int64_t xh = blockIdx.x;  // high part: global bits >= 13

    // constant part: C_HH(x_H) + sum_i A_i, accumulated by rows
    int cst = 0;
    if (tid < kLowBits) {
        int A = 0, D = 0;
        for (int j = kLowBits; j < n; ++j) {
            const int wij = wm[tid * n + j];
            D += wij;
            A += wij * (int)((xh >> (j - kLowBits)) & 1);
        }
        e[tid] = D - 2 * A;
        cst += A;
    } else if (tid < kLowBits + (n - kLowBits)) {
        const int i = tid;  // high vertex of this row
        const int bi = (int)((xh >> (i - kLowBits)) & 1);
        for (int j = i + 1; j < n; ++j) cst += wm[i * n + j] * (bi ^ (int)((xh >> (j - kLowBits)) & 1));
    }
    for (int off = 32; off >= 1; off >>= 1) cst += __shfl_xor(cst, off, 64);
    if ((tid & 63) == 0) part[tid >> 6] = cst;
    __syncthreads();
    const int base = part[0] + part[1] + part[2] + part[3];

    // low bits 2..9 come from the thread index, 10..12 from the store round m
    int st = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) st += ((tid >> k) & 1) * e[2 + k];
    const int e0 = e[0], e1 = e[1];
    int best = 0;
    const int4 *low4 = reinterpret_cast<const int4 *>(low);
    int4 *out4 = reinterpret_cast<int4 *>(diag + (xh << kLowBits));
    const int f4 = (int)(swz_fold(xh) << (kSwzDst - 2));  // swizzled layout, in int4 units
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int sm = (m & 1) * e[10] + ((m >> 1) & 1) * e[11] + ((m >> 2) & 1) * e[12];
        const int idx = m * 256 + tid;  // int4 index = (m*1024 + 4*tid) / 4
        const int4 t = low4[idx];
        const int b = base + st + sm;
        int4 v;
        v.x = b + t.x;
        v.y = b + e0 + t.y;
        v.z = b + e1 + t.z;
        v.w = b + e0 + e1 + t.w;
        out4[idx ^ f4] = v;
        best = max(best, max(max(v.x, v.y), max(v.z, v.w)));
    }
    for (int off = 32; off >= 1; off >>= 1) best = max(best, __shfl_xor(best, off, 64));
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) wg_max[blockIdx.x] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// Complement-symmetric layout: entry z (z < 2^(n-1)) holds C of the state
// x = y(z) with bit n-1 clear, y_q = z_q ^ z_(q+1) ^ ... ^ z_(n-2).  The
// high bits of y depend only on the high bits of z, and the low 13 bits of y
// are the low suffix-XOR of z's low bits, complemented when the high bits of
// z have odd parity.  So workgroup zh computes the natural-order block of
// y_H = y(zh) in LDS exactly as diag_main_kernel does, then writes it out
// permuted into z order with coalesced stores.
__device__ __forceinline__ int64_t suffix_xor(int64_t v)
{
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) v ^= (int64_t)((uint64_t)v >> sh);
    return v;
}

__global__ void __launch_bounds__(kDiagThreads) diag_sym_kernel(const int32_t *wm, int n, const int32_t *low,
                                                                int32_t *diag, int32_t *wg_max)
{
    __shared__ int e[kLowBits];
    __shared__ int red[kDiagThreads / 64];
    __shared__ int part[kDiagThreads / 64];
    __shared__ int4 blk[(1 << kLowBits) / 4];
    const int tid = threadIdx.x;
    const int64_t zh = blockIdx.x;
    const int64_t yh = suffix_xor(zh);          // y bits >= 13 (vertex n-1 stays 0)
    const int flip = (int)(yh & 1) ? (1 << kLowBits) - 1 : 0;

    int cst = 0;
    if (tid < kLowBits) {
        int A = 0, D = 0;
        for (int j = kLowBits; j < n; ++j) {
            const int wij = wm[tid * n + j];
            D += wij;
            A += wij * (int)((yh >> (j - kLowBits)) & 1);
        }
        e[tid] = D - 2 * A;
        cst += A;
    } else if (tid < kLowBits + (n - kLowBits)) {
        const int i = tid;
        const int bi = (int)((yh >> (i - kLowBits)) & 1);
        for (int j = i + 1; j < n; ++j) cst += wm[i * n + j] * (bi ^ (int)((yh >> (j - kLowBits)) & 1));
    }
    for (int off = 32; off >= 1; off >>= 1) cst += __shfl_xor(cst, off, 64);
    if ((tid & 63) == 0) part[tid >> 6] = cst;
    __syncthreads();
    const int base = part[0] + part[1] + part[2] + part[3];

    int st = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) st += ((tid >> k) & 1) * e[2 + k];
    const int e0 = e[0], e1 = e[1];
    int best = 0;
    const int4 *low4 = reinterpret_cast<const int4 *>(low);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int sm = (m & 1) * e[10] + ((m >> 1) & 1) * e[11] + ((m >> 2) & 1) * e[12];
        const int idx = m * 256 + tid;
        const int4 t = low4[idx];
        const int b = base + st + sm;
        int4 v;
        v.x = b + t.x;
        v.y = b + e0 + t.y;
        v.z = b + e1 + t.z;
        v.w = b + e0 + e1 + t.w;
        blk[idx] = v;
        best = max(best, max(max(v.x, v.y), max(v.z, v.w)));
    }
    __syncthreads();
    const int *blks = reinterpret_cast<const int *>(blk);
    int4 *out4 = reinterpret_cast<int4 *>(diag + (zh << kLowBits));
    const int f4 = (int)(swz_fold(zh) << (kSwzDst - 2));  // swizzled layout, in int4 units
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int idx = m * 256 + tid;
        const int z = 4 * idx;
        int4 v;
        v.x = blks[(int)suffix_xor(z) ^ flip];
        v.y = blks[(int)suffix_xor(z + 1) ^ flip];
        v.z = blks[(int)suffix_xor(z + 2) ^ flip];
        v.w = blks[(int)suffix_xor(z + 3) ^ flip];
        out4[idx ^ f4] = v;
    }
    for (int off = 32; off >= 1; off >>= 1) best = max(best, __shfl_xor(best, off, 64));
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) wg_max[blockIdx.x] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// max over in[0..count) by chunks of 4096 per workgroup.
__global__ void __launch_bounds__(256) max_kernel(const int32_t *in, int64_t count, int32_t *out)
{
    __shared__ int red[4];
    const int64_t lo = (int64_t)blockIdx.x * 4096;
    const int64_t hi = lo + 4096 < count ? lo + 4096 : count;
    int best = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) best = max(best, in[i]);
    for (int off = 32; off >= 1; off >>= 1) best = max(best, __shfl_xor(best, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = max(max(red[0], red[1]), max(red[2], red[3]));
}

}  // namespace

int64_t diag_wg_count(int n, int sym)
{
    if (sym) return (int64_t)1 << (n - 1 - kLowBits);
    if (n <= kLowBits) return ((int64_t)1 << n) / kDiagThreads + 1;
    return (int64_t)1 << (n - kLowBits);
}

hipError_t launch_cost_diagonal(int n, const int32_t *wm, int32_t *diag, int32_t *low_table, int32_t *wg_max,
                                int32_t *tmp_max, int32_t *cmax_dev, hipStream_t st, int sym)
{
    int64_t count;
    if (sym) {  // n - 1 >= 13 stored bits (checked by the caller)
        const int g0 = (1 << kLowBits) / kDiagThreads;
        hipLaunchKernelGGL(diag_low_kernel, dim3(g0), dim3(kDiagThreads), 0, st, wm, n, kLowBits, low_table,
                           (int32_t *)nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        count = diag_wg_count(n, 1);
        hipLaunchKernelGGL(diag_sym_kernel, dim3((unsigned)count), dim3(kDiagThreads), 0, st, wm, n,
                           (const int32_t *)low_table, diag, wg_max);
    } else if (n <= kLowBits) {
        const int64_t g = ((int64_t)1 << n) / kDiagThreads + 1;
        hipLaunchKernelGGL(diag_low_kernel, dim3((unsigned)g), dim3(kDiagThreads), 0, st, wm, n, n, diag, wg_max);
        count = g;
    } else {
        const int g0 = (1 << kLowBits) / kDiagThreads;
        hipLaunchKernelGGL(diag_low_kernel, dim3(g0), dim3(kDiagThreads), 0, st, wm, n, kLowBits, low_table,
                           (int32_t *)nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        count = (int64_t)1 << (n - kLowBits);
        hipLaunchKernelGGL(diag_main_kernel, dim3((unsigned)count), dim3(kDiagThreads), 0, st, wm, n,
                           (const int32_t *)low_table, diag, wg_max);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // two-level max: count -> ceil(count/4096) -> 1
    const int64_t nb = (count + 4095) / 4096;
    hipLaunchKernelGGL(max_kernel, dim3((unsigned)nb), dim3(256), 0, st, (const int32_t *)wg_max, count, tmp_max);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, (const int32_t *)tmp_max, nb, cmax_dev);
    return hipGetLastError();
}

}  // namespace qs
