// Exact distribution of the cut value under the state (arXiv:2604.26423,
// Sec. II-D: the noiseless reference distribution that the subsampled means
// and their 3-sigma thresholds are drawn from).  In the sampler's fixed point,
//   mass[c] = sum over x with C_t[x] = c of floor((re^2 + im^2) 2^62),
// with values outside 0..nbins-1 counted in the last bin.  Integer sums make
// the result independent of the order of accumulation, so it is reproducible
// bit for bit.
//
// One pass over psi and C_t (12 B per c64 amplitude).  Each workgroup owns a
// contiguous range and keeps a private histogram in LDS (64-bit LDS atomics);
// at the end it writes that histogram as one row of a scratch matrix, and a
// second kernel sums the rows per bin.  Histograms wider than the LDS budget
// add straight into one global row.  The FP64 sum of |a|^2 per workgroup is
// written beside it so that the host can reject states whose total mass would
// not fit in 64 bits.
#include "device.h"

namespace qs {

namespace {

constexpr int kHT = 512;  // threads per workgroup

// The state and the diagonal are read once: nontemporal (streaming) loads,
// which measured the n = 32 histogram 5% faster in both precisions.
template <typename V> struct Wide;
template <> struct Wide<float2> {  // two amplitudes per 16-byte load
    static constexpr int K = 2;
    __device__ static void load(const float2 *p, int64_t x, float2 (&a)[2])
    {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 v = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p + x));
        a[0] = make_float2(v.x, v.y);
        a[1] = make_float2(v.z, v.w);
    }
    __device__ static void load_c(const int32_t *d, int64_t x, int32_t (&c)[2])
    {
        typedef int i2 __attribute__((ext_vector_type(2)));
        const i2 v = __builtin_nontemporal_load(reinterpret_cast<const i2 *>(d + x));
        c[0] = v.x;
        c[1] = v.y;
    }
};
template <> struct Wide<double2> {
    static constexpr int K = 1;
    __device__ static void load(const double2 *p, int64_t x, double2 (&a)[1]) { a[0] = load_nt(p + x); }
    __device__ static void load_c(const int32_t *d, int64_t x, int32_t (&c)[1])
    {
        c[0] = __builtin_nontemporal_load(d + x);
    }
};

template <typename V, bool LDS>
__global__ void __launch_bounds__(kHT) hist_kernel(const V *__restrict__ psi, const int32_t *__restrict__ diag,
                                                   int64_t per, int nbins, uint64_t *rows, double *fsum,
                                                   int32_t *flag)
{
    using Wd = Wide<V>;
    constexpr int K = Wd::K;
    extern __shared__ uint64_t bins[];
    __shared__ double red[kHT / 64];
    const int tid = threadIdx.x;
    uint64_t *dst = LDS ? bins : rows;
    if (LDS) {
        for (int i = tid; i < nbins; i += kHT) bins[i] = 0;
        __syncthreads();
    }
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per;
    const unsigned last = (unsigned)nbins - 1u;
    double acc = 0.0;
    int32_t fl = 0;
    auto add = [&](const V (&a)[K], const int32_t (&c)[K]) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double P = prob_fp64((double)a[k].x, (double)a[k].y);
            acc += P;
            const uint64_t q = qmass(P, &fl);
            const unsigned b = (unsigned)c[k] > last ? last : (unsigned)c[k];
            if (q) atomicAdd((unsigned long long *)&dst[b], (unsigned long long)q);
        }
    };
    // U strides per step, all loads issued before the atomics (per is a
    // multiple of the stride; the tail loop takes what is left over)
    constexpr int U = 4;
    const int64_t S = (int64_t)kHT * K;
    int64_t x = lo + (int64_t)tid * K;
    for (; x + (U - 1) * S < hi; x += U * S) {
        V a[U][K];
        int32_t c[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            Wd::load(psi, x + u * S, a[u]);
            Wd::load_c(diag, x + u * S, c[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) add(a[u], c[u]);
    }
    for (; x < hi; x += S) {
        V a[K];
        int32_t c[K];
        Wd::load(psi, x, a);
        Wd::load_c(diag, x, c);
        add(a, c);
    }
    if (fl) *flag = fl;
    // fixed-order block sum of the FP64 mass
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < kHT / 64; ++w) s += red[w];
        fsum[blockIdx.x] = s;
    }
    if (LDS)
        for (int i = tid; i < nbins; i += kHT) rows[(int64_t)blockIdx.x * nbins + i] = bins[i];
}

__global__ void __launch_bounds__(256) hist_rows_kernel(const uint64_t *rows, int nrows, int nbins, int shift,
                                                        uint64_t *out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nbins) return;
    uint64_t s = 0;
    for (int r = 0; r < nrows; ++r) s += rows[(int64_t)r * nbins + i];
    out[i] = s << shift;
}

}  // namespace

HistGeom hist_geom(int prec, int n, int nbins)
{
    HistGeom g{};
    const int64_t dim = (int64_t)1 << n;
    const int K = prec == 0 ? 2 : 1;
    int64_t groups = 1;
    // about two workgroups per CU, each with at least one full sweep of its threads
    while (groups < 512 && dim / (groups * 2) >= (int64_t)kHT * K) groups *= 2;
    g.groups = groups;
    g.per = dim / groups;
    g.lds = (int64_t)nbins * 8 <= kHistLdsBytes;
    g.rows = g.lds ? groups : 1;
    return g;
}

hipError_t launch_histogram(int prec, const void *psi, const int32_t *diag, int nbins, const HistGeom &g,
                            uint64_t *rows, double *fsum, int32_t *flag, uint64_t *out, hipStream_t st, int shift)
{
    const size_t shm = g.lds ? (size_t)nbins * 8 : 0;
    const dim3 grid((unsigned)g.groups), block(kHT);
    if (prec == 0) {
        if (g.lds)
            hipLaunchKernelGGL((hist_kernel<float2, true>), grid, block, shm, st, (const float2 *)psi, diag, g.per,
                               nbins, rows, fsum, flag);
        else
            hipLaunchKernelGGL((hist_kernel<float2, false>), grid, block, 0, st, (const float2 *)psi, diag, g.per,
                               nbins, rows, fsum, flag);
    } else {
        if (g.lds)
            hipLaunchKernelGGL((hist_kernel<double2, true>), grid, block, shm, st, (const double2 *)psi, diag, g.per,
                               nbins, rows, fsum, flag);
        else
            hipLaunchKernelGGL((hist_kernel<double2, false>), grid, block, 0, st, (const double2 *)psi, diag, g.per,
                               nbins, rows, fsum, flag);
    }
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(hist_rows_kernel, dim3((unsigned)((nbins + 255) / 256)), dim3(256), 0, st, rows,
                       (int)g.rows, nbins, shift, out);
    return hipGetLastError();
}

}  // namespace qs
