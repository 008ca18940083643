// Elementwise kernels (initial state, stand-alone cost layer), the <C>/norm
// readout, and the fixed-order reduction of per-workgroup FP64 partial sums.
//
// <C> (arXiv:2604.26423, eq. 5 with exact probabilities): sum |a_x|^2 C(x)
// over the normalised state.  Partial sums are FP64, combined in a fixed
// order (no atomics), so the result is identical from run to run.
#include "device.h"

namespace qs {

namespace {

constexpr int kElemThreads = 256;
constexpr int64_t kElemMaxBlocks = 16384;
constexpr int kReduceChunk = 4096;

int64_t elem_grid(int64_t dim)
{
    int64_t g = (dim + kElemThreads - 1) / kElemThreads;
    return g < kElemMaxBlocks ? g : kElemMaxBlocks;
}

template <typename V>
__global__ void __launch_bounds__(kElemThreads) init_plus_kernel(V *psi, int64_t dim, double amp0)
{
    using R = typename Real<V>::T;
    const V a{(R)amp0, (R)0};
    for (int64_t x = (int64_t)blockIdx.x * kElemThreads + threadIdx.x; x < dim;
         x += (int64_t)gridDim.x * kElemThreads)
        psi[x] = a;
}

// exp(-i theta (W - 2C)/20), per element from an FP64 argument reduced mod 2 pi.
template <typename V>
__global__ void __launch_bounds__(kElemThreads) cost_layer_kernel(V *psi, const int32_t *diag,
                                                                  int64_t dim, int64_t W, double theta)
{
    for (int64_t x = (int64_t)blockIdx.x * kElemThreads + threadIdx.x; x < dim;
         x += (int64_t)gridDim.x * kElemThreads)
        psi[x] = cmul(psi[x], expi<V>(theta * (double)(2 * (int64_t)diag[x] - W) / 20.0));
}

template <typename V>
__global__ void __launch_bounds__(kElemThreads) expect_kernel(const V *psi, const int32_t *diag,
                                                              int64_t dim, double *partials)
{
    __shared__ double red[2 * (kElemThreads / 64)];
    double acc[2] = {0.0, 0.0};
    for (int64_t x = (int64_t)blockIdx.x * kElemThreads + threadIdx.x; x < dim;
         x += (int64_t)gridDim.x * kElemThreads) {
        const V a = psi[x];
        const double pr = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        acc[0] += pr;
        acc[1] += pr * (double)diag[x];
    }
    block_sum(acc, red, threadIdx.x, kElemThreads);
    if (threadIdx.x == 0) {
        partials[blockIdx.x * kSlots + 0] = acc[0];
        partials[blockIdx.x * kSlots + 1] = acc[1];
        partials[blockIdx.x * kSlots + 2] = 0.0;
        partials[blockIdx.x * kSlots + 3] = 0.0;
    }
}

// Level 1: workgroup b sums partials [b*4096, (b+1)*4096) slot by slot.
__global__ void __launch_bounds__(256) reduce_l1_kernel(const double *in, int64_t count, double *out)
{
    __shared__ double red[kSlots * 4];
    double acc[kSlots] = {0.0, 0.0, 0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * kReduceChunk;
    const int64_t hi = lo + kReduceChunk < count ? lo + kReduceChunk : count;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) acc[k] += in[i * kSlots + k];
    }
    block_sum(acc, red, threadIdx.x, 256);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) out[blockIdx.x * kSlots + k] = acc[k];
    }
}

struct SlotMap {
    int m[kSlots];
};

// Level 2: one workgroup sums all (<= 4096) rows and writes dst[map[k]].
__global__ void __launch_bounds__(256) reduce_l2_kernel(const double *in, int64_t count, double *dst,
                                                        SlotMap map, int accumulate)
{
    __shared__ double red[kSlots * 4];
    double acc[kSlots] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < count; i += 256) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) acc[k] += in[i * kSlots + k];
    }
    block_sum(acc, red, threadIdx.x, 256);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (map.m[k] >= 0) dst[map.m[k]] = (accumulate ? dst[map.m[k]] : 0.0) + acc[k];
    }
}

}  // namespace

namespace {
// Copies between index order and the swizzled state layout (internal.h).
template <typename V>
__global__ void __launch_bounds__(kElemThreads) gather_kernel(const V *psi, int64_t first, int64_t count, V *dst)
{
    for (int64_t i = (int64_t)blockIdx.x * kElemThreads + threadIdx.x; i < count; i += (int64_t)gridDim.x * kElemThreads)
        dst[i] = psi[swz(first + i)];
}

template <typename V>
__global__ void __launch_bounds__(kElemThreads) scatter_kernel(V *psi, int64_t first, int64_t count, const V *src)
{
    for (int64_t i = (int64_t)blockIdx.x * kElemThreads + threadIdx.x; i < count; i += (int64_t)gridDim.x * kElemThreads)
        psi[swz(first + i)] = src[i];
}
}  // namespace

hipError_t launch_copy_amplitudes(int prec, void *psi, int64_t first, int64_t count, void *buf, int to_state,
                                  hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const dim3 g((unsigned)elem_grid(count)), b(kElemThreads);
    if (prec == 0) {
        if (to_state) hipLaunchKernelGGL(scatter_kernel<float2>, g, b, 0, st, (float2 *)psi, first, count, (const float2 *)buf);
        else hipLaunchKernelGGL(gather_kernel<float2>, g, b, 0, st, (const float2 *)psi, first, count, (float2 *)buf);
    } else {
        if (to_state) hipLaunchKernelGGL(scatter_kernel<double2>, g, b, 0, st, (double2 *)psi, first, count, (const double2 *)buf);
        else hipLaunchKernelGGL(gather_kernel<double2>, g, b, 0, st, (const double2 *)psi, first, count, (double2 *)buf);
    }
    return hipGetLastError();
}

hipError_t launch_init_plus(int prec, void *psi, int n, int nq, hipStream_t st)
{
    const int64_t dim = (int64_t)1 << n;
    const double amp0 = sqrt(ldexp(1.0, -nq));
    if (prec == 0)
        hipLaunchKernelGGL(init_plus_kernel<float2>, dim3((unsigned)elem_grid(dim)), dim3(kElemThreads), 0, st,
                           (float2 *)psi, dim, amp0);
    else
        hipLaunchKernelGGL(init_plus_kernel<double2>, dim3((unsigned)elem_grid(dim)), dim3(kElemThreads), 0, st,
                           (double2 *)psi, dim, amp0);
    return hipGetLastError();
}

hipError_t launch_cost_layer(int prec, void *psi, const int32_t *diag, int n, int64_t W, double theta,
                             hipStream_t st)
{
    const int64_t dim = (int64_t)1 << n;
    if (prec == 0)
        hipLaunchKernelGGL(cost_layer_kernel<float2>, dim3((unsigned)elem_grid(dim)), dim3(kElemThreads), 0, st,
                           (float2 *)psi, diag, dim, W, theta);
    else
        hipLaunchKernelGGL(cost_layer_kernel<double2>, dim3((unsigned)elem_grid(dim)), dim3(kElemThreads), 0,
                           st, (double2 *)psi, diag, dim, W, theta);
    return hipGetLastError();
}

hipError_t launch_expect(int prec, const void *psi, const int32_t *diag, int n, double *partials,
                         int64_t *nblocks, hipStream_t st)
{
    const int64_t dim = (int64_t)1 << n;
    const int64_t g = elem_grid(dim);
    *nblocks = g;
    if (prec == 0)
        hipLaunchKernelGGL(expect_kernel<float2>, dim3((unsigned)g), dim3(kElemThreads), 0, st,
                           (const float2 *)psi, diag, dim, partials);
    else
        hipLaunchKernelGGL(expect_kernel<double2>, dim3((unsigned)g), dim3(kElemThreads), 0, st,
                           (const double2 *)psi, diag, dim, partials);
    return hipGetLastError();
}

int64_t reduce_tmp_doubles(int64_t count)
{
    return ((count + kReduceChunk - 1) / kReduceChunk) * kSlots;
}

hipError_t launch_reduce(const double *partials, int64_t count, double *tmp, double *dst, const int *map,
                         int accumulate, hipStream_t st)
{
    SlotMap sm;
    for (int k = 0; k < kSlots; ++k) sm.m[k] = map[k];
    if (count <= kReduceChunk) {
        hipLaunchKernelGGL(reduce_l2_kernel, dim3(1), dim3(256), 0, st, partials, count, dst, sm, accumulate);
        return hipGetLastError();
    }
    const int64_t nb = (count + kReduceChunk - 1) / kReduceChunk;
    hipLaunchKernelGGL(reduce_l1_kernel, dim3((unsigned)nb), dim3(256), 0, st, partials, count, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_l2_kernel, dim3(1), dim3(256), 0, st, (const double *)tmp, nb, dst, sm, accumulate);
    return hipGetLastError();
}

}  // namespace qs
