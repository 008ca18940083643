// Single-workgroup kernels for states that fit in LDS (n <= 13 for complex64,
// n <= 12 for complex128): the whole state (and, for the adjoint, the adjoint
// vector) stays in LDS for a chunk of up to kSmallMaxLayers layers.
//
// Layer k (arXiv:2604.26423, Sec. II-B): cost phase of eq. (2) on every
// amplitude, exp(-i theta_zz (W - 2C)/20) with an FP64 argument, then RX on
// each qubit in turn (eq. 3).  The adjoint walks the chunk backwards,
// accumulating dE/dtheta_x = Im <lam| sum_q X_q |psi> and
// dE/dtheta_zz = -2 Im <lam| C |psi> before undoing each layer on both vectors.
#include "device.h"

namespace qs {

namespace {

constexpr int kSmallThreads = 1024;

template <typename V> struct SmallCfg;
template <> struct SmallCfg<float2> { static constexpr int NMAX = kTileBitsC64; };
template <> struct SmallCfg<double2> { static constexpr int NMAX = kTileBitsC128; };

__device__ __forceinline__ int insert_zero_bit(int k, int q)
{
    const int low = (1 << q) - 1;
    return ((k & ~low) << 1) | (k & low);
}

template <typename V>
__device__ __forceinline__ void small_phase(V *s, const int32_t *diag, int dim, double theta, int64_t W,
                                            int sign, int tid)
{
    for (int x = tid; x < dim; x += kSmallThreads)
        s[x] = cmul(s[x], expi<V>(sign * theta * (double)(2 * (int64_t)diag[x] - W) / 20.0));
}

template <typename V, typename R>
__device__ __forceinline__ void small_rx(V *s, int n, int q, R c, R sn, int tid)
{
    const int half = 1 << (n - 1);
    for (int k = tid; k < half; k += kSmallThreads) {
        const int x0 = insert_zero_bit(k, q);
        V a0 = s[x0], a1 = s[x0 | (1 << q)];
        rx_pair(a0, a1, c, sn);
        s[x0] = a0;
        s[x0 | (1 << q)] = a1;
    }
}

template <typename V>
__global__ void __launch_bounds__(kSmallThreads) small_forward(SmallProg sp)
{
    using R = typename Real<V>::T;
    __shared__ V s[1 << SmallCfg<V>::NMAX];
    __shared__ double red[2 * (kSmallThreads / 64)];
    const int tid = threadIdx.x, n = sp.n, dim = 1 << n;
    V *psi = reinterpret_cast<V *>(sp.psi);

    for (int x = tid; x < dim; x += kSmallThreads) s[x] = sp.init ? V{(R)sp.amp0, (R)0} : psi[x];
    __syncthreads();
    for (int L = 0; L < sp.nlayers; ++L) {
        if (sp.do_phase[L]) {
            small_phase(s, sp.diag, dim, sp.tzz[L], sp.W, 1, tid);
            __syncthreads();
        }
        if (sp.do_mixer[L]) {
            const R c = (R)cos(0.5 * sp.tx[L]), sn = (R)sin(0.5 * sp.tx[L]);
            for (int q = 0; q < n; ++q) {
                small_rx(s, n, q, c, sn, tid);
                __syncthreads();
            }
        }
    }
    if (sp.readout) {
        double acc[2] = {0.0, 0.0};
        for (int x = tid; x < dim; x += kSmallThreads) {
            const double pr = (double)s[x].x * (double)s[x].x + (double)s[x].y * (double)s[x].y;
            acc[0] += pr;
            acc[1] += pr * (double)sp.diag[x];
        }
        block_sum(acc, red, tid, kSmallThreads);
        if (tid == 0) {
            sp.out[0] = acc[0];
            sp.out[1] = acc[1];
        }
    }
    for (int x = tid; x < dim; x += kSmallThreads) psi[x] = s[x];
}

// Accumulator layout in sp.out: [0] norm, [1] sum |a|^2 C_t, [2 + k] dE/dtheta_zz[k],
// [2 + ptotal + k] dE/dtheta_x[k].
template <typename V>
__global__ void __launch_bounds__(kSmallThreads) small_adjoint(SmallProg sp)
{
    using R = typename Real<V>::T;
    __shared__ V sp_[1 << SmallCfg<V>::NMAX];
    __shared__ V sl_[1 << SmallCfg<V>::NMAX];
    __shared__ double red[2 * (kSmallThreads / 64)];
    const int tid = threadIdx.x, n = sp.n, dim = 1 << n;
    const int ptotal = sp.ptotal;
    V *psi = reinterpret_cast<V *>(sp.psi);
    V *lam = reinterpret_cast<V *>(sp.lam);

    for (int x = tid; x < dim; x += kSmallThreads) {
        sp_[x] = psi[x];
        if (!sp.turnaround) sl_[x] = lam[x];
    }
    __syncthreads();
    if (sp.turnaround) {
        double acc[2] = {0.0, 0.0};
        for (int x = tid; x < dim; x += kSmallThreads) {
            const V a = sp_[x];
            const double pr = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
            acc[0] += pr;
            acc[1] += pr * (double)sp.diag[x];
            const R cu = (R)(((double)sp.diag[x] - sp.lam_shift) * 0.1);
            sl_[x] = V{cu * a.x, cu * a.y};
        }
        block_sum(acc, red, tid, kSmallThreads);
        if (tid == 0) {
            sp.out[0] = acc[0];
            sp.out[1] = acc[1];
        }
        __syncthreads();
    }
    for (int L = sp.nlayers - 1; L >= 0; --L) {
        const int k = sp.layer0 + L;
        if (sp.do_mixer[L]) {
            const R c = (R)cos(0.5 * sp.tx[L]), sn = (R)sin(0.5 * sp.tx[L]);
            double acc[1] = {0.0};
            for (int x = tid; x < dim; x += kSmallThreads) {
                for (int q = 0; q < n; ++q) {
                    const V l0 = sl_[x], p1 = sp_[x ^ (1 << q)];
                    acc[0] += (double)l0.x * (double)p1.y - (double)l0.y * (double)p1.x;
                }
            }
            block_sum(acc, red, tid, kSmallThreads);
            if (tid == 0) sp.out[2 + ptotal + k] += acc[0];
            __syncthreads();
            for (int q = n - 1; q >= 0; --q) {
                small_rx(sp_, n, q, c, (R)(-sn), tid);
                small_rx(sl_, n, q, c, (R)(-sn), tid);
                __syncthreads();
            }
        }
        if (sp.do_phase[L]) {
            double acc[1] = {0.0};
            for (int x = tid; x < dim; x += kSmallThreads) {
                const V l0 = sl_[x], p0 = sp_[x];
                acc[0] += -0.2 * ((double)sp.diag[x] - sp.lam_shift) *
                          ((double)l0.x * (double)p0.y - (double)l0.y * (double)p0.x);
            }
            block_sum(acc, red, tid, kSmallThreads);
            if (tid == 0) sp.out[2 + k] += acc[0];
            __syncthreads();
            small_phase(sp_, sp.diag, dim, sp.tzz[L], sp.W, -1, tid);
            small_phase(sl_, sp.diag, dim, sp.tzz[L], sp.W, -1, tid);
            __syncthreads();
        }
    }
    if (sp.store) {
        for (int x = tid; x < dim; x += kSmallThreads) {
            psi[x] = sp_[x];
            lam[x] = sl_[x];
        }
    }
}

}  // namespace

hipError_t launch_small_forward(int prec, const SmallProg &sp, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL(small_forward<float2>, dim3(1), dim3(kSmallThreads), 0, st, sp);
    else
        hipLaunchKernelGGL(small_forward<double2>, dim3(1), dim3(kSmallThreads), 0, st, sp);
    return hipGetLastError();
}

hipError_t launch_small_adjoint(int prec, const SmallProg &sp, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL(small_adjoint<float2>, dim3(1), dim3(kSmallThreads), 0, st, sp);
    else
        hipLaunchKernelGGL(small_adjoint<double2>, dim3(1), dim3(kSmallThreads), 0, st, sp);
    return hipGetLastError();
}

}  // namespace qs
