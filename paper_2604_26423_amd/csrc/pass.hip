// Tile-pass kernels: the fused layer passes of the forward circuit and of the
// adjoint (reverse) sweep.
//
// A layer of the circuit (arXiv:2604.26423, Sec. II-B) is the cost unitary of
// eq. (2), a diagonal phase exp(-i theta_zz (W - 2C(x))/20) once the
// n(n-1)/2 commuting RZZ gates are combined, followed by the mixer of
// eq. (3), RX(theta_x) on every qubit.  The RX gates commute, so one pass over
// memory applies all of them for the T qubits of a tile: a tile of 2^T
// amplitudes sits in registers (2^(T-8) per thread), butterflies act on the
// tile bits held in registers, and LDS exchanges rotate other tile bits into
// registers.  The cost phase is elementwise, so it is applied inside a pass,
// between the butterflies of one layer and the next (the "pre" and "post"
// stages).
#include "device.h"

namespace qs {

namespace {

constexpr int kTabMax = kPhaseTableMaxW / 64 + 64;

template <int T> struct TileCfg {
    static constexpr int RB = T - 8;
    static constexpr int NR = 1 << RB;
    static constexpr int LDS = (1 << T) + (1 << T) / 32;
};

// Phase factor exp(-i theta (W - 2C)/20) = A[C >> 6] * B[C & 63] with
//   A[h] = exp(i theta (128 h - W) / 20),  B[l] = exp(i theta l / 10),
// both evaluated with FP64 arguments reduced modulo 2 pi.
template <typename V>
__device__ __forceinline__ void build_phase_table(V *tab, int ht, double theta, int64_t W, int tid)
{
    for (int i = tid; i < ht + 64; i += kThreads) {
        const double a = (i < ht) ? theta * (double)(128 * (int64_t)i - W) / 20.0
                                  : theta * (double)(i - ht) / 10.0;
        tab[i] = expi<V>(a);
    }
}

template <typename V>
__device__ __forceinline__ V phase_factor(const V *tab, int ht, int32_t C, int table, double theta,
                                          int64_t W)
{
    if (table) {
        // C is in [0, W] for a matching diagonal; clamp so that any other
        // input stays inside the table
        const uint32_t h = min((uint32_t)C >> 6, (uint32_t)(ht - 1));
        return cmul(tab[h], tab[ht + (C & 63)]);
    }
    return expi<V>(theta * (double)(2 * (int64_t)C - W) / 20.0);
}

template <typename V>
__device__ __forceinline__ V conj_v(V a) { return V{a.x, -a.y}; }

// Call f(r, global index) for every register r of the window.
template <int NR, typename F>
__device__ __forceinline__ void for_each_reg(const Addr &a, F &&f)
{
    if (a.fast) {
#pragma unroll
        for (int r = 0; r < NR; ++r) f(r, a.fast_idx(r));
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) f(r, a.slow_idx(r));
    }
}

// Forward butterfly stage: walk the windows of `seq`, applying RX to each
// target bit once, in the first window that holds it.
template <typename V, int NR, typename R>
__device__ __forceinline__ void run_stage(V (&v)[NR], V *lds, const WinSeq &seq, uint32_t targets,
                                          R c, R s, int &cur, int tid, int rb)
{
    uint32_t done = 0;
    for (int i = 0; i < seq.cnt; ++i) {
        const int w = seq.s[i];
        if (w != cur) {
            exchange(v, lds, cur, w, tid, rb);
            cur = w;
        }
        const uint32_t mask = targets & (((1u << rb) - 1u) << w) & ~done;
        rx_reg_mask(v, mask >> w, c, s);
        done |= mask;
    }
}

// Reverse stage on psi and lambda together: windows in reverse order; for each
// target qubit accumulate Im <lam| X_q |psi> (invariant under RX applied to
// both), then apply RX(-theta) to both.
template <typename V, int NR, typename R>
__device__ __forceinline__ void unrun_stage(V (&p)[NR], V (&l)[NR], V *lds, const WinSeq &seq,
                                            uint32_t targets, R c, R s, int &cur, int tid, int rb,
                                            double &gx)
{
    uint32_t done = 0;
    for (int i = seq.cnt - 1; i >= 0; --i) {
        const int w = seq.s[i];
        if (w != cur) {
            exchange(p, lds, cur, w, tid, rb);
            exchange(l, lds, cur, w, tid, rb);
            cur = w;
        }
        const uint32_t mask = targets & (((1u << rb) - 1u) << w) & ~done;
        gx += imx_reg_mask(l, p, mask >> w);
        rx_reg_mask(p, mask >> w, c, -s);
        rx_reg_mask(l, mask >> w, c, -s);
        done |= mask;
    }
}

template <typename V, int T>
__global__ void __launch_bounds__(kThreads) pass_kernel(PassProg pp)
{
    using R = typename Real<V>::T;
    constexpr int RB = TileCfg<T>::RB, NR = TileCfg<T>::NR;
    __shared__ V lds[TileCfg<T>::LDS];
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (kThreads / 64)];

    const int tid = threadIdx.x;
    const int64_t w = xcd_tile(pp.xcd_remap);
    const int64_t base = tile_base(w, pp.c, pp.q0, T - pp.c);
    V *psi = reinterpret_cast<V *>(pp.psi);
    const int32_t *diag = pp.diag;
    const int ht = (int)(pp.W >> 6) + 1;

    if (pp.has_phase && pp.phase_table) {
        build_phase_table(tab, ht, pp.theta_zz, pp.W, tid);
        __syncthreads();
    }

    V v[NR];
    int cur = pp.load_win;
    if (pp.init) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = V{(R)pp.amp0, (R)0};
    } else {
        for_each_reg<NR>(win_addr(tid, cur, RB, base, pp.c, pp.q0), [&](int r, int64_t g) { v[r] = psi[g]; });
    }

    if (pp.has_pre) run_stage(v, lds, pp.A, pp.targets, (R)pp.pre_c, (R)pp.pre_s, cur, tid, RB);

    if (pp.has_phase) {
        for_each_reg<NR>(win_addr(tid, cur, RB, base, pp.c, pp.q0), [&](int r, int64_t g) {
            v[r] = cmul(v[r], phase_factor<V>(tab, ht, diag[g], pp.phase_table, pp.theta_zz, pp.W));
        });
    }

    if (pp.has_post) run_stage(v, lds, pp.B, pp.targets, (R)pp.post_c, (R)pp.post_s, cur, tid, RB);

    const Addr a = win_addr(tid, cur, RB, base, pp.c, pp.q0);
    if (pp.readout) {
        double acc[2] = {0.0, 0.0};
        for_each_reg<NR>(a, [&](int r, int64_t g) {
            const double pr = (double)v[r].x * (double)v[r].x + (double)v[r].y * (double)v[r].y;
            acc[0] += pr;
            acc[1] += pr * (double)diag[g];
        });
        block_sum(acc, red, tid, kThreads);
        if (tid == 0) {
            pp.partials[w * kSlots + 0] = acc[0];
            pp.partials[w * kSlots + 1] = acc[1];
        }
    }

    for_each_reg<NR>(a, [&](int r, int64_t g) { psi[g] = v[r]; });
}

// Reverse of one forward pass.  Slots: 0 = gx of the post layer, 1 = gzz of the
// phase layer, 2 = gx of the pre layer.  Turnaround (the last forward pass):
// apply the pass, read out norm and sum |a|^2 C (slots 1, 2), form
// lambda = C psi, undo the pass on both vectors (slot 0 = gx), store lambda.
template <typename V, int T>
__global__ void __launch_bounds__(kThreads) adjoint_kernel(PassProg pp, int turnaround)
{
    using R = typename Real<V>::T;
    constexpr int RB = TileCfg<T>::RB, NR = TileCfg<T>::NR;
    __shared__ V lds[TileCfg<T>::LDS];
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (kThreads / 64)];

    const int tid = threadIdx.x;
    const int64_t w = xcd_tile(pp.xcd_remap);
    const int64_t base = tile_base(w, pp.c, pp.q0, T - pp.c);
    V *psi = reinterpret_cast<V *>(pp.psi);
    V *lam = reinterpret_cast<V *>(pp.lam);
    const int32_t *diag = pp.diag;
    const int ht = (int)(pp.W >> 6) + 1;

    if (pp.has_phase && pp.phase_table) {
        build_phase_table(tab, ht, pp.theta_zz, pp.W, tid);
        __syncthreads();
    }

    V p[NR], l[NR];
    double acc[kSlots] = {0.0, 0.0, 0.0, 0.0};
    int cur = pp.load_win;
    if (turnaround) {
        for_each_reg<NR>(win_addr(tid, cur, RB, base, pp.c, pp.q0), [&](int r, int64_t g) { p[r] = psi[g]; });
        run_stage(p, lds, pp.B, pp.targets, (R)pp.post_c, (R)pp.post_s, cur, tid, RB);
        for_each_reg<NR>(win_addr(tid, cur, RB, base, pp.c, pp.q0), [&](int r, int64_t g) {
            const int32_t C = diag[g];
            const double pr = (double)p[r].x * (double)p[r].x + (double)p[r].y * (double)p[r].y;
            acc[1] += pr;
            acc[2] += pr * (double)C;
            const R cu = (R)((double)C * 0.1);
            l[r] = V{cu * p[r].x, cu * p[r].y};
        });
        unrun_stage(p, l, lds, pp.B, pp.targets, (R)pp.post_c, (R)pp.post_s, cur, tid, RB, acc[0]);
        for_each_reg<NR>(win_addr(tid, cur, RB, base, pp.c, pp.q0), [&](int r, int64_t g) { lam[g] = l[r]; });
    } else {
        for_each_reg<NR>(win_addr(tid, cur, RB, base, pp.c, pp.q0), [&](int r, int64_t g) {
            p[r] = psi[g];
            l[r] = lam[g];
        });
        if (pp.has_post)
            unrun_stage(p, l, lds, pp.B, pp.targets, (R)pp.post_c, (R)pp.post_s, cur, tid, RB, acc[0]);
        if (pp.has_phase) {
            for_each_reg<NR>(win_addr(tid, cur, RB, base, pp.c, pp.q0), [&](int r, int64_t g) {
                const int32_t C = diag[g];
                const double im = (double)l[r].x * (double)p[r].y - (double)l[r].y * (double)p[r].x;
                acc[1] += -0.2 * (double)C * im;
                if (!pp.init) {
                    const V f = conj_v(phase_factor<V>(tab, ht, C, pp.phase_table, pp.theta_zz, pp.W));
                    p[r] = cmul(p[r], f);
                    l[r] = cmul(l[r], f);
                }
            });
        }
        if (pp.has_pre)
            unrun_stage(p, l, lds, pp.A, pp.targets, (R)pp.pre_c, (R)pp.pre_s, cur, tid, RB, acc[2]);
        if (!pp.init) {
            for_each_reg<NR>(win_addr(tid, cur, RB, base, pp.c, pp.q0), [&](int r, int64_t g) {
                psi[g] = p[r];
                lam[g] = l[r];
            });
        }
    }

    block_sum(acc, red, tid, kThreads);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) pp.partials[w * kSlots + k] = acc[k];
    }
}

}  // namespace

hipError_t launch_pass(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL((pass_kernel<float2, kTileBitsC64>), dim3((unsigned)grid), dim3(kThreads), 0, st, pp);
    else
        hipLaunchKernelGGL((pass_kernel<double2, kTileBitsC128>), dim3((unsigned)grid), dim3(kThreads), 0, st, pp);
    return hipGetLastError();
}

hipError_t launch_adjoint_pass(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL((adjoint_kernel<float2, kTileBitsC64>), dim3((unsigned)grid), dim3(kThreads), 0, st,
                           pp, turnaround);
    else
        hipLaunchKernelGGL((adjoint_kernel<double2, kTileBitsC128>), dim3((unsigned)grid), dim3(kThreads), 0, st,
                           pp, turnaround);
    return hipGetLastError();
}

}  // namespace qs
