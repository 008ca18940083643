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
//
// The launch has one workgroup per tile (the kernels also accept fewer
// workgroups and then loop over tiles).
#include "device.h"

namespace qs {

namespace {

// Phase factor of the cost layer for cut value C (tenths):
//   exp(-i theta (W - 2C)/20) = G * prod_j T_j[d_j],  C = sum_j d_j 64^j,
// with T_j[d] = exp(i theta d 64^j / 10) and G = f exp(-i theta W / 20)
// folded into T_0 (f: real factor of the kernel's tangent-form stages).  The
// digits are 6 bits wide except the top one, which takes up to 7 bits, so
// W_t < 2^13 needs two levels (one complex multiply per amplitude) and
// W_t < 2^31 at most five.  Entries are evaluated once per workgroup with
// FP64 arguments reduced modulo 2 pi.
#ifndef QS_ADJ_PREFETCH
#define QS_ADJ_PREFETCH 1
#endif

constexpr int kTabLevels = 5;
constexpr int kTabMax = 64 * (kTabLevels - 1) + 128;

// Levels needed for cut values up to W: level j < L-1 holds 64 entries at
// offset 64 j, the top level L-1 holds 128 entries at offset 64 (L-1); L levels
// cover 6 (L-1) + 7 bits.
__host__ __device__ __forceinline__ int phase_levels(int64_t W)
{
    int L = 1;
    while (L < kTabLevels && (W >> (6 * (L - 1) + 7)) != 0) ++L;
    return L;
}

template <typename V>
__device__ __forceinline__ void build_phase_table(V *tab, int levels, double theta, int64_t W, double f, int tid,
                                                  int nthreads)
{
    using R = typename Real<V>::T;
    const int top = 64 * (levels - 1);
    for (int i = tid; i < top + 128; i += nthreads) {
        const int j = i < top ? (i >> 6) : levels - 1;
        const int d = i - 64 * j;
        const double a = theta * (double)d * (double)((int64_t)1 << (6 * j)) / 10.0;
        V t = expi<V>(j == 0 ? a - theta * (double)W / 20.0 : a);
        if (j == 0) t = scale_v(t, (R)f);
        tab[i] = t;
    }
}

template <typename V>
__device__ __forceinline__ V phase_factor(const V *tab, int levels, int32_t C)
{
    // C is in [0, W] for a matching diagonal; digits are masked so that any
    // other input stays inside the table
    const uint32_t u = (uint32_t)C;
    V f = tab[u & (levels == 1 ? 127u : 63u)];
    for (int j = 1; j < levels; ++j) {
        const uint32_t d = (u >> (6 * j)) & (j == levels - 1 ? 127u : 63u);
        f = cmul(f, tab[64 * j + d]);
    }
    return f;
}

template <typename V>
__device__ __forceinline__ V conj_v(V a) { return V{a.x, -a.y}; }

// Hide a uniform value from loop-invariant code motion: without this the
// compiler keeps every per-register offset of the persistent loop live in
// scalar registers for the whole kernel and spills them.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+s"(x));
    return x;
}

struct Geom {
    int c, q0, m;
};

__device__ __forceinline__ Geom geom_of(const PassProg &pp)
{
    return Geom{opaque(pp.c), opaque(pp.q0), opaque(pp.width)};
}

// Call f(r, global index) for every register r of the window.
template <int NR, typename F>
__device__ __forceinline__ void for_each_reg(const Addr &a, F &&f)
{
#pragma unroll
    for (int r = 0; r < NR; ++r) f(r, a.fast_idx(r));
}

// Forward butterfly stage: walk the windows of `seq`, applying RX to each
// target bit once, in the first window that holds it.
template <int RB, typename V, int NR>
__device__ __forceinline__ void run_stage(V (&v)[NR], V *lds, const WinSeq &seq, uint32_t targets,
                                          const RxStage &st, int &cur, int tid)
{
    uint32_t done = 0;
    for (int i = 0; i < seq.cnt; ++i) {
        const int w = seq.s[i];
        if (w != cur) {
            exchange<RB>(v, lds, cur, w, tid);
            cur = w;
        }
        const uint32_t mask = targets & (((1u << RB) - 1u) << w) & ~done;
        stage_rx(v, mask >> w, st, 1);
        done |= mask;
    }
}

// Reverse stage on psi and lambda together: windows in reverse order; for each
// target qubit accumulate Im <lam| X_q |psi> (invariant under RX applied to
// both), then apply RX(-theta) to both.  In tangent form both vectors carry
// 1/cos^j after j qubits, so the terms are rescaled by cos^(2j).
template <int RB, typename V, int NR>
__device__ __forceinline__ void unrun_stage(V (&p)[NR], V (&l)[NR], V *lds, const WinSeq &seq,
                                            uint32_t targets, const RxStage &st, int &cur, int tid, double &gx)
{
    uint32_t done = 0;
    double sc = 1.0;
    const double c2 = st.tan ? st.c * st.c : 1.0;
    for (int i = seq.cnt - 1; i >= 0; --i) {
        const int w = seq.s[i];
        if (w != cur) {
            exchange<RB>(p, lds, cur, w, tid);
            exchange<RB>(l, lds, cur, w, tid);
            cur = w;
        }
        const uint32_t mask = targets & (((1u << RB) - 1u) << w) & ~done;
        gx += sc * imx_reg_mask(l, p, mask >> w);
        stage_rx(p, mask >> w, st, -1);
        stage_rx(l, mask >> w, st, -1);
        for (uint32_t b = mask; b; b &= b - 1) sc *= c2;
        done |= mask;
    }
}

template <typename V, int T, int TB>
__global__ void __launch_bounds__(1 << TB) pass_kernel(PassProg pp)
{
    using R = typename Real<V>::T;
    constexpr int NT = 1 << TB, RB = T - TB, NR = 1 << RB;
    __shared__ V lds[1 << T];
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (NT / 64)];

    const int tid = threadIdx.x;
    V *psi = reinterpret_cast<V *>(pp.psi);
    const int32_t *diag = pp.diag;
    const int levels = pp.phase_levels;
    const R fac = (R)pp.factor;

    if (pp.has_phase) {
        build_phase_table(tab, levels, pp.theta_zz, pp.W, pp.factor, tid, NT);
        __syncthreads();
    }

    const bool need_diag = pp.has_phase || pp.readout;
    const int dwin = pp.has_phase ? pp.phase_win : pp.final_win;
    const int64_t G = gridDim.x;
    int64_t tile = xcd_tile(pp.xcd_remap);

    double acc[2] = {0.0, 0.0};
    for (; tile < pp.ntiles; tile += G) {
        const Geom g = geom_of(pp);
        const int64_t base = tile_base(tile, g.c, g.q0, g.m);
        V v[NR];
        int32_t dg[NR];
        // the diagonal is loaded first so that its latency overlaps stage A
        if (need_diag)
            for_each_reg<NR>(win_addr(tid, opaque(dwin), RB, base, g.c, g.q0),
                             [&](int r, int64_t x) { dg[r] = diag[x]; });
        int cur = opaque(pp.load_win);
        if (pp.init) {
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r] = V{(R)pp.amp0, (R)0};
        } else {
            for_each_reg<NR>(win_addr(tid, cur, RB, base, g.c, g.q0), [&](int r, int64_t x) { v[r] = psi[x]; });
        }
        if (pp.has_pre) run_stage<RB>(v, lds, pp.A, pp.targets, pp.pre, cur, tid);
        if (pp.has_phase) {
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r] = cmul(v[r], phase_factor<V>(tab, levels, dg[r]));
        }
        if (pp.has_post) run_stage<RB>(v, lds, pp.B, pp.targets, pp.post, cur, tid);
        if (!pp.has_phase && pp.factor != 1.0) {
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r] = scale_v(v[r], fac);
        }
        if (pp.readout) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double pr = (double)v[r].x * (double)v[r].x + (double)v[r].y * (double)v[r].y;
                acc[0] += pr;
                acc[1] += pr * (double)dg[r];
            }
        }
        for_each_reg<NR>(win_addr(tid, cur, RB, base, g.c, g.q0), [&](int r, int64_t x) { psi[x] = v[r]; });
    }

    if (pp.readout) {
        block_sum(acc, red, tid, NT);
        if (tid == 0) {
            pp.partials[blockIdx.x * kSlots + 0] = acc[0];
            pp.partials[blockIdx.x * kSlots + 1] = acc[1];
        }
    }
}

// Reverse of one forward pass.  Slots: 0 = gx of the post layer, 1 = gzz of the
// phase layer, 2 = gx of the pre layer.  Turnaround (the last forward pass):
// apply the pass, read out norm and sum |a|^2 C (slots 1, 2), form
// lambda = C psi, undo the pass on both vectors (slot 0 = gx), store lambda.
template <typename V, int T, int TB, bool turnaround>
__global__ void __launch_bounds__(1 << TB) adjoint_kernel(PassProg pp)
{
    using R = typename Real<V>::T;
    constexpr int NT = 1 << TB, RB = T - TB, NR = 1 << RB;
    __shared__ V lds[1 << T];
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (NT / 64)];

    const int tid = threadIdx.x;
    V *psi = reinterpret_cast<V *>(pp.psi);
    V *lam = reinterpret_cast<V *>(pp.lam);
    const int32_t *diag = pp.diag;
    const int levels = pp.phase_levels;
    const R fpre = (R)pp.fpre, fpost = (R)pp.fpost;

    if (pp.has_phase) {
        build_phase_table(tab, levels, pp.theta_zz, pp.W, 1.0, tid, NT);
        __syncthreads();
    }

    double acc[kSlots] = {0.0, 0.0, 0.0, 0.0};
    const int64_t G = gridDim.x;
    int64_t tile = xcd_tile(pp.xcd_remap);
    if constexpr (turnaround) {
        for (; tile < pp.ntiles; tile += G) {
            const Geom gg = geom_of(pp);
            const int64_t base = tile_base(tile, gg.c, gg.q0, gg.m);
            V p[NR], l[NR];
            int cur = opaque(pp.load_win);
            for_each_reg<NR>(win_addr(tid, cur, RB, base, gg.c, gg.q0), [&](int r, int64_t g) { p[r] = psi[g]; });
            run_stage<RB>(p, lds, pp.B, pp.targets, pp.post, cur, tid);
            for_each_reg<NR>(win_addr(tid, cur, RB, base, gg.c, gg.q0), [&](int r, int64_t g) {
                const int32_t C = diag[g];
                p[r] = scale_v(p[r], fpost);
                const double pr = (double)p[r].x * (double)p[r].x + (double)p[r].y * (double)p[r].y;
                acc[1] += pr;
                acc[2] += pr * (double)C;
                l[r] = scale_v(p[r], (R)((double)C * 0.1));
            });
            unrun_stage<RB>(p, l, lds, pp.B, pp.targets, pp.post, cur, tid, acc[0]);
            for_each_reg<NR>(win_addr(tid, cur, RB, base, gg.c, gg.q0),
                             [&](int r, int64_t g) { lam[g] = scale_v(l[r], fpost); });
        }
    } else {
        V p[NR], l[NR];
#if QS_ADJ_PREFETCH
        V np[NR], nl[NR];
#endif
        auto fetch = [&](int64_t t, V (&dp)[NR], V (&dl)[NR]) {
            const Geom gg = geom_of(pp);
            const int64_t base = tile_base(t, gg.c, gg.q0, gg.m);
            for_each_reg<NR>(win_addr(tid, opaque(pp.load_win), RB, base, gg.c, gg.q0), [&](int r, int64_t g) {
                dp[r] = psi[g];
                dl[r] = lam[g];
            });
        };
#if QS_ADJ_PREFETCH
        if (tile < pp.ntiles) fetch(tile, p, l);
#endif
        for (; tile < pp.ntiles; tile += G) {
            const Geom gg = geom_of(pp);
            const int64_t base = tile_base(tile, gg.c, gg.q0, gg.m);
            int cur = opaque(pp.load_win);
            // this tile's diagonal is requested before the next tile's vectors:
            // memory counters retire in order, so the phase step then waits
            // only for these loads
            int32_t dg[NR];
            if (pp.has_phase) {
                const int pw = opaque(pp.phase_win);
                for_each_reg<NR>(win_addr(tid, pw, RB, base, gg.c, gg.q0), [&](int r, int64_t g) { dg[r] = diag[g]; });
            }
#if QS_ADJ_PREFETCH
            if (tile + G < pp.ntiles) fetch(tile + G, np, nl);
#else
            fetch(tile, p, l);
#endif
            if (pp.has_post) {
                unrun_stage<RB>(p, l, lds, pp.B, pp.targets, pp.post, cur, tid, acc[0]);
                if (pp.post.tan) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        p[r] = scale_v(p[r], fpost);
                        l[r] = scale_v(l[r], fpost);
                    }
                }
            }
            if (pp.has_phase) {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int32_t C = dg[r];
                    const R im = l[r].x * p[r].y - l[r].y * p[r].x;
                    acc[1] += -0.2 * (double)C * (double)im;
                    if (!pp.init) {
                        const V f = conj_v(phase_factor<V>(tab, levels, C));
                        p[r] = cmul(p[r], f);
                        l[r] = cmul(l[r], f);
                    }
                }
            }
            if (pp.has_pre) {
                unrun_stage<RB>(p, l, lds, pp.A, pp.targets, pp.pre, cur, tid, acc[2]);
                if (pp.pre.tan) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        p[r] = scale_v(p[r], fpre);
                        l[r] = scale_v(l[r], fpre);
                    }
                }
            }
            if (!pp.init) {
                for_each_reg<NR>(win_addr(tid, cur, RB, base, gg.c, gg.q0), [&](int r, int64_t g) {
                    psi[g] = p[r];
                    lam[g] = l[r];
                });
            }
#if QS_ADJ_PREFETCH
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                p[r] = np[r];
                l[r] = nl[r];
            }
#endif
        }
    }

    block_sum(acc, red, tid, NT);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) pp.partials[blockIdx.x * kSlots + k] = acc[k];
    }
}

}  // namespace

int phase_table_levels(int64_t W) { return phase_levels(W); }

int64_t pass_grid(int prec, int adjoint, int64_t ntiles)
{
    // One tile per workgroup: the hardware dispatcher's dynamic assignment of
    // workgroups to CUs overlaps loads, butterflies and stores across
    // workgroups better than a persistent loop (measured on MI355X).
    (void)prec;
#if QS_ADJ_PREFETCH
    if (adjoint == 2) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        return (int64_t)cus < ntiles ? (int64_t)cus : ntiles;
    }
#endif
    (void)adjoint;
    return ntiles;
}

hipError_t launch_pass(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    constexpr int FT = kFwdThreadBits;
    if (prec == 0)
        hipLaunchKernelGGL((pass_kernel<float2, kTileBitsC64, FT>), dim3((unsigned)grid), dim3(1 << FT), 0, st, pp);
    else
        hipLaunchKernelGGL((pass_kernel<double2, kTileBitsC128, FT>), dim3((unsigned)grid), dim3(1 << FT), 0, st,
                           pp);
    return hipGetLastError();
}

hipError_t launch_adjoint_pass(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    constexpr int AT = kAdjThreadBits;
    const dim3 g((unsigned)grid), b(1 << AT);
    if (prec == 0) {
        if (turnaround) hipLaunchKernelGGL((adjoint_kernel<float2, kTileBitsC64, AT, true>), g, b, 0, st, pp);
        else hipLaunchKernelGGL((adjoint_kernel<float2, kTileBitsC64, AT, false>), g, b, 0, st, pp);
    } else {
        if (turnaround) hipLaunchKernelGGL((adjoint_kernel<double2, kTileBitsC128, AT, true>), g, b, 0, st, pp);
        else hipLaunchKernelGGL((adjoint_kernel<double2, kTileBitsC128, AT, false>), g, b, 0, st, pp);
    }
    return hipGetLastError();
}

}  // namespace qs
