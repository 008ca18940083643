// Tile-level device code shared by the single-circuit pass kernels and the
// batched kernel: phase tables, butterfly stages, and the bodies that process
// one tile of a forward pass, of the turnaround pass and of a reverse pass.
//
// A layer of the circuit (arXiv:2604.26423, Sec. II-B) is the cost unitary of
// eq. (2), a diagonal phase exp(-i theta_zz (W - 2C(x))/20) once the
// n(n-1)/2 commuting RZZ gates are combined, followed by the mixer of
// eq. (3), RX(theta_x) on every qubit.  The RX gates commute, so one pass over
// memory applies all of them for the T qubits of a tile: a tile of 2^T
// amplitudes sits in registers (2^(T-TB) per thread of a 2^TB-thread
// workgroup), butterflies act on the tile bits held in registers, and LDS
// exchanges rotate other tile bits into registers.  The cost phase is
// elementwise, so it is applied inside a pass, between the butterflies of one
// layer and the next (the "pre" and "post" stages).
#pragma once

#include "device.h"

namespace qs {

// Phase factor of the cost layer for cut value C (tenths):
//   exp(-i theta (W - 2C)/20) = G * prod_j T_j[d_j],  C = sum_j d_j 64^j,
// with T_j[d] = exp(i theta d 64^j / 10) and G = f exp(-i theta W / 20)
// folded into T_0 (f: real factor of the kernel's tangent-form stages).  The
// digits are 6 bits wide except the top one, which takes up to 7 bits, so
// W_t < 2^13 needs two levels (one complex multiply per amplitude) and
// W_t < 2^31 at most five.  Entries are evaluated once per workgroup with
// FP64 arguments reduced modulo 2 pi.
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

// Phase factors of a thread's NR amplitudes, level by level.  The loop over
// levels is uniform and each level's table reads for all registers issue
// together (a per-amplitude loop over levels would branch and wait once per
// amplitude).
template <typename V, int NR>
__device__ __forceinline__ void phase_factors(const V *tab, int levels, const int32_t (&C)[NR], V (&f)[NR])
{
    const uint32_t m0 = levels == 1 ? 127u : 63u;
#pragma unroll
    for (int r = 0; r < NR; ++r) f[r] = tab[(uint32_t)C[r] & m0];
#pragma unroll 1
    for (int j = 1; j < levels; ++j) {
        const uint32_t mj = j == levels - 1 ? 127u : 63u;
#pragma unroll
        for (int r = 0; r < NR; ++r) f[r] = cmul(f[r], tab[64 * j + (((uint32_t)C[r] >> (6 * j)) & mj)]);
    }
}

// v[r] *= conj(phase factor of C[r]) for two vectors, a quarter of the
// registers at a time: the runtime loop over levels carries only that
// quarter's factors, not the two vectors.
template <typename V, int NR>
__device__ __forceinline__ void unphase_quarters(const V *tab, int levels, const int32_t (&C)[NR], V (&a)[NR],
                                               V (&b)[NR])
{
    constexpr int H = NR >= 4 ? NR / 4 : 1;
#pragma unroll
    for (int h = 0; h < NR; h += H) {
        int32_t c[H];
        V f[H];
#pragma unroll
        for (int i = 0; i < H; ++i) c[i] = C[h + i];
        phase_factors(tab, levels, c, f);
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const V t = conj_v(f[i]);
            a[h + i] = cmul(a[h + i], t);
            b[h + i] = cmul(b[h + i], t);
        }
    }
}

// Hide a uniform value from loop-invariant code motion: without this the
// compiler keeps every per-register offset of the persistent loop live in
// scalar registers for the whole kernel and spills them.
__device__ __forceinline__ int opaque(int x)
{
    x = __builtin_amdgcn_readfirstlane(x);  // uniform by construction
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

// Call f(r, memory element) for every register r of the window (the
// element of global index a.fast_idx(r) in the swizzled layout).
template <int NR, typename F>
__device__ __forceinline__ void for_each_reg(const Addr &a, F &&f)
{
    const int64_t tgs = swz(a.tg);
    // The register part is uniform: compute its swizzle on the scalar unit.
    // readfirstlane also keeps the compiler from merging it into the
    // per-thread part, which would redo the fold per register in vector ALU.
    const int sh = __builtin_amdgcn_readfirstlane(a.sh);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int64_t o = swz((int64_t)r << sh);
        const int64_t off = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(o >> 32)) << 32) |
                                      (uint32_t)__builtin_amdgcn_readfirstlane((int)(o & 0xffffffff)));
        f(r, tgs ^ off);
    }
}

// Factors of a stage inside window w (register bits [w, w + RB)): single
// targets, and two-bit factors whose both bits lie in the window.
template <int RB>
__device__ __forceinline__ uint32_t win_singles(uint32_t targets, int w)
{
    return targets & (((1u << RB) - 1u) << w);
}
template <int RB>
__device__ __forceinline__ uint32_t win_pairs(uint32_t pairs, int w)
{
    return pairs & (((1u << (RB - 1)) - 1u) << w);
}

// Stage code paths.  kModeGeneral handles any stage with runtime branches per
// register bit; the tangent modes (every stage of the pass in tangent form)
// are branch-free: kModeTan for single-qubit factors anywhere in a window,
// kModeTanSym for the complement-symmetric layout (two-bit factors anywhere,
// single factors only at the window ends).
enum : int { kModeGeneral = 0, kModeTan = 1, kModeTanSym = 2 };

// Pass shapes: which parts a pass has.  A kernel instantiated for a shape
// (SH >= 0) has no runtime branch on them, so the compiler does not copy the
// register arrays at their joins; SH = -1 reads them from the PassProg.
enum : int { kShPre = 1, kShPhase = 2, kShPost = 4, kShInit = 8, kShReadout = 16 };

__host__ __device__ __forceinline__ int pass_shape(const PassProg &pp)
{
    return (pp.has_pre ? kShPre : 0) | (pp.has_phase ? kShPhase : 0) | (pp.has_post ? kShPost : 0) |
           (pp.init ? kShInit : 0) | (pp.readout ? kShReadout : 0);
}

template <int MODE, typename V, int NR>
__device__ __forceinline__ void apply_window(V (&v)[NR], uint32_t mask, uint32_t pmask, const RxStage &st, int sign)
{
    if constexpr (MODE == kModeGeneral) {
        stage_rx(v, mask, pmask, st, sign);
    } else {
        using R = typename Real<V>::T;
        const R u = (R)(sign * st.u);
        if constexpr (MODE == kModeTan) {
            rxt_reg_all(v, mask, u);
        } else {
            rxt_reg_ends(v, mask, u);
            rxt_reg_pairs_all(v, pmask, u);
        }
    }
}

template <int MODE, typename V, int NR>
__device__ __forceinline__ double imx_window(const V (&l)[NR], const V (&p)[NR], uint32_t mask, uint32_t pmask)
{
    if constexpr (MODE == kModeGeneral) {
        double g = imx_reg_mask(l, p, mask);
        if (pmask) g += imx_reg_pairs(l, p, pmask);
        return g;
    } else if constexpr (MODE == kModeTan) {
        return imx_reg_all(l, p, mask);
    } else {
        return imx_reg_ends(l, p, mask) + imx_reg_pairs_all(l, p, pmask);
    }
}

// Register bits that the last visited window of a stage updates when the
// kernel fixes the stage's tail at compile time (stage_tail in plan.h):
// TAIL = +k the lowest k, TAIL = -k the highest k.
template <int RB, int TAIL>
constexpr uint32_t tail_mask()
{
    constexpr int k = TAIL > 0 ? TAIL : -TAIL;
    return TAIL > 0 ? (1u << k) - 1u : ((1u << k) - 1u) << (RB - k);
}

// Forward butterfly stage: walk the windows of `seq`, applying each factor
// once, in the first window that holds it.  The first window of every stage
// is the current layout and consecutive windows differ (checked on the host),
// so the branch-free modes exchange unconditionally from the second window on.
// TAIL != 0 (tangent form, single factors only): every window but the last
// applies all its register bits and the last those of tail_mask, fixed at
// compile time, so no idle bit is updated with a zero angle.
template <int RB, int MODE, int TAIL = 0, typename V, int NR>
__device__ __forceinline__ void run_stage(V (&v)[NR], V *lds, const WinSeq &seq, uint32_t targets, uint32_t pairs,
                                          const RxStage &st, int &cur, int tid)
{
    if constexpr (TAIL != 0) {
        static_assert(MODE == kModeTan, "compile-time tails are for single-factor tangent-form stages");
        using R = typename Real<V>::T;
        const R u = (R)st.u;
        const int last = seq.cnt - 1;
        // window indices go through opaque(): the peeled last window's layout
        // is loop-invariant across tiles, and hoisted its per-register LDS
        // offsets would occupy scalar registers for the whole kernel
        for (int i = 0; i < last; ++i) {
            if (i > 0) {
                const int w = opaque(seq.s[i]);
                exchange<RB>(v, lds, cur, w, tid);
                cur = w;
            }
            rxt_reg_const<(1u << RB) - 1u>(v, u);
        }
        if (last > 0) {
            const int w = opaque(seq.s[last]);
            exchange<RB>(v, lds, cur, w, tid);
            cur = w;
        }
        rxt_reg_const<tail_mask<RB, TAIL>()>(v, u);
        return;
    }
    uint32_t done = 0, pdone = 0;
    for (int i = 0; i < seq.cnt; ++i) {
        const int w = seq.s[i];
        if constexpr (MODE == kModeGeneral) {
            if (w != cur) {
                exchange<RB>(v, lds, cur, w, tid);
                cur = w;
            }
        } else if (i > 0) {
            exchange<RB>(v, lds, cur, w, tid);
            cur = w;
        }
        const uint32_t mask = win_singles<RB>(targets, w) & ~done;
        const uint32_t pm = win_pairs<RB>(pairs, w) & ~pdone;
        apply_window<MODE>(v, mask >> w, pm >> w, st, 1);
        done |= mask;
        pdone |= pm;
    }
}

// Reverse stage on psi and lambda together: windows in reverse order; for each
// factor accumulate Im <lam| X.. |psi> (invariant under the stage applied to
// both), then apply RX(-theta) to both.  In tangent form both vectors carry
// 1/cos^j after j factors, so the terms of window i are rescaled by
// st.wsc[i] = cos^(2j) (evaluated on the host).
template <int RB, int MODE, bool PAIR, int TAIL = 0, typename V, int NR>
__device__ __forceinline__ void unrun_stage(V (&p)[NR], V (&l)[NR], V *lds, const WinSeq &seq,
                                            uint32_t targets, uint32_t pairs, const RxStage &st, int &cur, int tid,
                                            double &gx)
{
    if constexpr (TAIL != 0) {
        // windows in reverse order; all but the last visited (index 0) full
        static_assert(MODE == kModeTan, "compile-time tails are for single-factor tangent-form stages");
        using R = typename Real<V>::T;
        constexpr uint32_t FULL = (1u << RB) - 1u, LAST = tail_mask<RB, TAIL>();
        const R u = (R)(-st.u);
        auto to = [&](int w) {
            if constexpr (PAIR) {
                exchange2<RB>(p, l, lds, cur, w, tid);
            } else {
                exchange<RB>(p, lds, cur, w, tid);
                exchange<RB>(l, lds, cur, w, tid);
            }
            cur = w;
        };
        for (int i = seq.cnt - 1; i > 0; --i) {
            if (i < seq.cnt - 1) to(opaque(seq.s[i]));
            gx += st.wsc[i] * imx_reg_const<FULL>(l, p);
            rxt_reg_const<FULL>(p, u);
            rxt_reg_const<FULL>(l, u);
        }
        if (seq.cnt > 1) to(opaque(seq.s[0]));  // (opaque: see run_stage)
        gx += st.wsc[0] * imx_reg_const<LAST>(l, p);
        rxt_reg_const<LAST>(p, u);
        rxt_reg_const<LAST>(l, u);
        return;
    }
    uint32_t done = 0, pdone = 0;
    for (int i = seq.cnt - 1; i >= 0; --i) {
        const int w = seq.s[i];
        if (MODE == kModeGeneral ? w != cur : i < seq.cnt - 1) {
            if constexpr (PAIR) {
                exchange2<RB>(p, l, lds, cur, w, tid);  // LDS holds two tiles
            } else {
                exchange<RB>(p, lds, cur, w, tid);
                exchange<RB>(l, lds, cur, w, tid);
            }
            cur = w;
        }
        const uint32_t mask = win_singles<RB>(targets, w) & ~done;
        const uint32_t pm = win_pairs<RB>(pairs, w) & ~pdone;
        gx += st.wsc[i] * imx_window<MODE>(l, p, mask >> w, pm >> w);
        apply_window<MODE>(p, mask >> w, pm >> w, st, -1);
        apply_window<MODE>(l, mask >> w, pm >> w, st, -1);
        done |= mask;
        pdone |= pm;
    }
}

template <typename V, int T, int TB> struct TileCfg {
    using R = typename Real<V>::T;
    static constexpr int NT = 1 << TB, RB = T - TB, NR = 1 << RB;
};

// C_t of the thread's registers in window s, evaluated from the pass's cut
// table (see the cut-value notes in internal.h): the tile row and the
// register terms are uniform (scalar loads), the thread's entries are two
// vector loads, and each register then costs two integer adds.
template <int T, int TB, int NR>
__device__ __forceinline__ void cut_values(const PassProg &pp, int64_t tile, int s, int tid, int32_t (&C)[NR])
{
    constexpr int RB = T - TB;
    const uint32_t *ct = reinterpret_cast<const uint32_t *>(pp.ctab);
    const uint32_t *row = ct + kCtTile + tile * 16;
    const uint32_t *ent = ct + kCtThr + tid * 8;
    uint32_t c0 = row[0] + ent[0];
#pragma unroll
    for (int b = 0; b < TB; ++b) {
        const uint32_t db = row[1 + (b < s ? b : b + RB)];  // thread bit b is tile bit b or b + RB
        c0 -= ((tid >> b) & 1) ? 2u * db : 0u;
    }
    uint32_t a[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) a[k] = 0u - 2u * (row[1 + s + k] + ent[1 + k]);
    uint32_t P[NR];
    P[0] = c0;
#pragma unroll
    for (int r = 1; r < NR; ++r) {
        const int t = 31 - __builtin_clz(r);
        P[r] = P[r ^ (1 << t)] + a[t];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) C[r] = (int32_t)(P[r] + ct[kCtCreg + r]);
}

// C_t of the thread's registers in window s, loaded from the diagonal.
template <int T, int TB, int NR>
__device__ __forceinline__ void load_diag(const PassProg &pp, int s, int64_t base, int c, int q0, int tid,
                                          int32_t (&C)[NR])
{
    for_each_reg<NR>(win_addr(tid, s, T - TB, base, c, q0), [&](int r, int64_t x) { C[r] = pp.diag[x]; });
}

// C_t of the thread's registers in window s: from the cut table when the pass
// has a valid one, else loaded from the diagonal.
template <int T, int TB, int NR>
__device__ __forceinline__ void load_cut(const PassProg &pp, int64_t tile, int s, int64_t base, int c, int q0,
                                         int tid, int32_t (&C)[NR])
{
    if (pp.ctab && pp.ctab[kCtValid]) cut_values<T, TB>(pp, tile, s, tid, C);
    else load_diag<T, TB>(pp, s, base, c, q0, tid, C);
}

// Copy a phase table built in global memory into LDS.
template <typename V>
__device__ __forceinline__ void load_phase_table(V *tab, const V *src, int levels, int tid, int nthreads)
{
    const int n = 64 * (levels - 1) + 128;
    for (int i = tid; i < n; i += nthreads) tab[i] = src[i];
}

// Forward pass on one tile; with pp.readout, acc += (sum |a|^2, sum |a|^2 C_t).
// K > 0 (a fixed shape SH in tangent form): the stages' tails are fixed at
// compile time, +K for the first stage and -K for the second (run_stage).
template <typename V, int T, int TB, int MODE = kModeGeneral, int SH = -1, int K = 0>
__device__ __forceinline__ void fwd_tile(const PassProg &pp, int64_t tile, V *lds, const V *tab, double (&acc)[2],
                                         int tid)
{
    using Cfg = TileCfg<V, T, TB>;
    using R = typename Cfg::R;
    constexpr int RB = Cfg::RB, NR = Cfg::NR;
    constexpr bool KS = SH >= 0;
    const bool has_pre = KS ? (SH & kShPre) != 0 : pp.has_pre != 0;
    const bool has_phase = KS ? (SH & kShPhase) != 0 : pp.has_phase != 0;
    const bool has_post = KS ? (SH & kShPost) != 0 : pp.has_post != 0;
    const bool init = KS ? (SH & kShInit) != 0 : pp.init != 0;
    const bool readout = KS ? (SH & kShReadout) != 0 : pp.readout != 0;
    const V *psi = reinterpret_cast<const V *>(pp.psi);
    V *out = reinterpret_cast<V *>(pp.psi_out);
    const bool need_diag = has_phase || readout;
    const int dwin = has_phase ? pp.phase_win : pp.final_win;
    const Geom g = geom_of(pp);
    const int64_t base = tile_base(tile, g.c, g.q0, g.m);
    // A pass of the full layout that only applies a stage streams the state
    // with nontemporal loads and stores (measured: plain passes 9% faster, the
    // n = 32 forward 4%, the complex128 one 4-12%).  The passes that apply a
    // phase or read out ran up to 14% slower with them, and the
    // complement-symmetric layout (two-bit factors) 6% slower, so those keep
    // ordinary accesses.
    const bool stream = !has_phase && !readout && !pp.pairs;
    V v[NR];
    int32_t dg[NR];
    // C_t first, so that the latency of its loads overlaps stage A
    if (need_diag) load_cut<T, TB>(pp, tile, opaque(dwin), base, g.c, g.q0, tid, dg);
    int cur = opaque(pp.load_win);
    if (init) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = V{(R)pp.amp0, (R)0};
    } else if (stream) {
        for_each_reg<NR>(win_addr(tid, cur, RB, base, g.c, g.q0), [&](int r, int64_t x) { v[r] = load_nt(&psi[x]); });
    } else {
        for_each_reg<NR>(win_addr(tid, cur, RB, base, g.c, g.q0), [&](int r, int64_t x) { v[r] = psi[x]; });
    }
    static_assert(K == 0 || (SH >= 0 && MODE == kModeTan), "compile-time tails need a fixed tangent-form shape");
    constexpr int TAIL_B = K == 0 ? 0 : ((SH & kShPre) != 0 ? -K : K);  // B is the second stage after A
    if (has_pre) run_stage<RB, MODE, K>(v, lds, pp.A, pp.targets, pp.pairs, pp.pre, cur, tid);
    if (has_phase) {
        V f[NR];
        phase_factors(tab, pp.phase_levels, dg, f);
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = cmul(v[r], f[r]);
    }
    if (has_post) run_stage<RB, MODE, TAIL_B>(v, lds, pp.B, pp.targets, pp.pairs, pp.post, cur, tid);
    // tangent-form factor of a pass without a phase table (scaling by 1 when
    // it is 1 costs less than a branch in a fixed-shape kernel)
    if (!has_phase && (KS || pp.factor != 1.0)) {
        const R fac = (R)pp.factor;
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = scale_v(v[r], fac);
    }
    if (readout) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double pr = (double)v[r].x * (double)v[r].x + (double)v[r].y * (double)v[r].y;
            acc[0] += pr;
            acc[1] += pr * (double)dg[r];
        }
    }
    if (stream)
        for_each_reg<NR>(win_addr(tid, cur, RB, base, g.c, g.q0), [&](int r, int64_t x) { store_nt(&out[x], v[r]); });
    else
        for_each_reg<NR>(win_addr(tid, cur, RB, base, g.c, g.q0), [&](int r, int64_t x) { out[x] = v[r]; });
}

// Turnaround on one tile: apply the last forward pass, read out the norm and
// sum |a|^2 C_t (acc[1], acc[2]), form lambda = (C - c) psi (C and c in
// weight units, c = pp.lam_shift / 10), undo the pass on both vectors
// (acc[0] += gx of the pass's layer) and store lambda only.
//
// Any constant c gives the same gradients: the reverse sweep applies the same
// unitaries to both vectors, so the c psi part of lambda adds
// c Im <psi_k| X_q |psi_k> and c Im <psi_k| C |psi_k> to the mixer and cost
// terms, and both vanish (<psi|X_q|psi> and <psi|C|psi> are real).  Likewise
// the phase-gradient weights may be C - c for any c, since Im <lam_k|psi_k> =
// Im <psi|(C - c)|psi> = 0.  With c = W_t / 2 (the mean cut over all
// bitstrings) the terms, and with them the rounding of a complex64 sweep, are
// several times smaller than with c = 0, where they are of the size of <C>
// and cancel to a gradient of order 1.  Split
// into loads (psi in the load layout, C_t in the final layout) and
// the rest, so that a persistent kernel can load the next tile early.
template <typename V, int T, int TB>
__device__ __forceinline__ void turn_load(const PassProg &pp, int64_t tile, V (&p)[TileCfg<V, T, TB>::NR], int tid)
{
    using Cfg = TileCfg<V, T, TB>;
    const V *psi = reinterpret_cast<const V *>(pp.psi);
    const Geom gg = geom_of(pp);
    const int64_t base = tile_base(tile, gg.c, gg.q0, gg.m);
    for_each_reg<Cfg::NR>(win_addr(tid, opaque(pp.load_win), Cfg::RB, base, gg.c, gg.q0),
                          [&](int r, int64_t g) { p[r] = psi[g]; });
}

template <typename V, int T, int TB>
__device__ __forceinline__ void turn_load_diag(const PassProg &pp, int64_t tile, int32_t (&dg)[TileCfg<V, T, TB>::NR],
                                               int tid)
{
    const Geom gg = geom_of(pp);
    const int64_t base = tile_base(tile, gg.c, gg.q0, gg.m);
    load_cut<T, TB>(pp, tile, opaque(pp.final_win), base, gg.c, gg.q0, tid, dg);
}

template <typename V, int T, int TB, int MODE = kModeGeneral, bool PAIR = true, int K = 0>
__device__ __forceinline__ void turn_compute(const PassProg &pp, int64_t tile, V (&p)[TileCfg<V, T, TB>::NR],
                                             const int32_t (&dg)[TileCfg<V, T, TB>::NR], V *lds,
                                             double (&acc)[kSlots], int tid)
{
    using Cfg = TileCfg<V, T, TB>;
    using R = typename Cfg::R;
    constexpr int RB = Cfg::RB, NR = Cfg::NR;
    V *lam = reinterpret_cast<V *>(pp.lam);
    const R fpost = (R)pp.fpost;
    const Geom gg = geom_of(pp);
    const int64_t base = tile_base(tile, gg.c, gg.q0, gg.m);
    V l[NR];
    int cur = opaque(pp.load_win);
    // K > 0: the stage forward ends in +K, its reverse in -K (fixed at compile time)
    run_stage<RB, MODE, K>(p, lds, pp.B, pp.targets, pp.pairs, pp.post, cur, tid);
    // cur is now the final layout, the one C_t was obtained in
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int32_t C = dg[r];
        p[r] = scale_v(p[r], fpost);
        const double pr = (double)p[r].x * (double)p[r].x + (double)p[r].y * (double)p[r].y;
        acc[1] += pr;
        acc[2] += pr * (double)C;
        l[r] = scale_v(p[r], (R)(((double)C - pp.lam_shift) * 0.1));
    }
    unrun_stage<RB, MODE, PAIR, -K>(p, l, lds, pp.B, pp.targets, pp.pairs, pp.post, cur, tid, acc[0]);
    for_each_reg<NR>(win_addr(tid, cur, RB, base, gg.c, gg.q0),
                     [&](int r, int64_t g) { lam[g] = scale_v(l[r], fpost); });
}

template <typename V, int T, int TB, int MODE = kModeGeneral, int K = 0>
__device__ __forceinline__ void turn_tile(const PassProg &pp, int64_t tile, V *lds, double (&acc)[kSlots], int tid)
{
    constexpr int NR = TileCfg<V, T, TB>::NR;
    V p[NR];
    int32_t dg[NR];
    turn_load_diag<V, T, TB>(pp, tile, dg, tid);
    turn_load<V, T, TB>(pp, tile, p, tid);
    turn_compute<V, T, TB, MODE, true, K>(pp, tile, p, dg, lds, acc, tid);
}

// Reverse pass, loads: psi and lambda of a tile in the pass's load layout, and
// C_t in the layout of the phase step.
template <typename V, int T, int TB>
__device__ __forceinline__ void rev_load_vectors(const PassProg &pp, int64_t tile, V (&p)[TileCfg<V, T, TB>::NR],
                                                 V (&l)[TileCfg<V, T, TB>::NR], int tid)
{
    using Cfg = TileCfg<V, T, TB>;
    const V *psi = reinterpret_cast<const V *>(pp.psi);
    const V *lam = reinterpret_cast<const V *>(pp.lam);
    const Geom gg = geom_of(pp);
    const int64_t base = tile_base(tile, gg.c, gg.q0, gg.m);
    for_each_reg<Cfg::NR>(win_addr(tid, opaque(pp.load_win), Cfg::RB, base, gg.c, gg.q0), [&](int r, int64_t g) {
        p[r] = psi[g];
        l[r] = lam[g];
    });
}

template <typename V, int T, int TB>
__device__ __forceinline__ void rev_load_diag(const PassProg &pp, int64_t tile, int32_t (&dg)[TileCfg<V, T, TB>::NR],
                                              int tid)
{
    const Geom gg = geom_of(pp);
    const int64_t base = tile_base(tile, gg.c, gg.q0, gg.m);
    load_cut<T, TB>(pp, tile, opaque(pp.phase_win), base, gg.c, gg.q0, tid, dg);
}

// Reverse pass, compute and store.  acc[0] += gx of the post layer, acc[1] +=
// gzz of the phase layer, acc[2] += gx of the pre layer.  The reverse of the
// first forward pass (init) only accumulates and writes nothing; with
// pp.psi_out null only lambda is stored (checkpointed psi).  LATE: dg is
// loaded here at the phase point rather than by the caller.
template <typename V, int T, int TB, int MODE = kModeGeneral, int SH = -1, bool PAIR = true, bool LATE = false,
          int K = 0>
__device__ __forceinline__ void rev_tile(const PassProg &pp, int64_t tile, V (&p)[TileCfg<V, T, TB>::NR],
                                         V (&l)[TileCfg<V, T, TB>::NR], int32_t (&dg)[TileCfg<V, T, TB>::NR],
                                         V *lds, const V *tab, double (&acc)[kSlots], int tid)
{
    using Cfg = TileCfg<V, T, TB>;
    using R = typename Cfg::R;
    constexpr int RB = Cfg::RB, NR = Cfg::NR;
    constexpr bool KS = SH >= 0;
    constexpr bool TAN = MODE != kModeGeneral;  // every stage in tangent form
    const bool has_pre = KS ? (SH & kShPre) != 0 : pp.has_pre != 0;
    const bool has_phase = KS ? (SH & kShPhase) != 0 : pp.has_phase != 0;
    const bool has_post = KS ? (SH & kShPost) != 0 : pp.has_post != 0;
    const bool init = KS ? (SH & kShInit) != 0 : pp.init != 0;
    V *psi = reinterpret_cast<V *>(pp.psi_out);
    V *lam = reinterpret_cast<V *>(pp.lam);
    const R fpre = (R)pp.fpre, fpost = (R)pp.fpost;
    const Geom gg = geom_of(pp);
    const int64_t base = tile_base(tile, gg.c, gg.q0, gg.m);
    int cur = opaque(pp.load_win);
    // In tangent form, when the pass undoes a phase layer, the stages' real
    // factors fpost * fpre sit in the phase table (one scale per factor
    // instead of one per amplitude of each vector, see the kernel); the
    // gradient sums taken on the vectors without fpost (phase point) or with
    // an extra fpre (pre stage) are corrected by fpost^2 and 1 / fpre^2.
    const bool fold = TAN && has_phase && !init;
    // K > 0 (a fixed tangent-form shape): the post stage, undone first, ends
    // in +K when the pre stage follows it and in -K when it is the only stage
    static_assert(K == 0 || (SH >= 0 && MODE == kModeTan), "compile-time tails need a fixed tangent-form shape");
    constexpr int TAIL_B = K == 0 ? 0 : ((SH & kShPre) != 0 ? K : -K);
    if (has_post) {
        unrun_stage<RB, MODE, PAIR, TAIL_B>(p, l, lds, pp.B, pp.targets, pp.pairs, pp.post, cur, tid, acc[0]);
        if ((TAN || pp.post.tan) && !fold) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                p[r] = scale_v(p[r], fpost);
                l[r] = scale_v(l[r], fpost);
            }
        }
    }
    if (has_phase) {
        // (the late load reads the diagonal: within the one-tile junction's 128
        // registers the cut table's terms would spill)
        if constexpr (LATE) load_diag<T, TB>(pp, opaque(pp.phase_win), base, gg.c, gg.q0, tid, dg);
        // sum of (C - c) Im(conj(l) p) over the thread's amplitudes (c: see
        // turn_compute): each amplitude's Im(conj(l) p) in the state
        // precision, the products with C - c and their sum in FP64
        const double cs = pp.lam_shift;
        double gz = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            R im = l[r].x * p[r].y;
            im = fma(-l[r].y, p[r].x, im);
            gz = fma((double)dg[r] - cs, (double)im, gz);
        }
        // pin the sum here: sunk past the next stage, it would keep the
        // vectors' values at the phase point live through that stage
        asm volatile("" : "+v"(gz));
        acc[1] += -0.2 * gz * (fold && has_post ? pp.fpost * pp.fpost : 1.0);
        if (!init) unphase_quarters(tab, pp.phase_levels, dg, p, l);
    }
    if (has_pre) {
        double gpre = 0.0;
        unrun_stage<RB, MODE, PAIR, -K>(p, l, lds, pp.A, pp.targets, pp.pairs, pp.pre, cur, tid, gpre);
        acc[2] += fold ? gpre / (pp.fpre * pp.fpre) : gpre;
        if ((TAN || pp.pre.tan) && !fold) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                p[r] = scale_v(p[r], fpre);
                l[r] = scale_v(l[r], fpre);
            }
        }
    }
    if (!init) {
        if (psi) {
            for_each_reg<NR>(win_addr(tid, cur, RB, base, gg.c, gg.q0), [&](int r, int64_t g) {
                psi[g] = p[r];
                lam[g] = l[r];
            });
        } else {  // psi of the next reverse pass comes from a checkpoint
            for_each_reg<NR>(win_addr(tid, cur, RB, base, gg.c, gg.q0),
                             [&](int r, int64_t g) { lam[g] = l[r]; });
        }
    }
}

}  // namespace qs
