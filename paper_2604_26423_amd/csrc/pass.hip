// Tile-pass kernels of a single circuit: the fused layer passes of the
// forward circuit and of the adjoint (reverse) sweep.  The per-tile work is in
// tiles.h; these kernels build the workgroup's phase table, walk tiles and
// reduce the workgroup's partial sums.
//
// Forward passes launch one workgroup per tile.  The complex64 adjoint
// kernels in tangent form do the same, two workgroups per CU; the others run
// one persistent workgroup per CU that loads the next tile's vectors into
// registers while it works on the current tile (see adjoint_variant).
#include "plan.h"
#include "tiles.h"

namespace qs {

namespace {

template <typename V, int T, int TB, int MODE, int SH, int K = 0>
__global__ void __launch_bounds__(1 << TB) pass_kernel(PassProg pp)
{
    constexpr int NT = 1 << TB;
    __shared__ V lds[1 << T];
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (NT / 64)];
    const int tid = threadIdx.x;
    if (pp.has_phase) {
        load_phase_table(tab, static_cast<const V *>(pp.tab), pp.phase_levels, tid, NT);
        __syncthreads();
    }
    double acc[2] = {0.0, 0.0};
    for (int64_t tile = xcd_tile(pp.xcd_remap); tile < pp.ntiles; tile += gridDim.x)
        fwd_tile<V, T, TB, MODE, SH, K>(pp, tile, lds, tab, acc, tid);
    if (pp.readout) {
        block_sum(acc, red, tid, NT);
        if (tid == 0) {
            pp.partials[blockIdx.x * kSlots + 0] = acc[0];
            pp.partials[blockIdx.x * kSlots + 1] = acc[1];
        }
    }
}

// The phase table of a pass (see build_phase_table): the same for every
// workgroup, so it is evaluated once, by one workgroup, into pp.tab, and each
// workgroup of the pass copies it into LDS.
template <typename V>
__global__ void __launch_bounds__(256) phase_table_kernel(V *tab, int levels, double theta, int64_t W, double f)
{
    build_phase_table(tab, levels, theta, W, f, threadIdx.x, 256);
}

// ONE = false: persistent (one workgroup per CU), prefetching the next
// tile's vectors, psi and lambda exchanged together through a two-tile LDS
// buffer.  ONE = true: one tile per workgroup, no prefetch, one-tile LDS
// buffer, at most 128 registers (launch bounds), so that two workgroups share
// a CU and overlap each other's memory and compute phases.
template <typename V, int T, int TB, bool turnaround, int MODE, int SH, bool ONE, int K = 0>
__global__ void __launch_bounds__(1 << TB, ONE ? 4 : 1) adjoint_kernel(PassProg pp)
{
    using Cfg = TileCfg<V, T, TB>;
    constexpr int NT = Cfg::NT, NR = Cfg::NR;
    constexpr bool PAIR = !ONE;
    constexpr bool PREFETCH = !ONE;
    static_assert(TB == 9, "exchange2 assumes 512-thread tiles");
    __shared__ V lds[(PAIR ? 2 : 1) << T];
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (NT / 64)];
    const int tid = threadIdx.x;
    if (pp.has_phase) {
        load_phase_table(tab, static_cast<const V *>(pp.tab), pp.phase_levels, tid, NT);
        __syncthreads();
    }
    double acc[kSlots] = {0.0, 0.0, 0.0, 0.0};
    const int64_t G = gridDim.x;
    int64_t tile = xcd_tile(pp.xcd_remap);
    if constexpr (turnaround) {
        V p[NR];
        int32_t dg[NR];
        V np[PREFETCH ? NR : 1];
        if constexpr (PREFETCH)
            if (tile < pp.ntiles) turn_load<V, T, TB>(pp, tile, p, tid);
        for (; tile < pp.ntiles; tile += G) {
            turn_load_diag<V, T, TB>(pp, tile, dg, tid);
            if constexpr (PREFETCH) {
                if (tile + G < pp.ntiles) turn_load<V, T, TB>(pp, tile + G, np, tid);
            } else {
                turn_load<V, T, TB>(pp, tile, p, tid);
            }
            turn_compute<V, T, TB, MODE, PAIR, K>(pp, tile, p, dg, lds, acc, tid);
            if constexpr (PREFETCH) {
#pragma unroll
                for (int r = 0; r < NR; ++r) p[r] = np[r];
            }
        }
    } else {
        V p[NR], l[NR];
        int32_t dg[NR];
        V np[PREFETCH ? NR : 1], nl[PREFETCH ? NR : 1];
        if constexpr (PREFETCH)
            if (tile < pp.ntiles) rev_load_vectors<V, T, TB>(pp, tile, p, l, tid);
        for (; tile < pp.ntiles; tile += G) {
            // this tile's diagonal is requested before the next tile's vectors:
            // memory counters retire in order, so the phase step then waits
            // only for these loads.  The one-tile junction loads it at the
            // phase point instead (LATE), to stay within 128 registers.
            constexpr bool LATE = ONE && SH == (kShPre | kShPhase | kShPost);
            if (!LATE && (SH >= 0 ? (SH & kShPhase) != 0 : pp.has_phase != 0))
                rev_load_diag<V, T, TB>(pp, tile, dg, tid);
            if constexpr (PREFETCH) {
                if (tile + G < pp.ntiles) rev_load_vectors<V, T, TB>(pp, tile + G, np, nl, tid);
            } else {
                rev_load_vectors<V, T, TB>(pp, tile, p, l, tid);
            }
            rev_tile<V, T, TB, MODE, SH, PAIR, LATE, K>(pp, tile, p, l, dg, lds, tab, acc, tid);
            if constexpr (PREFETCH) {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    p[r] = np[r];
                    l[r] = nl[r];
                }
            }
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

size_t pass_table_bytes() { return (size_t)kTabMax * sizeof(double2); }

int64_t pass_grid(int prec, int adjoint, int64_t ntiles)
{
    // Forward passes: one tile per workgroup -- the hardware dispatcher's
    // dynamic assignment of workgroups to CUs overlaps loads, butterflies and
    // stores across workgroups better than a persistent loop (measured on
    // MI355X).  Persistent adjoint kernels: one workgroup per CU (the
    // one-tile adjoint variants launch one workgroup per tile, tile_grid).
    (void)prec;
    if (adjoint == 1 || adjoint == 2) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        return (int64_t)cus < ntiles ? (int64_t)cus : ntiles;
    }
    return ntiles;
}

// Stage code path of a pass (see tiles.h): branch-free when every stage is in
// tangent form, and, for the complement-symmetric layout, when every single
// factor sits at an end of its window.
int tile_mode(const PassProg &pp, int T, int tb)
{
    if ((pp.has_pre && !pp.pre.tan) || (pp.has_post && !pp.post.tan)) return kModeGeneral;
    if (!pp.pairs) return kModeTan;
    const int rb = T - tb;
    auto ends_only = [&](const WinSeq &w) {
        for (int i = 0; i < w.cnt; ++i) {
            const uint32_t in = (pp.targets >> w.s[i]) & ((1u << rb) - 1u);
            if (in & ~(1u | (1u << (rb - 1)))) return false;
        }
        return true;
    };
    if ((pp.has_pre && !ends_only(pp.A)) || (pp.has_post && !ends_only(pp.B))) return kModeGeneral;
    return kModeTanSym;
}

// Compile-time stage tail K of a fixed-shape tangent-form kernel (see
// stage_tail in plan.h and run_stage / unrun_stage in tiles.h), or 0 when the
// pass's windows do not have the pattern the kernel assumes.  kind: 0 =
// forward pass, 1 = turnaround, 2 = reverse pass.  The first stage a kernel
// visits must end in its lowest K bits, the second (if any) in its highest K.
int tail_k(const PassProg &pp, int T, int tb, int kind)
{
    if (pp.pairs) return 0;
    const int rb = T - tb;
    if (kind == 0) {
        if (pp.has_pre)
            return kernel_tail(stage_tail(pp.A, pp.targets, rb, false), stage_tail(pp.B, pp.targets, rb, false), true,
                               rb);
        return kernel_tail(stage_tail(pp.B, pp.targets, rb, false), 0, false, rb);
    }
    if (kind == 1)
        return kernel_tail(stage_tail(pp.B, pp.targets, rb, false), stage_tail(pp.B, pp.targets, rb, true), true, rb);
    if (pp.has_pre)
        return kernel_tail(stage_tail(pp.B, pp.targets, rb, true), stage_tail(pp.A, pp.targets, rb, true), true, rb);
    // a lone reverse stage ends in its highest K bits
    const int t = stage_tail(pp.B, pp.targets, rb, true);
    return t == rb ? rb : (t < 0 ? -t : 0);
}

namespace {
template <int MODE, int SH, int K = 0>
void launch_pass_s(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    constexpr int FT = kFwdThreadBits;
    if (prec == 0)
        hipLaunchKernelGGL((pass_kernel<float2, kTileBitsC64, FT, MODE, SH, K>), dim3((unsigned)grid), dim3(1 << FT),
                           0, st, pp);
    else
        hipLaunchKernelGGL((pass_kernel<double2, kTileBitsC128, FT, MODE, SH>), dim3((unsigned)grid), dim3(1 << FT),
                           0, st, pp);
}

// complex64 tangent-form fixed shapes: the instantiation for the pass's tail
template <int SH>
void launch_pass_k(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    const int k = prec == 0 ? tail_k(pp, kTileBitsC64, kFwdThreadBits, 0) : 0;
    switch (k) {
    case 1: launch_pass_s<kModeTan, SH, 1>(prec, pp, grid, st); break;
    case 2: launch_pass_s<kModeTan, SH, 2>(prec, pp, grid, st); break;
    case 3: launch_pass_s<kModeTan, SH, 3>(prec, pp, grid, st); break;
    case 4: launch_pass_s<kModeTan, SH, 4>(prec, pp, grid, st); break;
    case 5: launch_pass_s<kModeTan, SH, 5>(prec, pp, grid, st); break;
    default: launch_pass_s<kModeTan, SH>(prec, pp, grid, st); break;
    }
}

// Forward shapes with their own instantiation: the first pass (|+>, phase,
// stage), a junction (stage, phase, stage) and the last pass (stage and
// readout); anything else uses the runtime-shape kernel.  (A plain stage was
// measured 1 ms slower fixed than with the runtime shape at n = 32.)
template <int MODE>
void launch_pass_m(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    constexpr int kFirst = kShInit | kShPhase | kShPost, kJunc = kShPre | kShPhase | kShPost,
                  kLast = kShPost | kShReadout;
    if constexpr (MODE == kModeTan) {
        switch (pass_shape(pp)) {
        case kFirst: launch_pass_k<kFirst>(prec, pp, grid, st); return;
        case kJunc: launch_pass_k<kJunc>(prec, pp, grid, st); return;
        case kLast: launch_pass_k<kLast>(prec, pp, grid, st); return;
        default: launch_pass_s<MODE, -1>(prec, pp, grid, st); return;
        }
    }
    switch (pass_shape(pp)) {
    case kFirst: launch_pass_s<MODE, kFirst>(prec, pp, grid, st); break;
    case kJunc: launch_pass_s<MODE, kJunc>(prec, pp, grid, st); break;
    case kLast: launch_pass_s<MODE, kLast>(prec, pp, grid, st); break;
    default: launch_pass_s<MODE, -1>(prec, pp, grid, st); break;
    }
}

template <int MODE, bool TURN, int SH, bool ONE>
void launch_adjoint_s(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    constexpr int AT = kAdjThreadBits;
    const dim3 g((unsigned)grid), b(1 << AT);
    if (prec == 0) hipLaunchKernelGGL((adjoint_kernel<float2, kTileBitsC64, AT, TURN, MODE, SH, ONE>), g, b, 0, st, pp);
    else hipLaunchKernelGGL((adjoint_kernel<double2, kTileBitsC128, AT, TURN, MODE, SH, ONE>), g, b, 0, st, pp);
}

// complex64 one-tile tangent-form kernels: the instantiation for the pass's tail
template <bool TURN, int SH>
void launch_adjoint_k(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    constexpr int AT = kAdjThreadBits;
    const int k = prec == 0 ? tail_k(pp, kTileBitsC64, AT, TURN ? 1 : 2) : 0;
    const dim3 g((unsigned)grid), b(1 << AT);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, b, 0, st, pp); };
    switch (k) {
    case 1: go(adjoint_kernel<float2, kTileBitsC64, AT, TURN, kModeTan, SH, true, 1>); break;
    case 2: go(adjoint_kernel<float2, kTileBitsC64, AT, TURN, kModeTan, SH, true, 2>); break;
    case 3: go(adjoint_kernel<float2, kTileBitsC64, AT, TURN, kModeTan, SH, true, 3>); break;
    case 4: go(adjoint_kernel<float2, kTileBitsC64, AT, TURN, kModeTan, SH, true, 4>); break;
    default: launch_adjoint_s<kModeTan, TURN, SH, true>(prec, pp, grid, st); break;
    }
}

// Adjoint kernel variants.  kAdjPersistent: the runtime-shape persistent
// kernel with prefetch.  The others take one tile per workgroup and fit in
// 128 registers without prefetch, so two workgroups share a CU: the
// turnaround, a reverse pass of plain stages, the reverse of the first
// forward pass (phase of layer 1, no writes) and the reverse junction (stage,
// phase, stage; its diagonal is loaded at the phase point).  The turnaround
// and the junction are one-tile for complex64 only: in complex128 they spill
// at 128 registers.
enum { kAdjPersistent, kAdjOneTurn, kAdjOnePlain, kAdjOneFirst, kAdjOneJunc };

int adjoint_variant(int prec, const PassProg &pp, int turnaround, int mode)
{
    if (mode == kModeGeneral) return kAdjPersistent;
    if (turnaround) return prec == 0 ? kAdjOneTurn : kAdjPersistent;
    switch (pass_shape(pp)) {
    case kShPost: return kAdjOnePlain;
    case kShInit | kShPhase | kShPost: return kAdjOneFirst;
    case kShPre | kShPhase | kShPost: return prec == 0 ? kAdjOneJunc : kAdjPersistent;
    default: return kAdjPersistent;
    }
}

template <int MODE>
void launch_adjoint_m(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    if constexpr (MODE == kModeTan) {
        if (prec == 0) {
            switch (adjoint_variant(prec, pp, turnaround, MODE)) {
            case kAdjOneTurn: launch_adjoint_k<true, -1>(prec, pp, grid, st); return;
            // (the reverse of a plain pass and the reverse junction keep runtime
            // masks: with compile-time tails their code needs more than the 128
            // registers of two workgroups per CU and spills)
            case kAdjOneFirst: launch_adjoint_k<false, kShInit | kShPhase | kShPost>(prec, pp, grid, st); return;
            default: break;
            }
        }
    }
    switch (adjoint_variant(prec, pp, turnaround, MODE)) {
    case kAdjOneTurn: launch_adjoint_s<MODE, true, -1, true>(prec, pp, grid, st); break;
    case kAdjOnePlain: launch_adjoint_s<MODE, false, kShPost, true>(prec, pp, grid, st); break;
    case kAdjOneFirst: launch_adjoint_s<MODE, false, kShInit | kShPhase | kShPost, true>(prec, pp, grid, st); break;
    case kAdjOneJunc: launch_adjoint_s<MODE, false, kShPre | kShPhase | kShPost, true>(prec, pp, grid, st); break;
    default:
        if (turnaround) launch_adjoint_s<MODE, true, -1, false>(prec, pp, grid, st);
        else launch_adjoint_s<MODE, false, -1, false>(prec, pp, grid, st);
        break;
    }
}
}  // namespace

// Grid of the kernel that launch_pass / launch_adjoint_pass pick for pp.
int64_t tile_grid(int prec, int adjoint, const PassProg &pp)
{
    if (adjoint == 0) return pass_grid(prec, 0, pp.ntiles);
    const int mode = tile_mode(pp, tile_bits(prec), kAdjThreadBits);
    return adjoint_variant(prec, pp, adjoint == 1, mode) == kAdjPersistent ? pass_grid(prec, adjoint, pp.ntiles)
                                                                            : pp.ntiles;
}

namespace {
// Evaluate the table of a phase pass into pp.tab, ahead of the pass on the
// same stream.  f: the real factor folded into the table.
hipError_t launch_phase_table(int prec, const PassProg &pp, double f, hipStream_t st)
{
    if (!pp.has_phase) return hipSuccess;
    if (!pp.tab) return hipErrorInvalidValue;
    if (prec == 0)
        hipLaunchKernelGGL(phase_table_kernel<float2>, dim3(1), dim3(256), 0, st, static_cast<float2 *>(pp.tab),
                           pp.phase_levels, pp.theta_zz, pp.W, f);
    else
        hipLaunchKernelGGL(phase_table_kernel<double2>, dim3(1), dim3(256), 0, st, static_cast<double2 *>(pp.tab),
                           pp.phase_levels, pp.theta_zz, pp.W, f);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_pass(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    if (hipError_t e = launch_phase_table(prec, pp, pp.factor, st)) return e;
    switch (tile_mode(pp, tile_bits(prec), kFwdThreadBits)) {
    case kModeTan: launch_pass_m<kModeTan>(prec, pp, grid, st); break;
    case kModeTanSym: launch_pass_m<kModeTanSym>(prec, pp, grid, st); break;
    default: launch_pass_s<kModeGeneral, -1>(prec, pp, grid, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_pass(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    const int mode = tile_mode(pp, tile_bits(prec), kAdjThreadBits);
    // reverse passes in tangent form fold the stages' factors into the table
    // (see rev_tile)
    const bool fold = !turnaround && mode != kModeGeneral && !pp.init;
    if (hipError_t e = launch_phase_table(prec, pp, fold ? pp.factor : 1.0, st)) return e;
    switch (mode) {
    case kModeTan: launch_adjoint_m<kModeTan>(prec, pp, turnaround, grid, st); break;
    case kModeTanSym: launch_adjoint_m<kModeTanSym>(prec, pp, turnaround, grid, st); break;
    default:
        if (turnaround) launch_adjoint_s<kModeGeneral, true, -1, false>(prec, pp, grid, st);
        else launch_adjoint_s<kModeGeneral, false, -1, false>(prec, pp, grid, st);
        break;
    }
    return hipGetLastError();
}

}  // namespace qs
