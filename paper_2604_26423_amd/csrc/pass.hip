// Tile-pass kernels of a single circuit: the fused layer passes of the
// forward circuit and of the adjoint (reverse) sweep.  The per-tile work is in
// tiles.h; these kernels build the workgroup's phase table, walk tiles and
// reduce the workgroup's partial sums.
//
// Forward passes launch one workgroup per tile.  The turnaround and the
// reverse passes run one persistent workgroup per CU that loads the next
// tile's vectors into registers while it works on the current tile.
#include <stdlib.h>

#include "tiles.h"

#ifndef QS_ADJ_PREFETCH
#define QS_ADJ_PREFETCH 1
#endif

namespace qs {

namespace {

template <typename V, int T, int TB, int MODE, int SH>
__global__ void __launch_bounds__(1 << TB) pass_kernel(PassProg pp)
{
    constexpr int NT = 1 << TB;
    __shared__ V lds[1 << T];
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (NT / 64)];
    const int tid = threadIdx.x;
    if (pp.has_phase) {
        build_phase_table(tab, pp.phase_levels, pp.theta_zz, pp.W, pp.factor, tid, NT);
        __syncthreads();
    }
    double acc[2] = {0.0, 0.0};
    for (int64_t tile = xcd_tile(pp.xcd_remap); tile < pp.ntiles; tile += gridDim.x)
        fwd_tile<V, T, TB, MODE, SH>(pp, tile, lds, tab, acc, tid);
    if (pp.readout) {
        block_sum(acc, red, tid, NT);
        if (tid == 0) {
            pp.partials[blockIdx.x * kSlots + 0] = acc[0];
            pp.partials[blockIdx.x * kSlots + 1] = acc[1];
        }
    }
}

template <typename V, int T, int TB, bool turnaround, int MODE, int SH>
__global__ void __launch_bounds__(1 << TB) adjoint_kernel(PassProg pp)
{
    using Cfg = TileCfg<V, T, TB>;
    constexpr int NT = Cfg::NT, NR = Cfg::NR;
    static_assert(TB == 9, "exchange2 assumes 512-thread tiles");
    __shared__ V lds[2 << T];  // two tiles: psi and lambda move through LDS together
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (NT / 64)];
    const int tid = threadIdx.x;
    if (pp.has_phase) {
        build_phase_table(tab, pp.phase_levels, pp.theta_zz, pp.W, 1.0, tid, NT);
        __syncthreads();
    }
    double acc[kSlots] = {0.0, 0.0, 0.0, 0.0};
    const int64_t G = gridDim.x;
    int64_t tile = xcd_tile(pp.xcd_remap);
    if constexpr (turnaround) {
        V p[NR];
        int32_t dg[NR];
#if QS_ADJ_PREFETCH
        V np[NR];
        if (tile < pp.ntiles) turn_load<V, T, TB>(pp, tile, p, tid);
#endif
        for (; tile < pp.ntiles; tile += G) {
            turn_load_diag<V, T, TB>(pp, tile, dg, tid);
#if QS_ADJ_PREFETCH
            if (tile + G < pp.ntiles) turn_load<V, T, TB>(pp, tile + G, np, tid);
#else
            turn_load<V, T, TB>(pp, tile, p, tid);
#endif
            turn_compute<V, T, TB, MODE>(pp, tile, p, dg, lds, acc, tid);
#if QS_ADJ_PREFETCH
#pragma unroll
            for (int r = 0; r < NR; ++r) p[r] = np[r];
#endif
        }
    } else {
        V p[NR], l[NR];
        int32_t dg[NR];
#if QS_ADJ_PREFETCH
        V np[NR], nl[NR];
        if (tile < pp.ntiles) rev_load_vectors<V, T, TB>(pp, tile, p, l, tid);
#endif
        for (; tile < pp.ntiles; tile += G) {
            // this tile's diagonal is requested before the next tile's vectors:
            // memory counters retire in order, so the phase step then waits
            // only for these loads
            if (SH >= 0 ? (SH & kShPhase) != 0 : pp.has_phase != 0) rev_load_diag<V, T, TB>(pp, tile, dg, tid);
#if QS_ADJ_PREFETCH
            if (tile + G < pp.ntiles) rev_load_vectors<V, T, TB>(pp, tile + G, np, nl, tid);
#else
            rev_load_vectors<V, T, TB>(pp, tile, p, l, tid);
#endif
            rev_tile<V, T, TB, MODE, SH>(pp, tile, p, l, dg, lds, tab, acc, tid);
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
    if (adjoint == 1 || adjoint == 2) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        return (int64_t)cus < ntiles ? (int64_t)cus : ntiles;
    }
#endif
    (void)adjoint;
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

namespace {
template <int MODE, int SH>
void launch_pass_s(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    constexpr int FT = kFwdThreadBits;
    if (prec == 0)
        hipLaunchKernelGGL((pass_kernel<float2, kTileBitsC64, FT, MODE, SH>), dim3((unsigned)grid), dim3(1 << FT), 0,
                           st, pp);
    else
        hipLaunchKernelGGL((pass_kernel<double2, kTileBitsC128, FT, MODE, SH>), dim3((unsigned)grid), dim3(1 << FT),
                           0, st, pp);
}

// Forward shapes with their own instantiation: the first pass (|+>, phase,
// stage), a junction (stage, phase, stage) and the last pass (stage and
// readout); anything else uses the runtime-shape kernel.  (A plain stage was
// measured 1 ms slower fixed than with the runtime shape at n = 32.)
// QS_PASS_SHAPES=0 in the environment selects the runtime-shape kernels
// everywhere (for comparisons).
int shapes_enabled()
{
    static const int on = [] {
        const char *v = getenv("QS_PASS_SHAPES");
        return v && v[0] == '0' ? 0 : 1;
    }();
    return on;
}

template <int MODE>
void launch_pass_m(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    switch (shapes_enabled() ? pass_shape(pp) : -1) {
    case kShInit | kShPhase | kShPost: launch_pass_s<MODE, kShInit | kShPhase | kShPost>(prec, pp, grid, st); break;
    case kShPre | kShPhase | kShPost: launch_pass_s<MODE, kShPre | kShPhase | kShPost>(prec, pp, grid, st); break;
    case kShPost | kShReadout: launch_pass_s<MODE, kShPost | kShReadout>(prec, pp, grid, st); break;
    default: launch_pass_s<MODE, -1>(prec, pp, grid, st); break;
    }
}

template <int MODE, bool TURN, int SH>
void launch_adjoint_s(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    constexpr int AT = kAdjThreadBits;
    const dim3 g((unsigned)grid), b(1 << AT);
    if (prec == 0) hipLaunchKernelGGL((adjoint_kernel<float2, kTileBitsC64, AT, TURN, MODE, SH>), g, b, 0, st, pp);
    else hipLaunchKernelGGL((adjoint_kernel<double2, kTileBitsC128, AT, TURN, MODE, SH>), g, b, 0, st, pp);
}

// Reverse shapes with their own instantiation: a plain stage and the first
// forward pass undone (phase of layer 1, no writes).  The junction keeps the
// runtime shape: fixed, it needs more than 256 registers and spills.
template <int MODE>
void launch_adjoint_m(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    if (turnaround) {
        launch_adjoint_s<MODE, true, -1>(prec, pp, grid, st);
        return;
    }
    switch (shapes_enabled() ? pass_shape(pp) : -1) {
    case kShPost: launch_adjoint_s<MODE, false, kShPost>(prec, pp, grid, st); break;
    case kShInit | kShPhase | kShPost:
        launch_adjoint_s<MODE, false, kShInit | kShPhase | kShPost>(prec, pp, grid, st);
        break;
    default: launch_adjoint_s<MODE, false, -1>(prec, pp, grid, st); break;
    }
}
}  // namespace

hipError_t launch_pass(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    switch (tile_mode(pp, tile_bits(prec), kFwdThreadBits)) {
    case kModeTan: launch_pass_m<kModeTan>(prec, pp, grid, st); break;
    case kModeTanSym: launch_pass_m<kModeTanSym>(prec, pp, grid, st); break;
    default: launch_pass_s<kModeGeneral, -1>(prec, pp, grid, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_pass(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    switch (tile_mode(pp, tile_bits(prec), kAdjThreadBits)) {
    case kModeTan: launch_adjoint_m<kModeTan>(prec, pp, turnaround, grid, st); break;
    case kModeTanSym: launch_adjoint_m<kModeTanSym>(prec, pp, turnaround, grid, st); break;
    default:
        if (turnaround) launch_adjoint_s<kModeGeneral, true, -1>(prec, pp, grid, st);
        else launch_adjoint_s<kModeGeneral, false, -1>(prec, pp, grid, st);
        break;
    }
    return hipGetLastError();
}

}  // namespace qs
