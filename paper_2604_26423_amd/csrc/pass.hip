// Tile-pass kernels of a single circuit: the fused layer passes of the
// forward circuit and of the adjoint (reverse) sweep.  The per-tile work is in
// tiles.h; these kernels copy the pass's phase table into LDS, walk tiles and
// reduce the workgroup's partial sums.
//
// Forward passes launch one workgroup per tile.  The adjoint kernels in
// tangent form do the same, two workgroups per CU (256 threads in the full
// layout); the others run one persistent workgroup per CU that loads the next
// tile's vectors into registers while it works on the current tile (see
// adjoint_variant).
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

// Weights of the cut function that a full-layout diagonal encodes, and a
// check that they reproduce it (see the cut-value notes in internal.h).  One
// workgroup.  wts: kWtSize int32.
__global__ void __launch_bounds__(256) cut_weights_kernel(const int32_t *__restrict__ diag, int n, int64_t W,
                                                          int32_t *__restrict__ wts)
{
    __shared__ int32_t w[kWtStride * kWtStride];
    __shared__ int32_t deg[kWtStride];
    __shared__ int bad;
    __shared__ unsigned long long twice_w;
    const int tid = threadIdx.x;
    if (tid == 0) {
        bad = diag[0] != 0;
        twice_w = 0;
    }
    for (int i = tid; i < kWtStride; i += 256) deg[i] = i < n ? diag[swz((int64_t)1 << i)] : 0;
    __syncthreads();
    for (int idx = tid; idx < kWtStride * kWtStride; idx += 256) {
        const int i = idx / kWtStride, j = idx % kWtStride;
        int32_t v = 0;
        if (i < n && j < n && i != j) {
            const int64_t d = (int64_t)deg[i] + deg[j] - diag[swz(((int64_t)1 << i) | ((int64_t)1 << j))];
            if (d < 0 || (d & 1)) atomicOr(&bad, 1);
            v = (int32_t)(d >> 1);
        }
        w[idx] = v;
    }
    __syncthreads();
    // deg_i = sum_j w_ij and W_t = sum_{i<j} w_ij
    if (tid < n) {
        int64_t rs = 0;
        for (int j = 0; j < n; ++j) rs += w[tid * kWtStride + j];
        if (rs != deg[tid]) atomicOr(&bad, 1);
        atomicAdd(&twice_w, (unsigned long long)rs);
    }
    __syncthreads();
    if (tid == 0 && twice_w != 2ull * (unsigned long long)W) bad = 1;
    // sampled entries: C(x) = sum_{i in x} deg_i - 2 sum_{i<j in x} w_ij
    for (int k = tid; k < kCtSamples; k += 256) {
        const uint64_t x = n == 0 ? 0 : ((uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull) >> (64 - n);
        int64_t cx = 0;
        for (uint64_t a = x; a; a &= a - 1) {
            const int i = __builtin_ctzll(a);
            cx += deg[i];
            for (uint64_t b = a & (a - 1); b; b &= b - 1) cx -= 2 * (int64_t)w[i * kWtStride + __builtin_ctzll(b)];
        }
        if (cx != (int64_t)diag[swz((int64_t)x)]) atomicOr(&bad, 1);
    }
    __syncthreads();
    for (int idx = tid; idx < kWtStride * kWtStride; idx += 256) wts[idx] = w[idx];
    for (int i = tid; i < kWtStride; i += 256) wts[kWtDeg + i] = deg[i];
    if (tid == 0) wts[kWtOk] = bad ? 0 : 1;
}

// Cut table of a pass (layout in internal.h) for kernels of 2^tb threads whose
// tiles hold 2^T amplitudes, evaluated in window s.  Blocks 0 .. gridDim.x - 2
// write one tile row per thread; the last block writes the uniform and the
// per-thread entries.
__global__ void __launch_bounds__(256) cut_table_kernel(const int32_t *__restrict__ wts, int n, int c, int q0,
                                                        int T, int tb, int s, int64_t ntiles,
                                                        int32_t *__restrict__ ctab)
{
    __shared__ int32_t w[kWtStride * kWtStride];
    __shared__ int32_t deg[kWtStride];
    const int tid = threadIdx.x;
    for (int i = tid; i < n * kWtStride; i += 256) w[i] = wts[i];
    for (int i = tid; i < kWtStride; i += 256) deg[i] = wts[kWtDeg + i];
    __syncthreads();
    const int rb = T - tb;
    auto gbit = [&](int e) { return e < c ? e : q0 + (e - c); };  // tile bit -> global bit
    // C of the bit set a (uint32 arithmetic, exact for C < 2^31)
    auto cut = [&](uint64_t a) {
        uint32_t cx = 0;
        for (uint64_t m = a; m; m &= m - 1) {
            const int i = __builtin_ctzll(m);
            cx += (uint32_t)deg[i];
            for (uint64_t b = m & (m - 1); b; b &= b - 1) cx -= 2u * (uint32_t)w[i * kWtStride + __builtin_ctzll(b)];
        }
        return cx;
    };
    if (blockIdx.x + 1 < gridDim.x) {
        const int64_t tile = (int64_t)blockIdx.x * 256 + tid;
        if (tile >= ntiles) return;
        const uint64_t A = (uint64_t)tile_base(tile, c, q0, T - c);
        int32_t *row = ctab + kCtTile + tile * 16;
        row[0] = (int32_t)cut(A);
        for (int e = 0; e < 15; ++e) {
            uint32_t db = 0;
            if (e < T) {
                const int g = gbit(e);
                for (uint64_t m = A; m; m &= m - 1) db += (uint32_t)w[g * kWtStride + __builtin_ctzll(m)];
            }
            row[1 + e] = (int32_t)db;
        }
        return;
    }
    if (tid < (1 << rb)) {
        uint64_t D = 0;
        for (int k = 0; k < rb; ++k)
            if ((tid >> k) & 1) D |= 1ull << gbit(s + k);
        ctab[kCtCreg + tid] = (int32_t)cut(D);
    }
    if (tid == 0) ctab[kCtValid] = wts[kWtOk];
    for (int t = tid; t < (1 << tb); t += 256) {
        const int et = win_elem(0, t, s, rb);
        uint64_t B = 0;
        for (int e = 0; e < T; ++e)
            if ((et >> e) & 1) B |= 1ull << gbit(e);
        int32_t *ent = ctab + kCtThr + t * 8;
        ent[0] = (int32_t)cut(B);
        for (int k = 0; k < 7; ++k) {
            uint32_t dt = 0;
            if (k < rb) {
                const int g = gbit(s + k);
                for (uint64_t m = B; m; m &= m - 1) dt += (uint32_t)w[g * kWtStride + __builtin_ctzll(m)];
            }
            ent[1 + k] = (int32_t)dt;
        }
    }
}

// ONE = false: persistent (one workgroup per CU), prefetching the next
// tile's vectors, psi and lambda exchanged together through a two-tile LDS
// buffer.  ONE = true: one tile per workgroup, no prefetch, one-tile LDS
// buffer, registers for two workgroups per CU (launch bounds: 128 with 512
// threads, 256 with 256 threads), so that two workgroups share a CU and
// overlap each other's memory and compute phases.
template <typename V, int T, int TB, bool turnaround, int MODE, int SH, bool ONE, int K = 0>
__global__ void __launch_bounds__(1 << TB, ONE ? (TB == 9 ? 4 : 2) : 1) adjoint_kernel(PassProg pp)
{
    using Cfg = TileCfg<V, T, TB>;
    constexpr int NT = Cfg::NT, NR = Cfg::NR;
    constexpr bool PAIR = !ONE;
    constexpr bool PREFETCH = !ONE;
    static_assert(ONE || TB == 9, "exchange2 assumes 512-thread tiles");
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

int64_t cut_table_entries(int n, int prec)
{
    const int T = tile_bits(prec);
    return kCtTile + 16 * (n > T ? (int64_t)1 << (n - T) : 1);
}

hipError_t launch_cut_weights(const int32_t *diag, int n, int64_t W, int32_t *wts, hipStream_t st)
{
    if (n < 1 || n > kWtStride - 1 || !diag || !wts) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cut_weights_kernel, dim3(1), dim3(256), 0, st, diag, n, W, wts);
    return hipGetLastError();
}

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
// stage), a junction (stage, phase, stage), the last pass (stage and readout)
// and, in tangent form, a plain stage with its compile-time tail (102-136
// registers against 240 with runtime masks; bit-identical, a plain contiguous
// pass ~0.1 ms faster at n = 32); anything else uses the runtime-shape
// kernel.
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
        case kShPost: launch_pass_k<kShPost>(prec, pp, grid, st); return;
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

template <int MODE, bool TURN, int SH, bool ONE, int AT = kAdjThreadBits>
void launch_adjoint_s(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    const dim3 g((unsigned)grid), b(1 << AT);
    if (prec == 0) hipLaunchKernelGGL((adjoint_kernel<float2, kTileBitsC64, AT, TURN, MODE, SH, ONE>), g, b, 0, st, pp);
    else hipLaunchKernelGGL((adjoint_kernel<double2, kTileBitsC128, AT, TURN, MODE, SH, ONE>), g, b, 0, st, pp);
}

// complex64 one-tile tangent-form kernels: the instantiation for the pass's tail
template <bool TURN, int SH, int AT>
void launch_adjoint_k(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    const int k = prec == 0 ? tail_k(pp, kTileBitsC64, AT, TURN ? 1 : 2) : 0;
    const dim3 g((unsigned)grid), b(1 << AT);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, b, 0, st, pp); };
    switch (k) {
    case 1: go(adjoint_kernel<float2, kTileBitsC64, AT, TURN, kModeTan, SH, true, 1>); break;
    case 2: go(adjoint_kernel<float2, kTileBitsC64, AT, TURN, kModeTan, SH, true, 2>); break;
    case 3: go(adjoint_kernel<float2, kTileBitsC64, AT, TURN, kModeTan, SH, true, 3>); break;
    case 4: go(adjoint_kernel<float2, kTileBitsC64, AT, TURN, kModeTan, SH, true, 4>); break;
    default: launch_adjoint_s<kModeTan, TURN, SH, true, AT>(prec, pp, grid, st); break;
    }
}

// Adjoint kernel variants.  kAdjPersistent: the runtime-shape persistent
// kernel with prefetch (512 threads).  The others take one tile per
// workgroup, without prefetch, in the registers of two workgroups per CU: the
// turnaround, a reverse pass of plain stages, the reverse of the first
// forward pass (phase of layer 1, no writes) and the reverse junction (stage,
// phase, stage; its diagonal is loaded at the phase point).  They run 256
// threads (pp.tb = 8: 5-bit windows, up to 256 registers); planned for 512
// threads (128 registers) the complex128 turnaround and junction spill and
// take the persistent kernel instead.
enum { kAdjPersistent, kAdjOneTurn, kAdjOnePlain, kAdjOneFirst, kAdjOneJunc };

int adjoint_variant(int prec, const PassProg &pp, int turnaround, int mode)
{
    if (mode == kModeGeneral) return kAdjPersistent;
    const bool spills = prec != 0 && pp.tb == kAdjThreadBits;
    if (turnaround) return spills ? kAdjPersistent : kAdjOneTurn;
    switch (pass_shape(pp)) {
    case kShPost: return kAdjOnePlain;
    case kShInit | kShPhase | kShPost: return kAdjOneFirst;
    case kShPre | kShPhase | kShPost: return spills ? kAdjPersistent : kAdjOneJunc;
    default: return kAdjPersistent;
    }
}

// AT: thread bits of the one-tile kernels (pp.tb); the persistent kernels
// are 512-thread only.
template <int MODE, int AT>
void launch_adjoint_m_at(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    if constexpr (MODE == kModeTan) {
        if (prec == 0) {
            switch (adjoint_variant(prec, pp, turnaround, MODE)) {
            case kAdjOneTurn: launch_adjoint_k<true, -1, AT>(prec, pp, grid, st); return;
            // (the reverse of a plain pass and the reverse junction keep runtime
            // masks: with compile-time tails their 512-thread code needs more
            // than the 128 registers of two workgroups per CU and spills)
            case kAdjOneFirst: launch_adjoint_k<false, kShInit | kShPhase | kShPost, AT>(prec, pp, grid, st); return;
            default: break;
            }
        }
    }
    switch (adjoint_variant(prec, pp, turnaround, MODE)) {
    case kAdjOneTurn: launch_adjoint_s<MODE, true, -1, true, AT>(prec, pp, grid, st); break;
    case kAdjOnePlain: launch_adjoint_s<MODE, false, kShPost, true, AT>(prec, pp, grid, st); break;
    case kAdjOneFirst: launch_adjoint_s<MODE, false, kShInit | kShPhase | kShPost, true, AT>(prec, pp, grid, st); break;
    case kAdjOneJunc: launch_adjoint_s<MODE, false, kShPre | kShPhase | kShPost, true, AT>(prec, pp, grid, st); break;
    default:
        if constexpr (AT == kAdjThreadBits) {
            if (turnaround) launch_adjoint_s<MODE, true, -1, false>(prec, pp, grid, st);
            else launch_adjoint_s<MODE, false, -1, false>(prec, pp, grid, st);
        }
        break;
    }
}

template <int MODE>
void launch_adjoint_m(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    if (pp.tb == kAdjOneThreadBits) launch_adjoint_m_at<MODE, kAdjOneThreadBits>(prec, pp, turnaround, grid, st);
    else launch_adjoint_m_at<MODE, kAdjThreadBits>(prec, pp, turnaround, grid, st);
}

// Stage code path of an adjoint pass, for the threads its windows are planned for.
int adjoint_mode(int prec, const PassProg &pp) { return tile_mode(pp, tile_bits(prec), pp.tb); }
}  // namespace

// Whether the kernel that launch_pass / launch_adjoint_pass pick for pp (kind
// 0 = forward pass, 1 = turnaround, 2 = reverse pass) needs C_t and takes it
// from a cut table: every forward and turnaround kernel does, and every
// reverse kernel but the complex64 one-tile junction, which loads the
// diagonal.
bool pass_takes_cut_table(int prec, const PassProg &pp, int kind)
{
    if (kind == 0) return pp.has_phase || pp.readout;
    if (kind == 1) return true;
    if (!pp.has_phase) return false;
    return adjoint_variant(prec, pp, 0, adjoint_mode(prec, pp)) != kAdjOneJunc;
}

// The one-tile adjoint kernels run 256 threads of 32 amplitudes per vector
// (complex64) or 16 (complex128): their windows of 5 (4) register bits need
// fewer exchanges per stage than those of 512 threads (a 13-qubit stage three
// windows instead of four, a 9- or 10-qubit stage two instead of three), at
// 164-246 registers for two workgroups per CU; planned for 256 threads the
// complex128 turnaround and junction fit too.  The host plans a pass for 256
// threads first and falls back to 512 (the persistent kernel) when this
// returns false.
bool adjoint_one_tile(int prec, const PassProg &pp, int turnaround)
{
    return adjoint_variant(prec, pp, turnaround, adjoint_mode(prec, pp)) != kAdjPersistent;
}

// Grid of the kernel that launch_pass / launch_adjoint_pass pick for pp.
int64_t tile_grid(int prec, int adjoint, const PassProg &pp)
{
    if (adjoint == 0) return pass_grid(prec, 0, pp.ntiles);
    return adjoint_one_tile(prec, pp, adjoint == 1) ? pp.ntiles : pass_grid(prec, adjoint, pp.ntiles);
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

namespace {
// The window in which a pass evaluates C_t (the layout tiles.h loads the
// diagonal in): kind 0 = forward pass (the phase layout, or the final one
// for the readout), 1 = turnaround (final layout), 2 = reverse pass (phase
// layout).
int cut_window(const PassProg &pp, int kind)
{
    return kind == 0 ? (pp.has_phase ? pp.phase_win : pp.final_win) : kind == 1 ? pp.final_win : pp.phase_win;
}

// Write the pass's cut table (pp.ctab non-null only when the pass's kernel
// takes one, see pass_takes_cut_table).
hipError_t launch_cut_table(int prec, const PassProg &pp, int kind, int tb, hipStream_t st)
{
    if (!pp.ctab) return hipSuccess;
    if (!pp.wts || pp.n > kWtStride - 1) return hipErrorInvalidValue;
    const int T = tile_bits(prec);
    const int64_t blocks = (pp.ntiles + 255) / 256 + 1;
    hipLaunchKernelGGL(cut_table_kernel, dim3((unsigned)blocks), dim3(256), 0, st, pp.wts, pp.n, pp.c, pp.q0, T, tb,
                       cut_window(pp, kind), pp.ntiles, pp.ctab);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_pass(int prec, const PassProg &pp, int64_t grid, hipStream_t st)
{
    if (hipError_t e = launch_phase_table(prec, pp, pp.factor, st)) return e;
    if (hipError_t e = launch_cut_table(prec, pp, 0, kFwdThreadBits, st)) return e;
    switch (tile_mode(pp, tile_bits(prec), kFwdThreadBits)) {
    case kModeTan: launch_pass_m<kModeTan>(prec, pp, grid, st); break;
    case kModeTanSym: launch_pass_m<kModeTanSym>(prec, pp, grid, st); break;
    default: launch_pass_s<kModeGeneral, -1>(prec, pp, grid, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_pass(int prec, const PassProg &pp, int turnaround, int64_t grid, hipStream_t st)
{
    // a program planned for 256 threads must take a one-tile kernel
    if (pp.tb != kAdjThreadBits && (pp.tb != kAdjOneThreadBits || !adjoint_one_tile(prec, pp, turnaround)))
        return hipErrorInvalidValue;
    const int mode = adjoint_mode(prec, pp);
    // reverse passes in tangent form fold the stages' factors into the table
    // (see rev_tile)
    const bool fold = !turnaround && mode != kModeGeneral && !pp.init;
    if (hipError_t e = launch_phase_table(prec, pp, fold ? pp.factor : 1.0, st)) return e;
    if (hipError_t e = launch_cut_table(prec, pp, turnaround ? 1 : 2, pp.tb, st)) return e;
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
