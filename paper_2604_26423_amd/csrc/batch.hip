// Batched forward + adjoint gradient of many circuits in one persistent
// launch.  Each circuit runs the same pass sequence as a single circuit:
// forward passes, the turnaround, reverse passes.  Work items (a chunk of
// tiles of one pass of one circuit) are claimed from a global ticket counter
// in rounds -- step r of every circuit, largest circuits first -- so a
// circuit's previous pass has almost always finished when its next pass is
// claimed.  A workgroup that finds it unfinished waits on that pass's
// completion counter.  The wait only ever targets items with lower ticket
// numbers, which running workgroups hold and finish without waiting on later
// items, so the queue always drains; a bounded spin additionally lets every
// wave exit (and raise a flag) should a dependency never complete.
//
// Memory ordering between workgroups: stores of an item are released at
// agent scope before its completion counter is incremented, and a workgroup
// acquires at agent scope after observing a complete predecessor.
#include "tiles.h"

namespace qs {

namespace {

constexpr int TBB = kBatchThreadBits;

__device__ __forceinline__ int find_step(const BatchStep *steps, int nsteps, int64_t item)
{
    int lo = 0, hi = nsteps - 1;  // last step with item0 <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (steps[mid].item0 <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Tiles [t0, t1) of one step, with the stage code path of that step.
template <typename V, int T, int MODE>
__device__ __forceinline__ void run_item(const BatchStep &st, int64_t t0, int64_t t1, V *lds, const V *tab,
                                         double (&acc)[kSlots], int tid)
{
    constexpr int NR = TileCfg<V, T, TBB>::NR;
    const PassProg &pp = st.pp;
    if (st.kind == 0) {
        double fa[2] = {0.0, 0.0};
        for (int64_t t = t0; t < t1; ++t) fwd_tile<V, T, TBB, MODE>(pp, t, lds, tab, fa, tid);
        acc[0] = fa[0];
        acc[1] = fa[1];
    } else if (st.kind == 1) {
        for (int64_t t = t0; t < t1; ++t) turn_tile<V, T, TBB, MODE>(pp, t, lds, acc, tid);
    } else {
        for (int64_t t = t0; t < t1; ++t) {
            V p[NR], l[NR];
            int32_t dg[NR];
            if (pp.has_phase) rev_load_diag<V, T, TBB>(pp, t, dg, tid);
            rev_load_vectors<V, T, TBB>(pp, t, p, l, tid);
            rev_tile<V, T, TBB, MODE>(pp, t, p, l, dg, lds, tab, acc, tid);
        }
    }
}

template <typename V, int T>
__global__ void __launch_bounds__(1 << TBB) batch_kernel(BatchArgs a)
{
    using Cfg = TileCfg<V, T, TBB>;
    constexpr int NT = Cfg::NT;
    __shared__ V lds[2 << T];  // two tiles for the reverse passes
    __shared__ V tab[kTabMax];
    __shared__ double red[kSlots * (NT / 64)];
    __shared__ int64_t s_item;
    __shared__ int s_step, s_ok;
    const int tid = threadIdx.x;
    int tab_step = -1;
    const V *tabs = reinterpret_cast<const V *>(a.tabs);
    const BatchStep *__restrict__ steps = a.steps;

    for (;;) {
        if (tid == 0) {
            const int64_t item = (int64_t)atomicAdd(a.ticket, 1ull);
            int ok = 1, si = 0;
            if (item < a.nitems) {
                si = find_step(steps, a.nsteps, item);
                const int prev = steps[si].prev;
                if (prev >= 0) {
                    const unsigned need = (unsigned)steps[prev].chunks;
                    int64_t spins = 0;
                    while (__hip_atomic_load(&a.done[prev], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                            ++spins > a.spin_limit) {
                            __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            ok = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
            }
            s_item = item;
            s_step = si;
            s_ok = ok;
        }
        __syncthreads();
        // values shared through LDS are uniform; readfirstlane tells the
        // compiler so, keeping the step's descriptor in scalar registers
        const int64_t item = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(s_item >> 32)) << 32) |
                                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(s_item & 0xffffffff)));
        const int ok = __builtin_amdgcn_readfirstlane(s_ok);
        if (item >= a.nitems || !ok) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int si = __builtin_amdgcn_readfirstlane(s_step);
        const BatchStep &st = steps[si];
        const PassProg &pp = st.pp;
        if (pp.has_phase && si != tab_step) {
            load_phase_table(tab, tabs + st.tab_off, pp.phase_levels, tid, NT);
            __syncthreads();
            tab_step = si;
        }
        const int64_t chunk = item - st.item0;
        const int64_t t0 = chunk * st.tiles_per_chunk;
        const int64_t t1 = t0 + st.tiles_per_chunk < pp.ntiles ? t0 + st.tiles_per_chunk : pp.ntiles;
        double acc[kSlots] = {0.0, 0.0, 0.0, 0.0};
        if (st.mode == kModeTan) run_item<V, T, kModeTan>(st, t0, t1, lds, tab, acc, tid);
        else run_item<V, T, kModeGeneral>(st, t0, t1, lds, tab, acc, tid);
        block_sum(acc, red, tid, NT);
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < kSlots; ++k) a.partials[item * kSlots + k] = acc[k];
        }
        // every thread's stores (and the partial sums) are released before the
        // item is counted as done
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) __hip_atomic_fetch_add(&a.done[si], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One workgroup per step: that step's phase table.  Forward passes, and
// reverse passes in tangent form that undo a phase, carry the tangent-form
// factor of their stages (see rev_tile); the others use the plain phase.
template <typename V>
__global__ void __launch_bounds__(256) batch_table_kernel(const BatchStep *steps, V *tabs)
{
    const BatchStep &st = steps[blockIdx.x];
    if (!st.pp.has_phase || st.tab_off < 0) return;
    const bool fold = st.kind == 2 && st.mode == kModeTan && !st.pp.init;  // run_item runs kModeTan or general
    const double f = st.kind == 0 || fold ? st.pp.factor : 1.0;
    build_phase_table(tabs + st.tab_off, st.pp.phase_levels, st.pp.theta_zz, st.pp.W, f, threadIdx.x, 256);
}

// One workgroup per circuit, fixed order: steps in the listed order, items in order.
__global__ void __launch_bounds__(256) batch_reduce_kernel(const BatchStep *steps, const int *cstep,
                                                           const int *cstep_off, const int64_t *res_off,
                                                           const double *partials, double *res)
{
    __shared__ double red[kSlots * 4];
    const int c = blockIdx.x;
    for (int j = cstep_off[c]; j < cstep_off[c + 1]; ++j) {
        const BatchStep &st = steps[cstep[j]];
        double acc[kSlots] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t i = threadIdx.x; i < st.chunks; i += 256) {
#pragma unroll
            for (int k = 0; k < kSlots; ++k) acc[k] += partials[(st.item0 + i) * kSlots + k];
        }
        block_sum(acc, red, threadIdx.x, 256);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < kSlots; ++k)
                if (st.map[k] >= 0) res[res_off[c] + st.map[k]] += acc[k];
        }
        __syncthreads();
    }
}

}  // namespace

int batch_table_entries() { return kTabMax; }

int64_t batch_grid(int prec)
{
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (prec == 0)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<float2, kTileBitsC64>, 1 << TBB, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<double2, kTileBitsC128>, 1 << TBB,
                                                           0);
    if (per_cu < 1) per_cu = 1;
    return (int64_t)cus * per_cu;
}

hipError_t launch_batch_tables(int prec, const BatchStep *steps, int nsteps, void *tabs, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL(batch_table_kernel<float2>, dim3(nsteps), dim3(256), 0, st, steps, (float2 *)tabs);
    else
        hipLaunchKernelGGL(batch_table_kernel<double2>, dim3(nsteps), dim3(256), 0, st, steps, (double2 *)tabs);
    return hipGetLastError();
}

hipError_t launch_batch(int prec, const BatchArgs &a, int64_t grid, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL((batch_kernel<float2, kTileBitsC64>), dim3((unsigned)grid), dim3(1 << TBB), 0, st, a);
    else
        hipLaunchKernelGGL((batch_kernel<double2, kTileBitsC128>), dim3((unsigned)grid), dim3(1 << TBB), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchStep *steps, const int *cstep, const int *cstep_off, const int64_t *res_off,
                               const double *partials, double *res, int ncircuits, hipStream_t st)
{
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(ncircuits), dim3(256), 0, st, steps, cstep, cstep_off, res_off,
                       partials, res);
    return hipGetLastError();
}

}  // namespace qs
