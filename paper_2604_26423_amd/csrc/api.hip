// C ABI of libqs (declared in include/qs.h): argument checks, the pass plan of
// the fused forward circuit and of the adjoint sweep, scratch management and
// per-kernel event timing.  Every entry point checks its arguments before it
// queues GPU work, and converts every failure into a qs_status plus a
// thread-local message; no C++ exception leaves this file.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qs.h"
#include "../../include/qs_debug.h"
#include "internal.h"
#include "plan.h"

using namespace qs;

namespace {

thread_local std::string g_err;

qs_status fail(qs_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

qs_status hip_fail(hipError_t e, const char *where)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(QS_ERR_OOM, "%s: out of device memory (%s)", where, hipGetErrorString(e));
    return fail(QS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIPCHK(call, where)                           \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

int max_qubits(int prec) { return prec == QS_C64 ? QS_MAX_QUBITS_C64 : QS_MAX_QUBITS_C128; }

// Split a precision argument into the precision and the QS_SYM flag; false if invalid.
bool parse_prec(int arg, int *prec, int *sym)
{
    *sym = (arg & QS_SYM) ? 1 : 0;
    *prec = arg & ~QS_SYM;
    return *prec == QS_C64 || *prec == QS_C128;
}

// Qubit range of a layout: the symmetric one needs more than a tile of stored bits.
int min_qubits(int prec, int sym) { return sym ? (prec == QS_C64 ? kTileBitsC64 : kTileBitsC128) + 2 : 1; }
int max_qubits(int prec, int sym) { return sym ? max_qubits(prec) + 1 : max_qubits(prec); }
size_t amp_bytes(int prec) { return prec == QS_C64 ? 8 : 16; }
bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

struct ProfRec {
    int kind;
    double bytes;
    hipEvent_t a, b;
};

// Grow-only device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    hipError_t ensure(size_t need)
    {
        if (need <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, need);
        if (e == hipSuccess) bytes = need;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

}  // namespace

namespace qs {
qs_status set_error(qs_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}
}  // namespace qs

struct qs_state_s {
    int n = 0, prec = 0;  // n: stored index bits (qubits, or qubits - 1 when sym)
    int nq = 0, sym = 0;  // qubits; complement-symmetric layout
    void *psi = nullptr;
    bool own = false;
    hipStream_t stream = nullptr;
    DevBuf partials, tmp, results, sample, shots_out, lambda, hist, xfer, tab, wts, ctab;
    int cut_mode = 0;     // qs_debug_set_cut_mode
    bool cut_on = false;  // this call's passes take cut tables
    bool prof = false;
    std::vector<ProfRec> recs;
};

struct qs_noise_s {
    int n = 0, prec = 0;
    hipStream_t stream = nullptr;
    int64_t W = 0;
    int32_t cmax = 0;
    DevBuf diag, edges, layers, tabs;
    std::vector<double> layers_h;
};

struct qs_batch_s {
    int count = 0, prec = 0;
    hipStream_t stream = nullptr;
    std::vector<int> n, p;
    std::vector<int64_t> W, angle_off;
    std::vector<int32_t> cmax;
    std::vector<size_t> off_psi, off_lam, off_diag;
    void *mem = nullptr;
    DevBuf steps, tabs, partials, counters, results, index;
    std::vector<qs::BatchStep> steps_h;
    std::vector<int> idx_h;        // cstep list, then cstep offsets
    std::vector<int64_t> res_off_h;
    std::vector<double> res_h;
};

namespace {

// ---------------------------------------------------------------- profiling
struct Launch {
    qs_state s;
    int kind;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    Launch(qs_state s_, int k, double by) : s(s_), kind(k), bytes(by)
    {
        if (s && s->prof) {
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            (void)hipEventRecord(a, s->stream);
        }
    }
    void done()
    {
        if (s && s->prof && a) {
            (void)hipEventRecord(b, s->stream);
            s->recs.push_back(ProfRec{kind, bytes, a, b});
            a = b = nullptr;
        }
    }
    ~Launch()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

void clear_prof(qs_state s)
{
    for (auto &r : s->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    s->recs.clear();
}

struct Circuit {
    const int32_t *diag;
    int64_t W;
    int p;
    const double *tzz, *tx;
};

// RX(theta) of one stage over m qubits: tangent form when |cos(theta/2)| >= 1/2.
RxStage rx_stage(double theta, int m, double *factor)
{
    RxStage st{};
    st.c = cos(0.5 * theta);
    st.s = sin(0.5 * theta);
    st.tan = fabs(st.c) >= 0.5 ? 1 : 0;
    st.u = st.tan ? st.s / st.c : 0.0;
    *factor = st.tan ? pow(st.c, m) : 1.0;
    return st;
}

// Gradient scales of a reverse stage over the window sequence w of a kernel
// with 2^tb threads (RxStage::wsc): the windows are undone from the last, each
// undoing the factors of the stage it holds that no later window held.
void stage_scales(RxStage &st, const WinSeq &w, uint32_t targets, uint32_t pairs, int T, int tb)
{
    const int rb = T - tb;
    const double c2 = st.tan ? st.c * st.c : 1.0;
    double sc = 1.0;
    uint32_t done = 0, pdone = 0;
    for (int i = 0; i < kMaxWindows; ++i) st.wsc[i] = 1.0;
    for (int i = std::min(w.cnt, kMaxWindows) - 1; i >= 0; --i) {
        const uint32_t mask = targets & (((1u << rb) - 1u) << w.s[i]) & ~done;
        const uint32_t pm = pairs & (((1u << (rb - 1)) - 1u) << w.s[i]) & ~pdone;
        st.wsc[i] = sc;
        for (int b = __builtin_popcount(mask) + __builtin_popcount(pm); b > 0; --b) sc *= c2;
        done |= mask;
        pdone |= pm;
    }
}

// Last window of a sequence.  A sequence longer than kMaxWindows (flagged by
// plan_windows) never occurs for a supported n -- qs_plan_check verifies every
// plan -- and the clamp keeps the read inside the array regardless.
static int last_window(const WinSeq &w)
{
    return w.s[std::min(std::max(w.cnt, 1), kMaxWindows) - 1];
}

PassProg make_prog_raw(void *psi, int n, int prec, double *partials, const PassGeom &g, const KSpec &k,
                       const Circuit &cc, int tb, int sym = 0)
{
    const int T = tile_bits(prec);
    PassProg pp{};
    pp.psi = psi;
    pp.lam = nullptr;
    pp.psi_out = psi;
    pp.diag = cc.diag;
    pp.partials = partials;
    pp.ntiles = (int64_t)1 << (n - T);
    pp.tb = tb;
    pp.n = n;
    pp.c = g.c;
    pp.q0 = g.q0;
    pp.targets = g.targets;
    pp.pairs = g.pairs;
    pp.ntargets = __builtin_popcount(g.targets) + __builtin_popcount(g.pairs);
    pp.width = T - g.c;
    pp.init = k.init;
    pp.has_pre = k.pre >= 0;
    pp.has_phase = k.phase >= 0;
    pp.has_post = k.post >= 0;
    pp.readout = k.readout;
    pp.load_win = tb;
    pp.fpre = pp.fpost = 1.0;
    if (pp.has_pre) {
        pp.A = plan_windows(tb, g.targets, g.pairs, T, tb);
        pp.B = plan_windows(last_window(pp.A), g.targets, g.pairs, T, tb);
        pp.pre = rx_stage(cc.tx[k.pre], pp.ntargets, &pp.fpre);
    } else {
        pp.B = plan_windows(tb, g.targets, g.pairs, T, tb);
    }
    if (pp.has_post) pp.post = rx_stage(cc.tx[k.post], pp.ntargets, &pp.fpost);
    if (pp.has_pre) stage_scales(pp.pre, pp.A, g.targets, g.pairs, T, tb);
    if (pp.has_post) stage_scales(pp.post, pp.B, g.targets, g.pairs, T, tb);
    pp.factor = pp.fpre * pp.fpost;
    pp.phase_win = pp.has_pre ? last_window(pp.A) : pp.load_win;
    pp.final_win = last_window(pp.B);
    if (pp.has_phase) pp.theta_zz = cc.tzz[k.phase];
    pp.W = cc.W;
    pp.phase_levels = phase_table_levels(cc.W);
    pp.amp0 = sqrt(ldexp(1.0, -(n + sym)));
    pp.lam_shift = 0.5 * (double)cc.W;
    return pp;
}

// kind: 0 = forward pass, 1 = turnaround, 2 = reverse pass (the cut table is
// attached when the kernel for the pass takes one).
PassProg make_prog(qs_state s, const PassGeom &g, const KSpec &k, const Circuit &cc, int tb, int kind = 0)
{
    PassProg pp = make_prog_raw(s->psi, s->n, s->prec, (double *)s->partials.p, g, k, cc, tb, s->sym);
    if (s->cut_on && pass_takes_cut_table(s->prec, pp, kind)) {
        pp.ctab = (int32_t *)s->ctab.p;
        pp.wts = (const int32_t *)s->wts.p;
    }
    return pp;
}

// Tile passes of the full layout evaluate C_t in registers (see the cut-value
// notes in internal.h) from n = kCutMinQubits on, or as qs_debug_set_cut_mode
// says: recover the weights from the diagonal of this call and size the
// per-pass cut table.
qs_status prepare_cut(qs_state s, const Circuit &cc, const char *where)
{
    s->cut_on = false;
    if (s->sym || s->n <= tile_bits(s->prec)) return QS_OK;
    if (s->cut_mode == 2 || (s->cut_mode == 0 && s->n < kCutMinQubits)) return QS_OK;
    HIPCHK(s->wts.ensure((size_t)kWtSize * sizeof(int32_t)), where);
    HIPCHK(s->ctab.ensure((size_t)cut_table_entries(s->n, s->prec) * sizeof(int32_t)), where);
    HIPCHK(launch_cut_weights(cc.diag, s->n, cc.W, (int32_t *)s->wts.p, s->stream), where);
    s->cut_on = true;
    return QS_OK;
}

// Pass plan of a state's layout.
std::vector<PassGeom> plan_for(qs_state s)
{
    return s->sym ? plan_passes_sym(s->nq, s->prec) : plan_passes(s->n, s->prec);
}

// Launch one tile kernel over a persistent grid; returns the grid (the number
// of per-workgroup partial sums it writes).
qs_status launch_tiles(qs_state s, PassProg &pp, int adjoint, int turnaround, int kind, double bytes,
                       int64_t *grid_out, const char *where)
{
    // adjoint: 0 = forward pass, 1 = turnaround, 2 = reverse pass
    const int64_t grid = tile_grid(s->prec, adjoint, pp);
    pp.xcd_remap = (grid % 8 == 0) ? 1 : 0;
    pp.tab = s->tab.p;
    Launch L(s, kind, bytes);
    HIPCHK(adjoint ? launch_adjoint_pass(s->prec, pp, turnaround, grid, s->stream)
                   : launch_pass(s->prec, pp, grid, s->stream),
           where);
    L.done();
    if (grid_out) *grid_out = grid;
    return QS_OK;
}


double pass_bytes(qs_state s, const PassProg &pp)
{
    const double dim = ldexp(1.0, s->n), a = (double)amp_bytes(s->prec);
    double b = dim * a * (pp.init ? 1.0 : 2.0);
    if ((pp.has_phase || pp.readout) && !pp.ctab) b += dim * 4.0;
    return b;
}

hipError_t ensure_partials(qs_state s, int64_t count)
{
    hipError_t e = s->partials.ensure((size_t)count * kSlots * sizeof(double));
    if (e != hipSuccess) return e;
    e = s->tmp.ensure((size_t)std::max<int64_t>(reduce_tmp_doubles(count), kSlots) * sizeof(double));
    if (e != hipSuccess) return e;
    return s->tab.ensure(pass_table_bytes());
}

// Small zero-fill kernel (kept out of hipMemsetAsync so that the work can be
// captured into a graph).
__global__ void zero_kernel(double *p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

hipError_t zero_results(qs_state s, int count)
{
    hipLaunchKernelGGL(zero_kernel, dim3((count + 255) / 256), dim3(256), 0, s->stream, (double *)s->results.p,
                       count);
    return hipGetLastError();
}

qs_status read_results(qs_state s, double *host, int count, const char *where)
{
    HIPCHK(hipMemcpyAsync(host, s->results.p, count * sizeof(double), hipMemcpyDeviceToHost, s->stream), where);
    HIPCHK(hipStreamSynchronize(s->stream), where);
    return QS_OK;
}

qs_status check_state(qs_state s)
{
    if (!s) return fail(QS_ERR_ARG, "null state handle");
    return QS_OK;
}

qs_status check_angles(int p, const double *tzz, const double *tx)
{
    if (p < 0) return fail(QS_ERR_ARG, "p must be >= 0 (got %d)", p);
    if (p > 0 && (!tzz || !tx)) return fail(QS_ERR_ARG, "null angle array");
    for (int k = 0; k < p; ++k)
        if (!std::isfinite(tzz[k]) || !std::isfinite(tx[k])) return fail(QS_ERR_ARG, "non-finite angle at layer %d", k);
    return QS_OK;
}

qs_status check_diag(qs_state s, const int32_t *diag, int64_t W)
{
    if (!diag) return fail(QS_ERR_ARG, "null cost diagonal");
    if (!aligned(diag, 16)) return fail(QS_ERR_ARG, "cost diagonal must be 16-byte aligned");
    if (W < 0 || W >= ((int64_t)1 << 31)) return fail(QS_ERR_RANGE, "W_t out of range: %lld", (long long)W);
    (void)s;
    return QS_OK;
}

// ---------------------------------------------------------------- forward
qs_status run_small_forward(qs_state s, const Circuit &cc, bool readout, const char *where)
{
    // chunks of kSmallMaxLayers layers; readout in the last chunk
    int k0 = 0;
    bool first = true;
    do {
        SmallProg sp{};
        sp.psi = s->psi;
        sp.diag = cc.diag;
        sp.out = (double *)s->results.p;
        sp.n = s->n;
        sp.init = first ? 1 : 0;
        sp.nlayers = std::min(kSmallMaxLayers, cc.p - k0);
        sp.readout = (readout && k0 + sp.nlayers >= cc.p) ? 1 : 0;
        sp.W = cc.W;
        for (int L = 0; L < sp.nlayers; ++L) {
            sp.tzz[L] = cc.tzz[k0 + L];
            sp.tx[L] = cc.tx[k0 + L];
            sp.do_phase[L] = 1;
            sp.do_mixer[L] = 1;
        }
        sp.amp0 = sqrt(ldexp(1.0, -s->n));
        Launch L(s, QS_KIND_SMALL, ldexp(1.0, s->n) * amp_bytes(s->prec) * 2);
        HIPCHK(launch_small_forward(s->prec, sp, s->stream), where);
        L.done();
        k0 += sp.nlayers;
        first = false;
    } while (k0 < cc.p);
    return QS_OK;
}

qs_status run_reduce(qs_state s, int64_t count, const int *map, int accumulate, const char *where)
{
    Launch L(s, QS_KIND_REDUCE, (double)count * kSlots * 8);
    HIPCHK(launch_reduce((const double *)s->partials.p, count, (double *)s->tmp.p, (double *)s->results.p, map,
                         accumulate, s->stream),
           where);
    L.done();
    return QS_OK;
}

// Fused forward circuit.  With readout, results[0] = norm, results[1] = sum |a|^2 C_t.
qs_status run_forward(qs_state s, const Circuit &cc, bool readout, const char *where)
{
    const int T = tile_bits(s->prec);
    HIPCHK(s->results.ensure(64 * sizeof(double)), where);
    if (cc.p == 0) {
        Launch L(s, QS_KIND_ELEMENTWISE, ldexp(1.0, s->n) * amp_bytes(s->prec));
        HIPCHK(launch_init_plus(s->prec, s->psi, s->n, s->nq, s->stream), where);
        L.done();
        if (readout) {
            int64_t nb = 0;
            HIPCHK(ensure_partials(s, 16384), where);
            Launch E(s, QS_KIND_EXPECT, ldexp(1.0, s->n) * (amp_bytes(s->prec) + 4));
            HIPCHK(launch_expect(s->prec, s->psi, cc.diag, s->n, (double *)s->partials.p, &nb, s->stream), where);
            E.done();
            const int map[kSlots] = {0, 1, -1, -1};
            return run_reduce(s, nb, map, 0, where);
        }
        return QS_OK;
    }
    if (s->n <= T) return run_small_forward(s, cc, readout, where);

    const std::vector<PassGeom> geo = plan_for(s);
    std::vector<KSpec> ks = forward_specs((int)geo.size(), cc.p, !s->sym);
    if (readout) ks.back().readout = 1;
    HIPCHK(ensure_partials(s, pass_grid(s->prec, 0, (int64_t)1 << (s->n - T))), where);
    if (qs_status st = prepare_cut(s, cc, where)) return st;
    int64_t grid = 0;
    for (const KSpec &k : ks) {
        PassProg pp = make_prog(s, geo[k.pass], k, cc, kFwdThreadBits);
        if (qs_status st = launch_tiles(s, pp, 0, 0, pp.has_phase ? QS_KIND_PASS_PHASE : QS_KIND_PASS,
                                        pass_bytes(s, pp), &grid, where))
            return st;
    }
    if (readout) {
        const int map[kSlots] = {0, 1, -1, -1};
        return run_reduce(s, grid, map, 0, where);
    }
    return QS_OK;
}

// ---------------------------------------------------------------- adjoint
// results layout: [0] norm, [1] sum |a|^2 C_t, [2 + k] dE/dtheta_zz[k], [2 + p + k] dE/dtheta_x[k]
qs_status run_small_adjoint(qs_state s, const Circuit &cc, void *lam, const char *where)
{
    if (qs_status st = run_small_forward(s, cc, false, where)) return st;
    const int nch = (cc.p + kSmallMaxLayers - 1) / kSmallMaxLayers;
    for (int ch = nch - 1; ch >= 0; --ch) {
        SmallProg sp{};
        sp.psi = s->psi;
        sp.lam = lam;
        sp.diag = cc.diag;
        sp.out = (double *)s->results.p;
        sp.n = s->n;
        sp.layer0 = ch * kSmallMaxLayers;
        sp.nlayers = std::min(kSmallMaxLayers, cc.p - sp.layer0);
        sp.ptotal = cc.p;
        sp.W = cc.W;
        for (int L = 0; L < sp.nlayers; ++L) {
            sp.tzz[L] = cc.tzz[sp.layer0 + L];
            sp.tx[L] = cc.tx[sp.layer0 + L];
            sp.do_phase[L] = 1;
            sp.do_mixer[L] = 1;
        }
        sp.turnaround = (ch == nch - 1) ? 1 : 0;
        sp.store = 1;
        sp.amp0 = sqrt(ldexp(1.0, -s->n));
        sp.lam_shift = 0.5 * (double)cc.W;
        Launch L(s, QS_KIND_SMALL, ldexp(1.0, s->n) * amp_bytes(s->prec) * 4);
        HIPCHK(launch_small_adjoint(s->prec, sp, s->stream), where);
        L.done();
    }
    return QS_OK;
}

// Tile passes of the forward circuit for p layers (0 when one workgroup holds
// the state).
int64_t forward_pass_count(qs_state s, int p)
{
    if (s->n <= tile_bits(s->prec)) return 0;
    return (int64_t)forward_specs((int)plan_for(s).size(), p, !s->sym).size();
}

// States a checkpointing adjoint keeps besides the state buffer: the outputs
// of forward passes 0 .. P-3 (the output of pass P-2 stays in the state
// buffer, where the turnaround reads it).
int64_t ckpt_states(qs_state s, int p)
{
    const int64_t P = forward_pass_count(s, p);
    return P > 2 ? P - 2 : 0;
}

// ckpt == nullptr: uncompute (the reverse passes undo every pass on psi).
// Otherwise store: the forward writes the output of pass i to checkpoint i
// (ckpt + i states, the state buffer for i = P-2) and reverse pass i reads
// psi from checkpoint i and stores lambda only.
qs_status run_adjoint(qs_state s, const Circuit &cc, void *lam, const char *where, void *ckpt = nullptr)
{
    const int T = tile_bits(s->prec);
    const int nres = 2 + 2 * cc.p;
    HIPCHK(s->results.ensure((size_t)std::max(64, nres) * sizeof(double)), where);
    HIPCHK(zero_results(s, nres), where);
    if (s->n <= T) return run_small_adjoint(s, cc, lam, where);

    const std::vector<PassGeom> geo = plan_for(s);
    const std::vector<KSpec> ks = forward_specs((int)geo.size(), cc.p, !s->sym);
    const int64_t ntiles = (int64_t)1 << (s->n - T);
    HIPCHK(ensure_partials(s, ntiles), where);  // no tile kernel has more workgroups than tiles
    if (qs_status st = prepare_cut(s, cc, where)) return st;
    const double dim = ldexp(1.0, s->n), ab = (double)amp_bytes(s->prec);

    int64_t grid = 0;

    const int P = (int)ks.size();
    const size_t sb = qs_state_bytes(s->n, s->prec);
    auto ck = [&](int i) -> void * { return i == P - 2 ? s->psi : (void *)((char *)ckpt + (size_t)i * sb); };

    // forward, all but the last pass
    for (int i = 0; i + 1 < P; ++i) {
        PassProg pp = make_prog(s, geo[ks[i].pass], ks[i], cc, kFwdThreadBits);
        if (ckpt) {
            if (i > 0) pp.psi = ck(i - 1);
            pp.psi_out = ck(i);
        }
        if (qs_status st = launch_tiles(s, pp, 0, 0, pp.has_phase ? QS_KIND_PASS_PHASE : QS_KIND_PASS,
                                        pass_bytes(s, pp), &grid, where))
            return st;
    }
    // turnaround: the last pass forward, lambda = C psi, the pass undone
    {
        const KSpec &k = ks.back();
        // one-tile kernels run 256 threads (5-bit windows), the persistent
        // kernel 512; the complement-symmetric layout keeps 512 threads (256
        // measured no faster there)
        PassProg pp = make_prog(s, geo[k.pass], k, cc, kAdjOneThreadBits, 1);
        if (s->sym || !adjoint_one_tile(s->prec, pp, 1)) pp = make_prog(s, geo[k.pass], k, cc, kAdjThreadBits, 1);
        pp.lam = lam;
        if (qs_status st = launch_tiles(s, pp, 1, 1, QS_KIND_TURNAROUND, dim * (2.0 * ab + (pp.ctab ? 0.0 : 4.0)),
                                        &grid, where))
            return st;
        const int map[kSlots] = {2 + cc.p + k.post, 0, 1, -1};
        if (qs_status st = run_reduce(s, grid, map, 1, where)) return st;
    }
    // reverse passes
    for (int i = (int)ks.size() - 2; i >= 0; --i) {
        const KSpec &k = ks[i];
        PassProg pp = make_prog(s, geo[k.pass], k, cc, kAdjOneThreadBits, 2);
        if (s->sym || !adjoint_one_tile(s->prec, pp, 0)) pp = make_prog(s, geo[k.pass], k, cc, kAdjThreadBits, 2);
        pp.lam = lam;
        pp.load_win = pp.final_win;
        if (ckpt) {
            pp.psi = ck(i);
            pp.psi_out = nullptr;
        }
        const double by = dim * ab * (pp.init ? 2.0 : ckpt ? 3.0 : 4.0) + (pp.has_phase && !pp.ctab ? dim * 4.0 : 0.0);
        if (qs_status st = launch_tiles(s, pp, 2, 0, QS_KIND_ADJOINT, by, &grid, where)) return st;
        const int map[kSlots] = {k.post >= 0 ? 2 + cc.p + k.post : -1, k.phase >= 0 ? 2 + k.phase : -1,
                                 k.pre >= 0 ? 2 + cc.p + k.pre : -1, -1};
        if (qs_status st = run_reduce(s, grid, map, 1, where)) return st;
    }
    return QS_OK;
}

// Device-memory layout of a batch: per-circuit state, adjoint vector and
// diagonal offsets (256-byte aligned) and angle offsets; returns the bytes.
size_t layout_batch(qs_batch b, int count, const qs_circuit *circuits, int prec)
{
    b->count = count;
    b->prec = prec;
    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    int64_t aoff = 0;
    for (int i = 0; i < count; ++i) {
        const int n = circuits[i].n;
        b->n.push_back(n);
        b->p.push_back(circuits[i].p);
        b->angle_off.push_back(aoff);
        aoff += circuits[i].p;
        b->off_psi.push_back(place(qs_state_bytes(n, prec)));
        b->off_lam.push_back(place(qs_state_bytes(n, prec)));
        b->off_diag.push_back(place(((size_t)1 << n) * 4));
        int64_t W = 0;
        for (size_t e = 0; e < (size_t)n * (n - 1) / 2; ++e) W += circuits[i].w_tenths[e];
        b->W.push_back(W);
    }
    b->angle_off.push_back(aoff);
    return off;
}

struct BatchSchedule {
    int64_t items = 0, tabs = 0, nres = 0;
    int nidx = 0;
};

// The steps of every circuit (forward passes, turnaround, reverse passes) in
// round order -- step r of every circuit, largest circuits first -- with item
// numbers, predecessor links, table offsets and the per-circuit step lists
// used by the reduction.  Host only: pointers into b->mem are computed, never
// dereferenced.
BatchSchedule build_batch_schedule(qs_batch b, const double *theta_zz, const double *theta_x)
{
    BatchSchedule sch;
    const int T = tile_bits(b->prec);
    const int count = b->count;
    // per-circuit step lists (in the circuit's own order)
    std::vector<std::vector<BatchStep>> cs(count);
    for (int c = 0; c < count; ++c) {
        const int n = b->n[c], p = b->p[c];
        void *psi = (char *)b->mem + b->off_psi[c];
        void *lam = (char *)b->mem + b->off_lam[c];
        const int32_t *diag = (const int32_t *)((char *)b->mem + b->off_diag[c]);
        const Circuit cc{diag, b->W[c], p, theta_zz + b->angle_off[c], theta_x + b->angle_off[c]};
        const std::vector<PassGeom> geo = plan_passes(n, b->prec);
        const std::vector<KSpec> ks = forward_specs((int)geo.size(), p, true);
        auto add = [&](const KSpec &k, int kind) {
            BatchStep s{};
            s.pp = make_prog_raw(psi, n, b->prec, nullptr, geo[k.pass], k, cc, kBatchThreadBits);
            s.pp.xcd_remap = 0;
            s.kind = kind;
            s.circuit = c;
            for (int j = 0; j < kSlots; ++j) s.map[j] = -1;
            if (kind >= 1) s.pp.lam = lam;
            if (kind == 1) {
                s.map[0] = 2 + p + k.post;
                s.map[1] = 0;
                s.map[2] = 1;
            } else if (kind == 2) {
                s.pp.load_win = s.pp.final_win;
                s.map[0] = k.post >= 0 ? 2 + p + k.post : -1;
                s.map[1] = k.phase >= 0 ? 2 + k.phase : -1;
                s.map[2] = k.pre >= 0 ? 2 + p + k.pre : -1;
            }
            s.mode = tile_mode(s.pp, T, kBatchThreadBits);
            const int64_t ntiles = (int64_t)1 << (n - T);
            s.tiles_per_chunk = (int)std::min<int64_t>(ntiles, 16);
            s.chunks = (int)((ntiles + s.tiles_per_chunk - 1) / s.tiles_per_chunk);
            cs[c].push_back(s);
        };
        for (size_t i = 0; i + 1 < ks.size(); ++i) add(ks[i], 0);
        add(ks.back(), 1);
        for (int i = (int)ks.size() - 2; i >= 0; --i) add(ks[i], 2);
    }
    // rounds: step r of every circuit, the largest circuits first
    std::vector<int> order(count);
    for (int c = 0; c < count; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const double wx = ldexp((double)cs[x].size(), b->n[x]), wy = ldexp((double)cs[y].size(), b->n[y]);
        return wx > wy;
    });
    size_t maxsteps = 0;
    for (int c = 0; c < count; ++c) maxsteps = std::max(maxsteps, cs[c].size());
    b->steps_h.clear();
    std::vector<std::vector<int>> where_c(count);
    std::vector<int> last(count, -1);
    int64_t &items = sch.items, &tabs = sch.tabs;
    const int tabn = batch_table_entries();
    for (size_t r = 0; r < maxsteps; ++r)
        for (int c : order) {
            if (r >= cs[c].size()) continue;
            BatchStep s = cs[c][r];
            s.prev = last[c];
            s.item0 = items;
            items += s.chunks;
            s.tab_off = s.pp.has_phase ? (tabs++) * tabn : -1;
            last[c] = (int)b->steps_h.size();
            where_c[c].push_back(last[c]);
            b->steps_h.push_back(s);
        }
    b->idx_h.clear();
    std::vector<int> coff(count + 1, 0);
    for (int c = 0; c < count; ++c) {
        coff[c] = (int)b->idx_h.size();
        for (int j : where_c[c]) b->idx_h.push_back(j);
    }
    coff[count] = (int)b->idx_h.size();
    sch.nidx = (int)b->idx_h.size();
    b->idx_h.insert(b->idx_h.end(), coff.begin(), coff.end());
    b->res_off_h.assign(count + 1, 0);
    for (int c = 0; c < count; ++c) b->res_off_h[c + 1] = b->res_off_h[c] + 2 + 2 * b->p[c];
    sch.nres = b->res_off_h[count];
    return sch;
}

// ---------------------------------------------------------------- diagonal helpers
// Dense symmetric weight matrix from the lexicographic edge list, with checks.
// wm: n * n entries, filled (diagonal zero).
qs_status weight_matrix(int n, const int32_t *w, int32_t *wm, int64_t *W)
{
    const int64_t ne = (int64_t)n * (n - 1) / 2;
    if (ne > 0 && !w) return fail(QS_ERR_ARG, "null weight array");
    for (int64_t i = 0; i < (int64_t)n * n; ++i) wm[i] = 0;
    int64_t sum = 0, e = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j, ++e) {
            const int32_t x = w[e];
            if (x < 0 || x >= (1 << 20)) return fail(QS_ERR_ARG, "weight %lld = %d outside [0, 2^20)", (long long)e, x);
            wm[(size_t)i * n + j] = wm[(size_t)j * n + i] = x;
            sum += x;
        }
    if (sum >= ((int64_t)1 << 31)) return fail(QS_ERR_RANGE, "W_t = %lld does not fit in int32", (long long)sum);
    *W = sum;
    return QS_OK;
}

DiagScratch diag_scratch_layout(int nmax, int nres, int sym = 0)
{
    return diag_scratch_plan(nmax, nres, diag_wg_count(nmax, sym));
}

// Queue the diagonal of one circuit; its C_max lands in result slot `res`.
// `wm` must stay alive until the stream has run the copy.
hipError_t build_diagonal(int n, const int32_t *wm, int32_t *diag, char *scratch, const DiagScratch &L,
                          int res, hipStream_t st, int sym = 0)
{
    hipError_t e = hipMemcpyAsync(scratch, wm, (size_t)n * n * 4, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return launch_cost_diagonal(n, (const int32_t *)scratch, diag, (int32_t *)(scratch + L.off_low),
                                (int32_t *)(scratch + L.off_wg), (int32_t *)(scratch + L.off_tmp),
                                (int32_t *)(scratch + L.off_res) + res, st, sym);
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char *qs_last_error(void) { return g_err.c_str(); }

const char *qs_version(void) { return "libqs 0.1 (gfx950)"; }

size_t qs_state_bytes(int n, int prec_arg)
{
    int prec, sym;
    if (!parse_prec(prec_arg, &prec, &sym)) return 0;
    if (n < min_qubits(prec, sym) || n > max_qubits(prec, sym)) return 0;
    return ((size_t)1 << (n - sym)) * amp_bytes(prec);
}

qs_status qs_alloc(int n, int prec_arg, void *dev_buf, size_t buf_bytes, void *hip_stream, qs_state *out)
{
    try {
        if (!out) return fail(QS_ERR_ARG, "null output handle pointer");
        *out = nullptr;
        int prec, sym;
        if (!parse_prec(prec_arg, &prec, &sym)) return fail(QS_ERR_ARG, "bad precision %d", prec_arg);
        if (n < min_qubits(prec, sym) || n > max_qubits(prec, sym))
            return fail(QS_ERR_ARG, "n = %d outside %d..%d for this precision and layout", n, min_qubits(prec, sym),
                        max_qubits(prec, sym));
        const size_t need = qs_state_bytes(n, prec_arg);
        if (dev_buf) {
            if (buf_bytes < need) return fail(QS_ERR_ARG, "buffer too small: %zu < %zu bytes", buf_bytes, need);
            if (!aligned(dev_buf, 256)) return fail(QS_ERR_ARG, "state buffer must be 256-byte aligned");
        }
        qs_state s = new qs_state_s();
        s->n = n - sym;
        s->nq = n;
        s->sym = sym;
        s->prec = prec;
        s->stream = (hipStream_t)hip_stream;
        if (dev_buf) {
            s->psi = dev_buf;
        } else {
            hipError_t e = hipMalloc(&s->psi, need);
            if (e != hipSuccess) {
                delete s;
                return hip_fail(e, "qs_alloc");
            }
            s->own = true;
        }
        *out = s;
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_alloc: host allocation failed");
    }
}

qs_status qs_free(qs_state s)
{
    if (!s) return QS_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    clear_prof(s);
    if (s->own && s->psi) (void)hipFree(s->psi);
    s->partials.release();
    s->tmp.release();
    s->results.release();
    s->sample.release();
    s->shots_out.release();
    s->xfer.release();
    s->lambda.release();
    delete s;
    return QS_OK;
}

qs_status qs_state_ptr(qs_state s, void **dev_ptr)
{
    if (qs_status st = check_state(s)) return st;
    if (!dev_ptr) return fail(QS_ERR_ARG, "null output pointer");
    *dev_ptr = s->psi;
    return QS_OK;
}

qs_status qs_set_stream(qs_state s, void *hip_stream)
{
    if (qs_status st = check_state(s)) return st;
    s->stream = (hipStream_t)hip_stream;
    return QS_OK;
}

qs_status qs_init_plus(qs_state s)
{
    if (qs_status st = check_state(s)) return st;
    Launch L(s, QS_KIND_ELEMENTWISE, ldexp(1.0, s->n) * amp_bytes(s->prec));
    HIPCHK(launch_init_plus(s->prec, s->psi, s->n, s->nq, s->stream), "qs_init_plus");
    L.done();
    return QS_OK;
}

namespace {
// Scratch of qs_cost_diagonal: one grow-only buffer per device, held by a call
// from its first copy until its stream has finished (every call synchronises),
// so calls from several threads take turns instead of allocating.  The buffers
// live until the process ends.
struct DiagCache {
    std::mutex mu;
    DevBuf buf;
};

DiagCache *diag_cache(int dev)
{
    static std::mutex map_mu;
    static std::map<int, DiagCache *> caches;
    std::lock_guard<std::mutex> g(map_mu);
    DiagCache *&c = caches[dev];
    if (!c) c = new DiagCache();  // never freed: device memory outlives static destructors
    return c;
}

qs_status cost_diagonal_impl(int n, int sym, const int32_t *w_tenths, int32_t *diag_dev, int64_t *w_total_tenths,
                             int32_t *cmax_tenths, void *hip_stream)
{
    try {
        if (!diag_dev) return fail(QS_ERR_ARG, "null diagonal buffer");
        if (!aligned(diag_dev, 16)) return fail(QS_ERR_ARG, "diagonal buffer must be 16-byte aligned");
        std::vector<int32_t> wm((size_t)n * n);
        int64_t W = 0;
        if (qs_status st = weight_matrix(n, w_tenths, wm.data(), &W)) return st;
        hipStream_t st = (hipStream_t)hip_stream;
        const DiagScratch L = diag_scratch_layout(n, 1, sym);
        int dev = 0;
        HIPCHK(hipGetDevice(&dev), "qs_cost_diagonal");
        DiagCache *cache = diag_cache(dev);
        std::lock_guard<std::mutex> lock(cache->mu);
        HIPCHK(cache->buf.ensure(L.total), "qs_cost_diagonal");
        char *scratch = (char *)cache->buf.p;
        hipError_t he = build_diagonal(n, wm.data(), diag_dev, scratch, L, 0, st, sym);
        int32_t cmax = 0;
        if (he == hipSuccess) he = hipMemcpyAsync(&cmax, scratch + L.off_res, 4, hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return hip_fail(he, "qs_cost_diagonal");
        if (w_total_tenths) *w_total_tenths = W;
        if (cmax_tenths) *cmax_tenths = cmax;
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_cost_diagonal: host allocation failed");
    }
}
}  // namespace

qs_status qs_cost_diagonal(int n, const int32_t *w_tenths, int32_t *diag_dev, int64_t *w_total_tenths,
                           int32_t *cmax_tenths, void *hip_stream)
{
    if (n < 1 || n > QS_MAX_QUBITS_C64) return fail(QS_ERR_ARG, "n = %d outside 1..%d", n, QS_MAX_QUBITS_C64);
    return cost_diagonal_impl(n, 0, w_tenths, diag_dev, w_total_tenths, cmax_tenths, hip_stream);
}

qs_status qs_cost_diagonal_sym(int n, const int32_t *w_tenths, int32_t *diag_dev, int64_t *w_total_tenths,
                               int32_t *cmax_tenths, void *hip_stream)
{
    if (n < 14 || n > QS_MAX_QUBITS_C64 + 1)
        return fail(QS_ERR_ARG, "n = %d outside 14..%d", n, QS_MAX_QUBITS_C64 + 1);
    return cost_diagonal_impl(n, 1, w_tenths, diag_dev, w_total_tenths, cmax_tenths, hip_stream);
}

namespace {
// Scratch of qs_cost_diagonal_noalloc, sized for the largest diagonal
// (n = QS_MAX_QUBITS_C64: the weight matrix, the low-bit table, 2^21
// per-workgroup maxima, their partial maxima and the result; 8.04 MiB).  A
// static array in device memory: every device the library runs on holds its
// own copy until the process ends.  Host code never names the array except in
// the symbol lookup below; it passes the per-device address that lookup
// returns.  Nothing in it needs to start at zero: every kernel writes each
// word it later reads.
constexpr DiagScratch kNoallocDiag =
    diag_scratch_plan(QS_MAX_QUBITS_C64, 1, (int64_t)1 << (QS_MAX_QUBITS_C64 - kDiagLowBits));
__device__ __align__(256) char noalloc_diag_scratch[kNoallocDiag.total];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;                  // held for a whole call: calls in one process take turns
void *g_noalloc_ptr[kMaxDevices] = {};    // address of each device's copy, looked up once

qs_status noalloc_scratch(char **out, const char *where)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev), where);
    if (dev < 0 || dev >= kMaxDevices) return fail(QS_ERR_HIP, "%s: device %d beyond %d", where, dev, kMaxDevices);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_diag_scratch)), where);
        if (!p) return fail(QS_ERR_HIP, "%s: no device address for the scratch array", where);
        g_noalloc_ptr[dev] = p;
    }
    *out = (char *)g_noalloc_ptr[dev];
    return QS_OK;
}
}  // namespace

qs_status qs_cost_diagonal_noalloc(int n, const int32_t *w_tenths, int32_t *diag_dev, int64_t *w_total_tenths,
                                   int32_t *cmax_tenths, void *hip_stream)
{
    const char *where = "qs_cost_diagonal_noalloc";
    if (n < 1 || n > QS_MAX_QUBITS_C64)
        return fail(QS_ERR_ARG, "%s: n = %d outside 1..%d (the scratch array's limit)", where, n, QS_MAX_QUBITS_C64);
    if (!diag_dev) return fail(QS_ERR_ARG, "%s: null diagonal buffer", where);
    if (!aligned(diag_dev, 16)) return fail(QS_ERR_ARG, "%s: diagonal buffer must be 16-byte aligned", where);
    int32_t wm[QS_MAX_QUBITS_C64 * QS_MAX_QUBITS_C64];  // host, on the stack
    int64_t W = 0;
    if (qs_status st = weight_matrix(n, w_tenths, wm, &W)) return st;
    const DiagScratch L = diag_scratch_layout(n, 1);
    if (L.total > kNoallocDiag.total) return fail(QS_ERR_ARG, "%s: scratch of n = %d exceeds the array", where, n);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    char *scratch_dev = nullptr;
    if (qs_status st = noalloc_scratch(&scratch_dev, where)) return st;
    hipStream_t st = (hipStream_t)hip_stream;
    int32_t cmax = 0;
    hipError_t he = build_diagonal(n, wm, diag_dev, scratch_dev, L, 0, st);
    if (he == hipSuccess) he = hipMemcpyAsync(&cmax, scratch_dev + L.off_res, 4, hipMemcpyDeviceToHost, st);
    // always wait: the queued copies read wm and write cmax in this frame
    const hipError_t hs = hipStreamSynchronize(st);
    if (he == hipSuccess) he = hs;
    if (he != hipSuccess) return hip_fail(he, where);
    if (w_total_tenths) *w_total_tenths = W;
    if (cmax_tenths) *cmax_tenths = cmax;
    return QS_OK;
}

qs_status qs_apply_cost_layer(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, double theta_zz)
{
    if (qs_status st = check_state(s)) return st;
    if (qs_status st = check_diag(s, diag_dev, w_total_tenths)) return st;
    if (!std::isfinite(theta_zz)) return fail(QS_ERR_ARG, "non-finite angle");
    Launch L(s, QS_KIND_ELEMENTWISE, ldexp(1.0, s->n) * (2 * amp_bytes(s->prec) + 4));
    HIPCHK(launch_cost_layer(s->prec, s->psi, diag_dev, s->n, w_total_tenths, theta_zz, s->stream),
           "qs_apply_cost_layer");
    L.done();
    return QS_OK;
}

qs_status qs_apply_mixer(qs_state s, double theta_x)
{
    if (qs_status st = check_state(s)) return st;
    if (!std::isfinite(theta_x)) return fail(QS_ERR_ARG, "non-finite angle");
    const int T = tile_bits(s->prec);
    const char *where = "qs_apply_mixer";
    if (s->n <= T) {
        HIPCHK(s->results.ensure(64 * sizeof(double)), where);
        SmallProg sp{};
        sp.psi = s->psi;
        sp.out = (double *)s->results.p;
        sp.n = s->n;
        sp.nlayers = 1;
        sp.tx[0] = theta_x;
        sp.do_mixer[0] = 1;
        Launch L(s, QS_KIND_SMALL, ldexp(1.0, s->n) * amp_bytes(s->prec) * 2);
        HIPCHK(launch_small_forward(s->prec, sp, s->stream), where);
        L.done();
        return QS_OK;
    }
    const std::vector<PassGeom> geo = plan_for(s);
    HIPCHK(ensure_partials(s, pass_grid(s->prec, 0, (int64_t)1 << (s->n - T))), where);
    const double tx[1] = {theta_x}, tzz[1] = {0.0};
    Circuit cc{nullptr, 0, 1, tzz, tx};
    for (size_t i = 0; i < geo.size(); ++i) {
        KSpec k{(int)i, 0, -1, -1, 0, 0};
        PassProg pp = make_prog(s, geo[i], k, cc, kFwdThreadBits);
        if (qs_status st = launch_tiles(s, pp, 0, 0, QS_KIND_PASS, pass_bytes(s, pp), nullptr, where)) return st;
    }
    return QS_OK;
}

qs_status qs_forward(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, int p, const double *theta_zz,
                     const double *theta_x, double *exp_c, double *norm)
{
    try {
        if (qs_status st = check_state(s)) return st;
        if (qs_status st = check_angles(p, theta_zz, theta_x)) return st;
        const bool readout = exp_c != nullptr;
        if (p > 0 || readout)
            if (qs_status st = check_diag(s, diag_dev, w_total_tenths)) return st;
        Circuit cc{diag_dev, w_total_tenths, p, theta_zz, theta_x};
        if (qs_status st = run_forward(s, cc, readout, "qs_forward")) return st;
        if (readout) {
            double r[2];
            if (qs_status st = read_results(s, r, 2, "qs_forward")) return st;
            *exp_c = (r[1] / 10.0) / r[0];
            if (norm) *norm = r[0] * (s->sym ? 2.0 : 1.0);
        }
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_forward: host allocation failed");
    }
}

qs_status qs_expect(qs_state s, const int32_t *diag_dev, double *exp_c, double *norm)
{
    if (qs_status st = check_state(s)) return st;
    if (qs_status st = check_diag(s, diag_dev, 0)) return st;
    if (!exp_c) return fail(QS_ERR_ARG, "null exp_c");
    const char *where = "qs_expect";
    HIPCHK(s->results.ensure(64 * sizeof(double)), where);
    HIPCHK(ensure_partials(s, 16384), where);
    int64_t nb = 0;
    Launch L(s, QS_KIND_EXPECT, ldexp(1.0, s->n) * (amp_bytes(s->prec) + 4));
    HIPCHK(launch_expect(s->prec, s->psi, diag_dev, s->n, (double *)s->partials.p, &nb, s->stream), where);
    L.done();
    const int map[kSlots] = {0, 1, -1, -1};
    if (qs_status st = run_reduce(s, nb, map, 0, where)) return st;
    double r[2];
    if (qs_status st = read_results(s, r, 2, where)) return st;
    *exp_c = (r[1] / 10.0) / r[0];
    if (norm) *norm = r[0] * (s->sym ? 2.0 : 1.0);
    return QS_OK;
}

qs_status qs_sample(qs_state s, uint64_t seed, int64_t shots, uint64_t *out, int out_on_device)
{
    if (qs_status st = check_state(s)) return st;
    if (shots < 0) return fail(QS_ERR_ARG, "shots must be >= 0");
    if (shots > ((int64_t)1 << 31) * 256) return fail(QS_ERR_ARG, "too many shots");
    if (shots > 0 && !out) return fail(QS_ERR_ARG, "null output array");
    if (out_on_device && shots > 0 && !aligned(out, 8)) return fail(QS_ERR_ARG, "output must be 8-byte aligned");
    const char *where = "qs_sample";
    int64_t nsub, nblk, nchunk;
    sample_sizes(s->n, &nsub, &nblk, &nchunk);
    const size_t o_sub = 0;
    const size_t o_blk = o_sub + (size_t)nsub * 8;
    const size_t o_chunk = o_blk + (size_t)nblk * 8;
    const size_t o_flag = o_chunk + (size_t)(nchunk + 1) * 8;
    HIPCHK(s->sample.ensure(o_flag + 256), where);
    char *base = (char *)s->sample.p;
    SampleBufs b{(uint64_t *)(base + o_sub), (uint64_t *)(base + o_blk), (uint64_t *)(base + o_chunk),
                 (int32_t *)(base + o_flag)};
    uint64_t *dst = out;
    if (!out_on_device && shots > 0) {
        HIPCHK(s->shots_out.ensure((size_t)shots * 8), where);
        dst = (uint64_t *)s->shots_out.p;
    }
    HIPCHK(s->results.ensure(64 * sizeof(double)), where);
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s->stream, (double *)b.flag, 1);
    HIPCHK(hipGetLastError(), where);
    {
        Launch L(s, QS_KIND_SAMPLE, ldexp(1.0, s->n) * amp_bytes(s->prec) + (double)shots * 8);
        HIPCHK(launch_sample(s->prec, s->psi, s->n, b, seed, shots, dst, s->stream, s->sym ? s->nq : 0), where);
        L.done();
    }
    int32_t flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, b.flag, 4, hipMemcpyDeviceToHost, s->stream), where);
    if (!out_on_device && shots > 0)
        HIPCHK(hipMemcpyAsync(out, dst, (size_t)shots * 8, hipMemcpyDeviceToHost, s->stream), where);
    HIPCHK(hipStreamSynchronize(s->stream), where);
    if (flag == 1) return fail(QS_ERR_STATE, "qs_sample: state has zero norm");
    if (flag == 2) return fail(QS_ERR_STATE, "qs_sample: state norm too large (|a|^2 sums to 4 or more)");
    return QS_OK;
}

int64_t qs_layout_index(int64_t x) { return x < 0 ? -1 : swz(x); }

namespace {
qs_status copy_amplitudes(qs_state s, int64_t first, int64_t count, void *buf, int on_device, int to_state,
                          const char *where)
{
    if (qs_status st = check_state(s)) return st;
    const int64_t dim = (int64_t)1 << s->n;
    if (first < 0 || count < 0 || first > dim || count > dim - first)
        return fail(QS_ERR_ARG, "%s: range [%lld, %lld) outside 0..%lld", where, (long long)first,
                    (long long)(first + count), (long long)dim);
    if (count > 0 && !buf) return fail(QS_ERR_ARG, "%s: null buffer", where);
    if (count == 0) return QS_OK;
    const size_t bytes = (size_t)count * amp_bytes(s->prec);
    if (on_device) {
        if (!aligned(buf, 8)) return fail(QS_ERR_ARG, "%s: device buffer must be 8-byte aligned", where);
        HIPCHK(launch_copy_amplitudes(s->prec, s->psi, first, count, buf, to_state, s->stream), where);
        return QS_OK;
    }
    HIPCHK(s->xfer.ensure(bytes), where);
    if (to_state) HIPCHK(hipMemcpyAsync(s->xfer.p, buf, bytes, hipMemcpyHostToDevice, s->stream), where);
    HIPCHK(launch_copy_amplitudes(s->prec, s->psi, first, count, s->xfer.p, to_state, s->stream), where);
    if (!to_state) HIPCHK(hipMemcpyAsync(buf, s->xfer.p, bytes, hipMemcpyDeviceToHost, s->stream), where);
    HIPCHK(hipStreamSynchronize(s->stream), where);
    return QS_OK;
}
}  // namespace

qs_status qs_get_amplitudes(qs_state s, int64_t first, int64_t count, void *dst, int on_device)
{
    return copy_amplitudes(s, first, count, dst, on_device, 0, "qs_get_amplitudes");
}

qs_status qs_set_amplitudes(qs_state s, int64_t first, int64_t count, const void *src, int on_device)
{
    return copy_amplitudes(s, first, count, const_cast<void *>(src), on_device, 1, "qs_set_amplitudes");
}

qs_status qs_cost_histogram(qs_state s, const int32_t *diag_dev, int32_t nbins, uint64_t *mass, int out_on_device)
{
    if (qs_status st = check_state(s)) return st;
    if (qs_status st = check_diag(s, diag_dev, 0)) return st;
    if (nbins < 1 || nbins > kHistMaxBins) return fail(QS_ERR_ARG, "nbins = %d outside 1..%d", nbins, kHistMaxBins);
    if (!mass) return fail(QS_ERR_ARG, "null output array");
    if (out_on_device && !aligned(mass, 8)) return fail(QS_ERR_ARG, "output must be 8-byte aligned");
    const char *where = "qs_cost_histogram";
    const HistGeom g = hist_geom(s->prec, s->n, nbins);
    // scratch: rows of nbins uint64, the device output, per-workgroup FP64 sums, the flag
    const size_t o_rows = 0;
    const size_t o_out = o_rows + (((size_t)g.rows * nbins * 8 + 255) & ~(size_t)255);
    const size_t o_fsum = o_out + (((size_t)nbins * 8 + 255) & ~(size_t)255);
    const size_t o_flag = o_fsum + (((size_t)g.groups * 8 + 255) & ~(size_t)255);
    HIPCHK(s->hist.ensure(o_flag + 256), where);
    char *base = (char *)s->hist.p;
    uint64_t *rows = (uint64_t *)(base + o_rows);
    uint64_t *dst = out_on_device ? mass : (uint64_t *)(base + o_out);
    double *fsum = (double *)(base + o_fsum);
    int32_t *flag = (int32_t *)(base + o_flag);
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s->stream, (double *)flag, 1);
    HIPCHK(hipGetLastError(), where);
    if (!g.lds) {  // the global-atomic form adds into one zeroed row
        const int64_t words = nbins;
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s->stream,
                           (double *)rows, (int)words);
        HIPCHK(hipGetLastError(), where);
    }
    {
        Launch L(s, QS_KIND_HISTOGRAM, ldexp(1.0, s->n) * (amp_bytes(s->prec) + 4));
        HIPCHK(launch_histogram(s->prec, s->psi, diag_dev, nbins, g, rows, fsum, flag, dst, s->stream, s->sym), where);
        L.done();
    }
    std::vector<double> fs((size_t)g.groups);
    int32_t fl = 0;
    HIPCHK(hipMemcpyAsync(fs.data(), fsum, fs.size() * 8, hipMemcpyDeviceToHost, s->stream), where);
    HIPCHK(hipMemcpyAsync(&fl, flag, 4, hipMemcpyDeviceToHost, s->stream), where);
    if (!out_on_device) HIPCHK(hipMemcpyAsync(mass, dst, (size_t)nbins * 8, hipMemcpyDeviceToHost, s->stream), where);
    HIPCHK(hipStreamSynchronize(s->stream), where);
    double total = 0.0;
    for (double v : fs) total += v;
    if (s->sym) total *= 2.0;
    if (fl == 2 || !(total < 3.999))
        return fail(QS_ERR_STATE, "qs_cost_histogram: state norm too large (|a|^2 sums to 4 or more)");
    return QS_OK;
}

static bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

static qs_status adjoint_entry(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, int p,
                               const double *theta_zz, const double *theta_x, void *ckpt_buf, size_t ckpt_bytes,
                               bool store, void *lambda_buf, size_t lambda_bytes, double *exp_c,
                               double *d_theta_zz, double *d_theta_x, const char *where)
{
    try {
        if (qs_status st = check_state(s)) return st;
        if (p < 1) return fail(QS_ERR_ARG, "p must be >= 1 for a gradient (got %d)", p);
        if (qs_status st = check_angles(p, theta_zz, theta_x)) return st;
        if (qs_status st = check_diag(s, diag_dev, w_total_tenths)) return st;
        if (!d_theta_zz || !d_theta_x) return fail(QS_ERR_ARG, "null gradient output");
        if (s->n < 2) return fail(QS_ERR_ARG, "the adjoint needs n >= 2");
        const size_t need = qs_state_bytes(s->n, s->prec);
        if (lambda_buf) {
            if (lambda_bytes < need) return fail(QS_ERR_ARG, "lambda buffer too small: %zu < %zu", lambda_bytes, need);
            if (!aligned(lambda_buf, 256)) return fail(QS_ERR_ARG, "lambda buffer must be 256-byte aligned");
            if (lambda_buf == s->psi) return fail(QS_ERR_ARG, "lambda buffer aliases the state");
        }
        void *ckpt = nullptr;
        if (store) {
            const size_t cneed = (size_t)ckpt_states(s, p) * need;
            if (cneed > 0) {
                if (!ckpt_buf) return fail(QS_ERR_ARG, "null checkpoint buffer (%zu bytes needed)", cneed);
                if (ckpt_bytes < cneed)
                    return fail(QS_ERR_ARG, "checkpoint buffer too small: %zu < %zu", ckpt_bytes, cneed);
                if (!aligned(ckpt_buf, 256)) return fail(QS_ERR_ARG, "checkpoint buffer must be 256-byte aligned");
                if (overlaps(ckpt_buf, cneed, s->psi, need) ||
                    (lambda_buf && overlaps(ckpt_buf, cneed, lambda_buf, need)))
                    return fail(QS_ERR_ARG, "checkpoint buffer overlaps the state or the adjoint vector");
                ckpt = ckpt_buf;
            } else if (s->n > tile_bits(s->prec)) {
                ckpt = s->psi;  // two passes: the one checkpoint is the state buffer
            }
        }
        void *lam = lambda_buf;
        if (!lam) {
            HIPCHK(s->lambda.ensure(need), where);
            lam = s->lambda.p;
        }
        Circuit cc{diag_dev, w_total_tenths, p, theta_zz, theta_x};
        if (qs_status st = run_adjoint(s, cc, lam, where, ckpt)) return st;
        std::vector<double> r(2 + 2 * (size_t)p);
        if (qs_status st = read_results(s, r.data(), (int)r.size(), where)) return st;
        if (!lambda_buf) s->lambda.release();
        const double nrm = r[0];
        if (exp_c) *exp_c = (r[1] / 10.0) / nrm;
        for (int k = 0; k < p; ++k) {
            d_theta_zz[k] = r[2 + k] / nrm;
            d_theta_x[k] = r[2 + p + k] / nrm;
        }
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "%s: host allocation failed", where);
    }
}

qs_status qs_adjoint_grad(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, int p,
                          const double *theta_zz, const double *theta_x, void *lambda_buf, size_t lambda_bytes,
                          double *exp_c, double *d_theta_zz, double *d_theta_x)
{
    return adjoint_entry(s, diag_dev, w_total_tenths, p, theta_zz, theta_x, nullptr, 0, false, lambda_buf,
                         lambda_bytes, exp_c, d_theta_zz, d_theta_x, "qs_adjoint_grad");
}

qs_status qs_adjoint_ckpt_bytes(qs_state s, int p, size_t *bytes)
{
    if (qs_status st = check_state(s)) return st;
    if (p < 1) return fail(QS_ERR_ARG, "p must be >= 1 (got %d)", p);
    if (p > (1 << 20)) return fail(QS_ERR_ARG, "p must be <= 2^20 (got %d)", p);
    if (!bytes) return fail(QS_ERR_ARG, "null output");
    try {
        *bytes = (size_t)ckpt_states(s, p) * qs_state_bytes(s->n, s->prec);
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_adjoint_ckpt_bytes: host allocation failed");
    }
    return QS_OK;
}

qs_status qs_adjoint_grad_store(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, int p,
                                const double *theta_zz, const double *theta_x, void *ckpt_buf, size_t ckpt_bytes,
                                void *lambda_buf, size_t lambda_bytes, double *exp_c, double *d_theta_zz,
                                double *d_theta_x)
{
    return adjoint_entry(s, diag_dev, w_total_tenths, p, theta_zz, theta_x, ckpt_buf, ckpt_bytes, true,
                         lambda_buf, lambda_bytes, exp_c, d_theta_zz, d_theta_x, "qs_adjoint_grad_store");
}

qs_status qs_debug_set_cut_mode(qs_state s, int mode)
{
    if (qs_status st = check_state(s)) return st;
    if (mode < 0 || mode > 2) return fail(QS_ERR_ARG, "cut mode %d (0 automatic, 1 registers, 2 diagonal)", mode);
    s->cut_mode = mode;
    return QS_OK;
}

qs_status qs_profile(qs_state s, int enable)
{
    if (qs_status st = check_state(s)) return st;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    clear_prof(s);
    s->prof = enable != 0;
    return QS_OK;
}

qs_status qs_profile_read(qs_state s, int kind, int64_t *launches, double *total_ms, double *bytes)
{
    if (qs_status st = check_state(s)) return st;
    if (kind < 0 || kind >= QS_KIND_COUNT) return fail(QS_ERR_ARG, "bad kernel kind %d", kind);
    int64_t cnt = 0;
    double ms = 0.0, by = 0.0;
    for (auto &r : s->recs) {
        if (r.kind != kind) continue;
        HIPCHK(hipEventSynchronize(r.b), "qs_profile_read");
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b), "qs_profile_read");
        ++cnt;
        ms += t;
        by += r.bytes;
    }
    if (launches) *launches = cnt;
    if (total_ms) *total_ms = ms;
    if (bytes) *bytes = by;
    return QS_OK;
}

// ---------------------------------------------------------------- batch
qs_status qs_batch_create(int count, const qs_circuit *circuits, int prec, void *hip_stream, qs_batch *out)
{
    try {
        if (!out) return fail(QS_ERR_ARG, "null output handle pointer");
        *out = nullptr;
        if (count < 1) return fail(QS_ERR_ARG, "count must be >= 1");
        if (!circuits) return fail(QS_ERR_ARG, "null circuit array");
        if (prec != QS_C64 && prec != QS_C128) return fail(QS_ERR_ARG, "bad precision %d", prec);
        const int T = tile_bits(prec);
        std::vector<std::vector<int32_t>> wms(count);
        qs_batch b0 = nullptr;
        int nmax = 0;
        for (int i = 0; i < count; ++i) {
            const qs_circuit &c = circuits[i];
            if (c.n <= T || c.n > QS_BATCH_MAX_QUBITS)
                return fail(QS_ERR_ARG, "circuit %d: n = %d outside %d..%d", i, c.n, T + 1, QS_BATCH_MAX_QUBITS);
            if (c.p < 1) return fail(QS_ERR_ARG, "circuit %d: p must be >= 1", i);
            int64_t W = 0;
            if (c.n > 0) wms[i].resize((size_t)c.n * c.n);
            if (qs_status st = weight_matrix(c.n, c.w_tenths, wms[i].data(), &W)) return st;
            nmax = std::max(nmax, c.n);
        }
        qs_batch b = new qs_batch_s();
        b0 = b;
        b->stream = (hipStream_t)hip_stream;
        const size_t off = layout_batch(b, count, circuits, prec);
        hipError_t he = hipMalloc(&b->mem, off);
        if (he != hipSuccess) {
            delete b0;
            return hip_fail(he, "qs_batch_create");
        }
        const DiagScratch L = diag_scratch_layout(nmax, count);
        char *scratch = nullptr;
        he = hipMalloc(&scratch, L.total);
        for (int i = 0; i < count && he == hipSuccess; ++i)
            he = build_diagonal(b->n[i], wms[i].data(), (int32_t *)((char *)b->mem + b->off_diag[i]), scratch, L, i,
                                b->stream);
        b->cmax.assign(count, 0);
        if (he == hipSuccess)
            he = hipMemcpyAsync(b->cmax.data(), scratch + L.off_res, (size_t)count * 4, hipMemcpyDeviceToHost,
                                b->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(b->stream);
        if (scratch) (void)hipFree(scratch);
        if (he != hipSuccess) {
            (void)hipFree(b->mem);
            delete b0;
            return hip_fail(he, "qs_batch_create");
        }
        *out = b;
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_batch_create: host allocation failed");
    }
}

qs_status qs_batch_info(qs_batch b, int i, int64_t *w_total_tenths, int32_t *cmax_tenths, void **psi_dev,
                        int32_t **diag_dev)
{
    if (!b) return fail(QS_ERR_ARG, "null batch handle");
    if (i < 0 || i >= b->count) return fail(QS_ERR_ARG, "circuit index %d outside 0..%d", i, b->count - 1);
    if (w_total_tenths) *w_total_tenths = b->W[i];
    if (cmax_tenths) *cmax_tenths = b->cmax[i];
    if (psi_dev) *psi_dev = (char *)b->mem + b->off_psi[i];
    if (diag_dev) *diag_dev = (int32_t *)((char *)b->mem + b->off_diag[i]);
    return QS_OK;
}

qs_status qs_batch_forward_grad(qs_batch b, const double *theta_zz, const double *theta_x, double *exp_c,
                                double *d_theta_zz, double *d_theta_x)
{
    try {
        if (!b) return fail(QS_ERR_ARG, "null batch handle");
        if (!theta_zz || !theta_x) return fail(QS_ERR_ARG, "null angle array");
        if (!exp_c || !d_theta_zz || !d_theta_x) return fail(QS_ERR_ARG, "null output array");
        const int64_t nang = b->angle_off.back();
        for (int64_t k = 0; k < nang; ++k)
            if (!std::isfinite(theta_zz[k]) || !std::isfinite(theta_x[k]))
                return fail(QS_ERR_ARG, "non-finite angle at index %lld", (long long)k);
        const char *where = "qs_batch_forward_grad";
        const int count = b->count;

        const BatchSchedule sch = build_batch_schedule(b, theta_zz, theta_x);
        const int nsteps = (int)b->steps_h.size();
        const int64_t items = sch.items, tabs = sch.tabs, nres = sch.nres;
        const int nidx = sch.nidx;
        const int tabn = batch_table_entries();

        const size_t ab = b->prec == QS_C64 ? 8 : 16;
        HIPCHK(b->steps.ensure(sizeof(BatchStep) * nsteps), where);
        HIPCHK(b->tabs.ensure((size_t)std::max<int64_t>(tabs, 1) * tabn * ab), where);
        HIPCHK(b->partials.ensure((size_t)items * kSlots * sizeof(double)), where);
        // counters: ticket (8 B), abort flag, per-step done counters
        const size_t cnt_doubles = (16 + (size_t)nsteps * 4 + 7) / 8;
        HIPCHK(b->counters.ensure(cnt_doubles * 8), where);
        HIPCHK(b->results.ensure((size_t)nres * sizeof(double)), where);
        HIPCHK(b->index.ensure(b->idx_h.size() * sizeof(int) + 64 + b->res_off_h.size() * sizeof(int64_t)), where);
        char *idx_d = (char *)b->index.p;
        const size_t roff_pos = (b->idx_h.size() * sizeof(int) + 63) & ~(size_t)63;
        HIPCHK(hipMemcpyAsync(b->steps.p, b->steps_h.data(), sizeof(BatchStep) * nsteps, hipMemcpyHostToDevice,
                              b->stream), where);
        HIPCHK(hipMemcpyAsync(idx_d, b->idx_h.data(), b->idx_h.size() * sizeof(int), hipMemcpyHostToDevice, b->stream),
               where);
        HIPCHK(hipMemcpyAsync(idx_d + roff_pos, b->res_off_h.data(), b->res_off_h.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, b->stream), where);
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((cnt_doubles + 255) / 256)), dim3(256), 0, b->stream,
                           (double *)b->counters.p, (int)cnt_doubles);
        HIPCHK(hipGetLastError(), where);
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((nres + 255) / 256)), dim3(256), 0, b->stream,
                           (double *)b->results.p, (int)nres);
        HIPCHK(hipGetLastError(), where);
        HIPCHK(launch_batch_tables(b->prec, (const BatchStep *)b->steps.p, nsteps, b->tabs.p, b->stream), where);
        BatchArgs args{};
        args.steps = (const BatchStep *)b->steps.p;
        args.nsteps = nsteps;
        args.nitems = items;
        args.ticket = (unsigned long long *)b->counters.p;
        args.abort_flag = (int *)((char *)b->counters.p + 8);
        args.done = (unsigned *)((char *)b->counters.p + 16);
        args.partials = (double *)b->partials.p;
        args.tabs = b->tabs.p;
        args.spin_limit = 4000000;
        HIPCHK(launch_batch(b->prec, args, batch_grid(b->prec), b->stream), where);
        HIPCHK(launch_batch_reduce((const BatchStep *)b->steps.p, (const int *)idx_d, (const int *)idx_d + nidx,
                                   (const int64_t *)(idx_d + roff_pos), (const double *)b->partials.p,
                                   (double *)b->results.p, count, b->stream),
               where);
        b->res_h.assign(nres, 0.0);
        int32_t abort_flag = 0;
        HIPCHK(hipMemcpyAsync(b->res_h.data(), b->results.p, (size_t)nres * sizeof(double), hipMemcpyDeviceToHost,
                              b->stream), where);
        HIPCHK(hipMemcpyAsync(&abort_flag, args.abort_flag, 4, hipMemcpyDeviceToHost, b->stream), where);
        HIPCHK(hipStreamSynchronize(b->stream), where);
        if (abort_flag) return fail(QS_ERR_HIP, "%s: a work item waited too long for its predecessor", where);
        for (int c = 0; c < count; ++c) {
            const double *r = b->res_h.data() + b->res_off_h[c];
            const int p = b->p[c];
            exp_c[c] = (r[1] / 10.0) / r[0];
            for (int k = 0; k < p; ++k) {
                d_theta_zz[b->angle_off[c] + k] = r[2 + k] / r[0];
                d_theta_x[b->angle_off[c] + k] = r[2 + p + k] / r[0];
            }
        }
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_batch_forward_grad: host allocation failed");
    }
}

qs_status qs_noise_create(int n, int prec, const int32_t *w_tenths, void *hip_stream, qs_noise *out)
{
    try {
        if (!out) return fail(QS_ERR_ARG, "null output handle pointer");
        *out = nullptr;
        if (n < 2 || n > kNoiseMaxQubits) return fail(QS_ERR_ARG, "n = %d outside 2..%d", n, kNoiseMaxQubits);
        if (prec != QS_C64 && prec != QS_C128) return fail(QS_ERR_ARG, "bad precision %d", prec);
        std::vector<int32_t> wm((size_t)n * n);
        int64_t W = 0;
        if (qs_status st = weight_matrix(n, w_tenths, wm.data(), &W)) return st;
        const char *where = "qs_noise_create";
        std::unique_ptr<qs_noise_s> h(new qs_noise_s);
        h->n = n;
        h->prec = prec;
        h->stream = (hipStream_t)hip_stream;
        const int ne = n * (n - 1) / 2;
        std::vector<int32_t> edges((size_t)ne);
        for (int i = 0, e = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j, ++e) edges[(size_t)e] = i | (j << 4) | (w_tenths[e] << 8);
        HIPCHK(h->diag.ensure(sizeof(int32_t) << n), where);
        HIPCHK(h->edges.ensure(sizeof(int32_t) * (size_t)ne), where);
        HIPCHK(hipMemcpyAsync(h->edges.p, edges.data(), sizeof(int32_t) * (size_t)ne, hipMemcpyHostToDevice,
                              h->stream), where);
        if (qs_status st = cost_diagonal_impl(n, 0, w_tenths, (int32_t *)h->diag.p, &h->W, &h->cmax, hip_stream))
            return st;
        *out = h.release();
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_noise_create: host allocation failed");
    }
}

qs_status qs_noise_info(qs_noise h, int64_t *w_total_tenths, int32_t *cmax_tenths)
{
    if (!h) return fail(QS_ERR_ARG, "null noise handle");
    if (w_total_tenths) *w_total_tenths = h->W;
    if (cmax_tenths) *cmax_tenths = h->cmax;
    return QS_OK;
}

qs_status qs_noise_run(qs_noise h, int p, const double *theta_zz, const double *theta_x, double eps, uint64_t seed,
                       int64_t traj0, int64_t ntraj, double *exp_c, double *norm, int32_t *nerr, void *states)
{
    try {
        if (!h) return fail(QS_ERR_ARG, "null noise handle");
        if (p < 1 || p > QS_NOISE_MAX_LAYERS) return fail(QS_ERR_ARG, "p = %d outside 1..%d", p, QS_NOISE_MAX_LAYERS);
        if (!theta_zz || !theta_x) return fail(QS_ERR_ARG, "null angle array");
        for (int k = 0; k < p; ++k)
            if (!std::isfinite(theta_zz[k]) || !std::isfinite(theta_x[k]))
                return fail(QS_ERR_ARG, "non-finite angle in layer %d", k);
        if (!(eps >= 0.0 && eps <= 1.0)) return fail(QS_ERR_ARG, "eps outside [0, 1]");
        if (ntraj < 1 || ntraj > 0x7fffffff) return fail(QS_ERR_ARG, "ntraj = %lld outside 1..2^31-1", (long long)ntraj);
        if (traj0 < 0) return fail(QS_ERR_ARG, "negative first trajectory");
        if (!exp_c) return fail(QS_ERR_ARG, "null exp_c buffer");
        if (!aligned(exp_c, 8) || (norm && !aligned(norm, 8)) || (nerr && !aligned(nerr, 4)) ||
            (states && !aligned(states, h->prec ? 16 : 8)))
            return fail(QS_ERR_ARG, "misaligned output buffer");
        const char *where = "qs_noise_run";
        // per layer: theta_zz, then the mixer in tangent form (u = tan(theta/2), factor cos^n) when every
        // layer has |cos(theta_x / 2)| >= 1/2, else directly (cos, sin; factor 1)
        // (graphs whose phase table needs more than two levels use the direct form)
        const int levels = std::max(2, phase_table_levels(3 * h->W));
        bool tangent = levels == 2;
        for (int k = 0; k < p; ++k) tangent = tangent && std::fabs(std::cos(0.5 * theta_x[k])) >= 0.5;
        // the previous run may still be reading the uploaded table
        HIPCHK(h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize(), where);
        h->layers_h.assign((size_t)4 * p, 0.0);
        for (int k = 0; k < p; ++k) {
            double *L = &h->layers_h[(size_t)4 * k];
            const double c = std::cos(0.5 * theta_x[k]), sn = std::sin(0.5 * theta_x[k]);
            L[0] = theta_zz[k];
            if (tangent) {
                L[1] = sn / c;
                L[3] = std::pow(c, h->n);
            } else {
                L[1] = c;
                L[2] = sn;
                L[3] = 1.0;
            }
        }
        HIPCHK(h->layers.ensure(sizeof(double) * h->layers_h.size()), where);
        HIPCHK(hipMemcpyAsync(h->layers.p, h->layers_h.data(), sizeof(double) * h->layers_h.size(),
                              hipMemcpyHostToDevice, h->stream), where);
        HIPCHK(h->tabs.ensure((size_t)p * noise_table_entries() * (h->prec ? 16 : 8)), where);
        NoiseProg np{};
        np.tabs = h->tabs.p;
        np.diag = (const int32_t *)h->diag.p;
        np.edges = (const int32_t *)h->edges.p;
        np.layers = (const double *)h->layers.p;
        np.exp_c = exp_c;
        np.norm = norm;
        np.nerr = nerr;
        np.states = states;
        np.traj0 = (uint64_t)traj0;
        np.seed = seed;
        np.thr = (uint64_t)std::floor(eps * 9007199254740992.0);  // eps * 2^53
        np.W = h->W;
        np.n = h->n;
        np.p = p;
        np.levels = levels;
        np.amp0 = std::sqrt(std::ldexp(1.0, -h->n));
        HIPCHK(launch_noise(h->prec, tangent ? 1 : 0, np, ntraj, h->stream), where);
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_noise_run: host allocation failed");
    }
}

qs_status qs_noise_free(qs_noise h)
{
    if (!h) return QS_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    delete h;
    return QS_OK;
}

}  // extern "C"

namespace {
__attribute__((format(printf, 3, 4))) int plan_fail(char *msg, size_t len, const char *fmt, ...)
{
    if (msg && len) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(msg, len, fmt, ap);
        va_end(ap);
    }
    return 1;
}
}  // namespace

extern "C" {

int qs_batch_plan_check(int count, const qs_circuit *circuits, int prec, char *msg, size_t msg_len)
{
#define bad(...) plan_fail(msg, msg_len, __VA_ARGS__)
    if (msg && msg_len) msg[0] = 0;
    if (count < 1 || !circuits || (prec != QS_C64 && prec != QS_C128)) return 2;
    const int T = tile_bits(prec);
    for (int i = 0; i < count; ++i)
        if (circuits[i].n <= T || circuits[i].n > QS_BATCH_MAX_QUBITS || circuits[i].p < 1 || !circuits[i].w_tenths)
            return 2;
    qs_batch_s b;
    const size_t total = layout_batch(&b, count, circuits, prec);
    b.mem = (void *)(uintptr_t)((uint64_t)1 << 40);  // never dereferenced
    std::vector<double> tzz(b.angle_off.back(), 0.3), tx(b.angle_off.back(), 0.4);
    const BatchSchedule sch = build_batch_schedule(&b, tzz.data(), tx.data());
    const std::vector<BatchStep> &st = b.steps_h;
    const int nsteps = (int)st.size();
    const int tabn = batch_table_entries();
    const char *lo = (const char *)b.mem, *hi = lo + total;
    // circuit memory: inside the allocation, disjoint, 256-byte aligned
    for (int c = 0; c < count; ++c) {
        const size_t sb = qs_state_bytes(b.n[c], prec), db = ((size_t)1 << b.n[c]) * 4;
        if (b.off_psi[c] % 256 || b.off_lam[c] % 256 || b.off_diag[c] % 256) return bad("circuit %d: misaligned", c);
        if (b.off_psi[c] + sb > b.off_lam[c] || b.off_lam[c] + sb > b.off_diag[c] || b.off_diag[c] + db > total)
            return bad("circuit %d: buffers overlap or exceed the allocation", c);
        if (c + 1 < count && b.off_diag[c] + db > b.off_psi[c + 1]) return bad("circuits %d, %d overlap", c, c + 1);
    }
    // items: contiguous in step order; predecessors earlier and of the same circuit
    int64_t next = 0;
    std::vector<int> seen(count, 0), lastk(count, -1);
    for (int i = 0; i < nsteps; ++i) {
        const BatchStep &s = st[i];
        if (s.item0 != next) return bad("step %d: items not contiguous", i);
        next += s.chunks;
        const int64_t ntiles = (int64_t)1 << (b.n[s.circuit] - T);
        if (s.tiles_per_chunk < 1 || (int64_t)s.chunks * s.tiles_per_chunk < ntiles ||
            (int64_t)(s.chunks - 1) * s.tiles_per_chunk >= ntiles)
            return bad("step %d: chunks do not cover the tiles", i);
        if (s.pp.ntiles != ntiles) return bad("step %d: tile count", i);
        if (s.prev != lastk[s.circuit]) return bad("step %d: predecessor %d, expected %d", i, s.prev, lastk[s.circuit]);
        if (s.prev >= 0 && (st[s.prev].circuit != s.circuit || st[s.prev].item0 + st[s.prev].chunks > s.item0))
            return bad("step %d: predecessor not strictly earlier", i);
        if ((s.prev < 0) != (s.pp.init != 0 && s.kind == 0)) return bad("step %d: first step must start from |+>", i);
        lastk[s.circuit] = i;
        ++seen[s.circuit];
        const char *psi = (const char *)s.pp.psi, *dg = (const char *)s.pp.diag;
        if (psi != lo + b.off_psi[s.circuit] || s.pp.psi_out != s.pp.psi || dg != lo + b.off_diag[s.circuit] ||
            (s.kind >= 1 && (const char *)s.pp.lam != lo + b.off_lam[s.circuit]) || psi < lo || psi >= hi)
            return bad("step %d: buffer pointers", i);
        if (s.pp.has_phase != (s.tab_off >= 0)) return bad("step %d: phase table", i);
        if (s.tab_off >= 0 && (s.tab_off % tabn || s.tab_off / tabn >= sch.tabs)) return bad("step %d: table offset", i);
        for (int k = 0; k < kSlots; ++k)
            if (s.map[k] >= 2 + 2 * b.p[s.circuit]) return bad("step %d: result slot", i);
        if (s.mode != tile_mode(s.pp, T, kBatchThreadBits)) return bad("step %d: stage mode", i);
    }
    if (next != sch.items) return bad("item count");
    for (int c = 0; c < count; ++c) {
        const int P = (int)plan_passes(b.n[c], prec).size();
        const int fwd = b.p[c] * (P - 1) + 1;
        if (seen[c] != 2 * fwd - 1) return bad("circuit %d: %d steps, expected %d", c, seen[c], 2 * fwd - 1);
    }
    // the reduction's per-circuit step lists and result offsets
    const int *cstep = b.idx_h.data(), *coff = b.idx_h.data() + sch.nidx;
    for (int c = 0; c < count; ++c) {
        if (coff[c + 1] - coff[c] != seen[c]) return bad("circuit %d: step list", c);
        for (int j = coff[c]; j < coff[c + 1]; ++j)
            if (cstep[j] < 0 || cstep[j] >= nsteps || st[cstep[j]].circuit != c) return bad("circuit %d: step list entry", c);
        if (b.res_off_h[c + 1] - b.res_off_h[c] != 2 + 2 * b.p[c]) return bad("circuit %d: result offsets", c);
    }
#undef bad
    return 0;
}

qs_status qs_batch_free(qs_batch b)
{
    if (!b) return QS_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    if (b->mem) (void)hipFree(b->mem);
    b->steps.release();
    b->tabs.release();
    b->partials.release();
    b->counters.release();
    b->results.release();
    b->index.release();
    delete b;
    return QS_OK;
}

}  // extern "C"
