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
#include <string>
#include <vector>

#include "../../include/qs.h"
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

struct qs_state_s {
    int n = 0, prec = 0;
    void *psi = nullptr;
    bool own = false;
    hipStream_t stream = nullptr;
    DevBuf partials, tmp, results, sample, shots_out, lambda;
    bool prof = false;
    std::vector<ProfRec> recs;
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

PassProg make_prog(qs_state s, const PassGeom &g, const KSpec &k, const Circuit &cc, int tb)
{
    const int T = tile_bits(s->prec);
    PassProg pp{};
    pp.psi = s->psi;
    pp.lam = nullptr;
    pp.diag = cc.diag;
    pp.partials = (double *)s->partials.p;
    pp.ntiles = (int64_t)1 << (s->n - T);
    pp.n = s->n;
    pp.c = g.c;
    pp.q0 = g.q0;
    pp.targets = g.targets;
    pp.ntargets = __builtin_popcount(g.targets);
    pp.width = T - g.c;
    pp.init = k.init;
    pp.has_pre = k.pre >= 0;
    pp.has_phase = k.phase >= 0;
    pp.has_post = k.post >= 0;
    pp.readout = k.readout;
    pp.load_win = tb;
    pp.fpre = pp.fpost = 1.0;
    if (pp.has_pre) {
        pp.A = plan_windows(tb, g.targets, T, tb);
        pp.B = plan_windows(pp.A.s[pp.A.cnt - 1], g.targets, T, tb);
        pp.pre = rx_stage(cc.tx[k.pre], pp.ntargets, &pp.fpre);
    } else {
        pp.B = plan_windows(tb, g.targets, T, tb);
    }
    if (pp.has_post) pp.post = rx_stage(cc.tx[k.post], pp.ntargets, &pp.fpost);
    pp.factor = pp.fpre * pp.fpost;
    pp.phase_win = pp.has_pre ? pp.A.s[pp.A.cnt - 1] : pp.load_win;
    pp.final_win = pp.B.s[pp.B.cnt - 1];
    if (pp.has_phase) pp.theta_zz = cc.tzz[k.phase];
    pp.W = cc.W;
    pp.phase_levels = phase_table_levels(cc.W);
    pp.amp0 = sqrt(ldexp(1.0, -s->n));
    return pp;
}

// Launch one tile kernel over a persistent grid; returns the grid (the number
// of per-workgroup partial sums it writes).
qs_status launch_tiles(qs_state s, PassProg &pp, int adjoint, int turnaround, int kind, double bytes,
                       int64_t *grid_out, const char *where)
{
    // adjoint: 0 = forward pass, 1 = turnaround, 2 = reverse pass
    const int64_t grid = pass_grid(s->prec, adjoint, pp.ntiles);
    pp.xcd_remap = (grid % 8 == 0) ? 1 : 0;
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
    if (pp.has_phase || pp.readout) b += dim * 4.0;
    return b;
}

hipError_t ensure_partials(qs_state s, int64_t count)
{
    hipError_t e = s->partials.ensure((size_t)count * kSlots * sizeof(double));
    if (e != hipSuccess) return e;
    e = s->tmp.ensure((size_t)std::max<int64_t>(reduce_tmp_doubles(count), kSlots) * sizeof(double));
    return e;
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
        HIPCHK(launch_init_plus(s->prec, s->psi, s->n, s->stream), where);
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

    const std::vector<PassGeom> geo = plan_passes(s->n, s->prec);
    std::vector<KSpec> ks = forward_specs((int)geo.size(), cc.p);
    if (readout) ks.back().readout = 1;
    HIPCHK(ensure_partials(s, pass_grid(s->prec, 0, (int64_t)1 << (s->n - T))), where);
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
        Launch L(s, QS_KIND_SMALL, ldexp(1.0, s->n) * amp_bytes(s->prec) * 4);
        HIPCHK(launch_small_adjoint(s->prec, sp, s->stream), where);
        L.done();
    }
    return QS_OK;
}

qs_status run_adjoint(qs_state s, const Circuit &cc, void *lam, const char *where)
{
    const int T = tile_bits(s->prec);
    const int nres = 2 + 2 * cc.p;
    HIPCHK(s->results.ensure((size_t)std::max(64, nres) * sizeof(double)), where);
    HIPCHK(zero_results(s, nres), where);
    if (s->n <= T) return run_small_adjoint(s, cc, lam, where);

    const std::vector<PassGeom> geo = plan_passes(s->n, s->prec);
    const std::vector<KSpec> ks = forward_specs((int)geo.size(), cc.p);
    const int64_t ntiles = (int64_t)1 << (s->n - T);
    HIPCHK(ensure_partials(s, std::max(pass_grid(s->prec, 0, ntiles), pass_grid(s->prec, 1, ntiles))), where);
    const double dim = ldexp(1.0, s->n), ab = (double)amp_bytes(s->prec);
    int64_t grid = 0;

    // forward, all but the last pass
    for (size_t i = 0; i + 1 < ks.size(); ++i) {
        PassProg pp = make_prog(s, geo[ks[i].pass], ks[i], cc, kFwdThreadBits);
        if (qs_status st = launch_tiles(s, pp, 0, 0, pp.has_phase ? QS_KIND_PASS_PHASE : QS_KIND_PASS,
                                        pass_bytes(s, pp), &grid, where))
            return st;
    }
    // turnaround: the last pass forward, lambda = C psi, the pass undone
    {
        const KSpec &k = ks.back();
        PassProg pp = make_prog(s, geo[k.pass], k, cc, kAdjThreadBits);
        pp.lam = lam;
        if (qs_status st = launch_tiles(s, pp, 1, 1, QS_KIND_TURNAROUND, dim * (ab + 4 + ab), &grid, where))
            return st;
        const int map[kSlots] = {2 + cc.p + k.post, 0, 1, -1};
        if (qs_status st = run_reduce(s, grid, map, 1, where)) return st;
    }
    // reverse passes
    for (int i = (int)ks.size() - 2; i >= 0; --i) {
        const KSpec &k = ks[i];
        PassProg pp = make_prog(s, geo[k.pass], k, cc, kAdjThreadBits);
        pp.lam = lam;
        pp.load_win = pp.final_win;
        const double by = dim * ab * (pp.init ? 2.0 : 4.0) + (pp.has_phase ? dim * 4.0 : 0.0);
        if (qs_status st = launch_tiles(s, pp, 2, 0, QS_KIND_ADJOINT, by, &grid, where)) return st;
        const int map[kSlots] = {k.post >= 0 ? 2 + cc.p + k.post : -1, k.phase >= 0 ? 2 + k.phase : -1,
                                 k.pre >= 0 ? 2 + cc.p + k.pre : -1, -1};
        if (qs_status st = run_reduce(s, grid, map, 1, where)) return st;
    }
    return QS_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char *qs_last_error(void) { return g_err.c_str(); }

const char *qs_version(void) { return "libqs 0.1 (gfx950)"; }

size_t qs_state_bytes(int n, int prec)
{
    if (prec != QS_C64 && prec != QS_C128) return 0;
    if (n < 1 || n > max_qubits(prec)) return 0;
    return ((size_t)1 << n) * amp_bytes(prec);
}

qs_status qs_alloc(int n, int prec, void *dev_buf, size_t buf_bytes, void *hip_stream, qs_state *out)
{
    try {
        if (!out) return fail(QS_ERR_ARG, "null output handle pointer");
        *out = nullptr;
        if (prec != QS_C64 && prec != QS_C128) return fail(QS_ERR_ARG, "bad precision %d", prec);
        if (n < 1 || n > max_qubits(prec))
            return fail(QS_ERR_ARG, "n = %d outside 1..%d for this precision", n, max_qubits(prec));
        const size_t need = qs_state_bytes(n, prec);
        if (dev_buf) {
            if (buf_bytes < need) return fail(QS_ERR_ARG, "buffer too small: %zu < %zu bytes", buf_bytes, need);
            if (!aligned(dev_buf, 256)) return fail(QS_ERR_ARG, "state buffer must be 256-byte aligned");
        }
        qs_state s = new qs_state_s();
        s->n = n;
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
    HIPCHK(launch_init_plus(s->prec, s->psi, s->n, s->stream), "qs_init_plus");
    L.done();
    return QS_OK;
}

qs_status qs_cost_diagonal(int n, const int32_t *w_tenths, int32_t *diag_dev, int64_t *w_total_tenths,
                           int32_t *cmax_tenths, void *hip_stream)
{
    try {
        if (n < 1 || n > QS_MAX_QUBITS_C64) return fail(QS_ERR_ARG, "n = %d outside 1..%d", n, QS_MAX_QUBITS_C64);
        if (!diag_dev) return fail(QS_ERR_ARG, "null diagonal buffer");
        if (!aligned(diag_dev, 16)) return fail(QS_ERR_ARG, "diagonal buffer must be 16-byte aligned");
        const int64_t ne = (int64_t)n * (n - 1) / 2;
        if (ne > 0 && !w_tenths) return fail(QS_ERR_ARG, "null weight array");
        int64_t W = 0;
        std::vector<int32_t> wm((size_t)n * n, 0);
        int64_t e = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j, ++e) {
                const int32_t w = w_tenths[e];
                if (w < 0 || w >= (1 << 20)) return fail(QS_ERR_ARG, "weight %lld = %d outside [0, 2^20)", (long long)e, w);
                wm[(size_t)i * n + j] = wm[(size_t)j * n + i] = w;
                W += w;
            }
        if (W >= ((int64_t)1 << 31)) return fail(QS_ERR_RANGE, "W_t = %lld does not fit in int32", (long long)W);
        hipStream_t st = (hipStream_t)hip_stream;
        // scratch: weight matrix, low-bit table, per-workgroup maxima (+ second level, result)
        const int64_t nwg = diag_wg_count(n);
        const size_t off_low = ((size_t)n * n * 4 + 255) & ~(size_t)255;
        const size_t off_wg = off_low + 8192 * 4;
        const size_t off_tmp = off_wg + (((size_t)nwg * 4 + 255) & ~(size_t)255);
        const size_t off_res = off_tmp + (((size_t)(nwg / 4096 + 2) * 4 + 255) & ~(size_t)255);
        const size_t total = off_res + 256;
        char *scratch = nullptr;
        HIPCHK(hipMalloc(&scratch, total), "qs_cost_diagonal");
        auto cleanup = [&]() { (void)hipFree(scratch); };
        hipError_t he = hipMemcpyAsync(scratch, wm.data(), (size_t)n * n * 4, hipMemcpyHostToDevice, st);
        if (he == hipSuccess)
            he = launch_cost_diagonal(n, (const int32_t *)scratch, diag_dev, (int32_t *)(scratch + off_low),
                                      (int32_t *)(scratch + off_wg), (int32_t *)(scratch + off_tmp),
                                      (int32_t *)(scratch + off_res), st);
        int32_t cmax = 0;
        if (he == hipSuccess) he = hipMemcpyAsync(&cmax, scratch + off_res, 4, hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        cleanup();
        if (he != hipSuccess) return hip_fail(he, "qs_cost_diagonal");
        if (w_total_tenths) *w_total_tenths = W;
        if (cmax_tenths) *cmax_tenths = cmax;
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_OOM, "qs_cost_diagonal: host allocation failed");
    }
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
    const std::vector<PassGeom> geo = plan_passes(s->n, s->prec);
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
            if (norm) *norm = r[0];
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
    if (norm) *norm = r[0];
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
        HIPCHK(launch_sample(s->prec, s->psi, s->n, b, seed, shots, dst, s->stream), where);
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

qs_status qs_adjoint_grad(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, int p,
                          const double *theta_zz, const double *theta_x, void *lambda_buf, size_t lambda_bytes,
                          double *exp_c, double *d_theta_zz, double *d_theta_x)
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
        const char *where = "qs_adjoint_grad";
        void *lam = lambda_buf;
        if (!lam) {
            HIPCHK(s->lambda.ensure(need), where);
            lam = s->lambda.p;
        }
        Circuit cc{diag_dev, w_total_tenths, p, theta_zz, theta_x};
        if (qs_status st = run_adjoint(s, cc, lam, where)) return st;
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
        return fail(QS_ERR_OOM, "qs_adjoint_grad: host allocation failed");
    }
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

}  // extern "C"
