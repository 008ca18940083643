// Host-only verification of the pass plan (declared in include/qs_debug.h).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <random>
#include <vector>

#include "../../include/qs_debug.h"
#include "plan.h"

using namespace qs;

namespace {

template <int RB>
int lds_slot_host(int e)
{
    return qs::lds_slot<RB>(e);
}

struct Report {
    char *msg;
    size_t len;
    int bad = 0;
    int fail(const char *fmt, ...)
    {
        if (!bad && msg && len) {
            va_list ap;
            va_start(ap, fmt);
            vsnprintf(msg, len, fmt, ap);
            va_end(ap);
        }
        bad = 1;
        return 1;
    }
};

uint32_t window_mask(int s, int rb) { return ((1u << rb) - 1u) << s; }

int check_windows(Report &R, const WinSeq &w, uint32_t targets, uint32_t pairs, int T, int tb, const char *what)
{
    const int rb = T - tb;
    if (w.cnt < 1 || w.cnt > kMaxWindows) return R.fail("%s: %d windows", what, w.cnt);
    uint32_t cov = 0, pcov = 0;
    for (int i = 0; i < w.cnt; ++i) {
        // the branch-free stage code exchanges unconditionally between windows
        if (i > 0 && w.s[i] == w.s[i - 1]) return R.fail("%s: window %d repeats the previous one", what, i);
        if (w.s[i] < 0 || w.s[i] + rb > T) return R.fail("%s: window %d starts at %d", what, i, w.s[i]);
        cov |= window_mask(w.s[i], rb);
        pcov |= window_mask(w.s[i], rb - 1);  // pair (e, e+1) inside the window
    }
    if ((cov & targets) != targets) return R.fail("%s: windows miss targets (cover %x, targets %x)", what, cov, targets);
    if ((pcov & pairs) != pairs) return R.fail("%s: windows miss two-bit factors (cover %x, pairs %x)", what, pcov, pairs);
    return 0;
}

// Global index bit of tile bit e in a pass.
int global_bit(const PassGeom &g, int e) { return e < g.c ? e : g.q0 + (e - g.c); }

// Complement-symmetric plan: the n mixer factors (z0), (z_(j-1), z_j) for
// j = 1..n-2, and (z_(n-2)) are each applied by exactly one pass.
int check_sym_factors(Report &R, int n, int T, const std::vector<PassGeom> &geo)
{
    const int N = n - 1;
    std::vector<int> single(N, 0), pair(N, 0);  // pair[q]: factor on global bits (q, q+1)
    for (size_t i = 0; i < geo.size(); ++i) {
        const PassGeom &g = geo[i];
        for (int e = 0; e < T; ++e) {
            if (g.targets >> e & 1u) {
                if (e < g.c && i > 0) return R.fail("pass %zu: single factor on a carrier bit", i);
                single[global_bit(g, e)]++;
            }
            if (g.pairs >> e & 1u) {
                if (e + 1 >= T) return R.fail("pass %zu: pair factor at the top tile bit", i);
                if (i > 0 && e < g.c) return R.fail("pass %zu: pair factor on a carrier bit", i);
                const int a = global_bit(g, e), b = global_bit(g, e + 1);
                if (b != a + 1) return R.fail("pass %zu: pair factor on non-adjacent bits %d, %d", i, a, b);
                pair[a]++;
            }
        }
    }
    for (int q = 0; q < N; ++q) {
        const int want_single = (q == 0 || q == N - 1) ? 1 : 0;
        if (single[q] != want_single) return R.fail("single factor on z_%d applied %d times", q, single[q]);
        if (q + 1 < N && pair[q] != 1) return R.fail("pair factor (z_%d, z_%d) applied %d times", q, q + 1, pair[q]);
    }
    return 0;
}

int check_layout(Report &R, int s, int T, int tb)
{
    const int rb = T - tb, nr = 1 << rb;
    std::vector<char> seen(1u << T, 0);
    for (int tid = 0; tid < (1 << tb); ++tid)
        for (int r = 0; r < nr; ++r) {
            const int e = win_elem(r, tid, s, rb);
            if (e < 0 || e >= (1 << T)) return R.fail("window %d: element %d out of the tile", s, e);
            if (seen[e]++) return R.fail("window %d: element %d held twice", s, e);
        }
    // the XOR swizzle of LDS slots is a bijection of the tile
    std::vector<char> used(1u << T, 0);
    for (int e = 0; e < (1 << T); ++e) {
        const int sl = rb == 5 ? lds_slot_host<5>(e) : rb == 4 ? lds_slot_host<4>(e) : lds_slot_host<3>(e);
        if (sl < 0 || sl >= (1 << T) || used[sl]++) return R.fail("LDS swizzle (RB %d) is not a bijection", rb);
    }
    return 0;
}

int check_tile_maps(Report &R, int n, int T, int tb, const PassGeom &g, const WinSeq *seqs, int nseq)  // n: stored bits
{
    const int rb = T - tb, nr = 1 << rb, m = T - g.c;
    const int64_t grid = (int64_t)1 << (n - T), dim = (int64_t)1 << n;
    // workgroups to visit: all of them for n <= 24, else a sample
    std::vector<int64_t> ws;
    if (n <= 24) {
        for (int64_t w = 0; w < grid; ++w) ws.push_back(w);
    } else {
        std::mt19937_64 rng(12345);
        ws = {0, 1, grid / 2, grid - 2, grid - 1};
        for (int i = 0; i < 64; ++i) ws.push_back((int64_t)(rng() % (uint64_t)grid));
    }
    std::vector<uint8_t> seen(n <= 24 ? (size_t)dim : 0, 0);
    for (int64_t w : ws) {
        const int64_t base = tile_base(w, g.c, g.q0, m);
        if (base < 0 || base >= dim) return R.fail("pass c=%d q0=%d: base of tile %lld out of range", g.c, g.q0, (long long)w);
        std::vector<int64_t> idx;
        for (int e = 0; e < (1 << T); ++e) {
            const int64_t x = tile_gidx(e, base, g.c, g.q0);
            if (x < 0 || x >= dim) return R.fail("pass c=%d q0=%d: index %lld out of range", g.c, g.q0, (long long)x);
            if (n <= 24) {
                if (seen[x]++) return R.fail("pass c=%d q0=%d: index %lld visited twice", g.c, g.q0, (long long)x);
            }
        }
        // register-to-memory maps of every window this pass uses
        for (int q = 0; q < nseq; ++q)
            for (int i = 0; i < seqs[q].cnt; ++i) {
                const int s = seqs[q].s[i];
                for (int tid = 0; tid < (1 << tb); tid += 37) {
                    const Addr a = win_addr(tid, s, rb, base, g.c, g.q0);
                    if (!a.fast) return R.fail("window %d below the carrier bits (c = %d)", s, g.c);
                    for (int r = 0; r < nr; ++r) {
                        const int64_t want = tile_gidx(win_elem(r, tid, s, rb), base, g.c, g.q0);
                        if (a.fast_idx(r) != want) return R.fail("window %d: index map wrong", s);
                        if (a.mem_idx(swz(a.tg), r) != swz(want)) return R.fail("window %d: swizzled index wrong", s);
                        if (swz(swz(want)) != want || swz(want) >= dim) return R.fail("swizzle is not an involution of [0, 2^n)");
                    }
                }
            }
    }
    if (n <= 24)
        for (int64_t x = 0; x < dim; ++x)
            if (seen[x] != 1) return R.fail("pass c=%d q0=%d: index %lld not visited", g.c, g.q0, (long long)x);
    return 0;
}

int check_schedule(Report &R, int P, int p, bool mid)
{
    // walk the kernels in order and track, per layer, how many passes of the
    // mixer have run and whether the phase has run
    const std::vector<KSpec> ks = forward_specs(P, p, mid);
    std::vector<int> phase_done(p, 0), mixer_count(p, 0);
    std::vector<std::vector<int>> pass_seen(p, std::vector<int>(P, 0));
    if (ks.empty() || !ks[0].init || ks[0].phase != 0) return R.fail("first kernel must start from |+> with phase 0");
    for (size_t i = 0; i < ks.size(); ++i) {
        const KSpec &k = ks[i];
        if (i > 0 && k.init) return R.fail("kernel %zu re-initialises", i);
        auto rx = [&](int L) -> int {
            if (L < 0 || L >= p) return R.fail("kernel %zu: bad layer %d", i, L);
            if (!phase_done[L]) return R.fail("layer %d mixer before its phase", L);
            if (pass_seen[L][k.pass]++) return R.fail("layer %d: pass %d twice", L, k.pass);
            ++mixer_count[L];
            return 0;
        };
        if (k.pre >= 0 && rx(k.pre)) return 1;
        if (k.phase >= 0) {
            const int L = k.phase;
            if (L > 0 && mixer_count[L - 1] != P) return R.fail("layer %d phase before layer %d mixer finished", L, L - 1);
            if (phase_done[L]++) return R.fail("layer %d phase twice", L);
        }
        if (k.post >= 0 && rx(k.post)) return 1;
        if (k.pre >= 0 && k.post >= 0 && k.post != k.pre + 1) return R.fail("kernel %zu mixes layers %d and %d", i, k.pre, k.post);
    }
    for (int L = 0; L < p; ++L)
        if (!phase_done[L] || mixer_count[L] != P) return R.fail("layer %d incomplete", L);
    if (ks.size() != (size_t)(p * (P - 1) + 1)) return R.fail("kernel count %zu", ks.size());
    return 0;
}

}  // namespace

namespace {
int check_sym(Report &R, int n, int prec, int p)
{
    const int T = tile_bits(prec);
    const int N = n - 1;
    const std::vector<PassGeom> geo = plan_passes_sym(n, prec);
    if (geo.empty()) return R.fail("no plan for n = %d", n);
    if (check_sym_factors(R, n, T, geo)) return 1;
    for (size_t i = 0; i < geo.size(); ++i) {
        const PassGeom &g = geo[i];
        if (g.c < 0 || g.c > 8) return R.fail("pass %zu: carrier bits %d", i, g.c);
        if (i == 0 && (g.c != 0 || g.q0 != 0)) return R.fail("first pass must be the low tile");
        if (i > 0 && g.q0 < g.c) return R.fail("pass %zu: q0 below the carriers", i);
        if (g.q0 + (T - g.c) > N) return R.fail("pass %zu: tile beyond the stored bits", i);
    }
    for (int tb : {kFwdThreadBits, kAdjThreadBits}) {
        for (int s = 0; s <= tb; ++s)
            if (check_layout(R, s, T, tb)) return 1;
        for (const PassGeom &g : geo) {
            WinSeq seq[3];
            seq[0] = plan_windows(tb, g.targets, g.pairs, T, tb);
            seq[1] = plan_windows(tb, g.targets, g.pairs, T, tb);
            if (seq[1].cnt > kMaxWindows) return R.fail("pre stage: too many windows");
            seq[2] = plan_windows(seq[1].s[seq[1].cnt - 1], g.targets, g.pairs, T, tb);
            if (check_windows(R, seq[0], g.targets, g.pairs, T, tb, "single stage")) return 1;
            if (check_windows(R, seq[2], g.targets, g.pairs, T, tb, "post stage")) return 1;
            if (check_tile_maps(R, N, T, tb, g, seq, 3)) return 1;
        }
    }
    return check_schedule(R, (int)geo.size(), p, false);
}
}  // namespace

extern "C" int qs_plan_check(int n, int prec_arg, int p, char *msg, size_t msg_len)
{
    if (msg && msg_len) msg[0] = 0;
    const int sym = (prec_arg & 16) ? 1 : 0;  // QS_SYM
    const int prec = prec_arg & ~16;
    if ((prec != 0 && prec != 1) || p < 1) return 2;
    Report R{msg, msg_len};
    const int T = tile_bits(prec);
    if (sym) {
        if (n < T + 2 || n > 35) return 2;
        return check_sym(R, n, prec, p);
    }
    if (n < 1 || n > 34) return 2;
    if (n <= T) return 0;  // single-workgroup path
    const std::vector<PassGeom> geo = plan_passes(n, prec);
    // target qubits partition 0..n-1
    std::vector<int> owner(n, -1);
    for (size_t i = 0; i < geo.size(); ++i) {
        const PassGeom &g = geo[i];
        const int w = T - g.c;                       // strided tile bits
        const int m = __builtin_popcount(g.targets); // target qubits
        if (g.c < 0 || g.c > 8) return R.fail("pass %zu: carrier bits %d", i, g.c);
        if (m < 1 || g.targets != (((1u << T) - 1u) & ~((1u << (T - m)) - 1u)))
            return R.fail("pass %zu: targets must be the top tile bits", i);
        if (m > w) return R.fail("pass %zu: more targets than strided bits", i);
        if (i == 0 && (g.c != 0 || g.q0 != 0 || m != T)) return R.fail("first pass must be the low tile");
        if (i > 0 && g.q0 < g.c) return R.fail("pass %zu: q0 below the carriers", i);
        if (g.q0 + w > n) return R.fail("pass %zu: tile beyond n", i);
        for (int q = g.q0 + w - m; q < g.q0 + w; ++q) {
            if (owner[q] >= 0) return R.fail("qubit %d in passes %d and %zu", q, owner[q], i);
            owner[q] = (int)i;
        }
    }
    for (int q = 0; q < n; ++q)
        if (owner[q] < 0) return R.fail("qubit %d in no pass", q);
    for (int tb : {kFwdThreadBits, kAdjThreadBits}) {
        for (int s = 0; s <= tb; ++s)
            if (check_layout(R, s, T, tb)) return 1;
        for (const PassGeom &g : geo) {
            WinSeq seq[3];
            seq[0] = plan_windows(tb, g.targets, T, tb);                         // single stage
            seq[1] = plan_windows(tb, g.targets, T, tb);                         // pre stage
            if (seq[1].cnt > kMaxWindows) return R.fail("pre stage: too many windows");
            seq[2] = plan_windows(seq[1].s[seq[1].cnt - 1], g.targets, T, tb);   // post stage after pre
            if (check_windows(R, seq[0], g.targets, 0u, T, tb, "single stage")) return 1;
            if (check_windows(R, seq[2], g.targets, 0u, T, tb, "post stage")) return 1;
            if (check_tile_maps(R, n, T, tb, g, seq, 3)) return 1;
        }
    }
    if (check_schedule(R, (int)geo.size(), p, true)) return 1;
    // the XCD renumbering is a bijection whenever it is enabled (grid % 8 == 0)
    const int64_t grid = (int64_t)1 << (n - T);
    if (grid % 8 == 0 && grid <= (1 << 22)) {
        std::vector<uint8_t> seen((size_t)grid, 0);
        for (int64_t b = 0; b < grid; ++b) {
            const int64_t w = (b & 7) * (grid >> 3) + (b >> 3);
            if (w < 0 || w >= grid || seen[w]++) return R.fail("XCD renumbering is not a bijection");
        }
    }
    return 0;
}
