// Host-only driver for the pass planner (plan.h) under AddressSanitizer and
// UndefinedBehaviorSanitizer: every n, both precisions, both layouts, the
// window sequences for every kernel width.  Checks that each stage's windows
// stay inside the tile and cover its factors, computes every stage's tail in
// both directions, and drives the planner past its window limit.  Built and run by
// tests/test_sanitizers.py; prints "ok <windows>" and exits 0.
#include <cstdio>

#include "plan.h"

int main()
{
    long windows = 0, tails = 0;
    for (int prec = 0; prec < 2; ++prec) {
        const int T = qs::tile_bits(prec);
        for (int sym = 0; sym < 2; ++sym) {
            for (int n = 2; n <= 35; ++n) {
                const auto geo = sym ? qs::plan_passes_sym(n, prec) : qs::plan_passes(n, prec);
                for (const auto &g : geo) {
                    for (int tb : {qs::kFwdThreadBits, qs::kAdjThreadBits}) {
                        const int rb = T - tb;
                        const qs::WinSeq A = qs::plan_windows(tb, g.targets, g.pairs, T, tb);
                        if (A.cnt < 1 || A.cnt > qs::kMaxWindows) {
                            std::printf("window count %d (n=%d prec=%d sym=%d tb=%d)\n", A.cnt, n, prec, sym, tb);
                            return 1;
                        }
                        const qs::WinSeq B = qs::plan_windows(A.s[A.cnt - 1], g.targets, g.pairs, T, tb);
                        for (const qs::WinSeq *w : {&A, &B}) {
                            if (w->cnt < 1 || w->cnt > qs::kMaxWindows) {
                                std::printf("window count %d (n=%d prec=%d sym=%d tb=%d)\n", w->cnt, n, prec, sym, tb);
                                return 1;
                            }
                            uint32_t single = 0, pair = 0;
                            for (int i = 0; i < w->cnt; ++i) {
                                const int s = w->s[i];
                                if (s < 0 || s + rb > T) {
                                    std::printf("window %d outside the tile (n=%d)\n", s, n);
                                    return 1;
                                }
                                single |= ((1u << rb) - 1u) << s;
                                pair |= ((1u << (rb - 1)) - 1u) << s;
                            }
                            if ((g.targets & ~single) || (g.pairs & ~pair)) {
                                std::printf("factors not covered (n=%d prec=%d sym=%d tb=%d)\n", n, prec, sym, tb);
                                return 1;
                            }
                            windows += w->cnt;
                        }
                        // stage tails (compile-time masks of the last window), both directions
                        for (const qs::WinSeq *w : {&A, &B})
                            for (bool rev : {false, true}) {
                                const int t = qs::stage_tail(*w, g.pairs ? 0u : g.targets, rb, rev);
                                if (t < -rb || t > rb) {
                                    std::printf("tail %d outside +-%d (n=%d)\n", t, rb, n);
                                    return 1;
                                }
                                tails += t != 0;
                            }
                    }
                }
            }
        }
    }
    // a stage that needs more windows than a sequence holds (one-bit windows
    // over 13 targets): the planner flags it, and nothing reads past the array
    const qs::WinSeq over = qs::plan_windows(12, (1u << 13) - 1u, 13, 12);
    if (over.cnt != qs::kMaxWindows + 1 || qs::stage_tail(over, (1u << 13) - 1u, 1, false) != 0) {
        std::printf("overflow not flagged (cnt %d)\n", over.cnt);
        return 1;
    }
    std::printf("ok %ld %ld\n", windows, tails);
    return 0;
}
