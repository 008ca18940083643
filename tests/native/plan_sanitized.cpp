// Host-only driver for the pass planner (plan.h) under AddressSanitizer and
// UndefinedBehaviorSanitizer: every n, both precisions, both layouts, the
// window sequences for every kernel width.  Checks that each stage's windows
// stay inside the tile and cover its factors.  Built and run by
// tests/test_sanitizers.py; prints "ok <windows>" and exits 0.
#include <cstdio>

#include "plan.h"

int main()
{
    long windows = 0;
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
                    }
                }
            }
        }
    }
    std::printf("ok %ld\n", windows);
    return 0;
}
