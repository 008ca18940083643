// Host-side plan of the tile passes: which qubits each pass covers, the
// register windows of each butterfly stage, and the order in which the
// layers' mixer passes and cost phases are fused into kernels.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace qs {

struct PassGeom {
    int c, q0;
    uint32_t targets;     // single-bit factors (tile bits)
    uint32_t pairs = 0;   // bit e: two-bit factor on tile bits e, e+1
};

inline int cmin_for(int prec)
{
    // Minimum carrier bits of a strided pass: contiguous runs of 2^c amplitudes
    // (complex64: 8 x 8 B = 64 B; complex128: 8 x 16 B = 128 B).
    (void)prec;
    return 3;
}

// Passes of one mixer layer.  Pass 0 is the contiguous low tile (qubits
// 0..T-1).  The remaining n - T qubits are split as evenly as possible over
// strided passes of at most T - cmin targets.  A strided pass keeps c <= 8
// carrier bits (so every register window starts at or above them); when it
// has fewer than T - c targets, its lowest strided tile bits are qubits that
// an earlier pass already handled and are not targets.
inline std::vector<PassGeom> plan_passes(int n, int prec)
{
    const int T = tile_bits(prec);
    std::vector<PassGeom> v;
    v.push_back(PassGeom{0, 0, (1u << T) - 1u});
    const int rem = n - T;
    if (rem <= 0) return v;
    const int cap = T - cmin_for(prec);
    const int np = (rem + cap - 1) / cap;
    int qa = T;  // first target qubit of the next pass
    for (int i = 0; i < np; ++i) {
        const int m = rem / np + (i < rem % np ? 1 : 0);
        const int c = std::min(T - m, 8);
        const int q0 = qa + m - (T - c);  // strided bits end at the last target
        v.push_back(PassGeom{c, q0, ((1u << T) - 1u) & ~((1u << (T - m)) - 1u)});
        qa += m;
    }
    return v;
}

// Window sequence covering all factors (single target bits, and two-bit
// factors that need both bits in one window), starting from window `start`,
// for a kernel with 2^tb threads (windows start at or below tb).
inline WinSeq plan_windows(int start, uint32_t targets, uint32_t pairs, int T, int tb)
{
    const int rb = T - tb;
    WinSeq w{};
    w.cnt = 0;
    w.s[w.cnt++] = start;
    auto in_win = [&](int s, uint32_t &t, uint32_t &pr) {
        t = targets & (((1u << rb) - 1u) << s);
        pr = pairs & (((1u << (rb - 1)) - 1u) << s);
    };
    uint32_t done = 0, pdone = 0;
    in_win(start, done, pdone);
    while ((targets & ~done) || (pairs & ~pdone)) {
        int low = 32;
        if (targets & ~done) low = __builtin_ctz(targets & ~done);
        if (pairs & ~pdone) low = std::min(low, __builtin_ctz(pairs & ~pdone));
        const int s = std::min(low, tb);
        if (w.cnt == kMaxWindows) {  // reported by the plan checker
            w.cnt = kMaxWindows + 1;
            return w;
        }
        w.s[w.cnt++] = s;
        uint32_t t, pr;
        in_win(s, t, pr);
        done |= t;
        pdone |= pr;
    }
    return w;
}

inline WinSeq plan_windows(int start, uint32_t targets, int T, int tb)
{
    return plan_windows(start, targets, 0u, T, tb);
}

// Tail of a stage: the stage's windows visited forward or in reverse, each
// applying the single factors in it that no earlier-visited window applied.
// Returns +k when every window but the last visited applies all rb of its
// register bits and the last applies its lowest k; -k when the last applies
// its highest k; 0 for any other pattern.  (k = rb: the last window is full
// too, and +rb is returned.)  The planner's stages always have such a tail,
// which lets a kernel fix at compile time which register bits a window
// updates instead of updating idle bits with a zero angle.
inline int stage_tail(const WinSeq &w, uint32_t targets, int rb, bool reverse)
{
    if (w.cnt < 1 || w.cnt > kMaxWindows) return 0;
    const uint32_t full = (1u << rb) - 1u;
    uint32_t done = 0;
    for (int j = 0; j < w.cnt; ++j) {
        const int i = reverse ? w.cnt - 1 - j : j;
        const uint32_t m = (targets >> w.s[i]) & full & ~(done >> w.s[i]);
        done |= m << w.s[i];
        if (j < w.cnt - 1) {
            if (m != full) return 0;
            continue;
        }
        const int k = __builtin_popcount(m);
        if (k == 0) return 0;
        if (m == (1u << k) - 1u) return k;
        if (m == (((1u << k) - 1u) << (rb - k))) return -k;
        return 0;
    }
    return 0;
}

// Compile-time tail of a kernel that visits one or two stages of a pass:
// the first stage must end in the low k bits (+k) and the second, if any, in
// the high k bits (-k), with the same k (a full last window, k = rb, fits
// either).  Returns k, or 0 when the pass does not have this shape.
inline int kernel_tail(int first, int second, bool two_stages, int rb)
{
    if (first <= 0) return 0;
    if (!two_stages) return first;
    const int k = first;
    if (second == -k || (k == rb && second == rb)) return k;
    return 0;
}

// Complement-symmetric storage.  Every state of the circuit satisfies
// psi(x) = psi(~x) (the cost function is invariant under complementing all
// bits, and so are |+>^n and the mixer), so only the half with bit n-1 = 0
// is stored, indexed by z, the "domain-wall" coordinates of y = x mod 2^(n-1):
//   z_q = y_q XOR y_(q+1)  (q < N-1),  z_(N-1) = y_(N-1),  N = n - 1,
// i.e. y_q = z_q XOR ... XOR z_(N-1).  In these coordinates X on qubit 0
// flips z_0; X on qubit q (1 <= q <= N-1) flips z_(q-1) and z_q; and X on
// qubit n-1, which maps the stored half onto the other half and back through
// the complement, flips z_(N-1) alone.  So the mixer is n commuting factors
// exp(-i theta/2 X..) on one or two adjacent z bits, each paired like an RX.
//
// Pass 0 is the contiguous low tile: the single factor on z_0 and the pairs
// (z_(q-1), z_q), q = 1..T-1.  Each strided pass holds the bit below its
// first pair so that every pair has both bits in the tile; the last pass also
// holds the single factor on z_(N-1).
inline std::vector<PassGeom> plan_passes_sym(int n, int prec)
{
    const int T = tile_bits(prec);
    const int N = n - 1;
    std::vector<PassGeom> v;
    PassGeom g0{0, 0, 1u, ((1u << (T - 1)) - 1u)};
    const int rem = N - T;          // pair factors q = T..N-1
    if (rem <= 0) return v;         // such small states are not supported in this layout
    v.push_back(g0);
    const int cap = T - cmin_for(prec) - 1;
    const int np = (rem + cap - 1) / cap;
    int qa = T;  // first pair factor (bits qa-1, qa) of the next pass
    for (int i = 0; i < np; ++i) {
        const int m = rem / np + (i < rem % np ? 1 : 0);
        const int c = std::min(T - m - 1, 8);
        const int q0 = qa + m - (T - c);           // strided bits end at bit qa+m-1
        const int e0 = c + (qa - 1 - q0);          // tile bit of global bit qa-1
        PassGeom g{c, q0, 0u, ((1u << m) - 1u) << e0};
        if (i == np - 1) g.targets = 1u << (T - 1);  // z_(N-1) is the top tile bit
        v.push_back(g);
        qa += m;
    }
    return v;
}

struct KSpec {
    int pass;
    int init;
    int pre, phase, post;  // layer indices, -1 = none
    int readout;
};

// Forward kernel list: layer 1 walks the passes in one order, layer 2 in the
// reverse order, and so on; the pass where two layers meet applies the end of
// one layer's mixer, the next cost phase and the start of the next mixer.
// The passes at the ends of the order are the junctions (two stages and the
// phase: bound by latency and arithmetic more than by memory) and the first
// and last passes of the circuit; the ones in between are plain stages, bound
// by memory.  With mid set and three or more passes, the contiguous pass
// (pass 0, the fastest geometry) walks in second place, among the plain ones,
// and a strided pass takes its place at the end (K32 complex64: forward 101
// -> 96.5 ms, forward + adjoint 292 -> 275.5 ms).
inline std::vector<KSpec> forward_specs(int P, int p, bool mid)
{
    std::vector<KSpec> ks;
    std::vector<int> order(P);
    for (int i = 0; i < P; ++i) order[i] = i;
    if (mid && P >= 3) std::swap(order[0], order[1]);
    ks.push_back(KSpec{order[0], 1, -1, 0, 0, 0});
    for (int i = 1; i < P; ++i) ks.push_back(KSpec{order[i], 0, -1, -1, 0, 0});
    for (int k = 1; k < p; ++k) {
        std::reverse(order.begin(), order.end());
        KSpec &last = ks.back();
        last.pre = k - 1;
        last.phase = k;
        last.post = k;
        for (int i = 1; i < P; ++i) ks.push_back(KSpec{order[i], 0, -1, -1, k, 0});
    }
    return ks;
}

}  // namespace qs
