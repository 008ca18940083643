// Host-side plan of the tile passes: which qubits each pass covers, the
// register windows of each butterfly stage, and the order in which the
// layers' mixer passes and cost phases are fused into kernels.
#pragma once

#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace qs {

struct PassGeom {
    int c, q0;
    uint32_t targets;
};

inline int cmin_for(int prec)
{
    // Minimum carrier bits of a strided pass: contiguous runs of 2^c amplitudes
    // (complex64: 8 x 8 B = 64 B; complex128: 8 x 16 B = 128 B).  The
    // environment variable QS_CARRIER_BITS overrides it for tuning.
    const char *v = getenv("QS_CARRIER_BITS");
    const int env = v ? atoi(v) : 0;
    if (env >= 1 && env <= tile_bits(prec) - 1) return env;
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

// Window sequence covering all target bits, starting from window `start`,
// for a kernel with 2^tb threads (windows start at or below tb).
inline WinSeq plan_windows(int start, uint32_t targets, int T, int tb)
{
    const int rb = T - tb;
    WinSeq w{};
    w.cnt = 0;
    w.s[w.cnt++] = start;
    uint32_t done = targets & (((1u << rb) - 1u) << start);
    while (targets & ~done) {
        const int low = __builtin_ctz(targets & ~done);
        const int s = std::min(low, tb);
        w.s[w.cnt++] = s;
        done |= targets & (((1u << rb) - 1u) << s);
    }
    return w;
}

struct KSpec {
    int pass;
    int init;
    int pre, phase, post;  // layer indices, -1 = none
    int readout;
};

// Forward kernel list: layer 1 walks the passes in ascending order, layer 2
// descending, and so on; the pass where two layers meet applies the end of
// one layer's mixer, the next cost phase and the start of the next mixer.
inline std::vector<KSpec> forward_specs(int P, int p)
{
    std::vector<KSpec> ks;
    std::vector<int> order(P);
    for (int i = 0; i < P; ++i) order[i] = i;
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
