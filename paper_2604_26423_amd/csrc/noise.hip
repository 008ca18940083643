// Noisy LR-QAOA trajectories (arXiv:2604.26423, Sec. II-C): a two-qubit
// depolarizing channel of rate eps after every RZZ gate, unravelled into
// Pauli insertions.  One workgroup runs one trajectory of an n <= 12 qubit
// circuit with the whole state in registers (2^RB amplitudes per thread) and
// LDS (exchanges, the cost diagonal, the phase table).
//
// Draw rule (trajectory t, layer k, edge e in lexicographic order):
//   (r0, r1, ..) = Philox4x64-10(counter (t, k, e, 1), key (seed, 0));
//   the gate errs iff (r0 >> 11) < thr = floor(eps 2^53); its Pauli is
//   code = r1 & 15, P_a = code & 3 on the edge's lower qubit, P_b = code >> 2
//   on the upper one (0 I, 1 X, 2 Y = i X Z, 3 Z).
//
// The cost layer stays one fused diagonal.  Errors are moved to the end of
// the layer: an X component on qubit v anticommutes with Z_v Z_u, so every
// later gate touching v changes the sign of its angle.  With F the set of
// gates whose sign flipped an odd number of times,
//   prod_g E_g U_g = E_tot exp(-i theta/2 [sum_g w_g z_a z_b - 2 sum_{g in F} w_g z_a z_b]),
// and E_tot = i^a X^ex Z^ez (product of the layer's Paulis in gate order).
// X components are not applied to the state: they commute with every RX, so
// the trajectory keeps a frame m with psi_true = i^phi X^m psi_stored, and the
// next cost diagonal is read at x ^ m.  Z components are applied as signs.
// Per amplitude the layer's phase is exp(-i theta K / 20) with
//   K = (W - 2 C(y)) - 2 (W_F - 2 C_F(y)),  y = x ^ m,
// C_F the cut of y over the flipped gates (a short list, empty without
// errors).  The mixer is unchanged.
#include "tiles.h"

namespace qs {

namespace {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), words 0 and 1 of the
// output for counter (c0, c1, c2, c3) and key (k0, 0).
__device__ __forceinline__ void philox_w01(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                           uint64_t &w0, uint64_t &w1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = c3, ka = k0, kb = 0;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            ka += W0;
            kb += W1;
        }
        const uint64_t h0 = __umul64hi(M0, x0), l0 = M0 * x0;
        const uint64_t h1 = __umul64hi(M1, x2), l1 = M1 * x2;
        const uint64_t y0 = h1 ^ x1 ^ ka, y2 = h0 ^ x3 ^ kb;
        x0 = y0;
        x1 = l1;
        x2 = y2;
        x3 = l0;
    }
    w0 = x0;
    w1 = x1;
}

template <int N> struct NoiseCfg {
    // threads: 2^(n-4) from n = 10 (16 amplitudes each), one wave for n = 8, 9
    static constexpr int TB = N >= 10 ? N - 4 : (N >= 8 ? 6 : N - 2);
    static constexpr int RB = N - TB;
    static constexpr int NR = 1 << RB, NT = 1 << TB;
    static constexpr int WL = NT < 64 ? NT : 64;  // lanes of the bookkeeping wave
    static constexpr int NW = (N + RB - 1) / RB;  // register windows per layer
    static constexpr int G = N * (N - 1) / 2;     // gates per cost layer
    static constexpr int pos(int j) { return j * RB < N - RB ? j * RB : N - RB; }
    static constexpr uint32_t win(int j) { return ((1u << RB) - 1u) << pos(j); }
    // register-bit targets of window j when the windows run in ascending
    // (ASC) or descending order: its qubits not covered by an earlier window
    static constexpr uint32_t targets(int j, bool asc)
    {
        uint32_t done = 0;
        if (asc)
            for (int i = 0; i < j; ++i) done |= win(i);
        else
            for (int i = NW - 1; i > j; --i) done |= win(i);
        return (win(j) & ~done) >> pos(j);
    }
};

// Workgroup sum of two doubles into thread 0.  Fewer than 64 threads form
// one partial wave: shuffle only among its lanes.
template <int NT>
__device__ __forceinline__ void noise_sum(double (&x)[2], double *red, int tid)
{
    if constexpr (NT >= 64) {
        block_sum(x, red, tid, NT);
    } else {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
#pragma unroll
            for (int off = NT / 2; off >= 1; off >>= 1) x[k] += __shfl_xor(x[k], off, 64);
        }
    }
}

// LDS slot of cut value x: the low 4 bits are XORed with bits 6..9, so that
// the 64 lanes of a wave reading one register's values -- consecutive x in
// the layouts whose window holds the high bits, x 16 (or 2^RB) apart in the
// layout whose window holds the low bits, both XORed with the frame -- hit
// 64 different banks.
// The map is linear over XOR: slot(a ^ b) = slot(a) ^ slot(b).
__host__ __device__ constexpr int dg_slot(uint32_t x) { return (int)(x ^ ((x >> 6) & 15u)); }

struct NoiseShared {
    int nf, wf, ph, cnt;
    uint32_t ex, ez;
};

// LV = 2: two-level phase table (3 W < 2^13, every graph with weights up to
// 10 tenths at n <= 12); LV = 0: levels read at run time.
template <typename V, int LV>
__device__ __forceinline__ V noise_phase(const V *tab, int levels, int u)
{
    if constexpr (LV == 2) return cmul(tab[u & 63], tab[64 + ((u >> 6) & 127)]);
    else return phase_factor(tab, levels, u);
}

// Cost layer with its errors, then the mixer, for layer k.  The state enters
// in the layout of the first window of this layer's order and leaves in the
// layout of the last.
template <typename V, int N, int MODE, int LV, bool ASC>
__device__ __forceinline__ void noise_layer(const NoiseProg &np, int k, V (&v)[NoiseCfg<N>::NR], V *lds,
                                            const int32_t *dg, V *tab, uint8_t *codes, uint32_t *fm, int *fw,
                                            NoiseShared &sh, uint32_t &m, int &phi, int &nerr, double &fprev,
                                            int tid)
{
    using Cfg = NoiseCfg<N>;
    using R = typename Real<V>::T;
    constexpr int RB = Cfg::RB, NR = Cfg::NR, NT = Cfg::NT, G = Cfg::G, WL = Cfg::WL, NW = Cfg::NW;
    const double *lay = np.layers + 4 * k;

    // draws of the next chunk of layers (counter-based: any order gives the same codes)
    if (k % kNoiseChunk == 0) {
        const int len = np.p - k < kNoiseChunk ? np.p - k : kNoiseChunk;
        __syncthreads();  // the previous chunk's codes are no longer read
        for (int i = tid; i < len * G; i += NT) {
            uint8_t c = 0;
            if (np.thr != 0) {
                uint64_t r0, r1;
                philox_w01(np.traj0 + blockIdx.x, (uint64_t)(k + i / G), (uint64_t)(i % G), 1, np.seed, r0, r1);
                c = (r0 >> 11) < np.thr ? (uint8_t)(r1 & 15u) : (uint8_t)0;
            }
            codes[i] = c;
        }
    }
    __syncthreads();  // codes visible; the previous layer's table and F reads done

    // phase table of this layer (the same for every trajectory, built by noise_table_kernel)
    {
        const V *src = reinterpret_cast<const V *>(np.tabs) + (size_t)k * kTabMax;
        const int ntab = 64 * (np.levels - 1) + 128;
        for (int i = tid; i < ntab; i += NT) tab[i] = src[i];
    }

    // the layer's errors, moved to its end (one wave, gates in order)
    if (tid < WL) {
        const int lane = tid;
        const uint8_t *cl = codes + (k % kNoiseChunk) * G;
        uint32_t carry = 0, ez = 0;
        int nf = 0, wf = 0, ph = 0, cnt = 0;
        // most layers draw no error: then every sum below stays zero
        bool any = false;
        for (int base = 0; base < G; base += WL) any |= base + lane < G && cl[base + lane] != 0;
        const int first = __ballot(any) != 0 ? 0 : G;
        for (int base = first; base < G; base += WL) {
            const int e = base + lane;
            const bool valid = e < G;
            const int code = valid ? cl[e] : 0;
            const uint32_t ab = valid ? (uint32_t)np.edges[e] : 0u;
            const int a = ab & 15, b = (ab >> 4) & 15, wt = (int)(ab >> 8);
            const int pa = code & 3, pb = code >> 2;
            const uint32_t xm = ((uint32_t)(pa == 1 || pa == 2) << a) | ((uint32_t)(pb == 1 || pb == 2) << b);
            const uint32_t zm = ((uint32_t)(pa >= 2) << a) | ((uint32_t)(pb >= 2) << b);
            // prefix XOR of the X components over the gates before e
            uint32_t incl = xm;
#pragma unroll
            for (int d = 1; d < WL; d <<= 1) {
                const uint32_t t = __shfl_up(incl, d, 64);
                if (lane >= d) incl ^= t;
            }
            const uint32_t before = incl ^ xm ^ carry;
            const uint32_t emask = (1u << a) | (1u << b);
            const bool flip = valid && (__popc(before & emask) & 1);
            const uint64_t bal = __ballot(flip);
            if (flip) {
                const int at = nf + __popcll(bal & ((1ull << lane) - 1ull));
                fm[at] = emask;
                fw[at] = wt;
            }
            nf += __popcll(bal);
            int sw = flip ? wt : 0;
            // E_e (i^y X^xm Z^zm) multiplied onto the product of the earlier errors
            int sp = (pa == 2) + (pb == 2) + 2 * (__popc(zm & before) & 1);
            int sc = code != 0;
            uint32_t sz = zm;
#pragma unroll
            for (int off = WL / 2; off >= 1; off >>= 1) {
                sw += __shfl_xor(sw, off, 64);
                sp += __shfl_xor(sp, off, 64);
                sc += __shfl_xor(sc, off, 64);
                sz ^= __shfl_xor(sz, off, 64);
            }
            wf += sw;
            ph += sp;
            cnt += sc;
            ez ^= sz;
            carry ^= __shfl(incl, WL - 1, 64);
        }
        if (lane == 0) {
            sh.nf = nf;
            sh.wf = wf;
            sh.ph = ph & 3;
            sh.cnt = cnt;
            sh.ex = carry;
            sh.ez = ez;
        }
    }
    __syncthreads();

    const int nf = __builtin_amdgcn_readfirstlane(sh.nf);
    const int wf = __builtin_amdgcn_readfirstlane(sh.wf);
    const uint32_t ez = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.ez);
    const uint32_t ex = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.ex);

    // cost phase, in the layout of this layer's first window
    constexpr int s0 = ASC ? Cfg::pos(0) : Cfg::pos(NW - 1);
    const int xb = win_elem(0, tid, s0, RB);
    const int u0 = 2 * (int)np.W - wf;
    int cf[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) cf[r] = 0;
    for (int f = 0; f < nf; ++f) {
        const uint32_t mk = fm[f];
        const int wk = fw[f];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint32_t y = (uint32_t)(xb | (r << s0)) ^ m;
            cf[r] += (__popc(y & mk) & 1) ? wk : 0;
        }
    }
    V f[NR];
    const int db = dg_slot((uint32_t)xb ^ m);  // per-thread part of the slot; the register part is a constant
#pragma unroll
    for (int r = 0; r < NR; ++r)
        f[r] = noise_phase<V, LV>(tab, np.levels, u0 - dg[db ^ dg_slot((uint32_t)r << s0)] + 2 * cf[r]);
    if (ez != 0) {  // Z components of the layer's errors (rare): signs
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (__popc((uint32_t)(xb | (r << s0)) & ez) & 1) f[r] = V{-f[r].x, -f[r].y};
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = cmul(v[r], f[r]);
    phi = (phi + sh.ph + 2 * (__popc(ez & m) & 1)) & 3;
    m ^= ex;
    nerr += sh.cnt;

    // mixer: RX on every qubit, window by window
    const R a = (R)lay[1], b = (R)lay[2];
#pragma unroll
    for (int jj = 0; jj < NW; ++jj) {
        const int j = ASC ? jj : NW - 1 - jj;
        if (jj > 0) exchange<RB>(v, lds, Cfg::pos(ASC ? j - 1 : j + 1), Cfg::pos(j), tid);
        const uint32_t mask = Cfg::targets(j, ASC);
        if constexpr (MODE == kModeTan) rxt_reg_all(v, mask, a);
        else rx_reg_mask(v, mask, a, b);
    }
    fprev = lay[3];
}

template <typename V, int N, int MODE, int LV>
__global__ void __launch_bounds__(NoiseCfg<N>::NT) noise_kernel(NoiseProg np)
{
    using Cfg = NoiseCfg<N>;
    using R = typename Real<V>::T;
    constexpr int NR = Cfg::NR, NT = Cfg::NT, RB = Cfg::RB, NW = Cfg::NW, G = Cfg::G;
    __shared__ V lds[1 << N];
    __shared__ int32_t dg[1 << N];
    __shared__ V tab[kTabMax];
    __shared__ uint8_t codes[kNoiseChunk * G];
    __shared__ uint32_t fm[G];
    __shared__ int fw[G];
    __shared__ NoiseShared sh;
    __shared__ double red[2 * (NT < 64 ? 1 : NT / 64)];
    const int tid = threadIdx.x;

    for (int i = tid; i < (1 << N); i += NT) dg[dg_slot((uint32_t)i)] = np.diag[i];
    V v[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = V{(R)np.amp0, (R)0};
    uint32_t m = 0;
    int phi = 0, nerr = 0;
    double fprev = 1.0;

    int k = 0;
    for (; k + 1 < np.p; k += 2) {
        noise_layer<V, N, MODE, LV, true>(np, k, v, lds, dg, tab, codes, fm, fw, sh, m, phi, nerr, fprev, tid);
        noise_layer<V, N, MODE, LV, false>(np, k + 1, v, lds, dg, tab, codes, fm, fw, sh, m, phi, nerr, fprev, tid);
    }
    if (k < np.p)
        noise_layer<V, N, MODE, LV, true>(np, k, v, lds, dg, tab, codes, fm, fw, sh, m, phi, nerr, fprev, tid);
    const int s = (np.p & 1) ? Cfg::pos(NW - 1) : Cfg::pos(0);

    // readout: psi_true[x ^ m] = i^phi fprev psi_stored[x]
    const int xb = win_elem(0, tid, s, RB);
    const R fs = (R)fprev;
    double acc[2] = {0.0, 0.0};
    V *out = np.states ? reinterpret_cast<V *>(np.states) + ((int64_t)blockIdx.x << N) : nullptr;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const uint32_t x = (uint32_t)(xb | (r << s));
        V a = V{fs * v[r].x, fs * v[r].y};
        const double pr = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        acc[0] += pr;
        acc[1] += pr * (double)dg[dg_slot(x ^ m)];
        if (out) {
            V t = a;
            if (phi & 1) t = V{-a.y, a.x};
            if (phi & 2) t = V{-t.x, -t.y};
            out[x ^ m] = t;
        }
    }
    noise_sum<NT>(acc, red, tid);
    if (tid == 0) {
        np.exp_c[blockIdx.x] = acc[1] / acc[0] / 10.0;
        if (np.norm) np.norm[blockIdx.x] = acc[0];
        if (np.nerr) np.nerr[blockIdx.x] = nerr;
    }
}

// Phase table of every layer k: entry(u) = f_(k-1) exp(-i theta_zz,k (2u - 3W) / 20),
// f_(k-1) the tangent-form factor of the previous layer's mixer (1 for k = 0).
template <typename V>
__global__ void __launch_bounds__(256) noise_table_kernel(NoiseProg np)
{
    const int k = blockIdx.x;
    const double f = k == 0 ? 1.0 : np.layers[4 * (k - 1) + 3];
    build_phase_table(reinterpret_cast<V *>(np.tabs) + (size_t)k * kTabMax, np.levels, -np.layers[4 * k],
                      3 * np.W, f, threadIdx.x, 256);
}

template <typename V, int MODE, int LV>
hipError_t launch_noise_v(const NoiseProg &np, int64_t ntraj, hipStream_t st)
{
    hipLaunchKernelGGL(noise_table_kernel<V>, dim3(np.p), dim3(256), 0, st, np);
    const dim3 g((unsigned)ntraj);
    switch (np.n) {
#define QS_NOISE_CASE(NN)                                                                                       \
    case NN: hipLaunchKernelGGL((noise_kernel<V, NN, MODE, LV>), g, dim3(NoiseCfg<NN>::NT), 0, st, np); break;
        QS_NOISE_CASE(2)
        QS_NOISE_CASE(3)
        QS_NOISE_CASE(4)
        QS_NOISE_CASE(5)
        QS_NOISE_CASE(6)
        QS_NOISE_CASE(7)
        QS_NOISE_CASE(8)
        QS_NOISE_CASE(9)
        QS_NOISE_CASE(10)
        QS_NOISE_CASE(11)
        QS_NOISE_CASE(12)
#undef QS_NOISE_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int noise_table_entries() { return kTabMax; }

int noise_threads(int n)
{
    return n >= 10 ? 1 << (n - 4) : (n >= 8 ? 64 : 1 << (n - 2));
}

hipError_t launch_noise(int prec, int tangent, const NoiseProg &np, int64_t ntraj, hipStream_t st)
{
    if (np.n < 2 || np.n > kNoiseMaxQubits || ntraj < 1 || ntraj > 0x7fffffff) return hipErrorInvalidValue;
    // np.levels is 2 whenever 3 W < 2^13 (the host raises 1 to 2); larger graphs take the
    // run-time-levels kernel with the direct-form mixer
    if (np.levels == 2) {
        if (prec == 0)
            return tangent ? launch_noise_v<float2, kModeTan, 2>(np, ntraj, st)
                           : launch_noise_v<float2, kModeGeneral, 2>(np, ntraj, st);
        return tangent ? launch_noise_v<double2, kModeTan, 2>(np, ntraj, st)
                       : launch_noise_v<double2, kModeGeneral, 2>(np, ntraj, st);
    }
    return prec == 0 ? launch_noise_v<float2, kModeGeneral, 0>(np, ntraj, st)
                     : launch_noise_v<double2, kModeGeneral, 0>(np, ntraj, st);
}

}  // namespace qs
