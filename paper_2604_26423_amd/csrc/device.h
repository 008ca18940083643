// Device-side building blocks shared by the kernels of libqs (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace qs {

template <typename V> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };

template <typename V>
__device__ __forceinline__ V cmul(V a, V b)
{
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// FP64 phase argument reduced to about [-pi, pi].
__device__ __forceinline__ double reduce_2pi(double a)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double inv_two_pi = 0.15915494309189533576888376337251;
    return a - two_pi * rint(a * inv_two_pi);
}

// exp(i a) for an FP64 argument, rounded to the state precision.
template <typename V> __device__ __forceinline__ V expi(double a);
template <> __device__ __forceinline__ float2 expi<float2>(double a)
{
    double s, c;
    sincos(reduce_2pi(a), &s, &c);
    return float2{(float)c, (float)s};
}
template <> __device__ __forceinline__ double2 expi<double2>(double a)
{
    double s, c;
    sincos(reduce_2pi(a), &s, &c);
    return double2{c, s};
}

// Fixed-point probability mass of one amplitude, shared by the sampler and the
// cut-value histogram: P = re^2 + im^2 in FP64 with no fused multiply-add and
// q = floor(P 2^62) as uint64.  *flag becomes 2 when P >= 4 (or NaN): q would
// not fit in 64 bits.
__device__ __forceinline__ double prob_fp64(double re, double im)
{
    // hipcc contracts a * b + c into an FMA by default, also through the
    // __dmul_rn / __dadd_rn helpers; the rule needs two roundings of the
    // products and one of the sum
#pragma clang fp contract(off)
    const double a = re * re;
    const double b = im * im;
    return a + b;
}

__device__ __forceinline__ uint64_t qmass(double P, int32_t *flag)
{
    if (!(P < 4.0)) {
        *flag = 2;
        return 0;
    }
    return __double2ull_rz(__dmul_rn(P, 4611686018427387904.0));  // 2^62
}

__device__ __forceinline__ uint64_t qval(double re, double im, int32_t *flag)
{
    return qmass(prob_fp64(re, im), flag);
}

template <typename V>
__device__ __forceinline__ uint64_t qval_of(const V a, int32_t *flag)
{
    return qval((double)a.x, (double)a.y, flag);
}

// RX(theta) on a pair (a0 = bit clear, a1 = bit set), c = cos(theta/2), s = sin(theta/2):
//   a0' = c a0 - i s a1,  a1' = -i s a0 + c a1.
template <typename V, typename R>
__device__ __forceinline__ void rx_pair(V &a0, V &a1, R c, R s)
{
    V b0{c * a0.x + s * a1.y, c * a0.y - s * a1.x};
    V b1{c * a1.x + s * a0.y, c * a1.y - s * a0.x};
    a0 = b0;
    a1 = b1;
}

// Butterflies on register bit K of an array of NR amplitudes.
template <int K, typename V, int NR, typename R>
__device__ __forceinline__ void rx_reg_bit(V (&v)[NR], R c, R s)
{
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (!(r & (1 << K))) rx_pair(v[r], v[r | (1 << K)], c, s);
}

template <typename V, int NR, typename R>
__device__ __forceinline__ void rx_reg_mask(V (&v)[NR], uint32_t mask, R c, R s)
{
    if constexpr (NR > 1) { if (mask & 1u) rx_reg_bit<0>(v, c, s); }
    if constexpr (NR > 2) { if (mask & 2u) rx_reg_bit<1>(v, c, s); }
    if constexpr (NR > 4) { if (mask & 4u) rx_reg_bit<2>(v, c, s); }
    if constexpr (NR > 8) { if (mask & 8u) rx_reg_bit<3>(v, c, s); }
    if constexpr (NR >= 32) { if (mask & 16u) rx_reg_bit<4>(v, c, s); }
    if constexpr (NR >= 64) { if (mask & 32u) rx_reg_bit<5>(v, c, s); }
}

// Tangent form: (a0, a1) <- (a0 - i u a1, a1 - i u a0) = RX(theta)/cos(theta/2) on
// the pair when u = tan(theta/2).
template <typename V, typename R>
__device__ __forceinline__ void rxt_pair(V &a0, V &a1, R u)
{
    const V b0{a0.x + u * a1.y, a0.y - u * a1.x};
    const V b1{a1.x + u * a0.y, a1.y - u * a0.x};
    a0 = b0;
    a1 = b1;
}

template <int K, typename V, int NR, typename R>
__device__ __forceinline__ void rxt_reg_bit(V (&v)[NR], R u)
{
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (!(r & (1 << K))) rxt_pair(v[r], v[r | (1 << K)], u);
}

template <typename V, int NR, typename R>
__device__ __forceinline__ void rxt_reg_mask(V (&v)[NR], uint32_t mask, R u)
{
    if constexpr (NR > 1) { if (mask & 1u) rxt_reg_bit<0>(v, u); }
    if constexpr (NR > 2) { if (mask & 2u) rxt_reg_bit<1>(v, u); }
    if constexpr (NR > 4) { if (mask & 4u) rxt_reg_bit<2>(v, u); }
    if constexpr (NR > 8) { if (mask & 8u) rxt_reg_bit<3>(v, u); }
    if constexpr (NR >= 32) { if (mask & 16u) rxt_reg_bit<4>(v, u); }
    if constexpr (NR >= 64) { if (mask & 32u) rxt_reg_bit<5>(v, u); }
}

// Two-bit factors exp(-i theta/2 X_a X_b) on register bits K and K+1 (the
// mixer in complement-symmetric coordinates, see plan.h): the amplitudes at r
// and r ^ (3 << K) form the pair, with the same 2x2 update as RX.
template <int K, typename V, int NR, typename R>
__device__ __forceinline__ void rx_reg_bit2(V (&v)[NR], R c, R s)
{
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (!(r & (1 << K))) rx_pair(v[r], v[r ^ (3 << K)], c, s);
}

template <int K, typename V, int NR, typename R>
__device__ __forceinline__ void rxt_reg_bit2(V (&v)[NR], R u)
{
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (!(r & (1 << K))) rxt_pair(v[r], v[r ^ (3 << K)], u);
}

// Bit K of pmask selects the factor on register bits K and K+1.
template <typename V, int NR, typename R>
__device__ __forceinline__ void rx_reg_pairs(V (&v)[NR], uint32_t pmask, R c, R s)
{
    if constexpr (NR > 2) { if (pmask & 1u) rx_reg_bit2<0>(v, c, s); }
    if constexpr (NR > 4) { if (pmask & 2u) rx_reg_bit2<1>(v, c, s); }
    if constexpr (NR > 8) { if (pmask & 4u) rx_reg_bit2<2>(v, c, s); }
    if constexpr (NR >= 32) { if (pmask & 8u) rx_reg_bit2<3>(v, c, s); }
    if constexpr (NR >= 64) { if (pmask & 16u) rx_reg_bit2<4>(v, c, s); }
}

template <typename V, int NR, typename R>
__device__ __forceinline__ void rxt_reg_pairs(V (&v)[NR], uint32_t pmask, R u)
{
    if constexpr (NR > 2) { if (pmask & 1u) rxt_reg_bit2<0>(v, u); }
    if constexpr (NR > 4) { if (pmask & 2u) rxt_reg_bit2<1>(v, u); }
    if constexpr (NR > 8) { if (pmask & 4u) rxt_reg_bit2<2>(v, u); }
    if constexpr (NR >= 32) { if (pmask & 8u) rxt_reg_bit2<3>(v, u); }
    if constexpr (NR >= 64) { if (pmask & 16u) rxt_reg_bit2<4>(v, u); }
}

// Branch-free tangent-form stage on one register window.  Every register bit
// K gets the update with u_K = u when bit K of mask selects it and u_K = 0
// (the identity) otherwise.  With no branches between the updates the
// compiler keeps each amplitude in its registers; behind a runtime branch per
// bit it would copy the whole array at every join instead.
template <int K, typename R>
__device__ __forceinline__ R sel_u(uint32_t mask, R u)
{
    return ((mask >> K) & 1u) ? u : R(0);
}

template <typename V, int NR, typename R>
__device__ __forceinline__ void rxt_reg_all(V (&v)[NR], uint32_t mask, R u)
{
    if constexpr (NR > 1) rxt_reg_bit<0>(v, sel_u<0>(mask, u));
    if constexpr (NR > 2) rxt_reg_bit<1>(v, sel_u<1>(mask, u));
    if constexpr (NR > 4) rxt_reg_bit<2>(v, sel_u<2>(mask, u));
    if constexpr (NR > 8) rxt_reg_bit<3>(v, sel_u<3>(mask, u));
    if constexpr (NR > 16) rxt_reg_bit<4>(v, sel_u<4>(mask, u));
    if constexpr (NR > 32) rxt_reg_bit<5>(v, sel_u<5>(mask, u));
}

// Tangent-form updates on the register bits of a compile-time mask M only.
template <uint32_t M, typename V, int NR, typename R>
__device__ __forceinline__ void rxt_reg_const(V (&v)[NR], R u)
{
    if constexpr (NR > 1 && (M & 1u)) rxt_reg_bit<0>(v, u);
    if constexpr (NR > 2 && (M & 2u)) rxt_reg_bit<1>(v, u);
    if constexpr (NR > 4 && (M & 4u)) rxt_reg_bit<2>(v, u);
    if constexpr (NR > 8 && (M & 8u)) rxt_reg_bit<3>(v, u);
    if constexpr (NR > 16 && (M & 16u)) rxt_reg_bit<4>(v, u);
    if constexpr (NR > 32 && (M & 32u)) rxt_reg_bit<5>(v, u);
}

// Two-bit factors on register bits (K, K+1), K = 0..RB-2, selected by pmask.
template <typename V, int NR, typename R>
__device__ __forceinline__ void rxt_reg_pairs_all(V (&v)[NR], uint32_t pmask, R u)
{
    if constexpr (NR > 2) rxt_reg_bit2<0>(v, sel_u<0>(pmask, u));
    if constexpr (NR > 4) rxt_reg_bit2<1>(v, sel_u<1>(pmask, u));
    if constexpr (NR > 8) rxt_reg_bit2<2>(v, sel_u<2>(pmask, u));
    if constexpr (NR > 16) rxt_reg_bit2<3>(v, sel_u<3>(pmask, u));
    if constexpr (NR > 32) rxt_reg_bit2<4>(v, sel_u<4>(pmask, u));
}

// Single factors of the complement-symmetric layout sit only at the lowest or
// the highest register bit of a window (tile bits 0 and T-1).
template <typename V, int NR, typename R>
__device__ __forceinline__ void rxt_reg_ends(V (&v)[NR], uint32_t mask, R u)
{
    constexpr int top = __builtin_ctz(NR) - 1;
    rxt_reg_bit<0>(v, sel_u<0>(mask, u));
    if constexpr (top > 0) rxt_reg_bit<top>(v, sel_u<top>(mask, u));
}

// RX of a stage on the register bits in mask (and the two-bit factors in
// pmask); sign = -1 applies RX(-theta).
template <typename V, int NR>
__device__ __forceinline__ void stage_rx(V (&v)[NR], uint32_t mask, uint32_t pmask, const RxStage &st, int sign)
{
    using R = typename Real<V>::T;
    if (st.tan) {
        rxt_reg_mask(v, mask, (R)(sign * st.u));
        if (pmask) rxt_reg_pairs(v, pmask, (R)(sign * st.u));
    } else {
        rx_reg_mask(v, mask, (R)st.c, (R)(sign * st.s));
        if (pmask) rx_reg_pairs(v, pmask, (R)st.c, (R)(sign * st.s));
    }
}

// The gradient term of one amplitude pair (a0, a1) of a factor:
// Im(conj(l0) p1) + Im(conj(l1) p0), a four-product dot in the state
// precision (one fused multiply-add per product after the first).
template <typename V>
__device__ __forceinline__ typename Real<V>::T imx_pair(V l0, V l1, V p0, V p1)
{
    typename Real<V>::T t = l0.x * p1.y;
    t = fma(-l0.y, p1.x, t);
    t = fma(l1.x, p0.y, t);
    return fma(-l1.y, p0.x, t);
}

// Im <lam| X_q |psi> restricted to the pairs held in registers, for register
// bit K: the sum over the thread's NR/2 pairs of their terms.  Each pair's
// term is formed in the state precision and the sum over pairs is taken in
// FP64.
template <int K, typename V, int NR>
__device__ __forceinline__ double imx_reg_bit(const V (&l)[NR], const V (&p)[NR])
{
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (!(r & (1 << K))) acc += (double)imx_pair(l[r], l[r | (1 << K)], p[r], p[r | (1 << K)]);
    return acc;
}

template <typename V, int NR>
__device__ __forceinline__ double imx_reg_mask(const V (&l)[NR], const V (&p)[NR], uint32_t mask)
{
    double acc = 0.0;
    if constexpr (NR > 1) { if (mask & 1u) acc += imx_reg_bit<0>(l, p); }
    if constexpr (NR > 2) { if (mask & 2u) acc += imx_reg_bit<1>(l, p); }
    if constexpr (NR > 4) { if (mask & 4u) acc += imx_reg_bit<2>(l, p); }
    if constexpr (NR > 8) { if (mask & 8u) acc += imx_reg_bit<3>(l, p); }
    if constexpr (NR >= 32) { if (mask & 16u) acc += imx_reg_bit<4>(l, p); }
    if constexpr (NR >= 64) { if (mask & 32u) acc += imx_reg_bit<5>(l, p); }
    return acc;
}

// Branch-free sums of Im <lam| X.. |psi> over the selected register bits
// (weights 0 or 1), in FP64.
template <int K>
__device__ __forceinline__ double sel_w(uint32_t mask)
{
    return ((mask >> K) & 1u) ? 1.0 : 0.0;
}

template <typename V, int NR>
__device__ __forceinline__ double imx_reg_all(const V (&l)[NR], const V (&p)[NR], uint32_t mask)
{
    double g = 0.0;
    if constexpr (NR > 1) g += sel_w<0>(mask) * imx_reg_bit<0>(l, p);
    if constexpr (NR > 2) g += sel_w<1>(mask) * imx_reg_bit<1>(l, p);
    if constexpr (NR > 4) g += sel_w<2>(mask) * imx_reg_bit<2>(l, p);
    if constexpr (NR > 8) g += sel_w<3>(mask) * imx_reg_bit<3>(l, p);
    if constexpr (NR > 16) g += sel_w<4>(mask) * imx_reg_bit<4>(l, p);
    if constexpr (NR > 32) g += sel_w<5>(mask) * imx_reg_bit<5>(l, p);
    return g;
}

// The same sums over the register bits of a compile-time mask M.
template <uint32_t M, typename V, int NR>
__device__ __forceinline__ double imx_reg_const(const V (&l)[NR], const V (&p)[NR])
{
    double g = 0.0;
    if constexpr (NR > 1 && (M & 1u)) g += imx_reg_bit<0>(l, p);
    if constexpr (NR > 2 && (M & 2u)) g += imx_reg_bit<1>(l, p);
    if constexpr (NR > 4 && (M & 4u)) g += imx_reg_bit<2>(l, p);
    if constexpr (NR > 8 && (M & 8u)) g += imx_reg_bit<3>(l, p);
    if constexpr (NR > 16 && (M & 16u)) g += imx_reg_bit<4>(l, p);
    if constexpr (NR > 32 && (M & 32u)) g += imx_reg_bit<5>(l, p);
    return g;
}

template <typename V, int NR>
__device__ __forceinline__ double imx_reg_ends(const V (&l)[NR], const V (&p)[NR], uint32_t mask)
{
    constexpr int top = __builtin_ctz(NR) - 1;
    double g = sel_w<0>(mask) * imx_reg_bit<0>(l, p);
    if constexpr (top > 0) g += sel_w<top>(mask) * imx_reg_bit<top>(l, p);
    return g;
}

// Im <lam| X_a X_b |psi> for the two-bit factor on register bits K, K+1.
template <int K, typename V, int NR>
__device__ __forceinline__ double imx_reg_bit2(const V (&l)[NR], const V (&p)[NR])
{
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (!(r & (1 << K))) acc += (double)imx_pair(l[r], l[r ^ (3 << K)], p[r], p[r ^ (3 << K)]);
    return acc;
}

template <typename V, int NR>
__device__ __forceinline__ double imx_reg_pairs(const V (&l)[NR], const V (&p)[NR], uint32_t pmask)
{
    double acc = 0.0;
    if constexpr (NR > 2) { if (pmask & 1u) acc += imx_reg_bit2<0>(l, p); }
    if constexpr (NR > 4) { if (pmask & 2u) acc += imx_reg_bit2<1>(l, p); }
    if constexpr (NR > 8) { if (pmask & 4u) acc += imx_reg_bit2<2>(l, p); }
    if constexpr (NR >= 32) { if (pmask & 8u) acc += imx_reg_bit2<3>(l, p); }
    if constexpr (NR >= 64) { if (pmask & 16u) acc += imx_reg_bit2<4>(l, p); }
    return acc;
}

template <typename V, int NR>
__device__ __forceinline__ double imx_reg_pairs_all(const V (&l)[NR], const V (&p)[NR], uint32_t pmask)
{
    double g = 0.0;
    if constexpr (NR > 2) g += sel_w<0>(pmask) * imx_reg_bit2<0>(l, p);
    if constexpr (NR > 4) g += sel_w<1>(pmask) * imx_reg_bit2<1>(l, p);
    if constexpr (NR > 8) g += sel_w<2>(pmask) * imx_reg_bit2<2>(l, p);
    if constexpr (NR > 16) g += sel_w<3>(pmask) * imx_reg_bit2<3>(l, p);
    if constexpr (NR > 32) g += sel_w<4>(pmask) * imx_reg_bit2<4>(l, p);
    return g;
}

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that each
// XCD works on a contiguous range of tiles (neighbouring tiles share L2 lines
// of the cost diagonal and TLB pages).
__device__ __forceinline__ int64_t xcd_tile(int remap)
{
    const int64_t b = blockIdx.x, g = gridDim.x;
    if (!remap) return b;
    return (b & 7) * (g >> 3) + (b >> 3);
}

template <typename V>
__device__ __forceinline__ V scale_v(V a, typename Real<V>::T f)
{
    return V{a.x * f, a.y * f};
}

// Nontemporal (streaming) access to one amplitude: the load and the store
// carry the streaming cache policy, as plain vector accesses of the element's
// two components.
template <typename V> struct NtVec;
template <> struct NtVec<float2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct NtVec<double2> { typedef double T __attribute__((ext_vector_type(2))); };

template <typename V>
__device__ __forceinline__ V load_nt(const V *p)
{
    const typename NtVec<V>::T t = __builtin_nontemporal_load(reinterpret_cast<const typename NtVec<V>::T *>(p));
    return V{t.x, t.y};
}

template <typename V>
__device__ __forceinline__ void store_nt(V *p, V v)
{
    typename NtVec<V>::T t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<typename NtVec<V>::T *>(p));
}

// LDS byte offset of slot (thread part) XOR slot (register part).  The slot
// map is linear over XOR, so the address of register r in a layout is the
// thread's part XOR a part that depends only on r and the (uniform) window:
// computed on the scalar unit, it costs one vector XOR per access.  (Left to
// itself the compiler rebuilds the whole index per register, about six vector
// instructions.)
template <typename V>
__device__ __forceinline__ V &lds_at(V *lds, int byte_off)
{
    return *reinterpret_cast<V *>(reinterpret_cast<char *>(lds) + byte_off);
}

template <int RB, typename V>
__device__ __forceinline__ int lds_reg_bytes(int r, int win)
{
    return __builtin_amdgcn_readfirstlane(lds_slot<RB>(r << win) * (int)sizeof(V));
}

// Byte offset of the thread's part of a layout, kept opaque so that the
// compiler XORs it with the register part instead of rebuilding it.
template <int RB, typename V>
__device__ __forceinline__ int lds_thread_bytes(int tid, int win)
{
    int t = lds_slot<RB>(win_elem(0, tid, win, RB)) * (int)sizeof(V);
    asm volatile("" : "+v"(t));
    return t;
}

// Move the NR amplitudes of every thread from layout `from` to layout `to`
// through LDS.  Leading barrier: earlier LDS reads of this buffer are done.
template <int RB, typename V, int NR>
__device__ __forceinline__ void exchange(V (&v)[NR], V *lds, int from, int to, int tid)
{
    const int tf = lds_thread_bytes<RB, V>(tid, from);
    const int tt = lds_thread_bytes<RB, V>(tid, to);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) lds_at(lds, tf ^ lds_reg_bytes<RB, V>(r, from)) = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = lds_at(lds, tt ^ lds_reg_bytes<RB, V>(r, to));
}

// The same move for two arrays at once through an LDS buffer of two tiles:
// one pair of barriers instead of two.
template <int RB, typename V, int NR>
__device__ __forceinline__ void exchange2(V (&a)[NR], V (&b)[NR], V *lds, int from, int to, int tid)
{
    constexpr int TILE = NR << 9;  // 2^(RB + 9): tiles of the 512-thread kernels
    V *ldb = lds + TILE;
    const int tf = lds_thread_bytes<RB, V>(tid, from);
    const int tt = lds_thread_bytes<RB, V>(tid, to);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int o = tf ^ lds_reg_bytes<RB, V>(r, from);
        lds_at(lds, o) = a[r];
        lds_at(ldb, o) = b[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int o = tt ^ lds_reg_bytes<RB, V>(r, to);
        a[r] = lds_at(lds, o);
        b[r] = lds_at(ldb, o);
    }
}

// Deterministic workgroup sum of NV doubles (fixed shuffle tree, then waves in
// order).  Result valid in thread 0.  `red` holds NV * (blockDim/64) doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&x)[NV], double *red, int tid, int nthreads)
{
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x[k] += __shfl_xor(x[k], off, 64);
    }
    const int wave = tid >> 6, lane = tid & 63, nw = nthreads >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = x[k];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[w * NV + k];
            x[k] = s;
        }
    }
}

}  // namespace qs
