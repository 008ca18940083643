// Measurement shots (arXiv:2604.26423, Sec. II-B: repeated preparation and
// measurement), reproducible bit for bit:
//   P(x) = re^2 + im^2 in FP64 with no fused multiply-add, q(x) = floor(P 2^62),
//   F(x) = sum_{y<=x} q(y) (uint64), T = F(2^n - 1);
//   shot s: r = word 0 of Philox4x64-10(counter (s,0,0,0), key (seed,0)),
//   u = floor(r T / 2^64), x_s = min { x : F(x) > u }.
// The CDF is never stored.  Pass A writes exclusive prefix sums at three
// levels: 64-amplitude sub-blocks within 8192-amplitude blocks, blocks within
// 2^26-amplitude chunks, and chunks; integer sums make the result independent
// of summation order.  Each shot then descends the three levels by binary
// search and scans 64 amplitudes.  Small states (n < 13) use one workgroup
// and a full CDF in LDS.
#include "device.h"

namespace qs {

namespace {

constexpr int kBlockBits = 13;   // amplitudes per block: 8192
constexpr int kSubBits = 6;      // amplitudes per sub-block: 64
constexpr int kChunkBits = 26;   // amplitudes per chunk
constexpr int kSubPerBlock = 1 << (kBlockBits - kSubBits);            // 128
constexpr int kBlkPerChunk = 1 << (kChunkBits - kBlockBits);          // 8192

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), words 0 and 1 of the
// output for counter (c0, 0, 0, 0) and key (k0, 0).
__device__ __forceinline__ void philox_words01(uint64_t c0, uint64_t k0, uint64_t &w0, uint64_t &w1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = c0, x1 = 0, x2 = 0, x3 = 0, ka = k0, kb = 0;
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

__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t k0)
{
    uint64_t w0, w1;
    philox_words01(c0, k0, w0, w1);
    return w0;
}

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_scan_u64(uint64_t v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Two consecutive amplitudes (an even index): one 16-byte load for complex64.
// Pass A reads each amplitude once: nontemporal (streaming) loads, which
// measured pass A 10% faster at n = 32 in complex64 (6.25 -> 5.65 ms).
template <typename V> struct AmpPair;
template <> struct AmpPair<float2> {
    static __device__ __forceinline__ void load(const float2 *p, float2 &a, float2 &b)
    {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p));
        a = float2{t.x, t.y};
        b = float2{t.z, t.w};
    }
};
template <> struct AmpPair<double2> {
    static __device__ __forceinline__ void load(const double2 *p, double2 &a, double2 &b)
    {
        a = load_nt(p);
        b = load_nt(p + 1);
    }
};

// Pass A: one workgroup per block of 8192 amplitudes.  Thread t reads the
// pairs (i 512 + 2 t, +1), i = 0..15, all issued before any arithmetic; the 32
// lanes of half a wave then hold one 64-amplitude sub-block and sum it with
// five shuffles.
template <typename V>
__global__ void __launch_bounds__(256) sample_blocks_kernel(const V *psi, uint64_t *sub, uint64_t *blk,
                                                            int32_t *flag)
{
    constexpr int NL = (1 << kBlockBits) / 512;  // pairs per thread
    __shared__ uint64_t ssum[kSubPerBlock];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t b = blockIdx.x;
    const V *blkp = psi + (b << kBlockBits);
    // layout of the block's entries (internal.h): the fold moves bits 4..12 only,
    // so a pair at an even index stays a pair
    const int fb = (int)(swz_fold(b) << kSwzDst);
    V a[NL], c[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) AmpPair<V>::load(blkp + ((i * 512 + 2 * tid) ^ fb), a[i], c[i]);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        uint64_t q = qval_of(a[i], flag) + qval_of(c[i], flag);
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) q += __shfl_xor(q, off, 64);
        if ((lane & 31) == 0) ssum[i * 8 + 2 * wave + (lane >> 5)] = q;
    }
    __syncthreads();
    if (wave == 0) {
        const uint64_t a0 = ssum[2 * lane], a1 = ssum[2 * lane + 1];
        const uint64_t incl = wave_scan_u64(a0 + a1, lane);
        const uint64_t excl = incl - (a0 + a1);
        sub[b * kSubPerBlock + 2 * lane] = excl;
        sub[b * kSubPerBlock + 2 * lane + 1] = excl + a0;
        if (lane == 63) blk[b] = incl;
    }
}

// In-place exclusive scan of block sums within each chunk; chunk sums out.
__global__ void __launch_bounds__(256) scan_blocks_kernel(uint64_t *blk, int64_t nblk, uint64_t *chunk)
{
    __shared__ uint64_t tsum[256];
    const int tid = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int64_t lo = c * kBlkPerChunk;
    const int64_t len = (nblk - lo) < kBlkPerChunk ? (nblk - lo) : kBlkPerChunk;
    const int per = kBlkPerChunk / 256;  // 32 entries per thread
    uint64_t loc = 0;
    for (int k = 0; k < per; ++k) {
        const int64_t i = (int64_t)tid * per + k;
        if (i < len) loc += blk[lo + i];
    }
    tsum[tid] = loc;
    __syncthreads();
    if (tid == 0) {
        uint64_t acc = 0;
        for (int t = 0; t < 256; ++t) {
            const uint64_t v = tsum[t];
            tsum[t] = acc;
            acc += v;
        }
        chunk[c] = acc;
    }
    __syncthreads();
    uint64_t acc = tsum[tid];
    for (int k = 0; k < per; ++k) {
        const int64_t i = (int64_t)tid * per + k;
        if (i < len) {
            const uint64_t v = blk[lo + i];
            blk[lo + i] = acc;
            acc += v;
        }
    }
}

// Exclusive scan of chunk sums; total T at chunk[nchunk].  Flags a zero total
// or a 64-bit wrap.
__global__ void scan_chunks_kernel(uint64_t *chunk, int64_t nchunk, int32_t *flag)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t acc = 0;
    for (int64_t c = 0; c < nchunk; ++c) {
        const uint64_t v = chunk[c];
        chunk[c] = acc;
        if (acc + v < acc) *flag = 2;
        acc += v;
    }
    chunk[nchunk] = acc;
    if (acc == 0) *flag = 1;
}

// Largest i in [0, len) with a[i] <= u (a nondecreasing, a[0] = 0 <= u).
__device__ __forceinline__ int64_t last_le(const uint64_t *a, int64_t len, uint64_t u)
{
    int64_t lo = 0, hi = len - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (a[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename V>
__global__ void __launch_bounds__(256) sample_shots_kernel(const V *psi, const uint64_t *sub, const uint64_t *blk,
                                                           const uint64_t *chunk, int64_t nchunk, int64_t nblk,
                                                           uint64_t seed, int64_t shots, uint64_t *out,
                                                           int32_t *flag, int sym_n)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= shots) return;
    const uint64_t T = chunk[nchunk];
    uint64_t r0, r1;
    philox_words01((uint64_t)s, seed, r0, r1);
    uint64_t u = __umul64hi(r0, T);
    const int64_t c = last_le(chunk, nchunk, u);
    u -= chunk[c];
    const int64_t b0 = c * kBlkPerChunk;
    const int64_t blen = (nblk - b0) < kBlkPerChunk ? (nblk - b0) : kBlkPerChunk;
    const int64_t b = b0 + last_le(blk + b0, blen, u);
    u -= blk[b];
    const int64_t j = last_le(sub + b * kSubPerBlock, kSubPerBlock, u);
    u -= sub[b * kSubPerBlock + j];
    const int64_t x0 = (b << kBlockBits) + (j << kSubBits);
    const int64_t fb = swz_fold(b) << kSwzDst;
    uint64_t acc = 0;
    int64_t x = x0 + 63;
    for (int t = 0; t < 64; ++t) {
        acc += qval_of(psi[(x0 + t) ^ fb], flag);
        if (acc > u) {
            x = x0 + t;
            break;
        }
    }
    uint64_t xo = (uint64_t)x;
    if (sym_n) {  // z -> y(z) (suffix XOR), or its complement over sym_n bits
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) xo ^= xo >> sh;
        if (r1 >> 63) xo ^= (~0ull) >> (64 - sym_n);
    }
    out[s] = xo;
}

// n < 13: the whole CDF in LDS, one workgroup.
template <typename V>
__global__ void __launch_bounds__(256) sample_small_kernel(const V *psi, int n, uint64_t seed, int64_t shots,
                                                           uint64_t *out, int32_t *flag)
{
    __shared__ uint64_t F[1 << (kBlockBits - 1)];
    __shared__ uint64_t tsum[256];
    const int tid = threadIdx.x, dim = 1 << n;
    const int per = (dim + 255) / 256;
    uint64_t loc = 0;
    for (int k = 0; k < per; ++k) {
        const int x = tid * per + k;
        if (x < dim) {
            loc += qval_of(psi[x], flag);
            F[x] = loc;
        }
    }
    tsum[tid] = loc;
    __syncthreads();
    if (tid == 0) {
        uint64_t acc = 0;
        for (int t = 0; t < 256; ++t) {
            const uint64_t v = tsum[t];
            tsum[t] = acc;
            acc += v;
        }
        if (acc == 0) *flag = 1;
    }
    __syncthreads();
    for (int k = 0; k < per; ++k) {
        const int x = tid * per + k;
        if (x < dim) F[x] += tsum[tid];
    }
    __syncthreads();
    const uint64_t T = F[dim - 1];
    for (int64_t s = tid; s < shots; s += 256) {
        const uint64_t u = __umul64hi(philox_word0((uint64_t)s, seed), T);
        int lo = 0, hi = dim - 1;  // first x with F[x] > u
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (F[mid] > u) hi = mid;
            else lo = mid + 1;
        }
        out[s] = (uint64_t)lo;
    }
}

}  // namespace

void sample_sizes(int n, int64_t *nsub, int64_t *nblk, int64_t *nchunk)
{
    if (n < kBlockBits) {
        *nsub = *nblk = 0;
        *nchunk = 0;
        return;
    }
    *nsub = (int64_t)1 << (n - kSubBits);
    *nblk = (int64_t)1 << (n - kBlockBits);
    *nchunk = n > kChunkBits ? (int64_t)1 << (n - kChunkBits) : 1;
}

hipError_t launch_sample(int prec, const void *psi, int n, const SampleBufs &b, uint64_t seed, int64_t shots,
                         uint64_t *out, hipStream_t st, int sym_n)
{
    if (n < kBlockBits) {
        if (prec == 0)
            hipLaunchKernelGGL(sample_small_kernel<float2>, dim3(1), dim3(256), 0, st, (const float2 *)psi, n, seed,
                               shots, out, b.flag);
        else
            hipLaunchKernelGGL(sample_small_kernel<double2>, dim3(1), dim3(256), 0, st, (const double2 *)psi, n,
                               seed, shots, out, b.flag);
        return hipGetLastError();
    }
    int64_t nsub, nblk, nchunk;
    sample_sizes(n, &nsub, &nblk, &nchunk);
    if (prec == 0)
        hipLaunchKernelGGL(sample_blocks_kernel<float2>, dim3((unsigned)nblk), dim3(256), 0, st,
                           (const float2 *)psi, b.sub, b.blk, b.flag);
    else
        hipLaunchKernelGGL(sample_blocks_kernel<double2>, dim3((unsigned)nblk), dim3(256), 0, st,
                           (const double2 *)psi, b.sub, b.blk, b.flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)nchunk), dim3(256), 0, st, b.blk, nblk, b.chunk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scan_chunks_kernel, dim3(1), dim3(64), 0, st, b.chunk, nchunk, b.flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (shots > 0) {
        const int64_t g = (shots + 255) / 256;
        if (prec == 0)
            hipLaunchKernelGGL(sample_shots_kernel<float2>, dim3((unsigned)g), dim3(256), 0, st, (const float2 *)psi,
                               (const uint64_t *)b.sub, (const uint64_t *)b.blk, (const uint64_t *)b.chunk, nchunk,
                               nblk, seed, shots, out, b.flag, sym_n);
        else
            hipLaunchKernelGGL(sample_shots_kernel<double2>, dim3((unsigned)g), dim3(256), 0, st,
                               (const double2 *)psi, (const uint64_t *)b.sub, (const uint64_t *)b.blk,
                               (const uint64_t *)b.chunk, nchunk, nblk, seed, shots, out, b.flag, sym_n);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace qs
