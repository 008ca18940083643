// Internal declarations shared by the kernel translation units and the C ABI
// layer of libqs.  Not installed; the public interface is include/qs.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qs {

constexpr int kThreads = 256;         // threads per workgroup of the elementwise kernels
constexpr int kFwdThreadBits = 8;     // forward tile kernels: 256 threads
constexpr int kAdjThreadBits = 9;     // adjoint tile kernels: 512 threads (two vectors)
constexpr int kAdjOneThreadBits = 8;  // ... but the one-tile adjoint kernels: 256
constexpr int kTileBitsC64 = 13;      // 8192 amplitudes (64 KiB) per tile, complex64
constexpr int kTileBitsC128 = 12;     // 4096 amplitudes (64 KiB) per tile, complex128
constexpr int kMaxWindows = 8;        // register windows per butterfly stage
constexpr int kSmallMaxLayers = 32;   // layers per launch of the single-workgroup kernel
constexpr int kSlots = 4;             // FP64 partial sums per workgroup

inline int tile_bits(int prec) { return prec == 0 ? kTileBitsC64 : kTileBitsC128; }

// Butterfly stage: a sequence of register windows.  In window s a thread's
// register index r holds tile bits [s, s + RB); its thread index fills the
// remaining tile bits in order.  With 2^TB threads, s = TB is the "natural"
// layout (consecutive threads hold consecutive tile elements).
struct WinSeq {
    int cnt;
    int s[kMaxWindows];
};

// One tile pass over the state.  A tile is 2^T amplitudes: tile bits
// [0, c) are the "carrier" bits, equal to global bits [0, c) (contiguous
// runs in memory), and tile bits [c, T) are the target qubits
// [q0, q0 + T - c).  The workgroup index supplies the other global bits.
// RX(theta) on the targets of one butterfly stage.  With |cos(theta/2)| >= 1/2
// the stage applies the tangent form (a0 - i u a1, a1 - i u a0), u = tan(theta/2),
// which is RX(theta) / cos(theta/2): two fused multiply-adds per amplitude; the
// factor cos(theta/2)^m of the stage's m qubits is applied once per kernel.
// Otherwise it applies RX directly with c = cos(theta/2), s = sin(theta/2).
struct RxStage {
    double c, s, u;
    int tan;
    // Reverse stage: the gradient terms of window i (of the stage's window
    // sequence, walked from the last) are scaled by wsc[i] = cos(theta/2)^(2j),
    // j the factors undone before it (tangent form; 1 in the direct form).
    // Evaluated on the host: as uniform FP64 values they would take vector
    // registers for the whole pass.
    double wsc[kMaxWindows];
};

struct PassProg {
    void *psi;            // state (float2 / double2)
    void *lam;            // adjoint vector (reverse kernels only)
    void *psi_out;        // where the pass stores psi: psi (in place), another
                          // buffer (checkpointing forward), or null (reverse
                          // pass reading a checkpoint: psi is not stored)
    const int32_t *diag;  // cost diagonal in tenths
    void *tab;            // phase table of the pass's cost layer (kTabMax entries of float2 / double2),
                          // written by the launcher's table kernel just before the pass
    int32_t *ctab;        // cut table of the pass (layout kCt* below), written by the launcher just
                          // before the pass, from which the pass evaluates C_t in registers instead of
                          // loading the diagonal; null: the pass loads the diagonal
    const int32_t *wts;   // weights recovered from the diagonal (layout kWt* below), when ctab is set
    double *partials;     // kSlots doubles per workgroup
    int64_t ntiles;       // 2^(n - T); workgroups loop over tiles
    int tb;               // log2 threads of the kernel the window sequences are planned for
    int n, c, q0;
    uint32_t targets;     // mask of tile bits that are single-qubit gate targets
    uint32_t pairs;       // bit e: two-bit factor on tile bits e, e+1 (complement-symmetric storage)
    int ntargets;         // factors per stage: popcount(targets) + popcount(pairs)
    int width;            // strided tile bits T - c
    int xcd_remap;        // map consecutive tiles to one XCD
    int init;             // start from |+>^n instead of loading
    int has_pre, has_phase, has_post, readout;
    int load_win;         // layout of the first global access
    int phase_win;        // layout in which the phase is applied (end of stage A)
    int final_win;        // layout after stage B (store, readout)
    WinSeq A, B;          // windows of the pre and post butterfly stages
    RxStage pre, post;
    double fpre, fpost;   // tangent-form factors cos(theta/2)^m of the stages (1 if direct)
    double factor;        // fpre * fpost
    double theta_zz;      // phase angle of the fused cost layer
    int64_t W;            // W_t
    int phase_levels;     // digits of the phase table (see pass.hip)
    double amp0;          // 2^(-n/2)
    double lam_shift;     // adjoint: c (tenths) in lambda = (C - c) psi / 10 at the turnaround and in
                          // the weights (C - c) of the phase gradients; any c gives the same
                          // gradients, c = W_t / 2 keeps the terms small (see tiles.h)
};

// ---- cut values in registers ----
//
// C_t(x) = sum_{i<j} w_ij [x_i != x_j] is a cut function, so for disjoint bit
// sets A, B: C(A | B) = C(A) + C(B) - 2 w(A, B), w(A, B) = sum_{i in A, j in B}
// w_ij.  At the point of a pass where it needs C_t, a register r of thread t
// holds the amplitude x = A | B_t | D_r: A the tile's bits outside the tile
// (from the workgroup index), B_t the thread's tile bits, D_r the register
// bits of r.  With Db_i = sum_{j in A} w_ij and Dt_k = sum_{i in B_t} w_ik,
//   C(x) = C(A) + C(B_t) + C(D_r) - 2 sum_{i in B_t} Db_i
//          - 2 sum_{k in D_r} (Db_k + Dt_k).
// The cut table of a pass holds C(D_r) for every r (uniform), C(B_t) and Dt_k
// for every thread, and C(A) and Db_i for every tile (one 64-byte row, a
// scalar load); the sums above are exact in uint32 (C_t < 2^31).
//
// The weights are recovered from the diagonal itself: C(e_i) = deg_i and
// C(e_i | e_j) = deg_i + deg_j - 2 w_ij.  A sample of the diagonal is checked
// against them; if the diagonal is not the cut function of nonnegative
// integer weights summing to W_t, the table says so and the passes load the
// diagonal instead.
constexpr int kWtStride = 64;                     // row stride of the weight matrix
constexpr int kWtDeg = kWtStride * kWtStride;     // deg_i, i < 64
constexpr int kWtOk = kWtDeg + kWtStride;         // 1: weights reproduce the diagonal
constexpr int kWtSize = kWtOk + 1;
constexpr int kCtCreg = 0;                        // C(D_r), r < 2^RB (RB <= 5)
constexpr int kCtValid = 32;                      // copy of the weights' ok flag
constexpr int kCtThr = 64;                        // per thread: C(B_t), Dt_0 .. Dt_{RB-1}, 8 entries
constexpr int kCtTile = kCtThr + 8 * 512;         // per tile: C(A), Db_0 .. Db_{T-1}, 16 entries
constexpr int kCtSamples = 1024;                  // diagonal entries checked against the weights
// Smallest state (qubits, full layout) whose passes evaluate C_t in registers
// by default: the weights and tables cost ~0.1 ms per call, which the saved
// diagonal reads repay from n = 28 on (complex64 forward, p = 3: 1.8x slower
// at n = 16..22, even at n = 27, 3% faster at n = 28..30).
constexpr int kCutMinQubits = 28;

// ---- index maps of a tile pass (host and device) ----

// Tile element held by (register r, thread tid) in the layout of window s.
__host__ __device__ __forceinline__ int win_elem(int r, int tid, int s, int rb)
{
    return (tid & ((1 << s) - 1)) | (r << s) | ((tid >> s) << (s + rb));
}

// Global amplitude index of tile element e.
__host__ __device__ __forceinline__ int64_t tile_gidx(int e, int64_t base, int c, int q0)
{
    return base | (int64_t)(e & ((1 << c) - 1)) | ((int64_t)(e >> c) << q0);
}

// Workgroup index -> global bits outside the tile.  Bits [c, q0) come from the
// low part of w, bits [q0 + m, n) from the high part (m = T - c).
__host__ __device__ __forceinline__ int64_t tile_base(int64_t w, int c, int q0, int m)
{
    const int nlow = q0 - c;
    const int64_t wl = w & (((int64_t)1 << nlow) - 1);
    const int64_t wh = w >> nlow;
    return (wl << c) | (wh << (q0 + m));
}

// Memory layout of states, adjoint vectors and cost diagonals: entry x is
// stored at element swz(x) = x ^ (f(x >> 13) << 4), f the XOR of the 9-bit
// digits of x >> 13.  Tiles whose amplitudes are 2^q0 apart for large q0 would
// otherwise send all their rows to the same HBM channels; folding the high
// index bits into bits 4..12 spreads them while keeping 16-entry runs (128 B
// of complex64) and every aligned 2^13 block intact.  swz is linear over XOR
// and its own inverse; it is the identity below 2^13 entries.
constexpr int kSwzSrc = 13, kSwzDst = 4, kSwzWidth = 9;

__host__ __device__ __forceinline__ int64_t swz_fold(int64_t y)
{
    y ^= y >> kSwzWidth;
    y ^= y >> (2 * kSwzWidth);
    return y & ((1 << kSwzWidth) - 1);
}

__host__ __device__ __forceinline__ int64_t swz(int64_t x)
{
    return x ^ (swz_fold(x >> kSwzSrc) << kSwzDst);
}

// LDS slot of tile element e: an XOR of bits [RB, RB + 5) into the low five
// bits.  Every window layout of a 256- or 512-thread kernel then puts the 32
// lanes of each half-wave on distinct banks (checked for 32 and 64 banks of
// 4 bytes).  The map is linear over GF(2), so the slot of (thread part |
// register part) is the XOR of the two slots: a per-thread constant and a
// per-register uniform value; and it is a bijection (bits >= 5 are kept, and
// bit 4 for RB = 4 depends only on bit 8).
template <int RB>
__host__ __device__ __forceinline__ int lds_slot(int e)
{
    return e ^ ((e >> RB) & 31);
}

// Global index of (register r, thread) in window s.  Every window starts at
// or above the carrier bits (s >= c, guaranteed by the pass plan), so its
// register bits are contiguous global bits and the index is the thread's
// r = 0 element plus r << sh; the two parts occupy disjoint bits, so the
// memory element is swz(tg) ^ swz(r << sh), a per-thread and a uniform part.
struct Addr {
    int64_t tg;
    int sh;
    bool fast;  // s >= c (checked by the host plan checker)
    __host__ __device__ __forceinline__ int64_t fast_idx(int r) const { return tg + ((int64_t)r << sh); }
    __host__ __device__ __forceinline__ int64_t mem_idx(int64_t tgs, int r) const { return tgs ^ swz((int64_t)r << sh); }
};

__host__ __device__ __forceinline__ Addr win_addr(int tid, int s, int rb, int64_t base, int c, int q0)
{
    return Addr{tile_gidx(win_elem(0, tid, s, rb), base, c, q0), q0 + s - c, s >= c};
}

// Host-side launchers (one per kernel family); all return hipError_t.
hipError_t launch_pass(int prec, const PassProg &pp, int64_t grid, hipStream_t st);
// Whether launch_adjoint_pass runs pp (turnaround: 1), with its windows
// planned for pp.tb threads, on a one-tile kernel rather than the persistent
// 512-thread one.
bool adjoint_one_tile(int prec, const PassProg &pp, int turnaround);
// Bytes of the device buffer PassProg::tab points to (any precision).
size_t pass_table_bytes();
// Recover the weights of the cut function in diag (2^n entries, full layout)
// into wts (kWtSize int32) and check them against the diagonal.
hipError_t launch_cut_weights(const int32_t *diag, int n, int64_t W, int32_t *wts, hipStream_t st);
// int32 entries of a cut table (PassProg::ctab) for 2^n amplitudes.
int64_t cut_table_entries(int n, int prec);
// Whether the kernel picked for pp (kind 0 = forward pass, 1 = turnaround,
// 2 = reverse pass) takes C_t from a cut table; pp.ctab must be null otherwise.
bool pass_takes_cut_table(int prec, const PassProg &pp, int kind);
int phase_table_levels(int64_t W);
hipError_t launch_adjoint_pass(int prec, const PassProg &pp, int turnaround, int64_t grid,
                               hipStream_t st);
// Stage code path of a pass for a kernel with 2^tb threads: 0 = general,
// 1 = branch-free tangent form, 2 = the same for the complement-symmetric layout.
int tile_mode(const PassProg &pp, int T, int tb);
// Grid of a tile kernel (kind 0 = forward, 1 = turnaround, 2 = reverse pass):
// the largest one of that kind, and the one launched for a given pass.
int64_t pass_grid(int prec, int adjoint, int64_t ntiles);
int64_t tile_grid(int prec, int adjoint, const PassProg &pp);

// ---- batched circuits: one persistent launch over a ticket queue ----
constexpr int kBatchThreadBits = 9;   // batched tile kernels: 512 threads

// One pass of one circuit.  Its tiles are split into `chunks` work items; the
// items of all steps are numbered in rounds (step r of every circuit that has
// one), largest circuits first, and workgroups claim them in that order.
struct BatchStep {
    PassProg pp;
    int kind;             // 0 = forward pass, 1 = turnaround, 2 = reverse pass
    int mode;             // stage code path (tile_mode)
    int circuit;
    int prev;             // previous step of the same circuit, -1 if none
    int chunks;           // work items of this step
    int tiles_per_chunk;
    int map[kSlots];      // accumulator index of each partial-sum slot (-1: unused)
    int64_t item0;        // first item number of this step
    int64_t tab_off;      // offset of this step's phase table (entries), -1 if none
};

struct BatchArgs {
    const BatchStep *steps;
    int nsteps;
    int64_t nitems;
    unsigned long long *ticket;  // next item to claim
    unsigned *done;              // finished items per step
    int *abort_flag;             // set when a dependency wait exceeds spin_limit
    double *partials;            // kSlots doubles per item
    void *tabs;                  // phase tables (float2 / double2)
    int64_t spin_limit;
};

hipError_t launch_batch_tables(int prec, const BatchStep *steps, int nsteps, void *tabs, hipStream_t st);
hipError_t launch_batch(int prec, const BatchArgs &a, int64_t grid, hipStream_t st);
int64_t batch_grid(int prec);
// Fixed-order per-circuit reduction: for circuit c, res[res_off[c] + map[k]] +=
// sum over its steps' items of slot k (steps listed in cstep[cstep_off[c]..]).
hipError_t launch_batch_reduce(const BatchStep *steps, const int *cstep, const int *cstep_off,
                               const int64_t *res_off, const double *partials, double *res, int ncircuits,
                               hipStream_t st);
int batch_table_entries();

// Single-workgroup kernels for n <= T: a chunk of up to kSmallMaxLayers layers.
struct SmallProg {
    void *psi;
    void *lam;
    const int32_t *diag;
    double *out;          // readout / gradient accumulators (device)
    int n;
    int init, readout;
    int nlayers;
    int64_t W;
    double tzz[kSmallMaxLayers];
    double tx[kSmallMaxLayers];
    int do_phase[kSmallMaxLayers];
    int do_mixer[kSmallMaxLayers];
    int layer0;           // index of the first layer of the chunk (gradient slots)
    int ptotal;           // total layers of the circuit (gradient slot layout)
    int turnaround;       // adjoint: build lambda = (C - lam_shift) psi / 10 from the loaded psi first
    int store;            // adjoint: write psi and lambda back
    double amp0;          // 2^(-n/2)
    double lam_shift;     // adjoint: shift of the cost in lambda and in the phase-gradient weights (tenths)
};
hipError_t launch_small_forward(int prec, const SmallProg &sp, hipStream_t st);
hipError_t launch_small_adjoint(int prec, const SmallProg &sp, hipStream_t st);

// ---- noisy trajectories (noise.hip): one workgroup per trajectory ----
constexpr int kNoiseMaxQubits = 12;
constexpr int kNoiseChunk = 32;  // layers whose error draws are made together

struct NoiseProg {
    const int32_t *diag;     // 2^n cut values (tenths)
    const int32_t *edges;    // per edge: a | b << 4 | w << 8 (a < b, w in tenths)
    const double *layers;    // per layer: theta_zz, u or cos, 0 or sin, mixer factor
    void *tabs;              // per layer: kTabMax phase-table entries (float2 / double2)
    double *exp_c;           // [ntraj] normalized <C> in units
    double *norm;            // [ntraj] or null
    int32_t *nerr;           // [ntraj] non-identity errors, or null
    void *states;            // [ntraj][2^n] final states, or null
    uint64_t traj0, seed, thr;
    int64_t W;
    int n, p, levels;
    double amp0;
};

int noise_threads(int n);
int noise_table_entries();  // phase-table entries per layer
hipError_t launch_noise(int prec, int tangent, const NoiseProg &np, int64_t ntraj, hipStream_t st);

// Elementwise and readout kernels.
// |+>: 2^n stored amplitudes, each 2^(-nq/2) (nq = n, or n + 1 in the
// complement-symmetric layout).
hipError_t launch_init_plus(int prec, void *psi, int n, int nq, hipStream_t st);
// Amplitudes [first, first + count) between index order in buf and the state
// (to_state = 1 writes the state).
hipError_t launch_copy_amplitudes(int prec, void *psi, int64_t first, int64_t count, void *buf, int to_state,
                                  hipStream_t st);
hipError_t launch_cost_layer(int prec, void *psi, const int32_t *diag, int n, int64_t W,
                             double theta, hipStream_t st);
hipError_t launch_expect(int prec, const void *psi, const int32_t *diag, int n,
                         double *partials, int64_t *nblocks, hipStream_t st);
// Fixed-order reduction of kSlots-wide partials into dst[map[k]] (+= if accumulate).
hipError_t launch_reduce(const double *partials, int64_t count, double *tmp, double *dst,
                         const int *map, int accumulate, hipStream_t st);
int64_t reduce_tmp_doubles(int64_t count);

// Cost diagonal.
// sym = 1: the 2^(n-1) entries of the complement-symmetric layout (plan.h)
// in z order; n is the qubit count of the graph.
hipError_t launch_cost_diagonal(int n, const int32_t *wmat_dev, int32_t *diag, int32_t *low_table,
                                int32_t *wg_max, int32_t *tmp_max, int32_t *cmax_dev,
                                hipStream_t st, int sym = 0);
int64_t diag_wg_count(int n, int sym = 0);

// Vertices 0..12 (the low index bits) form the diagonal builder's shared
// table; each workgroup of its main kernel owns one value of the other bits.
constexpr int kDiagLowBits = 13;

// Scratch for building diagonals of up to nmax qubits with nwg workgroups of
// the main kernel: the weight matrix (nmax x nmax int32), the low-bit table
// (2^13 int32), per-workgroup maxima, their partial maxima and `nres` int32
// results, each at a 256-byte aligned offset.
struct DiagScratch {
    size_t off_low, off_wg, off_tmp, off_res, total;
};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr DiagScratch diag_scratch_plan(int nmax, int nres, int64_t nwg)
{
    DiagScratch L{};
    L.off_low = align256((size_t)nmax * nmax * 4);
    L.off_wg = L.off_low + 8192 * 4;
    L.off_tmp = L.off_wg + align256((size_t)nwg * 4);
    L.off_res = L.off_tmp + align256((size_t)(nwg / 4096 + 2) * 4);
    L.total = L.off_res + align256((size_t)nres * 4);
    return L;
}

// Sampling.
struct SampleBufs {
    uint64_t *sub;     // in-block exclusive prefix of 64-amplitude sub-block sums
    uint64_t *blk;     // in-chunk exclusive prefix of block sums
    uint64_t *chunk;   // global exclusive prefix of chunk sums, then the total at [nchunks]
    int32_t *flag;     // overflow / zero-total flag
};
void sample_sizes(int n, int64_t *nsub, int64_t *nblk, int64_t *nchunk);
// sym_n > 0: psi is the complement-symmetric layout of sym_n qubits (n =
// sym_n - 1 stored bits); each drawn z is returned as the full index y(z) or
// its complement, chosen by bit 63 of word 1 of the same Philox output.
hipError_t launch_sample(int prec, const void *psi, int n, const SampleBufs &b, uint64_t seed,
                         int64_t shots, uint64_t *out, hipStream_t st, int sym_n = 0);

// Cut-value histogram.
constexpr int64_t kHistLdsBytes = 64 << 10;   // private LDS histograms up to 8192 bins
constexpr int kHistMaxBins = 1 << 24;
struct HistGeom {
    int64_t groups;   // workgroups
    int64_t per;      // amplitudes per workgroup (a power of two)
    int64_t rows;     // scratch rows of nbins uint64 (groups, or 1 for the global-atomic form)
    bool lds;         // private histograms in LDS
};
HistGeom hist_geom(int prec, int n, int nbins);
// shift: the per-bin sums are multiplied by 2^shift (1 for the complement-symmetric layout,
// where each stored amplitude stands for two basis states).
hipError_t launch_histogram(int prec, const void *psi, const int32_t *diag, int nbins, const HistGeom &g,
                            uint64_t *rows, double *fsum, int32_t *flag, uint64_t *out, hipStream_t st,
                            int shift = 0);

}  // namespace qs
