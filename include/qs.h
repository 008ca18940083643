/*
 * qs.h -- C ABI of libqs, a single-GPU (MI355X, gfx950) state-vector
 * simulator for linear-ramp QAOA (LR-QAOA) circuits on weighted complete
 * graphs (arXiv:2604.26423, Sec. II-B).
 *
 * The circuit: |+>^n (a Hadamard on every qubit), then p layers, each the
 * cost unitary of eq. (2) followed by the mixer of eq. (3).  The library
 * works in gate angles, which makes it independent of the sign and scale
 * convention used for (gamma_k, beta_k):
 *   layer k = [prod_{i<j} RZZ(theta_zz[k] * w_ij)] then [prod_q RX(theta_x[k])]
 *   RZZ(t) = exp(-i t/2 Z(x)Z),   RX(t) = exp(-i t/2 X).
 * The paper's unitaries exp(-i gamma H_C) and exp(+i beta sum_q X_q) are
 * theta_zz = 2 gamma, theta_x = -2 beta.
 *
 * Conventions shared by every call
 *   - Qubit q is bit q of the amplitude index.  An n-qubit state is a
 *     contiguous array of 2^n complex numbers (interleaved re, im; float for
 *     QS_C64, double for QS_C128) in which amplitude x sits at element
 *     qs_layout_index(x), an XOR swizzle of x that spreads the passes over
 *     the HBM channels (identity for x < 2^13).  Cost diagonals use the same
 *     layout.  qs_get_amplitudes / qs_set_amplitudes copy in index order.
 *   - Edge weights are integers in tenths (w_ij = w_t / 10), listed for
 *     pairs i<j in lexicographic order (0,1),(0,2),...,(0,n-1),(1,2),...
 *   - The cost diagonal is int32 C_t[x] = 10 * C(x), C(x) the cut value of
 *     eq. (6); W_t = sum of the weights in tenths.  H_C(x) = (W_t - 2 C_t[x])/10.
 *   - Every function returns a qs_status; QS_OK is 0.  On any other value
 *     qs_last_error() returns a message for the calling thread.  No C++
 *     exception, abort or exit crosses this interface.  Arguments are
 *     checked before any GPU work is queued.
 *   - Device pointers are HIP device pointers on the current device.  All
 *     GPU work of a state is queued on the HIP stream given to qs_alloc;
 *     functions that return host values synchronise that stream first.
 *   - A state handle is not thread-safe: calls on one handle must not
 *     overlap.  Different handles are independent.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QS_OK = 0,
    QS_ERR_ARG = 1,   /* invalid argument (null pointer, size, range of n, p, ...) */
    QS_ERR_OOM = 2,   /* device allocation failed */
    QS_ERR_HIP = 3,   /* any other HIP runtime error; message has the HIP string */
    QS_ERR_RANGE = 4, /* an integer result would not fit (e.g. W_t >= 2^31) */
    QS_ERR_STATE = 5  /* state content unusable (e.g. zero norm when sampling) */
} qs_status;

typedef enum { QS_C64 = 0, QS_C128 = 1 } qs_prec;

/* Largest supported qubit counts: 2^34 complex64 = 128 GiB, 2^33 complex128 = 128 GiB. */
#define QS_MAX_QUBITS_C64 34
#define QS_MAX_QUBITS_C128 33

/*
 * Complement-symmetric layout, OR'ed into the precision argument of
 * qs_state_bytes and qs_alloc (e.g. QS_C64 | QS_SYM).
 *
 * Every state the circuit produces from |+>^n satisfies psi(x) = psi(~x),
 * ~x the complement of all n bits, because the cut value of eq. (6), |+>^n
 * and the mixer of eq. (3) are all invariant under flipping every qubit.  The
 * layout stores only the 2^(n-1) amplitudes with bit n-1 clear, at index z:
 *   y = x mod 2^(n-1),  z_q = y_q XOR y_(q+1) (q < n-2),  z_(n-2) = y_(n-2);
 * conversely y_q = z_q XOR z_(q+1) XOR ... XOR z_(n-2), and psi(x) is the
 * stored value at z(y) for x = y and for x = ~y.  Memory and traffic are
 * halved, so one more qubit fits (n <= 35 complex64, 34 complex128); the
 * layout needs n >= 15 (complex64) or n >= 14 (complex128).
 * A symmetric state uses a diagonal from qs_cost_diagonal_sym (same z order).
 * Results refer to the full state: qs_expect and qs_forward report the full
 * norm, qs_cost_histogram the full masses, qs_sample full indices x (rule in
 * qs_sample).  qs_state_ptr returns the stored half.
 */
#define QS_SYM 16

typedef struct qs_state_s *qs_state;

/* Message for the calling thread's last failed call ("" if none). */
const char *qs_last_error(void);

/* Library version string. */
const char *qs_version(void);

/* Bytes of an n-qubit state: 2^n * 8 (QS_C64) or 2^n * 16 (QS_C128);
 * 0 if n or prec is out of range.  (Sec. II-E: FP32 needs 2^(N+3) bytes.) */
size_t qs_state_bytes(int n, int prec);

/*
 * Create a state handle for n qubits (1 <= n <= QS_MAX_QUBITS_*).
 * dev_buf: NULL -> the library allocates 2^n amplitudes and frees them in
 *          qs_free; otherwise a caller-owned device buffer of buf_bytes >=
 *          qs_state_bytes(n, prec), 256-byte aligned, that must outlive the
 *          handle.
 * hip_stream: hipStream_t for all work on this state (NULL = null stream).
 * The amplitudes are not initialised.  The handle also owns grow-only
 * device scratch for reductions and sampling, freed by qs_free.
 */
qs_status qs_alloc(int n, int prec, void *dev_buf, size_t buf_bytes, void *hip_stream,
                   qs_state *out);

/* Release the handle, its scratch and (if library-owned) its amplitudes. */
qs_status qs_free(qs_state s);

/* Device pointer of the amplitudes (2^n complex numbers, layout of qs_layout_index). */
qs_status qs_state_ptr(qs_state s, void **dev_ptr);

/*
 * Element of index x in the state and diagonal layout:
 *   qs_layout_index(x) = x XOR (f(x >> 13) << 4),
 * f(y) = (y XOR (y >> 9) XOR (y >> 18) XOR (y >> 27)) & 511, the 9-bit digits
 * of y folded by XOR.  Tiles of amplitudes 2^q apart for large q (the strided
 * mixer passes) otherwise put all their memory rows on the same HBM channels.
 * The map is its own inverse, keeps every aligned run of 16 entries and every
 * aligned block of 2^13 entries together, and is the identity below 2^13.
 * Returns -1 for x < 0.
 */
int64_t qs_layout_index(int64_t x);

/*
 * Copy amplitudes [first, first + count) of the state, in index order (z
 * order for QS_SYM states), to dst or from src: count complex numbers on the
 * device if on_device (8-byte aligned), else on the host (these calls then
 * synchronise the stream).
 * Errors: QS_ERR_ARG (range outside the stored amplitudes, null buffer).
 */
qs_status qs_get_amplitudes(qs_state s, int64_t first, int64_t count, void *dst, int on_device);
qs_status qs_set_amplitudes(qs_state s, int64_t first, int64_t count, const void *src, int on_device);

/* Change the stream used for later work on this state. */
qs_status qs_set_stream(qs_state s, void *hip_stream);

/* |+>^n: every amplitude 2^(-n/2) (Sec. II-B, initial state). */
qs_status qs_init_plus(qs_state s);

/*
 * Cost diagonal of eq. (6) on the device.
 * w_tenths: host array of n(n-1)/2 weights in tenths, each in [0, 2^20).
 * diag_dev: caller-owned device array of 2^n int32 (layout of
 *           qs_layout_index), written in full.
 * w_total_tenths (out, host, nullable): W_t.
 * cmax_tenths (out, host, nullable): max_x C_t[x] = 10 * C(x*) of eq. (5).
 * hip_stream: stream to use.  Synchronises it when cmax_tenths is non-null.
 * Errors: QS_ERR_ARG (n outside 1..34, null pointers, negative or too large
 * weight), QS_ERR_RANGE (W_t >= 2^31).
 */
qs_status qs_cost_diagonal(int n, const int32_t *w_tenths, int32_t *diag_dev,
                           int64_t *w_total_tenths, int32_t *cmax_tenths, void *hip_stream);

/*
 * Cost diagonal for the complement-symmetric layout: 2^(n-1) int32 in z order
 * (see QS_SYM), entry z = C_t[x] for x = y(z) with bit n-1 clear.  Same
 * arguments, outputs and errors as qs_cost_diagonal, for 14 <= n <= 35.
 */
qs_status qs_cost_diagonal_sym(int n, const int32_t *w_tenths, int32_t *diag_dev,
                               int64_t *w_total_tenths, int32_t *cmax_tenths, void *hip_stream);

/*
 * qs_cost_diagonal without any device allocation, for callers that cannot
 * allocate: code that runs under stream capture or in tight serving loops,
 * and harnesses that forbid hipMalloc.  Same arguments, outputs and errors as
 * qs_cost_diagonal, for 1 <= n <= 34 (larger n: QS_ERR_ARG).  Its scratch is
 * a static array in device memory (8.04 MiB; each device the library runs on
 * holds its own copy until the process ends), shared by every call on that
 * device: calls that overlapped on one device would race, so the library
 * lets one call at a time use it (calls from several host threads wait for
 * each other).  Synchronises hip_stream before it returns.
 */
qs_status qs_cost_diagonal_noalloc(int n, const int32_t *w_tenths, int32_t *diag_dev,
                                   int64_t *w_total_tenths, int32_t *cmax_tenths, void *hip_stream);

/*
 * One cost layer, eq. (2): prod_{i<j} RZZ(theta_zz * w_ij), applied as the
 * diagonal phase exp(-i theta_zz (W_t - 2 C_t[x]) / 20) on every amplitude.
 * The phase argument is reduced modulo 2 pi in FP64.
 */
qs_status qs_apply_cost_layer(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths,
                              double theta_zz);

/* One mixer layer, eq. (3): RX(theta_x) on every qubit. */
qs_status qs_apply_mixer(qs_state s, double theta_x);

/*
 * The whole circuit: |+>^n, then layers k = 0..p-1 with angles
 * theta_zz[k], theta_x[k] (host arrays of length p; p >= 0).  Same result
 * as qs_init_plus followed by p pairs of qs_apply_cost_layer and
 * qs_apply_mixer, computed with fewer passes over memory.
 * exp_c, norm (host, nullable): when exp_c is non-null the readout of
 * qs_expect is fused into the last pass and returned (synchronises).
 * diag_dev is the cost diagonal of the graph (qs_cost_diagonal).  In the full
 * layout, for states larger than one workgroup's tile, the passes evaluate
 * C_t[x] in registers from the weights the diagonal encodes (C_t at the
 * one- and two-hot indices: C(e_i) = deg_i, C(e_i + e_j) = deg_i + deg_j -
 * 2 w_ij) instead of reading it: the same integers, without the diagonal's
 * 4 bytes per amplitude.  The weights are checked against 1024 sampled
 * entries, diag[0] = 0, their degrees and w_total_tenths; a diagonal that
 * fails (not the cut function of nonnegative integer weights) is read entry
 * by entry.  The same holds for qs_adjoint_grad and qs_adjoint_grad_store.
 */
qs_status qs_forward(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, int p,
                     const double *theta_zz, const double *theta_x, double *exp_c, double *norm);

/*
 * <C> and the norm, FP64 reductions in a fixed order (run-to-run identical):
 *   norm = sum_x |a_x|^2,  exp_c = (sum_x |a_x|^2 C_t[x] / 10) / norm.
 * exp_c is the expected cut (eq. 5 with exact probabilities), in weight units.
 */
qs_status qs_expect(qs_state s, const int32_t *diag_dev, double *exp_c, double *norm);

/*
 * Measurement shots (Sec. II-B), reproducible bit for bit:
 *   P(x) = re^2 + im^2 in FP64 (single precision promoted first, no fused
 *   multiply-add), q(x) = floor(P(x) 2^62) as uint64, F(x) = sum_{y<=x} q(y),
 *   T = F(2^n - 1); shot s uses r = word 0 of Philox4x64-10 with counter
 *   (s, 0, 0, 0) and key (seed, 0), u = floor(r T / 2^64), and returns
 *   x_s = min { x : F(x) > u }.
 * out: shots uint64 values, on the device if out_on_device, else on the host.
 * Complement-symmetric states (QS_SYM) apply the rule to the stored half in
 * z order, which draws z, and return x = y(z) if bit 63 of word 1 of the same
 * Philox output is clear, else its complement ~y(z) over n bits.
 * Errors: QS_ERR_ARG (shots < 0, null out), QS_ERR_STATE (T = 0 or the
 * state norm is 4 or more, where q would overflow).
 */
qs_status qs_sample(qs_state s, uint64_t seed, int64_t shots, uint64_t *out, int out_on_device);

/*
 * Exact distribution of the cut value under the state: the noiseless
 * reference distribution that Sec. II-D subsamples (mean of n_s shots and its
 * 3-sigma threshold), without sampling noise.  In the fixed point of
 * qs_sample,
 *   mass[c] = sum over x with C_t[x] = c of q(x),  c = 0..nbins-1,
 * q(x) = floor((re^2 + im^2) 2^62); a value of C_t outside 0..nbins-1 counts
 * in bin nbins - 1, so nbins = W_t + 1 covers every cut.  Integer sums: the
 * result is identical run to run and equal to any exact evaluation of the
 * same rule.  The sum of mass is the sampler's T; mass / T is the probability.
 * mass: nbins uint64 values, on the device if out_on_device (8-byte aligned),
 * else on the host.  One pass over the state and the diagonal.
 * Errors: QS_ERR_ARG (nbins outside 1..2^24, null pointers, bad alignment),
 * QS_ERR_STATE (the state norm is 4 or more, where the sums would overflow).
 */
qs_status qs_cost_histogram(qs_state s, const int32_t *diag_dev, int32_t nbins, uint64_t *mass, int out_on_device);

/*
 * Forward circuit plus the adjoint (reverse state-vector) gradient of
 * E = <psi_p| C |psi_p> / <psi_p|psi_p> with C(x) = C_t[x] / 10:
 *   d_theta_zz[k] = dE/dtheta_zz[k],  d_theta_x[k] = dE/dtheta_x[k]
 * (host arrays of length p >= 1; exp_c receives E).  The reverse sweep
 * undoes every layer on the state and on the adjoint vector (no stored
 * checkpoints; qs_adjoint_grad_store below keeps them instead), so it needs
 * exactly two state vectors for any p.
 * lambda_buf: caller-owned device buffer of lambda_bytes >= qs_state_bytes
 * for the adjoint vector, or NULL to let the library allocate it for the call.
 * On return the state buffer holds an intermediate of the reverse sweep (its
 * contents are unspecified); qs_forward recomputes psi_p.  The adjoint buffer
 * is overwritten too.  Needs n >= 2.  Synchronises.
 */
qs_status qs_adjoint_grad(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, int p,
                          const double *theta_zz, const double *theta_x, void *lambda_buf,
                          size_t lambda_bytes, double *exp_c, double *d_theta_zz,
                          double *d_theta_x);

/*
 * The same gradient with stored checkpoints instead of uncomputing psi (the
 * "store" mode of the reverse sweep, for states small enough that the
 * checkpoints fit; the uncompute mode above needs only two state vectors).
 * The forward keeps the state after every tile pass but the last two in
 * ckpt_buf and the one after the second-to-last in the state buffer; each
 * reverse pass then reads psi from its checkpoint and stores lambda only, so
 * psi carries no error accumulated by undoing passes.  Same results as
 * qs_adjoint_grad up to rounding.
 * ckpt_buf: caller-owned device buffer of ckpt_bytes >= the size that
 * qs_adjoint_ckpt_bytes reports for p (256-byte aligned, not overlapping
 * the state or lambda_buf); it may be NULL when that size is 0 (one
 * workgroup holds the whole state, or the circuit has two tile passes).
 * The reverse passes do not write the state buffer: on return it holds the
 * output of the second-to-last forward pass.  Other arguments, errors and
 * synchronisation as qs_adjoint_grad.
 */
qs_status qs_adjoint_grad_store(qs_state s, const int32_t *diag_dev, int64_t w_total_tenths, int p,
                                const double *theta_zz, const double *theta_x, void *ckpt_buf,
                                size_t ckpt_bytes, void *lambda_buf, size_t lambda_bytes,
                                double *exp_c, double *d_theta_zz, double *d_theta_x);

/*
 * Checkpoint bytes qs_adjoint_grad_store needs for p layers on this state:
 * (P - 2) state sizes for a circuit of P tile passes (P = p (passes per
 * layer - 1) + 1), 0 when one workgroup holds the state.
 * Errors: QS_ERR_ARG (p < 1 or p > 2^20, null bytes).
 */
qs_status qs_adjoint_ckpt_bytes(qs_state s, int p, size_t *bytes);

/*
 * Per-kernel timing.  While enabled, HIP events bracket every kernel the
 * handle launches.  qs_profile_read synchronises and reports, for one kernel
 * kind, the launch count, the summed event time and the summed algorithmic
 * bytes (the bytes each launch must move at minimum).  Enabling clears.
 */
/*
 * Batched circuits (target workload: hundreds of small, uneven circuits).
 * Each circuit has its own instance, depth and angles; all of them run the
 * forward circuit and the adjoint gradient of qs_adjoint_grad in one
 * persistent kernel launch that hands out (circuit, pass, chunk of tiles)
 * work items from a global queue in rounds (pass r of every circuit, largest
 * circuits first); a work item waits for its circuit's previous pass through
 * completion counters.  Single-circuit tile kernels and the batched kernel
 * compute the same arithmetic.
 */
#define QS_BATCH_MAX_QUBITS 30

typedef struct qs_circuit {
    int n;                   /* qubits: more than 13 (complex64) / 12 (complex128), at most 30 */
    int p;                   /* layers, >= 1 */
    const int32_t *w_tenths; /* host, n(n-1)/2 weights in tenths (as qs_cost_diagonal) */
} qs_circuit;

typedef struct qs_batch_s *qs_batch;

/*
 * Allocate device memory for every circuit (state, adjoint vector, cost
 * diagonal; one allocation) and build the cost diagonals and C(x*).
 * The weight arrays are read during the call only.  Synchronises.
 */
qs_status qs_batch_create(int count, const qs_circuit *circuits, int prec, void *hip_stream, qs_batch *out);

/* W_t, C(x*) (tenths) and device pointers of circuit i (all outputs nullable). */
qs_status qs_batch_info(qs_batch b, int i, int64_t *w_total_tenths, int32_t *cmax_tenths, void **psi_dev,
                        int32_t **diag_dev);

/*
 * Forward circuit and adjoint gradient of every circuit (as qs_adjoint_grad).
 * theta_zz, theta_x, d_theta_zz, d_theta_x: host arrays with the circuits'
 * per-layer values concatenated in circuit order (sum of p entries);
 * exp_c: host array of count values.  Synchronises.
 * Errors: QS_ERR_ARG, QS_ERR_HIP (including a dependency wait that exceeded
 * its bound, which cannot happen while the queue drains normally).
 */
qs_status qs_batch_forward_grad(qs_batch b, const double *theta_zz, const double *theta_x, double *exp_c,
                                double *d_theta_zz, double *d_theta_x);

/* Release the batch and its device memory. */
qs_status qs_batch_free(qs_batch b);

/*
 * Noisy trajectories (arXiv:2604.26423, Sec. II-C): every RZZ gate is followed
 * by a two-qubit depolarizing channel of rate eps,
 *   rho -> (1 - eps) rho + eps Tr_ab(rho) (x) I_ab / 4,
 * unravelled into Pauli insertions.  Trajectory t draws, for layer k
 * (0-based) and edge e (lexicographic (0,1),(0,2),...):
 *   (r0, r1, r2, r3) = Philox4x64-10(counter (t, k, e, 1), key (seed, 0));
 *   the gate errs iff (r0 >> 11) < floor(eps * 2^53), with the Pauli
 *   code = r1 & 15: code & 3 on the edge's lower qubit, code >> 2 on the upper
 *   one (0 = I, 1 = X, 2 = Y, 3 = Z; Y = [[0, -i], [i, 0]]); it is applied right
 *   after that gate.
 * The average of a per-trajectory quantity over trajectories estimates its
 * value under the channel.  States of n = 2..QS_NOISE_MAX_QUBITS qubits; one
 * workgroup runs one trajectory.
 */
#define QS_NOISE_MAX_QUBITS 12
#define QS_NOISE_MAX_LAYERS 4096
typedef struct qs_noise_s *qs_noise;

/*
 * Graph of the trajectories: n qubits, w_tenths as in qs_cost_diagonal (host,
 * n(n-1)/2 values, copied), prec QS_C64 or QS_C128, all work on
 * hip_stream (NULL: the default stream).  Builds the cost diagonal on the
 * device.  Errors: QS_ERR_ARG (n outside 2..QS_NOISE_MAX_QUBITS, bad weights
 * or precision, null pointers), QS_ERR_OOM, QS_ERR_HIP.
 */
qs_status qs_noise_create(int n, int prec, const int32_t *w_tenths, void *hip_stream, qs_noise *out);

/* W_t and C(x*) in tenths (both nullable). */
qs_status qs_noise_info(qs_noise h, int64_t *w_total_tenths, int32_t *cmax_tenths);

/*
 * Run trajectories traj0 .. traj0 + ntraj - 1 (1 <= ntraj <= 2^31 - 1) of the
 * p-layer circuit (host angle arrays theta_zz[p], theta_x[p], as in
 * qs_forward; 1 <= p <= QS_NOISE_MAX_LAYERS) with error rate eps in [0, 1]
 * and the given seed.  Device outputs, caller-owned, indexed by
 * trajectory - traj0:
 *   exp_c   double[ntraj]: <C> / <psi|psi> of the final state, in units;
 *   norm    double[ntraj] or NULL: <psi|psi> (1 up to rounding);
 *   nerr    int32_t[ntraj] or NULL: the number of non-identity Paulis drawn;
 *   states  [ntraj][2^n] complex (float2 for QS_C64, double2 for QS_C128) or
 *           NULL: the final state vector of each trajectory, global phase
 *           included (bit q of the index is qubit q).
 * Asynchronous on the handle's stream: outputs are complete when the stream
 * is.  Calls on one handle must not overlap (the angle upload is reused).
 * Errors: QS_ERR_ARG, QS_ERR_HIP.
 */
qs_status qs_noise_run(qs_noise h, int p, const double *theta_zz, const double *theta_x, double eps,
                       uint64_t seed, int64_t traj0, int64_t ntraj, double *exp_c, double *norm, int32_t *nerr,
                       void *states);

/* Release the handle and its device memory (synchronises its stream). */
qs_status qs_noise_free(qs_noise h);

typedef enum {
    QS_KIND_PASS = 0,        /* forward tile passes without a cost phase */
    QS_KIND_PASS_PHASE = 1,  /* forward tile passes that also apply a cost phase (same kernel) */
    QS_KIND_ADJOINT = 2,     /* reverse-sweep passes (two vectors) */
    QS_KIND_EXPECT = 3,      /* stand-alone <C>/norm readout */
    QS_KIND_SAMPLE = 4,      /* sampling kernels */
    QS_KIND_ELEMENTWISE = 5, /* init and stand-alone cost-layer kernels */
    QS_KIND_REDUCE = 6,      /* small reductions of per-workgroup partials */
    QS_KIND_SMALL = 7,       /* single-workgroup kernels for states of <= 8192 amplitudes */
    QS_KIND_TURNAROUND = 8,  /* the pass where the forward sweep turns into the reverse sweep */
    QS_KIND_HISTOGRAM = 9,   /* cut-value histogram */
    QS_KIND_COUNT = 10
} qs_kernel_kind;

qs_status qs_profile(qs_state s, int enable);
qs_status qs_profile_read(qs_state s, int kind, int64_t *launches, double *total_ms,
                          double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
