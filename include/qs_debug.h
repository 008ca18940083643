/*
 * qs_debug.h -- host-only diagnostics and test controls of libqs.  Nothing
 * here touches a GPU.
 */
#ifndef QS_DEBUG_H
#define QS_DEBUG_H

#include <stddef.h>

#include "qs.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Check, on the host, the pass plan that qs_forward / qs_adjoint_grad use for
 * an n-qubit state of precision prec and p layers:
 *   - the passes' target qubits partition 0..n-1;
 *   - every register window lies inside the tile and the windows of each
 *     butterfly stage cover the pass's targets;
 *   - each window layout is a bijection of the tile, and the fast and general
 *     register-to-memory index maps agree;
 *   - the tiles of each pass cover every amplitude index exactly once and stay
 *     below 2^n (exhaustive for n <= 24, sampled workgroups above);
 *   - the fused kernel sequence applies, for every layer k, the cost phase once
 *     after all of layer k-1's mixer and before any of layer k's, and every
 *     pass's mixer once per layer.
 * With prec | QS_SYM (16) the complement-symmetric plan is checked instead:
 * each of the n mixer factors in z coordinates (z_0; z_(j-1) z_j for
 * j = 1..n-2; z_(n-2)) is applied by exactly one pass, on adjacent bits, and
 * every window sequence covers them; tile maps are checked over the 2^(n-1)
 * stored indices.
 * Returns 0 when every check holds, else 1 with a description in msg
 * (msg may be NULL).  n outside 1..34 (15..35 or 14..34 with QS_SYM), or
 * prec not 0/1, returns 2.
 */
int qs_plan_check(int n, int prec, int p, char *msg, size_t msg_len);

/*
 * Check, on the host, the schedule qs_batch_forward_grad would run for these
 * circuits (structure from qs.h): every circuit's buffers lie inside one
 * allocation without overlap; work items are numbered contiguously in step
 * order; each step's predecessor is the previous step of the same circuit and
 * all its items carry lower numbers (which is what lets the persistent queue
 * drain); chunks cover each pass's tiles; table offsets, result slots and the
 * reduction's per-circuit step lists are in range; each circuit has
 * 2 (p (P - 1) + 1) - 1 steps.  Returns 0 if every check holds, 1 with a
 * message otherwise, 2 for invalid arguments.
 */
struct qs_circuit;
int qs_batch_plan_check(int count, const struct qs_circuit *circuits, int prec, char *msg, size_t msg_len);

/*
 * How the tile passes of a full-layout state s obtain the cut value C_t[x] of
 * eq. (6) in the calls that follow (qs_forward, qs_adjoint_grad,
 * qs_adjoint_grad_store): 0 = automatic (evaluated in registers from the
 * weights the diagonal encodes for n >= 28 qubits, read from the diagonal
 * below), 1 = evaluated in registers at any size, 2 = read from the diagonal
 * at any size.  The two ways give the same integers, so results are
 * bit-identical across modes; the mode changes only speed.  For tests and
 * measurements.  The complement-symmetric layout always reads its diagonal.
 * Errors: QS_ERR_ARG (mode outside 0..2, null state).
 */
qs_status qs_debug_set_cut_mode(qs_state s, int mode);

#ifdef __cplusplus
}
#endif

#endif /* QS_DEBUG_H */
