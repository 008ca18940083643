/*
 * Reference ("oracle") implementation of noiseless LR-QAOA state-vector
 * simulation on a weighted complete graph, in plain C with complex128
 * arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two only see the same
 * seeded inputs.
 *
 * What it follows (arXiv:2604.26423):
 *   - Sec. II-B, eq. (1):  H_C = sum_{i<j} w_ij Z_i Z_j on the complete graph.
 *   - Sec. II-B, eq. (2):  cost unitary  U_C = exp(-j gamma_k H_C).
 *   - Sec. II-B, eq. (3):  mixer unitary U_B = exp(+j beta_k H_B),
 *                          H_B = sum_i X_i; start state |+>^N.
 *   - Sec. II-B, eq. (6):  cut value C(x) = sum_{k<l} w_kl (x_k + x_l - 2 x_k x_l).
 *   - Sec. II-B, eq. (5):  approximation ratio uses C(x*) = max_x C(x).
 *   - Sec. II-E:           each gate updates disjoint pairs (one-qubit gate)
 *                          or quadruples (two-qubit gate) of amplitudes.
 *   - Sec. II-C:           noise as a two-qubit depolarizing channel of uniform
 *                          rate eps after every two-qubit gate, sampled here as
 *                          Pauli insertions (quantum trajectories).
 *
 * Angles are passed as gate angles: layer k applies RZZ(theta_zz[k] * w_ij)
 * on every pair (i<j) and then RX(theta_x[k]) on every qubit, with
 *   RZZ(t) = exp(-i t/2 Z(x)Z),  RX(t) = exp(-i t/2 X).
 * The mapping from the paper's (gamma_k, beta_k) lives in the Python side
 * of the oracle.  Weights are integers in tenths: w_ij = w_t[e] / 10.
 * Edge e enumerates pairs (i<j) lexicographically: (0,1),(0,2),...,(n-2,n-1).
 * Qubit q is bit q of the amplitude index.
 *
 * Build with -ffp-contract=off so that |a|^2 = re*re + im*im is evaluated
 * without fused multiply-adds (the sampling rule depends on it).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Index of edge (i<j) in lexicographic order. */
static int64_t edge_id(int n, int i, int j)
{
    return (int64_t)i * n - (int64_t)i * (i + 1) / 2 + (j - i - 1);
}

static int64_t n_edges(int n) { return (int64_t)n * (n - 1) / 2; }

/* ------------------------------------------------------------------ */
/* Cut function, eq. (6): C(x) = sum_{k<l} w_kl (x_k + x_l - 2 x_k x_l).  */
/* Returned in tenths (integer, exact).                                   */
/* ------------------------------------------------------------------ */
static int64_t cut_value(int n, const int32_t *w, uint64_t x)
{
    int64_t c = 0;
    for (int k = 0; k < n; k++) {
        int64_t xk = (int64_t)((x >> k) & 1u);
        for (int l = k + 1; l < n; l++) {
            int64_t xl = (int64_t)((x >> l) & 1u);
            c += (int64_t)w[edge_id(n, k, l)] * (xk + xl - 2 * xk * xl);
        }
    }
    return c;
}

/* Full cost diagonal C_t[x] for all 2^n basis states, by the double loop. */
int oracle_cost_diagonal(int n, const int32_t *w, int32_t *diag)
{
    if (n < 1 || n > 40 || !w || !diag) return 1;
    const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < dim; x++) diag[x] = (int32_t)cut_value(n, w, (uint64_t)x);
    return 0;
}

/* Cut value of a single basis state (for sampled checks at large n). */
int64_t oracle_cut_value(int n, const int32_t *w, uint64_t x) { return cut_value(n, w, x); }

/* Cut values of a list of basis states. */
int oracle_cut_values(int n, const int32_t *w, const uint64_t *xs, int64_t count, int64_t *out)
{
    if (n < 1 || n > 64 || !w || (count > 0 && (!xs || !out))) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; i++) out[i] = cut_value(n, w, xs[i]);
    return 0;
}

/* Sum of the weights in tenths (W_t). */
int64_t oracle_weight_total(int n, const int32_t *w)
{
    int64_t s = 0;
    for (int64_t e = 0; e < n_edges(n); e++) s += w[e];
    return s;
}

/* C(x*) by exhaustive evaluation of eq. (6) over all 2^n states. */
int64_t oracle_cmax_direct(int n, const int32_t *w)
{
    const int64_t dim = (int64_t)1 << n;
    int64_t best = 0;
#pragma omp parallel for reduction(max : best) schedule(static)
    for (int64_t x = 0; x < dim; x++) {
        int64_t c = cut_value(n, w, (uint64_t)x);
        if (c > best) best = c;
    }
    return best;
}

/*
 * C(x*) by a Gray-code walk.  A cut does not change when every bit is
 * complemented, so vertex n-1 is held at 0 and the other n-1 vertices run
 * through all 2^(n-1) assignments, one vertex flip per step.  With spins
 * s = 1 - 2x the cut is sum_{i<j} w_ij (1 - s_i s_j)/2; flipping vertex i
 * changes it by s_i * f_i with the local field f_i = sum_{j != i} w_ij s_j.
 */
int64_t oracle_cmax_gray(int n, const int32_t *w)
{
    if (n < 2) return 0;
    const int m = n - 1;                      /* free vertices 0..n-2 */
    const int64_t steps = (int64_t)1 << m;
    int64_t *wm = (int64_t *)calloc((size_t)n * n, sizeof(int64_t));
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) wm[i * n + j] = wm[j * n + i] = w[edge_id(n, i, j)];
    int64_t best = 0;
#pragma omp parallel reduction(max : best)
    {
        int nt = omp_get_num_threads(), t = omp_get_thread_num();
        int64_t lo = steps * t / nt, hi = steps * (t + 1) / nt;
        int64_t s[64], f[64];
        if (lo < hi) {
            uint64_t g = (uint64_t)lo ^ ((uint64_t)lo >> 1);
            for (int i = 0; i < n; i++) s[i] = ((g >> i) & 1u) ? -1 : 1; /* vertex n-1: bit 0 */
            int64_t c = 0;
            for (int i = 0; i < n; i++) {
                f[i] = 0;
                for (int j = 0; j < n; j++)
                    if (j != i) f[i] += wm[i * n + j] * s[j];
                for (int j = i + 1; j < n; j++) c += wm[i * n + j] * (1 - s[i] * s[j]) / 2;
            }
            if (c > best) best = c;
            for (int64_t k = lo + 1; k < hi; k++) {
                int i = __builtin_ctzll((uint64_t)k);
                c += s[i] * f[i];
                int64_t twice = 2 * s[i];
                s[i] = -s[i];
                for (int j = 0; j < n; j++)
                    if (j != i) f[j] -= twice * wm[i * n + j];
                if (c > best) best = c;
            }
        }
    }
    free(wm);
    return best;
}

/* ------------------------------------------------------------------ */
/* Gate-by-gate state-vector updates (Sec. II-E).                       */
/* ------------------------------------------------------------------ */

/* One-qubit gate [[m00, m01], [m10, m11]] on qubit q: disjoint pairs. */
static void apply_1q(int n, cplx *psi, int q, cplx m00, cplx m01, cplx m10, cplx m11)
{
    const int64_t half = (int64_t)1 << (n - 1);
    const uint64_t bit = (uint64_t)1 << q, low = bit - 1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < half; k++) {
        uint64_t x0 = (((uint64_t)k & ~low) << 1) | ((uint64_t)k & low);
        uint64_t x1 = x0 | bit;
        cplx a0 = psi[x0], a1 = psi[x1];
        psi[x0] = m00 * a0 + m01 * a1;
        psi[x1] = m10 * a0 + m11 * a1;
    }
}

/* Insert a zero bit at position b into k. */
static uint64_t insert_zero(uint64_t k, int b)
{
    uint64_t low = ((uint64_t)1 << b) - 1;
    return ((k & ~low) << 1) | (k & low);
}

/*
 * Two-qubit gate RZZ(t) = exp(-i t/2 Z_i Z_j) on qubits i<j: its 4x4 matrix
 * is diagonal, diag(e^{-it/2}, e^{+it/2}, e^{+it/2}, e^{-it/2}) over
 * |x_j x_i> = 00, 01, 10, 11; applied to disjoint quadruples.
 */
static void apply_rzz(int n, cplx *psi, int i, int j, double t)
{
    const int64_t quarter = (int64_t)1 << (n - 2);
    const uint64_t bi = (uint64_t)1 << i, bj = (uint64_t)1 << j;
    const cplx same = cexp(-I * (t / 2.0)), diff = cexp(I * (t / 2.0));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < quarter; k++) {
        uint64_t x = insert_zero(insert_zero((uint64_t)k, i), j);
        psi[x] *= same;
        psi[x | bi] *= diff;
        psi[x | bj] *= diff;
        psi[x | bi | bj] *= same;
    }
}

/* RX(t) = exp(-i t/2 X) = [[cos t/2, -i sin t/2], [-i sin t/2, cos t/2]]. */
static void apply_rx(int n, cplx *psi, int q, double t)
{
    cplx c = cos(t / 2.0), ms = -I * sin(t / 2.0);
    apply_1q(n, psi, q, c, ms, ms, c);
}

/* H_C(x) of eq. (1) in units: sum_{i<j} (w_ij/10) z_i z_j with z = 1 - 2 x. */
static double hamiltonian_value(int n, const int32_t *w, uint64_t x)
{
    double h = 0.0;
    for (int i = 0; i < n; i++) {
        double zi = ((x >> i) & 1u) ? -1.0 : 1.0;
        for (int j = i + 1; j < n; j++) {
            double zj = ((x >> j) & 1u) ? -1.0 : 1.0;
            h += ((double)w[edge_id(n, i, j)] / 10.0) * zi * zj;
        }
    }
    return h;
}

/* Layer k's cost unitary: the product of RZZ(theta * w_ij) over all pairs. */
static void apply_cost(int n, const int32_t *w, cplx *psi, double theta, int mode)
{
    if (mode == 0) {
        /* gate by gate, pairs in lexicographic order (Sec. II-E) */
        for (int i = 0; i < n; i++)
            for (int j = i + 1; j < n; j++)
                apply_rzz(n, psi, i, j, theta * ((double)w[edge_id(n, i, j)] / 10.0));
    } else {
        /* eq. (2) directly: H_C is diagonal, so the product of the commuting
         * RZZ gates is exp(-i theta/2 H_C(x)) on each basis state */
        const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < dim; x++)
            psi[x] *= cexp(-I * (theta / 2.0) * hamiltonian_value(n, w, (uint64_t)x));
    }
}

static void apply_mixer(int n, cplx *psi, double theta)
{
    for (int q = 0; q < n; q++) apply_rx(n, psi, q, theta);
}

/* |0...0> followed by a Hadamard on every qubit. */
static void prepare_plus(int n, cplx *psi)
{
    const int64_t dim = (int64_t)1 << n;
    memset(psi, 0, (size_t)dim * sizeof(cplx));
    psi[0] = 1.0;
    const double r = 1.0 / sqrt(2.0);
    for (int q = 0; q < n; q++) apply_1q(n, psi, q, r, r, r, -r);
}

static void run_circuit(int n, const int32_t *w, int p, const double *tzz, const double *tx,
                        int mode, cplx *psi)
{
    prepare_plus(n, psi);
    for (int k = 0; k < p; k++) {
        apply_cost(n, w, psi, tzz[k], mode);
        apply_mixer(n, psi, tx[k]);
    }
}

/*
 * Final state of the LR-QAOA circuit.  psi_out holds 2^n complex numbers,
 * interleaved (re, im).  mode 0 = RZZ gates one by one on quadruples;
 * mode 1 = each layer's cost unitary as the diagonal exp(-i theta/2 H_C).
 */
int oracle_simulate(int n, const int32_t *w, int p, const double *tzz, const double *tx, int mode,
                    double *psi_out)
{
    if (n < 1 || n > 34 || p < 0 || !w || !psi_out) return 1;
    run_circuit(n, w, p, tzz, tx, mode, (cplx *)psi_out);
    return 0;
}

/* Pairwise (recursive halving) sum: a fixed, order-defined FP64 reduction. */
static double pairwise_sum(const double *v, int64_t len)
{
    if (len <= 64) {
        double s = 0.0;
        for (int64_t i = 0; i < len; i++) s += v[i];
        return s;
    }
    int64_t h = len / 2;
    return pairwise_sum(v, h) + pairwise_sum(v + h, len - h);
}

/*
 * <C> (eq. 5 with exact probabilities) and the norm:
 *   norm = sum |a_x|^2,  exp_c = (sum |a_x|^2 C_t[x] / 10) / norm.
 */
int oracle_expect(int n, const double *psi, const int32_t *diag, double *exp_c, double *norm)
{
    const int64_t dim = (int64_t)1 << n;
    double *pr = (double *)malloc((size_t)dim * sizeof(double));
    double *pc = (double *)malloc((size_t)dim * sizeof(double));
    if (!pr || !pc) { free(pr); free(pc); return 2; }
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < dim; x++) {
        double re = psi[2 * x], im = psi[2 * x + 1];
        pr[x] = re * re + im * im;
        pc[x] = pr[x] * (double)diag[x];
    }
    double s = pairwise_sum(pr, dim), sc = pairwise_sum(pc, dim);
    free(pr);
    free(pc);
    *norm = s;
    *exp_c = (sc / 10.0) / s;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of a    */
/* multiply-xorshift S-box on a 4x64-bit counter under a 2x64-bit key.   */
/* ------------------------------------------------------------------ */
static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t h0, l0, h1, l1;
        mul128(M0, x0, &h0, &l0);
        mul128(M1, x2, &h1, &l1);
        uint64_t y0 = h1 ^ x1 ^ k0, y1 = l1, y2 = h0 ^ x3 ^ k1, y3 = l0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * Measurement sampling (Sec. II-B: repeated preparation and measurement),
 * made exactly reproducible:
 *   P(x) = re^2 + im^2 in FP64, q(x) = floor(P(x) * 2^62) as uint64,
 *   F(x) = sum_{y<=x} q(y), T = F(2^n - 1);
 *   shot s: r = word 0 of Philox4x64-10(counter = (s,0,0,0), key = (seed,0)),
 *   u = floor(r * T / 2^64), x_s = min { x : F(x) > u }.
 * psi holds 2^n interleaved FP64 (re, im); single-precision states are passed
 * promoted to FP64, which is exact.
 */
int oracle_sample(int n, const double *psi, uint64_t seed, int64_t shots, uint64_t *out)
{
    const int64_t dim = (int64_t)1 << n;
    uint64_t *F = (uint64_t *)malloc((size_t)dim * sizeof(uint64_t));
    if (!F) return 2;
    uint64_t acc = 0;
    for (int64_t x = 0; x < dim; x++) {
        double re = psi[2 * x], im = psi[2 * x + 1];
        double P = re * re + im * im;
        acc += (uint64_t)(P * 4611686018427387904.0); /* 2^62 */
        F[x] = acc;
    }
    const uint64_t T = acc;
    if (T == 0) { free(F); return 3; }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < shots; s++) {
        uint64_t ctr[4] = {(uint64_t)s, 0, 0, 0}, key[2] = {seed, 0}, r[4];
        oracle_philox4x64_10(ctr, key, r);
        uint64_t hi, lo;
        mul128(r[0], T, &hi, &lo);
        const uint64_t u = hi;
        int64_t a = 0, b = dim - 1; /* F[b] = T > u */
        while (a < b) {
            int64_t mid = a + (b - a) / 2;
            if (F[mid] > u) b = mid; else a = mid + 1;
        }
        out[s] = (uint64_t)a;
    }
    free(F);
    return 0;
}

/*
 * Complement-symmetric storage.  psi(x) = psi(~x) for every state of the
 * circuit (C(x) = C(~x) for the cut of eq. 6; |+> and the mixer of eq. 3 are
 * invariant under flipping all qubits), so a state is fixed by the half with
 * bit n-1 clear.  That half is indexed by z with y = x mod 2^(n-1):
 *   y_q = z_q XOR z_(q+1) XOR ... XOR z_(n-2),
 * computed here bit by bit from the top.
 */
uint64_t oracle_sym_y_of_z(int n, uint64_t z)
{
    uint64_t y = 0, acc = 0;
    for (int q = n - 2; q >= 0; q--) {
        acc ^= (z >> q) & 1u;
        y |= acc << q;
    }
    return y;
}

/* The stored half of a full state: half[z] = psi[y(z)] (interleaved re, im). */
int oracle_sym_half(int n, const double *psi, double *half)
{
    if (n < 2 || !psi || !half) return 1;
    const int64_t h = (int64_t)1 << (n - 1);
    for (int64_t z = 0; z < h; z++) {
        const uint64_t y = oracle_sym_y_of_z(n, (uint64_t)z);
        half[2 * z] = psi[2 * y];
        half[2 * z + 1] = psi[2 * y + 1];
    }
    return 0;
}

/*
 * Shots from a complement-symmetric half state (z order): the rule of
 * oracle_sample applied to the half draws z with probability |half[z]|^2 / sum;
 * the shot is y(z) when bit 63 of word 1 of the same Philox output is clear,
 * else the complement of y(z) over n bits -- each of x, ~x with half the
 * mass, as in the full state.
 */
int oracle_sample_sym(int n, const double *half, uint64_t seed, int64_t shots, uint64_t *out)
{
    const int64_t dim = (int64_t)1 << (n - 1);
    uint64_t *F = (uint64_t *)malloc((size_t)dim * sizeof(uint64_t));
    if (!F) return 2;
    uint64_t acc = 0;
    for (int64_t z = 0; z < dim; z++) {
        double re = half[2 * z], im = half[2 * z + 1];
        double P = re * re + im * im;
        acc += (uint64_t)(P * 4611686018427387904.0); /* 2^62 */
        F[z] = acc;
    }
    const uint64_t T = acc;
    if (T == 0) { free(F); return 3; }
    const uint64_t full = (n == 64) ? ~(uint64_t)0 : (((uint64_t)1 << n) - 1);
    for (int64_t s = 0; s < shots; s++) {
        uint64_t ctr[4] = {(uint64_t)s, 0, 0, 0}, key[2] = {seed, 0}, r[4];
        oracle_philox4x64_10(ctr, key, r);
        uint64_t hi, lo;
        mul128(r[0], T, &hi, &lo);
        int64_t a = 0, b = dim - 1;
        while (a < b) {
            int64_t mid = a + (b - a) / 2;
            if (F[mid] > hi) b = mid; else a = mid + 1;
        }
        uint64_t x = oracle_sym_y_of_z(n, (uint64_t)a);
        if (r[1] >> 63) x ^= full;
        out[s] = x;
    }
    free(F);
    return 0;
}

/*
 * Exact distribution of the cut value under the state: the noiseless
 * reference distribution of Sec. II-D without subsampling noise.  In the
 * sampler's fixed point,
 *   mass[c] = sum over x with C_t[x] = c of floor((re^2 + im^2) 2^62),
 * with every value outside 0..nbins-1 counted in bin nbins - 1.
 */
int oracle_cost_histogram(int n, const double *psi, const int32_t *diag, int64_t nbins, uint64_t *mass)
{
    if (n < 1 || nbins < 1 || !psi || !diag || !mass) return 1;
    const int64_t dim = (int64_t)1 << n;
    for (int64_t c = 0; c < nbins; c++) mass[c] = 0;
    for (int64_t x = 0; x < dim; x++) {
        double re = psi[2 * x], im = psi[2 * x + 1];
        double P = re * re + im * im;
        int64_t c = diag[x];
        if (c < 0 || c >= nbins) c = nbins - 1;
        mass[c] += (uint64_t)(P * 4611686018427387904.0); /* 2^62 */
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Adjoint gradient of E = <psi_p| C |psi_p> (C in units), gate by gate. */
/* For a gate G(t) = exp(-i t/2 P) applied as state phi = G psi, with     */
/* lambda = (later gates)^dagger C psi_p: dE/dt = Im <lambda| P |phi>.    */
/* Every gate is then undone on both vectors.                             */
/* ------------------------------------------------------------------ */
static double im_inner_x(int n, const cplx *lam, const cplx *psi, int q)
{
    const int64_t dim = (int64_t)1 << n;
    const uint64_t bit = (uint64_t)1 << q;
    double *t = (double *)malloc((size_t)dim * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < dim; x++) t[x] = cimag(conj(lam[x]) * psi[(uint64_t)x ^ bit]);
    double s = pairwise_sum(t, dim);
    free(t);
    return s;
}

static double im_inner_zz(int n, const cplx *lam, const cplx *psi, int i, int j)
{
    const int64_t dim = (int64_t)1 << n;
    double *t = (double *)malloc((size_t)dim * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < dim; x++) {
        double z = ((((uint64_t)x >> i) ^ ((uint64_t)x >> j)) & 1u) ? -1.0 : 1.0;
        t[x] = z * cimag(conj(lam[x]) * psi[x]);
    }
    double s = pairwise_sum(t, dim);
    free(t);
    return s;
}

int oracle_adjoint(int n, const int32_t *w, int p, const double *tzz, const double *tx,
                   double *exp_c, double *g_zz, double *g_x)
{
    if (n < 2 || n > 24 || p < 1) return 1;
    const int64_t dim = (int64_t)1 << n;
    cplx *psi = (cplx *)malloc((size_t)dim * sizeof(cplx));
    cplx *lam = (cplx *)malloc((size_t)dim * sizeof(cplx));
    int32_t *diag = (int32_t *)malloc((size_t)dim * sizeof(int32_t));
    if (!psi || !lam || !diag) { free(psi); free(lam); free(diag); return 2; }
    run_circuit(n, w, p, tzz, tx, 0, psi);
    oracle_cost_diagonal(n, w, diag);
    double nrm;
    oracle_expect(n, (const double *)psi, diag, exp_c, &nrm);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < dim; x++) lam[x] = ((double)diag[x] / 10.0) * psi[x];
    for (int k = p - 1; k >= 0; k--) {
        g_x[k] = 0.0;
        for (int q = n - 1; q >= 0; q--) {
            g_x[k] += im_inner_x(n, lam, psi, q);
            apply_rx(n, psi, q, -tx[k]);
            apply_rx(n, lam, q, -tx[k]);
        }
        g_zz[k] = 0.0;
        for (int i = n - 1; i >= 0; i--)
            for (int j = n - 1; j > i; j--) {
                double wij = (double)w[edge_id(n, i, j)] / 10.0;
                g_zz[k] += wij * im_inner_zz(n, lam, psi, i, j);
                apply_rzz(n, psi, i, j, -tzz[k] * wij);
                apply_rzz(n, lam, i, j, -tzz[k] * wij);
            }
    }
    free(psi);
    free(lam);
    free(diag);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Noisy trajectories (Sec. II-C).  The depolarizing channel of rate eps  */
/* on the two qubits (a, b) of a gate,                                    */
/*   rho -> (1 - eps) rho + eps Tr_ab(rho) (x) I_ab / 4                   */
/*        = (1 - eps) rho + (eps / 16) sum_P P rho P,                     */
/* P over the 16 two-qubit Paulis, is unravelled into trajectories: after */
/* each RZZ gate, with probability eps, one of the 16 Paulis drawn        */
/* uniformly is applied to the state.                                     */
/*                                                                        */
/* Draw rule, for trajectory t, layer k (0-based) and edge e (the         */
/* lexicographic pair index):                                             */
/*   (r0, r1, r2, r3) = Philox4x64-10(counter = (t, k, e, 1),             */
/*                                    key = (seed, 0));                   */
/*   error iff (r0 >> 11) < thr, with thr = floor(eps * 2^53);            */
/*   Pauli code c = r1 & 15: P_a = c & 3 on the lower qubit a of the      */
/*   edge, P_b = c >> 2 on the upper qubit b (0 = I, 1 = X, 2 = Y,        */
/*   3 = Z).  Code 0 is the identity and changes nothing.                 */
/* ------------------------------------------------------------------ */
static void apply_pauli(int n, cplx *psi, int q, int code)
{
    switch (code) {
    case 1: apply_1q(n, psi, q, 0.0, 1.0, 1.0, 0.0); break;  /* X */
    case 2: apply_1q(n, psi, q, 0.0, -I, I, 0.0); break;     /* Y = [[0, -i], [i, 0]] */
    case 3: apply_1q(n, psi, q, 1.0, 0.0, 0.0, -1.0); break; /* Z */
    default: break;
    }
}

/*
 * The circuit with explicit Pauli insertions: error t (err_layer[t],
 * err_edge[t], err_code[t]) is applied right after the RZZ gate of that edge
 * in that layer, before the next gate.  Several errors on one gate are
 * applied in list order.  psi_out: 2^n interleaved complex128.
 */
int oracle_pauli_circuit(int n, const int32_t *w, int p, const double *tzz, const double *tx, int64_t nerr,
                         const int32_t *err_layer, const int32_t *err_edge, const int32_t *err_code,
                         double *psi_out)
{
    if (n < 2 || n > 24 || p < 0 || !w || !psi_out || nerr < 0) return 1;
    if (nerr > 0 && (!err_layer || !err_edge || !err_code)) return 1;
    cplx *psi = (cplx *)psi_out;
    prepare_plus(n, psi);
    for (int k = 0; k < p; k++) {
        for (int i = 0; i < n; i++)
            for (int j = i + 1; j < n; j++) {
                const int64_t e = edge_id(n, i, j);
                apply_rzz(n, psi, i, j, tzz[k] * ((double)w[e] / 10.0));
                for (int64_t t = 0; t < nerr; t++)
                    if (err_layer[t] == k && err_edge[t] == e) {
                        apply_pauli(n, psi, i, err_code[t] & 3);
                        apply_pauli(n, psi, j, (err_code[t] >> 2) & 3);
                    }
            }
        apply_mixer(n, psi, tx[k]);
    }
    return 0;
}

/*
 * The non-identity errors of trajectory traj by the draw rule above, in
 * (layer, edge) order.  Writes at most cap of them and the total to *count;
 * returns 4 when the total exceeds cap.
 */
int oracle_noise_draws(int n, int p, uint64_t thr, uint64_t seed, uint64_t traj, int64_t cap, int32_t *err_layer,
                       int32_t *err_edge, int32_t *err_code, int64_t *count)
{
    if (n < 2 || p < 0 || cap < 0 || !count) return 1;
    const int64_t m = n_edges(n);
    int64_t c = 0;
    for (int k = 0; k < p; k++)
        for (int64_t e = 0; e < m; e++) {
            uint64_t ctr[4] = {traj, (uint64_t)k, (uint64_t)e, 1}, key[2] = {seed, 0}, r[4];
            oracle_philox4x64_10(ctr, key, r);
            if ((r[0] >> 11) >= thr) continue;
            const int code = (int)(r[1] & 15u);
            if (code == 0) continue;
            if (c < cap) {
                err_layer[c] = k;
                err_edge[c] = (int32_t)e;
                err_code[c] = code;
            }
            c++;
        }
    *count = c;
    return c > cap ? 4 : 0;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }
