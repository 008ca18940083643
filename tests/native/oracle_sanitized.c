/* Host-only driver for the oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every exported routine once on a small
 * instance with exactly sized buffers.  Built and run by
 * tests/test_oracle_sanitized.py; prints "ok" and exits 0 when every call
 * succeeds and no sanitizer reports. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_cost_diagonal(int n, const int32_t *w, int32_t *diag);
int oracle_cut_values(int n, const int32_t *w, const uint64_t *xs, int64_t count, int64_t *out);
int oracle_simulate(int n, const int32_t *w, int p, const double *tzz, const double *tx, int mode,
                    double *psi_out);
int oracle_expect(int n, const double *psi, const int32_t *diag, double *exp_c, double *norm);
int oracle_sample(int n, const double *psi, uint64_t seed, int64_t shots, uint64_t *out);
int oracle_sym_half(int n, const double *psi, double *half);
int oracle_sample_sym(int n, const double *half, uint64_t seed, int64_t shots, uint64_t *out);
int oracle_cost_histogram(int n, const double *psi, const int32_t *diag, int64_t nbins, uint64_t *mass);
int oracle_adjoint(int n, const int32_t *w, int p, const double *tzz, const double *tx, double *exp_c,
                   double *g_zz, double *g_x);
int oracle_pauli_circuit(int n, const int32_t *w, int p, const double *tzz, const double *tx, int64_t nerr,
                         const int32_t *err_layer, const int32_t *err_edge, const int32_t *err_code,
                         double *psi_out);
int oracle_noise_draws(int n, int p, uint64_t thr, uint64_t seed, uint64_t traj, int64_t cap, int32_t *err_layer,
                       int32_t *err_edge, int32_t *err_code, int64_t *count);

#define CHECK(call)                                                  \
    do {                                                             \
        if ((call) != 0) {                                           \
            fprintf(stderr, "failed: %s\n", #call);                  \
            return 1;                                                \
        }                                                            \
    } while (0)

int main(void)
{
    enum { N = 9, P = 3, M = N * (N - 1) / 2, DIM = 1 << N, SHOTS = 257, CAP = 64 };
    int32_t *w = malloc(M * sizeof(int32_t));
    for (int e = 0; e < M; e++) w[e] = 1 + (7 * e + 3) % 10;
    const double tzz[P] = {0.1, 0.2, 0.3}, tx[P] = {-0.9, -0.6, -0.3};

    int32_t *diag = malloc(DIM * sizeof(int32_t));
    CHECK(oracle_cost_diagonal(N, w, diag));
    int W = 0;
    for (int e = 0; e < M; e++) W += w[e];

    uint64_t xs[5] = {0, 1, DIM - 1, 77, 300};
    int64_t cuts[5];
    CHECK(oracle_cut_values(N, w, xs, 5, cuts));

    double *psi = malloc(2 * DIM * sizeof(double)), *psi1 = malloc(2 * DIM * sizeof(double));
    CHECK(oracle_simulate(N, w, P, tzz, tx, 0, psi));
    CHECK(oracle_simulate(N, w, P, tzz, tx, 1, psi1));
    double e = 0, nrm = 0;
    CHECK(oracle_expect(N, psi, diag, &e, &nrm));

    uint64_t *shots = malloc(SHOTS * sizeof(uint64_t));
    CHECK(oracle_sample(N, psi, 5, SHOTS, shots));
    double *half = malloc(2 * (DIM / 2) * sizeof(double));
    CHECK(oracle_sym_half(N, psi, half));
    CHECK(oracle_sample_sym(N, half, 5, SHOTS, shots));
    uint64_t *mass = malloc((W + 1) * sizeof(uint64_t));
    CHECK(oracle_cost_histogram(N, psi, diag, W + 1, mass));

    double ea = 0, gzz[P], gx[P];
    CHECK(oracle_adjoint(N, w, P, tzz, tx, &ea, gzz, gx));

    int32_t el[CAP], ee[CAP], ec[CAP];
    int64_t cnt = 0;
    CHECK(oracle_noise_draws(N, P, (uint64_t)1 << 50, 9, 3, CAP, el, ee, ec, &cnt));
    CHECK(oracle_pauli_circuit(N, w, P, tzz, tx, cnt < CAP ? cnt : CAP, el, ee, ec, psi1));

    printf("ok %.12f %.12f %.12f %lld\n", e, nrm, ea, (long long)cnt);
    free(w); free(diag); free(psi); free(psi1); free(shots); free(half); free(mass);
    return 0;
}
