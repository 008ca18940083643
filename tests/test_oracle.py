"""Pins for the CPU oracle: each check ties it to something other than itself.

Dense matrix exponentials of eqs. (1)-(3), closed forms, exact integer
identities of the cut function, brute force, published Philox known-answer
vectors and numpy's independent Philox, the paper's printed gate counts and
memory sizes, and finite differences.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def inst(n, seed):
    return workloads.complete_graph_tenths(n, seed)


# ---------------------------------------------------------------- circuit
@pytest.mark.parametrize("n", [2, 3, 5, 7, 8])
@pytest.mark.parametrize("convention", ["paper", "literal"])
def test_simulate_matches_dense_expm(n, convention):
    """Eqs. (2)-(3) by scipy expm of H_C and H_B vs both oracle cost modes."""
    w = inst(n, 10 + n)
    for p, seed in [(1, 0), (3, 1), (4, 2)]:
        g, b = workloads.random_angles(p, seed, scale=1.3)
        tzz, tx = oracle.gate_angles(g, b, convention)
        ref = oracle.dense_state(n, w, g, b, convention)
        for mode in (0, 1):
            psi = oracle.simulate(n, w, tzz, tx, mode)
            assert np.abs(psi - ref).max() < 1e-12


def test_gate_by_gate_equals_diagonal_mode():
    n = 11
    w = inst(n, 3)
    g, b = oracle.ramp_midpoint(3, 0.6, 0.6)
    tzz, tx = oracle.gate_angles(g, b)
    assert np.abs(oracle.simulate(n, w, tzz, tx, 0) - oracle.simulate(n, w, tzz, tx, 1)).max() < 1e-13


@pytest.mark.parametrize("convention", ["paper", "literal"])
def test_two_qubit_closed_form(convention):
    for wt in (1, 4, 10):
        for gamma, beta in [(0.3, 0.2), (0.9, -0.4), (1.7, 0.05)]:
            tzz, tx = oracle.gate_angles([gamma], [beta], convention)
            e = oracle.expect_of(2, [wt], tzz, tx)
            assert abs(e - oracle.k2_expect(wt / 10, gamma, beta, convention)) < 1e-14


@pytest.mark.parametrize("n", [3, 4, 6, 9, 10])
def test_single_layer_closed_form(n):
    """Heisenberg-picture <C> after one layer (independent derivation)."""
    w = inst(n, 40 + n)
    for seed in range(3):
        g, b = workloads.random_angles(1, seed, scale=1.5)
        tzz, tx = oracle.gate_angles(g, b)
        e = oracle.expect_of(n, w, tzz, tx, mode=0)
        assert abs(e - oracle.p1_expect(n, w, tzz[0], tx[0])) < 1e-12 * max(1, abs(e))


def test_invariants():
    n = 9
    w = inst(n, 7)
    W = oracle.weight_total(w) / 10
    diag = oracle.cost_diagonal(n, w)
    # p = 0: the |+> state, <C> = W/2
    e, nrm = oracle.expect(oracle.simulate(n, w, [], []), diag)
    assert abs(e - W / 2) < 1e-12 and abs(nrm - 1) < 1e-14
    # gamma = 0 or beta = 0 leave <C> = W/2
    for tzz, tx in [([0.0, 0.0], [0.7, -0.3]), ([0.5, 1.1], [0.0, 0.0])]:
        e, nrm = oracle.expect(oracle.simulate(n, w, tzz, tx), diag)
        assert abs(e - W / 2) < 1e-12 and abs(nrm - 1) < 1e-13
    # mixer only: |+> picks up the global phase exp(-i n theta/2) per layer
    psi = oracle.simulate(n, w, [0.0, 0.0], [0.7, -0.2])
    assert np.abs(psi - 2 ** (-n / 2) * np.exp(-1j * n * 0.5 / 2)).max() < 1e-14
    # cost only: amplitude = 2^{-n/2} exp(-i theta (W - 2C)/2) since H_C = W - 2C
    theta = 0.83
    psi = oracle.simulate(n, w, [theta], [0.0], mode=0)
    ref = 2 ** (-n / 2) * np.exp(-1j * theta * (W - 2 * diag / 10) / 2)
    assert np.abs(psi - ref).max() < 1e-14
    # Z2 symmetry: psi[x] == psi[~x] exactly, for both modes
    g, b = oracle.ramp_midpoint(3, 0.6, 0.6)
    tzz, tx = oracle.gate_angles(g, b)
    for mode in (0, 1):
        psi = oracle.simulate(n, w, tzz, tx, mode)
        x = np.arange(1 << n)
        assert np.array_equal(psi, psi[(~x) & ((1 << n) - 1)])
        assert abs(np.vdot(psi, psi).real - 1) < 1e-13


def test_noiseless_ratio_grows_with_depth_only_in_paper_convention():
    """Sec. II-C: noiseless r rises towards 1 with p.  This fixes the sign reading."""
    n = 10
    w = inst(n, 0)
    cmax = oracle.cmax_direct(n, w) / 10
    r = {}
    for conv in ("paper", "literal"):
        r[conv] = [oracle.expect_of(n, w, *oracle.gate_angles(*oracle.ramp_midpoint(p, 0.6, 0.6), conv)) / cmax
                   for p in (1, 3, 10)]
    assert r["paper"][0] < r["paper"][1] < r["paper"][2] < 1
    assert not (r["literal"][0] < r["literal"][1] < r["literal"][2])


# ---------------------------------------------------------------- cut function
@pytest.mark.parametrize("n", [2, 5, 12, 18])
def test_cost_diagonal_identities(n):
    w = inst(n, n)
    diag = oracle.cost_diagonal(n, w).astype(np.int64)
    W = int(np.sum(w, dtype=np.int64))
    s2 = int(np.sum(w.astype(np.int64) ** 2))
    assert int(diag.sum()) == (W << (n - 1))
    assert int((diag ** 2).sum()) == ((W * W + s2) << (n - 2)) if n >= 2 else True
    x = np.arange(1 << n)
    assert np.array_equal(diag, diag[(~x) & ((1 << n) - 1)])      # complement symmetry
    assert diag[0] == 0
    assert diag.min() >= 0 and diag.max() <= W


def test_cost_diagonal_matches_hamiltonian():
    """Eq. (1) vs eq. (6): H_C(x) = W - 2 C(x)."""
    n = 8
    w = inst(n, 2)
    hc, _ = oracle.dense_hamiltonians(n, w)
    diag = oracle.cost_diagonal(n, w)
    assert np.abs(hc - (oracle.weight_total(w) - 2 * diag) / 10).max() < 1e-12


def test_single_vertex_cut_is_its_degree():
    n = 9
    w = inst(n, 5)
    W = np.zeros((n, n), dtype=np.int64)
    W[np.triu_indices(n, 1)] = w
    W = W + W.T
    for i in range(n):
        assert oracle.cut_value(n, w, 1 << i) == W[i].sum()


@pytest.mark.parametrize("n", [2, 3, 7, 13, 16])
def test_cmax_gray_vs_direct(n):
    for seed in range(3):
        w = inst(n, 100 + seed)
        c = oracle.cmax_direct(n, w)
        assert oracle.cmax_gray(n, w) == c == int(oracle.cost_diagonal(n, w).max())
        assert 2 * c >= int(np.sum(w))    # the mean cut is W/2


def test_cmax_large_weights():
    rng = np.random.default_rng(9)
    n = 12
    w = rng.integers(0, 30000, size=n * (n - 1) // 2).astype(np.int32)
    assert oracle.cmax_gray(n, w) == oracle.cmax_direct(n, w)


# ---------------------------------------------------------------- Philox / sampling
def test_philox_known_answers():
    """Known-answer vectors of Philox4x64-10 (Salmon et al., SC'11)."""
    out = oracle.philox4x64_10([0, 0, 0, 0], [0, 0])
    assert [int(v) for v in out] == [0x16554d9eca36314c, 0xdb20fe9d672d0fdc,
                                    0xd7e772cee186176b, 0x7e68b68aec7ba23b]
    ctr = [0x243f6a8885a308d3, 0x13198a2e03707344, 0xa4093822299f31d0, 0x082efa98ec4e6c89]
    key = [0x452821e638d01377, 0xbe5466cf34e90c6c]
    assert [int(v) for v in oracle.philox4x64_10(ctr, key)] == [
        0xa528f45403e61d95, 0x38c72dbd566e9788, 0xa5a1610e72fd18b5, 0x57bd43b5e52b7fe6]


def test_philox_vs_numpy():
    """numpy's Philox advances the counter by one before each block."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        ctr = rng.integers(1, 2 ** 63, size=4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=np.array([ctr[0] - np.uint64(1)] + list(ctr[1:]),
                                                        dtype=np.uint64))
        assert np.array_equal(bg.random_raw(4), oracle.philox4x64_10(ctr, key))


def test_sampling_uniform_state_closed_form():
    """Uniform state: q = 2^(62-n), so x_s is the top n bits of the Philox word."""
    n, seed, shots = 10, 12345, 4000
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    got = oracle.sample(psi, seed, shots)
    want = np.array([int(oracle.philox4x64_10([s, 0, 0, 0], [seed, 0])[0]) >> (64 - n)
                     for s in range(shots)], dtype=np.uint64)
    assert np.array_equal(got, want)


def test_sampling_delta_and_two_point_states():
    n = 7
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[77] = 1j
    assert np.all(oracle.sample(psi, 3, 500) == 77)
    psi[:] = 0
    psi[5], psi[100] = np.sqrt(0.25), 1j * np.sqrt(0.75)
    s = oracle.sample(psi, 4, 2000)
    assert set(np.unique(s)) <= {5, 100}
    # the threshold: u < 2^60 (a quarter of T = 2^62) picks 5
    r = np.array([int(oracle.philox4x64_10([i, 0, 0, 0], [4, 0])[0]) for i in range(2000)], dtype=object)
    assert np.array_equal(s == 5, np.array([int(v) * (1 << 62) >> 64 < (1 << 60) for v in r]))


def test_sampling_distribution_g_test():
    """Shots follow |a|^2: G-test on a small circuit (p-value not tiny)."""
    from scipy.stats import chi2
    n = 8
    w = inst(n, 1)
    g, b = oracle.ramp_midpoint(3, 0.6, 0.6)
    psi = oracle.simulate(n, w, *oracle.gate_angles(g, b))
    shots = 200000
    s = oracle.sample(psi, 7, shots)
    obs = np.bincount(s.astype(np.int64), minlength=1 << n)
    exp = np.abs(psi) ** 2 * shots
    m = obs > 0
    G = 2 * np.sum(obs[m] * np.log(obs[m] / exp[m]))
    assert chi2.sf(G, (1 << n) - 1) > 1e-4


def test_sampling_single_precision_input_is_promoted():
    n = 9
    w = inst(n, 4)
    psi = oracle.simulate(n, w, [0.4], [-0.3]).astype(np.complex64)
    a = oracle.sample(psi, 11, 3000)
    b = oracle.sample(psi.astype(np.complex128), 11, 3000)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- complement-symmetric storage
def test_sym_index_map_and_factor_rule():
    """z -> y(z) pairs every basis state with its complement exactly once, and
    X on qubit q moves z by the factor mask (z0 | z_(q-1) z_q | z_(n-2))."""
    n = 6
    full = (1 << n) - 1
    zs = {}
    for z in range(1 << (n - 1)):
        y = oracle.sym_y_of_z(n, z)
        assert y < (1 << (n - 1))
        zs[y] = z
        zs[y ^ full] = z
    assert len(zs) == 1 << n
    for x in range(1 << n):
        for q in range(n):
            mask = 1 if q == 0 else (1 << (n - 2)) if q == n - 1 else 3 << (q - 1)
            assert zs[x ^ (1 << q)] == zs[x] ^ mask, (x, q)


def test_circuit_states_are_complement_symmetric():
    n = 9
    w = inst(n, 6)
    psi = oracle.simulate(n, w, *oracle.gate_angles(*oracle.ramp_midpoint(4, 0.8, 0.4)))
    comp = np.arange(1 << n) ^ ((1 << n) - 1)
    assert np.abs(psi - psi[comp]).max() < 1e-13
    half = oracle.sym_half(psi)
    for z in (0, 1, 77, 255):
        assert half[z] == psi[oracle.sym_y_of_z(n, z)]


def test_sample_sym_delta_and_complement_bit():
    n, seed = 8, 99
    half = np.zeros(1 << (n - 1), dtype=np.complex128)
    z0 = 45
    half[z0] = 1.0
    y = oracle.sym_y_of_z(n, z0)
    s = oracle.sample_sym(half, n, seed, 400)
    bits = np.array([int(oracle.philox4x64_10([i, 0, 0, 0], [seed, 0])[1]) >> 63 for i in range(400)])
    want = np.where(bits == 1, y ^ ((1 << n) - 1), y).astype(np.uint64)
    assert np.array_equal(s, want) and 0 < bits.sum() < 400


def test_sample_sym_distribution_g_test():
    """Shots from the half state follow |psi(x)|^2 of the full state."""
    from scipy.stats import chi2
    n = 8
    w = inst(n, 7)
    psi = oracle.simulate(n, w, *oracle.gate_angles(*oracle.ramp_midpoint(3, 0.6, 0.6)))
    shots = 200000
    s = oracle.sample_sym(oracle.sym_half(psi), n, 5, shots)
    obs = np.bincount(s.astype(np.int64), minlength=1 << n)
    exp = np.abs(psi) ** 2 * shots
    m = obs > 0
    G = 2 * np.sum(obs[m] * np.log(obs[m] / exp[m]))
    assert chi2.sf(G, (1 << n) - 1) > 1e-4


# ---------------------------------------------------------------- cut-value histogram
def test_histogram_uniform_state_counts_the_diagonal():
    """On |+>^n every q(x) is 2^(62-n) exactly, so the histogram is the count
    of basis states per cut value times that mass."""
    n = 11
    w = inst(n, 2)
    diag = oracle.cost_diagonal(n, w)
    W = oracle.weight_total(w)
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    got = oracle.cost_histogram(psi, diag, W + 1)
    want = np.bincount(diag, minlength=W + 1).astype(np.uint64) * np.uint64(1 << (62 - n))
    assert np.array_equal(got, want)


def test_histogram_delta_state_and_overflow_bin():
    n = 9
    w = inst(n, 3)
    diag = oracle.cost_diagonal(n, w)
    psi = np.zeros(1 << n, dtype=np.complex128)
    x0 = 300
    psi[x0] = -1j
    W = oracle.weight_total(w)
    h = oracle.cost_histogram(psi, diag, W + 1)
    assert h[diag[x0]] == 1 << 62 and int(h.sum()) == 1 << 62
    # values at or above nbins land in the last bin
    nb = int(diag[x0])
    h2 = oracle.cost_histogram(psi, diag, nb)
    assert h2[-1] == 1 << 62 and int(h2.sum()) == 1 << 62


def test_histogram_moments_match_the_state():
    """Total mass = 2^62 norm and mean cut = <C>, up to the floor of each q."""
    n = 10
    w = inst(n, 5)
    diag = oracle.cost_diagonal(n, w)
    psi = oracle.simulate(n, w, *oracle.gate_angles(*oracle.ramp_midpoint(3, 0.7, 0.5)))
    h = oracle.cost_histogram(psi, diag, oracle.weight_total(w) + 1).astype(np.float64)
    e, nrm = oracle.expect(psi, diag)
    total = h.sum() / 2.0 ** 62
    assert abs(total - nrm) <= (1 << n) * 2.0 ** -62 + 1e-15
    mean = (np.arange(len(h)) * h).sum() / h.sum() / 10
    assert abs(mean - e) <= 1e-12 * e
    # the distribution differs from the uniform one (the circuit moves mass up)
    assert mean > oracle.weight_total(w) / 20


# ---------------------------------------------------------------- gradient
@pytest.mark.parametrize("convention", ["paper", "literal"])
def test_adjoint_vs_finite_differences(convention):
    n = 7
    w = inst(n, 8)
    g, b = oracle.ramp_midpoint(3, 0.6, 0.6)
    tzz, tx = oracle.gate_angles(g, b, convention)
    e, gzz, gx = oracle.adjoint(n, w, tzz, tx)
    fzz, fx = oracle.fd_gradient(n, w, tzz, tx, h=1e-4)
    assert abs(e - oracle.expect_of(n, w, tzz, tx)) < 1e-12
    assert np.abs(gzz - fzz).max() < 1e-6 and np.abs(gx - fx).max() < 1e-6


@pytest.mark.parametrize("n", [4, 8, 10])
def test_adjoint_vs_single_layer_closed_form(n):
    w = inst(n, 20 + n)
    tzz, tx = 0.63, -0.41
    e, gzz, gx = oracle.adjoint(n, w, [tzz], [tx])
    czz, cx = oracle.p1_gradient(n, w, tzz, tx)
    assert abs(gzz[0] - czz) < 1e-11 and abs(gx[0] - cx) < 1e-11


# ---------------------------------------------------------------- schedule / paper values
def test_ramps():
    g, b = oracle.ramp_paper(4, 0.8, 0.4)
    assert np.allclose(g, [0.2, 0.4, 0.6, 0.8]) and np.allclose(b, [0.4, 0.3, 0.2, 0.1])
    g, b = oracle.ramp_midpoint(3, 0.6, 0.6)
    assert np.allclose(g, [0.1, 0.3, 0.5]) and np.allclose(b, [0.5, 0.3, 0.1])


def test_paper_printed_values():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        pv = json.load(f)
    for row in pv["two_qubit_gates"]:
        assert oracle.gate_counts(row["n"], row["p"])[0] == row["count"]
    for row in pv["fp32_state_bytes"]:
        assert oracle.state_bytes_fp32(row["n"]) == row["bytes"]
    assert oracle.gate_counts(40, 3)[1] == 4 * 40


def test_golden_instance_values():
    """Stored C(x*) and W of the benchmark instances (written by make_golden.py)."""
    path = os.path.join(GOLDEN, "instances.json")
    with open(path) as f:
        gold = json.load(f)
    for row in gold["instances"]:
        w = inst(row["n"], row["seed"])
        assert oracle.weight_total(w) == row["w_total_tenths"]
        if row["n"] <= 16:
            assert oracle.cmax_direct(row["n"], w) == row["cmax_tenths"]


# ---------------------------------------------------------------- noise (Sec. II-C)
def _angles(p, d=0.6):
    return oracle.gate_angles(*oracle.ramp_midpoint(p, d, d))


def test_noise_threshold():
    assert oracle.noise_threshold(0.0) == 0
    assert oracle.noise_threshold(1.0) == 1 << 53
    assert oracle.noise_threshold(0.5) == 1 << 52
    assert oracle.noise_threshold(2.0 ** -53) == 1
    with pytest.raises(ValueError):
        oracle.noise_threshold(1.5)


def test_noise_free_trajectory_is_the_noiseless_circuit():
    n = 5
    w = inst(n, 11)
    tzz, tx = _angles(3)
    psi, nerr = oracle.noisy_trajectory(n, w, tzz, tx, 0.0, 3, 17)
    assert nerr == 0
    assert np.array_equal(psi, oracle.simulate(n, w, tzz, tx, 0))


def test_noise_draw_statistics():
    """Error rate eps, each of the 16 Paulis equally likely (15 of them non-identity)."""
    n, p, eps, N = 6, 3, 0.3, 400
    gates = N * p * n * (n - 1) // 2
    codes = []
    for t in range(N):
        lay, edg, cod = oracle.noise_draws(n, p, eps, 5, t)
        assert np.all(np.diff(lay * 1000 + edg) > 0)  # (layer, edge) order, one draw per gate
        assert np.all((cod >= 1) & (cod <= 15))
        codes.append(cod)
    cod = np.concatenate(codes)
    mean = gates * eps * 15 / 16
    sd = np.sqrt(gates * eps * 15 / 16 * (1 - eps * 15 / 16))
    assert abs(len(cod) - mean) < 5 * sd
    counts = np.bincount(cod, minlength=16)[1:]
    chi2 = float(((counts - len(cod) / 15) ** 2 / (len(cod) / 15)).sum())
    assert chi2 < 60  # 14 degrees of freedom: P(chi2 > 60) ~ 1e-7
    # eps = 1: every gate errs
    lay, edg, cod = oracle.noise_draws(n, p, 1.0, 5, 0)
    g = p * n * (n - 1) // 2
    assert abs(len(cod) - g * 15 / 16) < 5 * np.sqrt(g * 15 / 256)


def test_pauli_insertion_xx_commutes_with_the_mixer():
    """X_a X_b after the last gate of the last layer: it commutes with every RX,
    so the final state is the noiseless one with bits a and b flipped."""
    n = 6
    w = inst(n, 12)
    tzz, tx = _angles(3)
    g = n * (n - 1) // 2
    psi = oracle.pauli_circuit(n, w, tzz, tx, ([2], [g - 1], [1 | (1 << 2)]))
    ref = oracle.simulate(n, w, tzz, tx, 0)
    x = np.arange(1 << n)
    assert np.abs(psi - ref[x ^ (3 << (n - 2))]).max() < 1e-13


def test_pauli_insertion_y_and_zz_closed_forms():
    """With an identity mixer (theta_x = 0) in the layer:
    Y on the lower qubit a of the last edge after its gate: (Y psi)[x] = (x_a ? i : -i) psi[x ^ 2^a];
    Z_0 Z_1 after the first gate commutes with every later RZZ: a sign (-1)^(x_0 xor x_1)."""
    n = 5
    w = inst(n, 13)
    tzz = np.array([0.7])
    tx = np.array([0.0])
    ref = oracle.simulate(n, w, tzz, tx, 0)
    x = np.arange(1 << n)
    g = n * (n - 1) // 2
    a = n - 2
    psi = oracle.pauli_circuit(n, w, tzz, tx, ([0], [g - 1], [2]))
    want = np.where((x >> a) & 1, 1j, -1j) * ref[x ^ (1 << a)]
    assert np.abs(psi - want).max() < 1e-13
    psi = oracle.pauli_circuit(n, w, tzz, tx, ([0], [0], [3 | (3 << 2)]))
    want = np.where(((x ^ (x >> 1)) & 1) == 1, -1.0, 1.0) * ref
    assert np.abs(psi - want).max() < 1e-13
    # a misplaced error (before its gate instead of after) would differ: X on qubit 0 of edge (0,1)
    psi = oracle.pauli_circuit(n, w, tzz, tx, ([0], [0], [1]))
    assert np.abs(psi - ref[x ^ 1]).max() > 1e-3


def test_density_matrix_special_cases():
    n = 4
    w = inst(n, 14)
    tzz, tx = _angles(2)
    pure = oracle.expect(oracle.simulate(n, w, tzz, tx, 0), oracle.cost_diagonal(n, w))[0]
    assert abs(oracle.density_expect(n, w, tzz, tx, 0.0) - pure) < 1e-12
    # eps = 1: every qubit is fully depolarized at its last gate of the layer -> I / 2^n
    assert abs(oracle.density_expect(n, w, tzz, tx, 1.0) - oracle.weight_total(w) / 20.0) < 1e-12
    w2 = np.array([7], dtype=np.int32)
    for p in (1, 2, 4):
        a, b = _angles(p)
        e0 = oracle.expect(oracle.simulate(2, w2, a, b, 0), oracle.cost_diagonal(2, w2))[0]
        for eps in (0.05, 0.5):
            assert abs(oracle.density_expect(2, w2, a, b, eps) - oracle.k2_noisy_expect(0.7, e0, eps, p)) < 1e-12


@pytest.mark.parametrize("n,p,eps", [(4, 2, 0.2), (3, 3, 0.05)])
def test_trajectory_average_matches_density_matrix(n, p, eps):
    w = inst(n, 15)
    tzz, tx = _angles(p)
    diag = oracle.cost_diagonal(n, w)
    N = 2000
    es = np.array([oracle.expect(oracle.noisy_trajectory(n, w, tzz, tx, eps, 21, t)[0], diag)[0]
                   for t in range(N)])
    dm = oracle.density_expect(n, w, tzz, tx, eps)
    assert abs(es.mean() - dm) < 5 * es.std() / np.sqrt(N) + 1e-12
