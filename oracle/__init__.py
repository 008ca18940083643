"""Oracle for LR-QAOA state-vector simulation: a plain, slow CPU reference.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library and never imports it; both sides only read the same seeded
inputs from ``workloads``.

Contents (arXiv:2604.26423):
  * ``liboracle.so`` (oracle.c): complex128 gate-by-gate simulation
    (Sec. II-E), cut function (eq. 6), C(x*) by brute force, <C> (eq. 5 with
    exact probabilities), the reproducible sampling rule, the gate-by-gate
    adjoint gradient;
  * the linear ramp (eq. 4) and its midpoint variant, and the map from the
    paper's (gamma_k, beta_k) to gate angles (eqs. 2-3);
  * dense matrix-exponential references of eqs. (1)-(3) for tiny n;
  * closed forms: two-qubit circuit and single-layer <C> on any complete graph;
  * noise (Sec. II-C): the circuit with explicit Pauli insertions, the
    trajectory draw rule, and a density-matrix reference of the depolarizing
    channel for tiny n, with its two-qubit closed form.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    """Load liboracle.so, compiling it with gcc if it is missing or stale."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.oracle_cost_diagonal.argtypes = [ctypes.c_int, _i32p, _i32p]
        L.oracle_cut_value.argtypes = [ctypes.c_int, _i32p, ctypes.c_uint64]
        L.oracle_cut_value.restype = ctypes.c_int64
        L.oracle_cut_values.argtypes = [ctypes.c_int, _i32p, _u64p, ctypes.c_int64, _i64p]
        L.oracle_weight_total.argtypes = [ctypes.c_int, _i32p]
        L.oracle_weight_total.restype = ctypes.c_int64
        L.oracle_cmax_direct.argtypes = [ctypes.c_int, _i32p]
        L.oracle_cmax_direct.restype = ctypes.c_int64
        L.oracle_cmax_gray.argtypes = [ctypes.c_int, _i32p]
        L.oracle_cmax_gray.restype = ctypes.c_int64
        L.oracle_simulate.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, _f64p, _f64p,
                                      ctypes.c_int, _f64p]
        L.oracle_expect.argtypes = [ctypes.c_int, _f64p, _i32p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        L.oracle_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.oracle_philox4x64_10.restype = None
        L.oracle_sample.argtypes = [ctypes.c_int, _f64p, ctypes.c_uint64, ctypes.c_int64, _u64p]
        L.oracle_sym_y_of_z.argtypes = [ctypes.c_int, ctypes.c_uint64]
        L.oracle_sym_y_of_z.restype = ctypes.c_uint64
        L.oracle_sym_half.argtypes = [ctypes.c_int, _f64p, _f64p]
        L.oracle_sample_sym.argtypes = [ctypes.c_int, _f64p, ctypes.c_uint64, ctypes.c_int64, _u64p]
        L.oracle_cost_histogram.argtypes = [ctypes.c_int, _f64p, _i32p, ctypes.c_int64, _u64p]
        L.oracle_adjoint.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, _f64p, _f64p,
                                     ctypes.POINTER(ctypes.c_double), _f64p, _f64p]
        L.oracle_pauli_circuit.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, _f64p, _f64p, ctypes.c_int64,
                                           _i32p, _i32p, _i32p, _f64p]
        L.oracle_noise_draws.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_int64, _i32p, _i32p, _i32p,
                                         ctypes.POINTER(ctypes.c_int64)]
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _w(w) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(w, dtype=np.int32))


def n_from_edges(m: int) -> int:
    n = int(round((1 + (1 + 8 * m) ** 0.5) / 2))
    assert n * (n - 1) // 2 == m
    return n


# --------------------------------------------------------------------------
# Cut function (eq. 6), C(x*) (eq. 5 denominator)
# --------------------------------------------------------------------------
def cost_diagonal(n: int, w) -> np.ndarray:
    """C_t[x] in tenths for all 2^n states, by the double loop of eq. (6)."""
    out = np.empty(1 << n, dtype=np.int32)
    _check(lib().oracle_cost_diagonal(n, _w(w), out), "cost_diagonal")
    return out


def cut_value(n: int, w, x: int) -> int:
    return int(lib().oracle_cut_value(n, _w(w), int(x)))


def cut_values(n: int, w, xs) -> np.ndarray:
    """C_t[x] (eq. 6) for each basis state in xs."""
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.uint64))
    out = np.empty(len(xs), dtype=np.int64)
    _check(lib().oracle_cut_values(n, _w(w), xs, len(xs), out), "cut_values")
    return out


def weight_total(w) -> int:
    w = _w(w)
    return int(lib().oracle_weight_total(n_from_edges(len(w)), w))


def cmax_direct(n: int, w) -> int:
    return int(lib().oracle_cmax_direct(n, _w(w)))


def cmax_gray(n: int, w) -> int:
    return int(lib().oracle_cmax_gray(n, _w(w)))


# --------------------------------------------------------------------------
# Simulation, <C>, sampling, gradient
# --------------------------------------------------------------------------
def simulate(n: int, w, theta_zz, theta_x, mode: int = 1) -> np.ndarray:
    """Final state (complex128) for gate angles theta_zz[k], theta_x[k].

    mode 0 applies every RZZ gate on its quadruples; mode 1 applies each
    layer's cost unitary as the diagonal exp(-i theta/2 H_C(x)) of eq. (2).
    """
    tzz = np.ascontiguousarray(theta_zz, dtype=np.float64)
    tx = np.ascontiguousarray(theta_x, dtype=np.float64)
    assert tzz.shape == tx.shape
    out = np.empty(2 << n, dtype=np.float64)
    _check(lib().oracle_simulate(n, _w(w), len(tzz), tzz, tx, mode, out), "simulate")
    return out.view(np.complex128)


def _as_c128(psi) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(psi).astype(np.complex128, copy=False))


def expect(psi, diag) -> tuple:
    """(<C> in units, normalised by the norm; norm = sum |a|^2)."""
    psi = _as_c128(psi)
    n = int(psi.size).bit_length() - 1
    e, s = ctypes.c_double(), ctypes.c_double()
    _check(lib().oracle_expect(n, psi.view(np.float64), np.ascontiguousarray(diag, dtype=np.int32),
                               ctypes.byref(e), ctypes.byref(s)), "expect")
    return e.value, s.value


def philox4x64_10(counter, key) -> np.ndarray:
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.empty(4, dtype=np.uint64)
    lib().oracle_philox4x64_10(ctr, k, out)
    return out


def sample(psi, seed: int, shots: int) -> np.ndarray:
    """Shots by the fixed-point inverse-CDF rule (see oracle.c)."""
    psi = _as_c128(psi)
    n = int(psi.size).bit_length() - 1
    out = np.empty(shots, dtype=np.uint64)
    _check(lib().oracle_sample(n, psi.view(np.float64), int(seed), int(shots), out), "sample")
    return out


def sym_y_of_z(n: int, z: int) -> int:
    """Basis state (bit n-1 clear) of complement-symmetric index z."""
    return int(lib().oracle_sym_y_of_z(n, int(z)))


def sym_half(psi) -> np.ndarray:
    """Stored half (z order) of a complement-symmetric full state."""
    p = _as_c128(psi)
    n = int(p.size).bit_length() - 1
    out = np.empty(p.size // 2, dtype=np.complex128)
    _check(lib().oracle_sym_half(n, p.view(np.float64), out.view(np.float64)), "sym_half")
    return out


def sample_sym(half, n: int, seed: int, shots: int) -> np.ndarray:
    """Shots of n-qubit basis states from a complement-symmetric half state."""
    h = _as_c128(half)
    out = np.empty(shots, dtype=np.uint64)
    _check(lib().oracle_sample_sym(n, h.view(np.float64), int(seed), int(shots), out), "sample_sym")
    return out


def cost_histogram(psi, diag, nbins: int) -> np.ndarray:
    """Fixed-point mass (2^62 = probability 1) of every cut value in tenths,
    0..nbins-1; values outside fall into the last bin."""
    p = _as_c128(psi)
    n = int(p.size).bit_length() - 1
    out = np.empty(int(nbins), dtype=np.uint64)
    _check(lib().oracle_cost_histogram(n, p.view(np.float64), np.ascontiguousarray(diag, dtype=np.int32),
                                       int(nbins), out), "cost_histogram")
    return out


def adjoint(n: int, w, theta_zz, theta_x) -> tuple:
    """(E, dE/dtheta_zz[k], dE/dtheta_x[k]) for E = <psi|C|psi>, gate by gate."""
    tzz = np.ascontiguousarray(theta_zz, dtype=np.float64)
    tx = np.ascontiguousarray(theta_x, dtype=np.float64)
    p = len(tzz)
    gzz, gx, e = np.empty(p), np.empty(p), ctypes.c_double()
    _check(lib().oracle_adjoint(n, _w(w), p, tzz, tx, ctypes.byref(e), gzz, gx), "adjoint")
    return e.value, gzz, gx


def expect_of(n: int, w, theta_zz, theta_x, mode: int = 1) -> float:
    return expect(simulate(n, w, theta_zz, theta_x, mode), cost_diagonal(n, w))[0]


def fd_gradient(n: int, w, theta_zz, theta_x, h: float = 1e-4, mode: int = 1) -> tuple:
    """Central finite differences of <C> with step h in every gate angle."""
    tzz = np.asarray(theta_zz, dtype=np.float64)
    tx = np.asarray(theta_x, dtype=np.float64)
    diag = cost_diagonal(n, w)

    def f(a, b):
        return expect(simulate(n, w, a, b, mode), diag)[0]

    gzz, gx = np.zeros(len(tzz)), np.zeros(len(tx))
    for k in range(len(tzz)):
        e = np.zeros(len(tzz)); e[k] = h
        gzz[k] = (f(tzz + e, tx) - f(tzz - e, tx)) / (2 * h)
        gx[k] = (f(tzz, tx + e) - f(tzz, tx - e)) / (2 * h)
    return gzz, gx


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# --------------------------------------------------------------------------
# Linear ramp (eq. 4) and the gate-angle conventions (eqs. 2-3)
# --------------------------------------------------------------------------
def ramp_paper(p: int, delta_gamma: float, delta_beta: float) -> tuple:
    """Eq. (4): beta_i = (1 - i/p) D_beta, gamma_i = (i+1)/p D_gamma, i = 0..p-1."""
    i = np.arange(p, dtype=np.float64)
    return (i + 1) / p * delta_gamma, (1 - i / p) * delta_beta


def ramp_midpoint(p: int, delta_gamma: float, delta_beta: float) -> tuple:
    """Midpoint form: gamma_k = (k-1/2)/p D_gamma, beta_k = (1-(k-1/2)/p) D_beta."""
    k = np.arange(1, p + 1, dtype=np.float64)
    return (k - 0.5) / p * delta_gamma, (1 - (k - 0.5) / p) * delta_beta


def gate_angles(gammas, betas, convention: str = "paper") -> tuple:
    """Map (gamma_k, beta_k) to (theta_zz, theta_x) of RZZ(theta_zz w), RX(theta_x).

    paper:   exp(-i gamma H_C) = prod RZZ(2 gamma w_ij); exp(+i beta H_B) = prod RX(-2 beta)
    literal: RZZ(gamma w_ij) and RX(2 beta) read with the standard gate definitions
    """
    g = np.asarray(gammas, dtype=np.float64)
    b = np.asarray(betas, dtype=np.float64)
    if convention == "paper":
        return 2.0 * g, -2.0 * b
    if convention == "literal":
        return g.copy(), 2.0 * b
    raise ValueError(convention)


# --------------------------------------------------------------------------
# Dense references of eqs. (1)-(3) (tiny n)
# --------------------------------------------------------------------------
def dense_hamiltonians(n: int, w) -> tuple:
    """H_C (eq. 1, units) as a diagonal vector and H_B = sum_i X_i as a dense matrix."""
    w = np.asarray(w, dtype=np.float64) / 10.0
    dim = 1 << n
    x = np.arange(dim)
    hc = np.zeros(dim)
    e = 0
    for i in range(n):
        for j in range(i + 1, n):
            zi = 1 - 2 * ((x >> i) & 1)
            zj = 1 - 2 * ((x >> j) & 1)
            hc += w[e] * zi * zj
            e += 1
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    hb = np.zeros((dim, dim))
    for q in range(n):
        # qubit q is bit q of the index: it is the q-th factor from the right
        op = np.array([[1.0]])
        for k in reversed(range(n)):
            op = np.kron(op, X if k == q else np.eye(2))
        hb += op
    return hc, hb


def dense_state(n: int, w, gammas, betas, convention: str = "paper") -> np.ndarray:
    """|psi> = prod_k U_B(beta_k) U_C(gamma_k) |+>^n with scipy's expm."""
    from scipy.linalg import expm
    hc, hb = dense_hamiltonians(n, w)
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
    for g, b in zip(gammas, betas):
        if convention == "paper":
            uc = np.exp(-1j * g * hc)                   # eq. (2)
            ub = expm(1j * b * hb)                      # eq. (3)
        else:
            uc = np.exp(-1j * (g / 2.0) * hc)           # prod RZZ(g w_ij)
            ub = expm(-1j * b * hb)                     # prod RX(2 b)
        psi = ub @ (uc * psi)
    return psi


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------
def k2_expect(w_units: float, gamma: float, beta: float, convention: str = "paper") -> float:
    """<C> for one edge (n = 2), p = 1."""
    if convention == "paper":
        return w_units / 2 + (w_units / 2) * np.sin(4 * beta) * np.sin(2 * gamma * w_units)
    return w_units / 2 - (w_units / 2) * np.sin(4 * beta) * np.sin(gamma * w_units)


def p1_expect(n: int, w, theta_zz, theta_x):
    """<C> after one layer on any complete graph, O(n^3) (Heisenberg picture).

    With a_uv = theta_zz w_uv / 2 and b = theta_x / 2:
      <Z_u Z_v> = 1/2 sin 4b sin 2a_uv (P_u + P_v) - 1/2 sin^2 2b (Q+ - Q-),
      P_u = prod_{x != u,v} cos 2a_ux,  Q(+/-) = prod_{x != u,v} cos 2(a_ux +/- a_vx),
    and <C> = sum_{u<v} w_uv (1 - <Z_u Z_v>) / 2.  Accepts complex angles so
    that complex-step differentiation works.
    """
    wu = np.asarray(w, dtype=np.float64) / 10.0
    W = np.zeros((n, n))
    e = 0
    for i in range(n):
        for j in range(i + 1, n):
            W[i, j] = W[j, i] = wu[e]
            e += 1
    a = theta_zz * W / 2.0
    b = theta_x / 2.0
    c2 = np.cos(2 * a)
    total = 0.0
    for u in range(n):
        for v in range(u + 1, n):
            mask = np.ones(n, dtype=bool)
            mask[[u, v]] = False
            Pu = np.prod(c2[u, mask])
            Pv = np.prod(c2[v, mask])
            Qp = np.prod(np.cos(2 * (a[u, mask] + a[v, mask])))
            Qm = np.prod(np.cos(2 * (a[u, mask] - a[v, mask])))
            zz = 0.5 * np.sin(4 * b) * np.sin(2 * a[u, v]) * (Pu + Pv) \
                - 0.5 * np.sin(2 * b) ** 2 * (Qp - Qm)
            total = total + W[u, v] * (1 - zz) / 2
    return total


def p1_gradient(n: int, w, theta_zz: float, theta_x: float, h: float = 1e-30) -> tuple:
    """(d<C>/dtheta_zz, d<C>/dtheta_x) of the single-layer closed form, by complex step."""
    gzz = np.imag(p1_expect(n, w, theta_zz + 1j * h, theta_x)) / h
    gx = np.imag(p1_expect(n, w, theta_zz, theta_x + 1j * h)) / h
    return float(gzz), float(gx)


def gate_counts(n: int, p: int) -> tuple:
    """(two-qubit, one-qubit) gate counts of the circuit, Sec. II-B."""
    return p * n * (n - 1) // 2, (p + 1) * n


def state_bytes_fp32(n: int) -> int:
    """Memory of an n-qubit complex single-precision state, Sec. II-E: 2^(n+3) B."""
    return 1 << (n + 3)


# --------------------------------------------------------------------------
# Noise (Sec. II-C): depolarizing channel of uniform rate eps after every
# two-qubit gate.  Trajectories apply one of the 16 two-qubit Paulis
# (uniformly) after a gate with probability eps; the density-matrix reference
# applies the channel itself.  Draw rule and Pauli codes: see oracle.c.
# --------------------------------------------------------------------------
PAULI_NAMES = "IXYZ"


def noise_threshold(eps: float) -> int:
    """thr = floor(eps * 2^53): a gate errs when (r0 >> 11) < thr."""
    eps = float(eps)
    if not 0.0 <= eps <= 1.0:
        raise ValueError("eps must lie in [0, 1]")
    return int(np.floor(eps * 2.0 ** 53))


def noise_draws(n: int, p: int, eps: float, seed: int, traj: int) -> tuple:
    """Non-identity errors of one trajectory: (layer, edge, code) arrays in
    (layer, edge) order."""
    cap = p * n * (n - 1) // 2
    lay = np.empty(max(cap, 1), dtype=np.int32)
    edg = np.empty_like(lay)
    cod = np.empty_like(lay)
    cnt = ctypes.c_int64()
    _check(lib().oracle_noise_draws(n, p, noise_threshold(eps), int(seed), int(traj), cap, lay, edg, cod,
                                    ctypes.byref(cnt)), "noise_draws")
    c = cnt.value
    return lay[:c].copy(), edg[:c].copy(), cod[:c].copy()


def pauli_circuit(n: int, w, theta_zz, theta_x, errors) -> np.ndarray:
    """Final state with Pauli error (layer, edge, code) applied right after
    that edge's RZZ gate in that layer (gate by gate, Sec. II-E)."""
    lay, edg, cod = (np.ascontiguousarray(a, dtype=np.int32) for a in errors)
    tzz = np.ascontiguousarray(theta_zz, dtype=np.float64)
    tx = np.ascontiguousarray(theta_x, dtype=np.float64)
    out = np.empty(2 << n, dtype=np.float64)
    one = np.zeros(1, dtype=np.int32)
    _check(lib().oracle_pauli_circuit(n, _w(w), len(tzz), tzz, tx, len(lay),
                                      lay if len(lay) else one, edg if len(edg) else one,
                                      cod if len(cod) else one, out), "pauli_circuit")
    return out.view(np.complex128)


def noisy_trajectory(n: int, w, theta_zz, theta_x, eps: float, seed: int, traj: int) -> tuple:
    """(final state, number of non-identity errors) of trajectory traj."""
    errs = noise_draws(n, len(theta_zz), eps, seed, traj)
    return pauli_circuit(n, w, theta_zz, theta_x, errs), len(errs[0])


def _pauli_1q(code: int) -> np.ndarray:
    return [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]),
            np.array([[1, 0], [0, -1]])][code].astype(np.complex128)


def _op_on(n: int, ops: dict) -> np.ndarray:
    """Dense operator with ops[q] on qubit q (bit q of the index), identity elsewhere."""
    m = np.array([[1.0 + 0j]])
    for q in reversed(range(n)):
        m = np.kron(m, ops.get(q, np.eye(2)))
    return m


def density_expect(n: int, w, theta_zz, theta_x, eps: float) -> float:
    """<C> (units) of the noisy circuit from its density matrix, tiny n.

    Gate by gate in lexicographic order: rho -> U rho U^+ for RZZ(theta w)
    then rho -> (1 - eps) rho + (eps / 16) sum_P P rho P over the 16 Paulis
    on the gate's two qubits; each layer ends with RX(theta_x) on every qubit.
    """
    if n > 7:
        raise ValueError("density matrix reference is for n <= 7")
    dim = 1 << n
    x = np.arange(dim)
    z = 1 - 2 * ((x[:, None] >> np.arange(n)[None, :]) & 1)
    rho = np.full((dim, dim), 1.0 / dim, dtype=np.complex128)
    wt = np.asarray(w, dtype=np.float64) / 10.0
    for k in range(len(theta_zz)):
        e = 0
        for i in range(n):
            for j in range(i + 1, n):
                d = np.exp(-1j * (theta_zz[k] * wt[e] / 2.0) * z[:, i] * z[:, j])
                rho = d[:, None] * rho * np.conj(d)[None, :]
                if eps > 0.0:
                    acc = np.zeros_like(rho)
                    for c in range(16):
                        P = _op_on(n, {i: _pauli_1q(c & 3), j: _pauli_1q(c >> 2)})
                        acc += P @ rho @ P.conj().T
                    rho = (1.0 - eps) * rho + (eps / 16.0) * acc
                e += 1
        c, s = np.cos(theta_x[k] / 2.0), np.sin(theta_x[k] / 2.0)
        rx = np.array([[c, -1j * s], [-1j * s, c]])
        M = _op_on(n, {q: rx for q in range(n)})
        rho = M @ rho @ M.conj().T
    C = cost_diagonal(n, w).astype(np.float64) / 10.0
    return float(np.real(np.sum(np.diag(rho) * C)))


def k2_noisy_expect(w_units: float, exp_noiseless: float, eps: float, p: int) -> float:
    """Two qubits, one gate per layer: the channel keeps the state's coherent
    part with weight (1 - eps) and replaces the rest by I/4, which every later
    gate and mixer leaves alone, so <C> = (1-eps)^p <C>_0 + (1 - (1-eps)^p) W/2."""
    keep = (1.0 - eps) ** p
    return keep * exp_noiseless + (1.0 - keep) * w_units / 2.0
