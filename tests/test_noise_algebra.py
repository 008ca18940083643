"""The noisy-trajectory kernel moves each layer's Pauli errors to the end of
its fused cost layer: X components flip the sign of later gates on their
qubit (a list F of flipped gates corrects the fused phase), the X part of the
product becomes a frame m (psi_true = i^phi X^m psi_stored) that commutes with
the mixer, and Z components become signs.  This CPU model of that algebra,
written with numpy (no GPU code), must reproduce the oracle's literal
gate-by-gate circuit with the same Pauli insertions."""
import numpy as np
import pytest

import oracle
import workloads


def popc(v):
    return bin(int(v)).count("1")


def commuted_trajectory(n, w, tzz, tx, errors):
    lay, edg, cod = errors
    dim = 1 << n
    x = np.arange(dim)
    C = oracle.cost_diagonal(n, w).astype(np.int64)
    W = int(np.sum(w))
    edges = [(i, j) for i in range(n) for j in range(i + 1, n)]
    psi = np.full(dim, 2.0 ** (-n / 2), dtype=np.complex128)
    m, phi = 0, 0
    parity = np.vectorize(lambda v, mk: popc(v & mk) & 1)
    for k in range(len(tzz)):
        codes = np.zeros(len(edges), dtype=int)
        for L, E, c in zip(lay, edg, cod):
            if L == k:
                codes[E] = c
        before, ez, ph, F = 0, 0, 0, []
        for e, (a, b) in enumerate(edges):
            c = int(codes[e])
            pa, pb = c & 3, c >> 2
            xm = (int(pa in (1, 2)) << a) | (int(pb in (1, 2)) << b)
            zm = (int(pa >= 2) << a) | (int(pb >= 2) << b)
            if popc(before & ((1 << a) | (1 << b))) & 1:
                F.append(((1 << a) | (1 << b), int(w[e])))
            ph += int(pa == 2) + int(pb == 2) + 2 * (popc(zm & before) & 1)
            ez ^= zm
            before ^= xm
        ex = before
        y = x ^ m
        wf = sum(wt for _, wt in F)
        cf = np.zeros(dim, dtype=np.int64)
        for mk, wt in F:
            cf += wt * parity(y, mk)
        K = (W - 2 * C[y]) - 2 * (wf - 2 * cf)
        sign = np.where(parity(x, ez) == 1, -1.0, 1.0)
        psi = psi * np.exp(-1j * tzz[k] * K / 20.0) * sign
        phi = (phi + ph + 2 * (popc(ez & m) & 1)) & 3
        m ^= ex
        c_, s_ = np.cos(tx[k] / 2), np.sin(tx[k] / 2)
        for q in range(n):
            lo = x[(x >> q) & 1 == 0]
            hi = lo | (1 << q)
            a0, a1 = psi[lo].copy(), psi[hi].copy()
            psi[lo] = c_ * a0 - 1j * s_ * a1
            psi[hi] = -1j * s_ * a0 + c_ * a1
    out = np.empty(dim, dtype=np.complex128)
    out[x ^ m] = (1j ** phi) * psi
    return out


@pytest.mark.parametrize("n,p,eps", [(3, 2, 0.5), (4, 3, 0.3), (5, 2, 0.6), (6, 2, 1.0)])
def test_commuted_errors_reproduce_the_literal_circuit(n, p, eps):
    w = workloads.complete_graph_tenths(n, 40 + n)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(p, 0.7, 0.7))
    for t in range(12):
        errs = oracle.noise_draws(n, p, eps, 5, t)
        got = commuted_trajectory(n, w, tzz, tx, errs)
        ref = oracle.pauli_circuit(n, w, tzz, tx, errs)
        assert np.abs(got - ref).max() < 1e-12


def test_every_single_pauli_at_every_position():
    n = 4
    w = workloads.complete_graph_tenths(n, 3)
    tzz, tx = np.array([0.8, 0.5]), np.array([0.6, 0.9])
    g = n * (n - 1) // 2
    for layer in range(2):
        for e in range(g):
            for code in range(1, 16):
                errs = ([layer], [e], [code])
                got = commuted_trajectory(n, w, tzz, tx, errs)
                ref = oracle.pauli_circuit(n, w, tzz, tx, errs)
                assert np.abs(got - ref).max() < 1e-12, (layer, e, code)
