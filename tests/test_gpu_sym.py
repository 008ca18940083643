"""Complement-symmetric layout (QS_SYM) on the GPU against the oracle's full
state, mapped to the stored half by the oracle's own index map."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)


def angles(p, seed):
    return oracle.gate_angles(*oracle.ramp_midpoint(p, 0.3 + 0.1 * (seed % 5), 0.7 - 0.05 * (seed % 4)))


def half_of_int(n, a):
    """Oracle map of an integer array over 2^n states to the stored half."""
    return oracle.sym_half(np.asarray(a, dtype=np.float64).astype(np.complex128)).real.astype(np.int64)


CASES = [(14, 1), (14, 3), (15, 2), (16, 3), (18, 4), (20, 3), (22, 2)]


def with_precisions(cases):
    """Each case in both precisions, except complex64 below n = 15 (the
    complex64 half-state layout needs n >= 15)."""
    return [(*c, prec) for prec in ("c64", "c128") for c in cases if not (prec == "c64" and c[0] < 15)]


@pytest.mark.parametrize("n,p,precision", with_precisions(CASES))
def test_sym_forward_vs_oracle(n, p, precision):
    from paper_2604_26423_amd import Simulator
    say(f"sym forward n={n} p={p} {precision}")
    w = workloads.complete_graph_tenths(n, 500 + n)
    s = Simulator(w, precision, symmetric=True)
    diag_full = oracle.cost_diagonal(n, w)
    assert np.array_equal(s.diagonal().cpu().numpy().astype(np.int64), half_of_int(n, diag_full))
    assert s.cmax == int(diag_full.max())
    tzz, tx = angles(p, n)
    e, nrm = s.forward(tzz, tx)
    ref = oracle.simulate(n, w, tzz, tx)
    half = oracle.sym_half(ref)
    got = s.amplitudes().cpu().numpy().astype(np.complex128)
    tol = 1e-12 if precision == "c128" else 1e-5
    assert np.abs(got - half).max() <= tol
    er, nr = oracle.expect(ref, diag_full)
    assert abs(nrm - nr) <= (1e-12 if precision == "c128" else 1e-5)
    assert abs(e - er) <= (1e-12 if precision == "c128" else 1e-6) * er
    full = s.full_state().cpu().numpy().astype(np.complex128)
    assert np.abs(full - ref).max() <= tol
    s.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_sym_separate_ops(precision):
    from paper_2604_26423_amd import Simulator
    n = 17
    w = workloads.complete_graph_tenths(n, 3)
    s = Simulator(w, precision, symmetric=True)
    tzz, tx = [0.41, -0.9], [1.1, 0.35]
    s.init_plus()
    for a, b in zip(tzz, tx):
        s.apply_cost_layer(a)
        s.apply_mixer(b)
    half = oracle.sym_half(oracle.simulate(n, w, tzz, tx))
    tol = 1e-12 if precision == "c128" else 1e-5
    assert np.abs(s.amplitudes().cpu().numpy().astype(np.complex128) - half).max() <= tol
    s.close()


# one precision is enough for the multi-chunk case (n = 28)
@pytest.mark.parametrize("n,shots,precision", [(15, 5000, "c64"), (20, 20000, "c64"), (28, 30000, "c64"),
                                               (15, 5000, "c128"), (20, 20000, "c128")])
def test_sym_sampling_bit_exact_on_same_state(n, shots, precision):
    from paper_2604_26423_amd import Simulator
    say(f"sym sampling n={n} {precision}")
    w = workloads.complete_graph_tenths(n, 60 + n)
    s = Simulator(w, precision, symmetric=True)
    s.forward(*angles(3, n))
    got = s.sample(shots, 1234 + n)
    want = oracle.sample_sym(s.amplitudes().cpu().numpy(), n, 1234 + n, shots)
    assert np.array_equal(got, want)
    dev = s.sample(shots, 1234 + n, on_device=True)
    assert np.array_equal(dev.cpu().numpy().astype(np.uint64), want)
    assert int(got.max()) < (1 << n) and (got >> np.uint64(n - 1)).any()  # both halves drawn
    s.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_sym_histogram_equals_full(precision):
    from paper_2604_26423_amd import Simulator
    n = 19
    w = workloads.complete_graph_tenths(n, 8)
    s = Simulator(w, precision, symmetric=True)
    s.forward(*angles(3, 2))
    full = s.full_state().cpu().numpy()
    got = s.cost_histogram()
    want = oracle.cost_histogram(full, oracle.cost_diagonal(n, w), s.w_total + 1)
    assert np.array_equal(got, want)
    s.close()


@pytest.mark.parametrize("n,p,precision", with_precisions([(14, 2), (16, 3), (19, 2)]))
def test_sym_adjoint_vs_oracle(n, p, precision):
    from paper_2604_26423_amd import Simulator
    say(f"sym adjoint n={n} p={p} {precision}")
    w = workloads.complete_graph_tenths(n, 70 + n)
    tzz, tx = angles(p, n + 1)
    s = Simulator(w, precision, symmetric=True)
    e, gzz, gx = s.adjoint(tzz, tx)
    er, rzz, rx = oracle.adjoint(n, w, tzz, tx)
    scale = max(np.abs(rzz).max(), np.abs(rx).max())
    tol = 1e-10 if precision == "c128" else 1e-4
    assert abs(e - er) <= max(tol, 1e-6) * er
    assert np.abs(gzz - rzz).max() <= tol * scale and np.abs(gx - rx).max() <= tol * scale
    s.close()
