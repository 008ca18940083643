"""Noisy trajectories (Sec. II-C) on the GPU against the oracle's gate-by-gate
circuit with the same Pauli draws: final states (global phase included),
error counts and <C> per trajectory."""
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


def angles(p, d=0.6):
    return oracle.gate_angles(*oracle.ramp_midpoint(p, d, d))


TOL = {"c64": (1e-5, 1e-6), "c128": (1e-12, 1e-12)}

CASES = [(2, 1, 0.3), (3, 2, 0.5), (4, 3, 0.25), (5, 3, 0.2), (6, 2, 0.0), (7, 2, 0.1), (8, 3, 0.05),
         (9, 2, 0.1), (10, 3, 0.02), (11, 2, 0.05), (12, 3, 0.01), (12, 2, 1.0)]


def check(tr, n, w, tzz, tx, eps, seed, traj0, ntraj, precision, sample=None):
    out = tr.run(tzz, tx, eps, seed, ntraj, traj0, states=True)
    torch.cuda.synchronize()
    st = out["states"].cpu().numpy().astype(np.complex128)
    e = out["exp_c"].cpu().numpy()
    ne = out["nerr"].cpu().numpy()
    nrm = out["norm"].cpu().numpy()
    atol, rtol = TOL[precision]
    diag = oracle.cost_diagonal(n, w)
    for i in (range(ntraj) if sample is None else sample):
        ref, rn = oracle.noisy_trajectory(n, w, tzz, tx, eps, seed, traj0 + i)
        assert ne[i] == rn, (i, ne[i], rn)
        err = np.abs(st[i] - ref).max()
        assert err <= atol, (i, err)
        er, nr = oracle.expect(ref, diag)
        assert abs(e[i] - er) <= rtol * er, (i, e[i], er)
        assert abs(nrm[i] - nr) <= atol
    return out


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,p,eps", CASES)
def test_trajectories_vs_oracle(n, p, eps, precision):
    from paper_2604_26423_amd import Trajectories
    say(f"noise n={n} p={p} eps={eps} {precision}")
    w = workloads.complete_graph_tenths(n, 300 + n)
    tzz, tx = angles(p)
    tr = Trajectories(w, precision)
    ntraj = 12 if n <= 10 else 5
    check(tr, n, w, tzz, tx, eps, 77 + n, 1000 * n, ntraj, precision)
    tr.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_noise_free_trajectory_is_the_noiseless_state(precision):
    from paper_2604_26423_amd import Trajectories
    n = 10
    w = workloads.complete_graph_tenths(n, 5)
    tzz, tx = angles(4)
    tr = Trajectories(w, precision)
    out = tr.run(tzz, tx, 0.0, 1, 3, states=True)
    ref = oracle.simulate(n, w, tzz, tx, 0)
    st = out["states"].cpu().numpy().astype(np.complex128)
    assert np.abs(st - ref[None, :]).max() <= TOL[precision][0]
    assert int(out["nerr"].sum()) == 0
    tr.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_direct_form_mixer(precision):
    """|cos(theta_x / 2)| < 1/2 in one layer: the kernel uses the direct RX form."""
    from paper_2604_26423_amd import Trajectories
    n, p, eps = 9, 3, 0.08
    w = workloads.complete_graph_tenths(n, 6)
    tzz = np.array([0.3, 0.9, -0.4])
    tx = np.array([2.6, -0.7, 3.0])
    tr = Trajectories(w, precision)
    check(tr, n, w, tzz, tx, eps, 11, 0, 8, precision)
    tr.close()


def test_many_layers_cross_draw_chunks():
    """p = 70 spans three chunks of error draws."""
    from paper_2604_26423_amd import Trajectories
    n, p, eps = 6, 70, 0.03
    w = workloads.complete_graph_tenths(n, 7)
    tzz, tx = angles(p, 0.9)
    tr = Trajectories(w, "c64")
    check(tr, n, w, tzz, tx, eps, 12, 5, 6, "c64")
    tr.close()


def test_full_size_sampled():
    """The benchmark shape (n = 12, p = 10, 4096 trajectories): sampled
    trajectories against the oracle, error counts against their expectation,
    and every norm 1."""
    from paper_2604_26423_amd import Trajectories
    n, p, eps, ntraj = 12, 10, 0.005, 4096
    w = workloads.complete_graph_tenths(n, 12)
    tzz, tx = angles(p)
    tr = Trajectories(w, "c64")
    out = check(tr, n, w, tzz, tx, eps, 2024, 0, ntraj, "c64", sample=[0, 1, 2047, 4095])
    ne = out["nerr"].cpu().numpy()
    g = p * n * (n - 1) // 2
    mean = ntraj * g * eps * 15 / 16
    assert abs(ne.sum() - mean) < 5 * np.sqrt(mean)
    assert np.abs(out["norm"].cpu().numpy() - 1).max() < 1e-4
    tr.close()


def test_trajectory_mean_matches_density_matrix():
    """Mean over many GPU trajectories vs the oracle's density matrix."""
    from paper_2604_26423_amd import Trajectories
    n, p, eps = 5, 2, 0.15
    w = workloads.complete_graph_tenths(n, 9)
    tzz, tx = angles(p)
    tr = Trajectories(w, "c128")
    e = tr.run(tzz, tx, eps, 31, 20000)["exp_c"].cpu().numpy()
    dm = oracle.density_expect(n, w, tzz, tx, eps)
    assert abs(e.mean() - dm) < 5 * e.std() / np.sqrt(len(e))
    tr.close()
