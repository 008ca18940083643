"""Cut-value histogram on the GPU vs the oracle's, bit for bit on the same state."""
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
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=p), rng.uniform(-1, 1, size=p)


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,p", [(1, 1), (2, 2), (5, 3), (12, 3), (13, 2), (14, 3), (20, 3), (24, 2)])
def test_histogram_bit_exact_on_same_state(n, p, precision):
    from paper_2604_26423_amd import Simulator
    say(f"histogram n={n} p={p} {precision}")
    w = workloads.complete_graph_tenths(n, 40 + n)
    s = Simulator(w, precision)
    s.forward(*angles(p, n))
    got = s.cost_histogram()
    psi = s.psi.cpu().numpy()
    diag = s.diag.cpu().numpy()
    want = oracle.cost_histogram(psi, diag, s.w_total + 1)
    assert np.array_equal(got, want)
    assert np.array_equal(s.cost_histogram(), got)                  # run to run
    dev = s.cost_histogram(on_device=True)
    assert np.array_equal(dev.cpu().numpy().view(np.uint64), got)
    # moments: total mass = 2^62 norm, mean cut = <C> (up to the floor of each q)
    e, nrm = s.expect()
    h = got.astype(np.float64)
    assert abs(h.sum() / 2.0 ** 62 - nrm) <= 1e-12 + (1 << n) * 2.0 ** -62
    if e > 0:
        assert abs((np.arange(len(h)) * h).sum() / h.sum() / 10 - e) <= 1e-12 * e
    s.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_histogram_wide_and_clipped(precision):
    """More than 8192 bins (global-atomic form) and values beyond the last bin."""
    from paper_2604_26423_amd import Simulator
    from paper_2604_26423_amd import qs
    n = 15
    w = np.random.default_rng(9).integers(1, 400, size=n * (n - 1) // 2).astype(np.int32)
    s = Simulator(w, precision)
    assert s.w_total + 1 > 8192
    s.forward(*angles(3, 1))
    psi, diag = s.psi.cpu().numpy(), s.diag.cpu().numpy()
    assert np.array_equal(s.cost_histogram(), oracle.cost_histogram(psi, diag, s.w_total + 1))
    for nb in (1, 100, 5000, 9000):
        got = qs.qs_cost_histogram(s.handle, s.diag, nb)
        assert np.array_equal(got, oracle.cost_histogram(psi, diag, nb)), nb
    s.close()


def test_histogram_uniform_state_and_errors():
    from paper_2604_26423_amd import Simulator
    from paper_2604_26423_amd import qs
    n = 18
    w = workloads.complete_graph_tenths(n, 3)
    s = Simulator(w, "c64")
    s.init_plus()
    got = s.cost_histogram()
    counts = np.bincount(s.diag.cpu().numpy(), minlength=s.w_total + 1).astype(np.uint64)
    assert np.array_equal(got, counts * np.uint64(1 << (62 - n)))
    r, prob = s.ratio_distribution()
    mu, sd, thr = __import__("paper_2604_26423_amd").mean_of_means(r, prob, 100)
    assert abs(mu - s.w_total / 2 / s.cmax) < 1e-12 and thr > mu
    with pytest.raises(qs.QSError) as ei:
        qs.qs_cost_histogram(s.handle, s.diag, 0)
    assert ei.value.status == qs.QS_ERR_ARG
    s.psi.mul_(2.0)                     # norm 4: the fixed-point total would overflow
    with pytest.raises(qs.QSError) as ei:
        s.cost_histogram()
    assert ei.value.status == qs.QS_ERR_STATE
    s.close()
