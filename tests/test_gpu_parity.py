"""GPU parity of libqs against the CPU oracle, element by element.

Sizes span the single-workgroup path (n <= 13 / 12), tile passes with one and
two strided passes, passes with more than 8 carrier bits (n = 14..17 in
complex64), the per-element phase path (W_t >= 8192) and ragged shapes.
Tolerances: cost diagonal and shots bit-exact; complex64 amplitudes max-abs
<= 1e-5 and <C> within 1e-6 relative; complex128 within 1e-12 (both sides are
FP64 with different rounding order).
"""
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
    from paper_2604_26423_amd import qs
    qs.lib()


def sim_for(w, precision):
    from paper_2604_26423_amd import Simulator
    return Simulator(w, precision)


def say(*a):
    print(*a, flush=True)


def host_state(sim):
    torch.cuda.synchronize()
    return sim.amplitudes().cpu().numpy()


# ---------------------------------------------------------------- diagonal
@pytest.mark.parametrize("n", [1, 2, 3, 7, 12, 13, 14, 17, 20, 22])
def test_cost_diagonal_bit_exact(n):
    say(f"diag n={n}")
    w = workloads.complete_graph_tenths(n, 100 + n)
    sim = sim_for(w, "c64")
    got = sim.diagonal().cpu().numpy()
    want = oracle.cost_diagonal(n, w)
    assert np.array_equal(got, want)
    assert sim.w_total == oracle.weight_total(w)
    assert sim.cmax == (int(want.max()) if n > 1 else 0)
    sim.close()


def test_cost_diagonal_large_weights():
    n = 16
    w = np.random.default_rng(3).integers(0, 1 << 20, size=n * (n - 1) // 2).astype(np.int32)
    sim = sim_for(w, "c64")
    assert np.array_equal(sim.diagonal().cpu().numpy(), oracle.cost_diagonal(n, w))
    assert sim.cmax == oracle.cmax_direct(n, w)
    sim.close()


def test_k12_config_vs_oracle():
    """The 12-qubit configuration (K12, seed 0, p = 3, D = 0.6, complex128):
    amplitudes, <C>, brute-force C(x*), r and 1,000 shots against the oracle."""
    run = workloads.SMALL
    n, w = run.n, run.weights()
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(run.p, run.delta_gamma, run.delta_beta))
    sim = sim_for(w, "c128")
    e, nrm = sim.forward(tzz, tx)
    psi = host_state(sim)
    ref = oracle.simulate(n, w, tzz, tx, mode=0)
    e_ref, n_ref = oracle.expect(ref, oracle.cost_diagonal(n, w))
    cmax = oracle.cmax_direct(n, w)
    assert np.abs(psi - ref).max() <= 1e-12
    assert abs(e - e_ref) <= 1e-12 * e_ref and abs(nrm - 1) <= 1e-12
    assert sim.cmax == cmax and abs(sim.ratio(e) - e_ref / (cmax / 10)) <= 1e-12
    shots = sim.sample(run.shots, run.seed)
    assert np.array_equal(shots, oracle.sample(psi, run.seed, run.shots))
    say(f"K12: <C> {e:.12f}, r {sim.ratio(e):.9f}, r_shots {sim.shots_ratio(shots):.4f}")
    sim.close()


# ---------------------------------------------------------------- forward
CASES = [(2, 1), (5, 3), (12, 3), (13, 2), (14, 3), (15, 4), (17, 1), (18, 3), (20, 4), (22, 2), (24, 3)]


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,p", CASES)
def test_forward_amplitudes(n, p, precision):
    say(f"forward n={n} p={p} {precision}")
    w = workloads.complete_graph_tenths(n, 7 * n + p)
    g, b = oracle.ramp_midpoint(p, 0.6, 0.6)
    tzz, tx = oracle.gate_angles(g, b)
    sim = sim_for(w, precision)
    e, nrm = sim.forward(tzz, tx)
    psi = host_state(sim)
    ref = oracle.simulate(n, w, tzz, tx, mode=1)
    e_ref, _ = oracle.expect(ref, oracle.cost_diagonal(n, w))
    err = np.abs(psi - ref).max()
    l2 = np.linalg.norm(psi - ref)
    say(f"  max-abs {err:.3e}  L2 {l2:.3e}  <C> rel {abs(e - e_ref) / e_ref:.3e}  norm-1 {nrm - 1:.3e}")
    if precision == "c64":
        assert err <= 1e-5 and l2 <= 1e-5
        assert abs(e - e_ref) <= 1e-6 * abs(e_ref)
        assert abs(nrm - 1) < 1e-5
    else:
        assert err <= 1e-12
        assert abs(e - e_ref) <= 1e-12 * abs(e_ref)
    sim.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("wmax,levels", [(2, 1), (300, 3), (1 << 20, 5)])
def test_forward_random_angles_and_weight_ranges(precision, wmax, levels):
    """Phase tables of 1, 3 and 5 levels (W_t < 128, < 2^19, < 2^31) and arbitrary angles."""
    n, p = 16, 3
    w = np.random.default_rng(5).integers(0, wmax, size=n * (n - 1) // 2).astype(np.int32)
    W = int(w.sum())
    assert (levels == 1 and W < 128) or (levels == 3 and 8192 <= W < 1 << 19) or (levels == 5 and W >= 1 << 25)
    tzz, tx = workloads.random_angles(p, 9, scale=2.5)
    if levels == 5:
        tzz = tzz * 1e-4   # keep the phases of order one for such large cuts
    sim = sim_for(w, precision)
    e, _ = sim.forward(tzz, tx)
    ref = oracle.simulate(n, w, tzz, tx, mode=1)
    tol = 1e-5 if precision == "c64" else 1e-12
    assert np.abs(host_state(sim) - ref).max() <= tol
    sim.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,p", [(14, 3), (17, 2), (21, 4), (24, 3)])
def test_cut_in_registers_and_from_the_diagonal_bit_identical(n, p, precision):
    """The tile passes either evaluate C_t in registers from the weights the
    diagonal encodes or read the diagonal; both give the same integers, so the
    state, <C> and the gradients (both adjoint modes) must agree bit for bit.
    (The diagonal path is held to the oracle by the tests above.)"""
    from paper_2604_26423_amd import qs
    w = workloads.complete_graph_tenths(n, 3 * n + p)
    g, b = oracle.ramp_midpoint(p, 0.6, 0.6)
    tzz, tx = oracle.gate_angles(g, b)
    sim = sim_for(w, precision)
    res = {}
    for mode in ("diagonal", "registers"):
        qs.qs_debug_set_cut_mode(sim.handle, mode)
        e, nrm = sim.forward(tzz, tx)
        psi = sim.amplitudes().clone()
        grads = [sim.adjoint(tzz, tx, mode=m) for m in ("uncompute", "store")]
        res[mode] = (e, nrm, psi, grads)
    (e0, n0, p0, g0), (e1, n1, p1, g1) = res["diagonal"], res["registers"]
    assert e0 == e1 and n0 == n1
    assert torch.equal(p0.view(torch.float32 if precision == "c64" else torch.float64),
                       p1.view(torch.float32 if precision == "c64" else torch.float64))
    for a, b in zip(g0, g1):
        assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    sim.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_diagonal_that_is_not_a_cut_is_read_entry_by_entry(precision):
    """The tile passes evaluate C_t from the weights a cut diagonal encodes; a
    diagonal that is not a cut function (here C_t + 1, nonzero at x = 0) must
    be read entry by entry instead.  Each layer's phase exp(-i theta (W - 2C)/20)
    then gains exp(i theta / 10), so the state gains exp(i sum(theta_zz) / 10),
    <C> grows by 0.1 and the gradients are unchanged."""
    n, p = 18, 3
    w = workloads.complete_graph_tenths(n, 4)
    g, b = oracle.ramp_midpoint(p, 0.6, 0.6)
    tzz, tx = oracle.gate_angles(g, b)
    sim = sim_for(w, precision)
    from paper_2604_26423_amd import qs
    qs.qs_debug_set_cut_mode(sim.handle, "registers")   # the in-register path at this size too
    e0, _ = sim.forward(tzz, tx)
    psi0 = host_state(sim)
    ea0, gzz0, gx0 = sim.adjoint(tzz, tx)
    sim.diag += 1
    e1, _ = sim.forward(tzz, tx)
    psi1 = host_state(sim)
    ea1, gzz1, gx1 = sim.adjoint(tzz, tx)
    tol = 1e-5 if precision == "c64" else 1e-12
    err = np.abs(psi1 - np.exp(1j * np.sum(tzz) / 10) * psi0).max() / np.abs(psi0).max()
    scale = max(np.abs(gzz0).max(), np.abs(gx0).max())
    gerr = max(np.abs(gzz1 - gzz0).max(), np.abs(gx1 - gx0).max()) / scale
    say(f"  amplitudes rel {err:.2e}, <C> shift {e1 - e0:.12f}, gradient rel {gerr:.2e}")
    assert err <= tol
    assert abs(e1 - e0 - 0.1) <= tol * e0 and abs(ea1 - ea0 - 0.1) <= tol * e0
    assert gerr <= (1e-4 if precision == "c64" else 1e-10)
    sim.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n", [11, 16, 21])
def test_separate_ops_match_oracle(n, precision):
    """qs_init_plus, qs_apply_cost_layer, qs_apply_mixer one by one."""
    say(f"ops n={n} {precision}")
    w = workloads.complete_graph_tenths(n, n)
    tzz, tx = workloads.random_angles(2, n, scale=1.2)
    sim = sim_for(w, precision)
    sim.init_plus()
    for k in range(2):
        sim.apply_cost_layer(tzz[k])
        sim.apply_mixer(tx[k])
    ref = oracle.simulate(n, w, tzz, tx, mode=0)
    tol = 1e-5 if precision == "c64" else 1e-12
    assert np.abs(host_state(sim) - ref).max() <= tol
    e, nrm = sim.expect()
    e_ref, _ = oracle.expect(ref, oracle.cost_diagonal(n, w))
    assert abs(e - e_ref) <= (1e-6 if precision == "c64" else 1e-12) * e_ref
    sim.close()


def test_p0_and_mixer_invariants():
    n = 18
    w = workloads.complete_graph_tenths(n, 1)
    sim = sim_for(w, "c128")
    e, nrm = sim.forward([], [])
    assert abs(e - sim.w_total / 20) < 1e-10 and abs(nrm - 1) < 1e-12
    sim.forward([0.0, 0.0], [0.7, -0.4])   # mixer on |+>: global phase exp(-i n sum(theta)/2)
    psi = host_state(sim)
    assert np.abs(psi - 2 ** (-n / 2) * np.exp(-1j * n * 0.3 / 2)).max() < 1e-13
    sim.close()


def test_z2_symmetry_and_determinism():
    n = 20
    w = workloads.complete_graph_tenths(n, 4)
    g, b = oracle.ramp_midpoint(5, 0.7, 0.5)
    tzz, tx = oracle.gate_angles(g, b)
    sim = sim_for(w, "c64")
    e1, n1 = sim.forward(tzz, tx)
    psi1 = host_state(sim).copy()
    e2, n2 = sim.forward(tzz, tx)
    assert e1 == e2 and n1 == n2
    assert np.array_equal(psi1, host_state(sim))
    # Z2 symmetry psi[x] = psi[~x]: exact in exact arithmetic; the GPU's fused
    # multiply-adds round the two members of a pair differently
    x = np.arange(1 << n)
    assert np.abs(psi1 - psi1[(~x) & ((1 << n) - 1)]).max() <= 1e-6 * np.abs(psi1).max()
    sim.close()


# ---------------------------------------------------------------- degenerate inputs
@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_single_qubit_without_edges(precision):
    """n = 1: no edges, so W_t = 0 and the cost layer of eq. (2) is the
    identity; each mixer layer (eq. (3)) multiplies |+> by exp(-i theta_x / 2).
    Layer 2's angle takes the direct (non-tangent) RX.  The adjoint needs an
    edge and refuses."""
    from paper_2604_26423_amd import qs
    w = np.zeros(0, dtype=np.int32)
    tzz, tx = np.array([0.4, -1.1, 0.9]), np.array([0.7, 2.9, -0.3])
    sim = sim_for(w, precision)
    assert sim.n == 1 and sim.w_total == 0 and sim.cmax == 0
    e, nrm = sim.forward(tzz, tx)
    psi = host_state(sim)
    tol = 1e-6 if precision == "c64" else 1e-15
    assert np.abs(psi - 2 ** -0.5 * np.exp(-0.5j * tx.sum())).max() <= tol
    assert np.abs(psi - oracle.simulate(1, w, tzz, tx, mode=1)).max() <= tol
    assert e == 0.0 and abs(nrm - 1) <= 10 * tol
    assert np.array_equal(sim.sample(1000, 3), oracle.sample(psi, 3, 1000))
    with pytest.raises(qs.QSError) as ei:
        sim.adjoint(tzz, tx)
    assert ei.value.status == qs.QS_ERR_ARG
    sim.close()


@pytest.mark.parametrize("n,precision", [(16, "c64"), (16, "c128"), (28, "c64")])
def test_zero_weights(n, precision):
    """All weights zero: C(x) = 0 for every x, so the circuit multiplies |+>^n
    by the global phase exp(-i n sum(theta_x) / 2), <C> = 0, lambda = 0 at the
    turnaround and every gradient component is exactly zero.  At n = 28 the
    tile passes evaluate C_t in registers from the weights recovered from the
    (all-zero) diagonal."""
    w = np.zeros(n * (n - 1) // 2, dtype=np.int32)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(3, 0.6, 0.6))
    sim = sim_for(w, precision)
    assert sim.w_total == 0 and sim.cmax == 0
    e, nrm = sim.forward(tzz, tx)
    amp = 2 ** (-n / 2) * np.exp(-0.5j * n * np.sum(tx))
    rel = 2e-5 if precision == "c64" else 1e-12
    dev = torch.abs(sim.psi - torch.tensor(amp, dtype=sim.psi.dtype, device=sim.psi.device)).max().item()
    say(f"  zero weights n={n} {precision}: max-abs {dev:.2e} (amplitude {abs(amp):.2e}), norm - 1 {nrm - 1:.2e}")
    assert dev <= rel * abs(amp) and e == 0.0 and abs(nrm - 1) <= rel
    if n <= 20:
        assert np.abs(host_state(sim) - oracle.simulate(n, w, tzz, tx, mode=1)).max() <= rel * abs(amp)
    for mode in ("uncompute", "store"):
        ea, gzz, gx = sim.adjoint(tzz, tx, mode=mode)
        assert ea == 0.0 and np.all(np.asarray(gzz) == 0.0) and np.all(np.asarray(gx) == 0.0), mode
    sim.close()


# ---------------------------------------------------------------- sampling
@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,shots", [(3, 500), (12, 1000), (13, 3000), (14, 5000), (20, 10000), (27, 20000)])
def test_sampling_bit_exact_on_same_state(n, shots, precision):
    """GPU sampler vs oracle sampler on the GPU's own state: identical shots."""
    say(f"sample n={n} shots={shots} {precision}")
    w = workloads.complete_graph_tenths(n, n)
    g, b = oracle.ramp_midpoint(3, 0.6, 0.6)
    sim = sim_for(w, precision)
    sim.forward(*oracle.gate_angles(g, b), readout=False)
    got = sim.sample(shots, seed=n)
    want = oracle.sample(host_state(sim), n, shots)
    assert np.array_equal(got, want)
    again = sim.sample(shots, seed=n)
    assert np.array_equal(got, again)
    dev = sim.sample(shots, seed=n, on_device=True).cpu().numpy().view(np.uint64)
    assert np.array_equal(dev, got)
    sim.close()


def test_sampling_c128_path_vs_oracle_state():
    """c128 GPU circuit vs the oracle's own state: mismatches only at CDF boundaries."""
    n, shots, seed = 14, 100000, 0
    w = workloads.complete_graph_tenths(n, 0)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(3, 0.6, 0.6))
    sim = sim_for(w, "c128")
    sim.forward(tzz, tx, readout=False)
    got = sim.sample(shots, seed)
    ref = oracle.simulate(n, w, tzz, tx, mode=1)
    want = oracle.sample(ref, seed, shots)
    mism = np.nonzero(got != want)[0]
    say(f"  mismatched shots: {len(mism)} of {shots}")
    if len(mism):
        q = lambda psi: np.floor((psi.real.astype(np.float64) ** 2 + psi.imag ** 2) * 2.0 ** 62).astype(np.uint64)
        Fg = np.cumsum(q(host_state(sim)).astype(object))
        Fo = np.cumsum(q(ref).astype(object))
        dF = max(abs(int(a) - int(b)) for a, b in zip(Fg, Fo))
        T = int(Fo[-1])
        for s in mism:
            r = int(oracle.philox4x64_10([int(s), 0, 0, 0], [seed, 0])[0])
            u = r * T >> 64
            x = int(want[s])
            assert min(abs(u - int(Fo[x])), abs(u - (int(Fo[x - 1]) if x else 0))) <= dF + 2
    assert len(mism) <= 5
    sim.close()


def test_sampling_delta_state_and_zero_state():
    from paper_2604_26423_amd import qs
    n = 15
    w = workloads.complete_graph_tenths(n, 2)
    sim = sim_for(w, "c64")
    delta = torch.zeros_like(sim.psi)
    delta[12345] = 1j
    sim.set_amplitudes(delta)
    assert np.all(sim.sample(300, 1) == 12345)
    sim.psi.zero_()
    with pytest.raises(qs.QSError) as ei:
        sim.sample(10, 1)
    assert ei.value.status == qs.QS_ERR_STATE
    sim.psi.fill_(1.0)   # norm 2^15: |a|^2 sums far above 4
    with pytest.raises(qs.QSError) as ei:
        sim.sample(10, 1)
    assert ei.value.status == qs.QS_ERR_STATE
    sim.close()


# ---------------------------------------------------------------- gradient
@pytest.mark.parametrize("n,p", [(2, 2), (4, 1), (9, 3), (12, 2), (13, 3), (14, 3), (16, 4), (19, 2)])
def test_adjoint_c128_vs_oracle(n, p):
    say(f"adjoint n={n} p={p}")
    w = workloads.complete_graph_tenths(n, 50 + n)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(p, 0.6, 0.6))
    sim = sim_for(w, "c128")
    e, gzz, gx = sim.adjoint(tzz, tx)
    e_ref, rzz, rx = oracle.adjoint(n, w, tzz, tx)
    scale = max(np.abs(rzz).max(), np.abs(rx).max())
    say(f"  E {e:.12f} vs {e_ref:.12f}; grad err {max(np.abs(gzz - rzz).max(), np.abs(gx - rx).max()) / scale:.2e}")
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)
    assert np.abs(gzz - rzz).max() <= 1e-10 * scale
    assert np.abs(gx - rx).max() <= 1e-10 * scale
    sim.close()


# n = 14, 18: junctions whose stages end in one-bit windows; n = 19: a
# junction of two-bit last windows; n = 20: three-bit (the generic kernel)
@pytest.mark.parametrize("n,p", [(2, 2), (9, 3), (14, 3), (18, 5), (19, 3), (20, 2)])
def test_adjoint_c64_vs_oracle(n, p):
    w = workloads.complete_graph_tenths(n, 60 + n)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(p, 0.6, 0.6))
    sim = sim_for(w, "c64")
    e, gzz, gx = sim.adjoint(tzz, tx)
    e_ref, rzz, rx = oracle.adjoint(n, w, tzz, tx)
    scale = max(np.abs(rzz).max(), np.abs(rx).max())
    err = max(np.abs(gzz - rzz).max(), np.abs(gx - rx).max()) / scale
    say(f"  c64 n={n}: <C> rel {abs(e - e_ref) / e_ref:.2e}, gradient rel {err:.2e}")
    assert abs(e - e_ref) <= 1e-6 * abs(e_ref)
    # measured 0.8e-7 .. 5.3e-7 over these cases
    assert err <= 5e-6
    sim.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("mode", ["uncompute", "store"])
def test_adjoint_large_angles_general_stage_code(precision, mode):
    """Mixer angles with |cos(theta_x / 2)| < 1/2 in some layers: those passes
    take the general (non-tangent) stage code in both directions."""
    n, p = 16, 4
    w = workloads.complete_graph_tenths(n, 33)
    tzz = np.array([0.3, -0.7, 0.5, 0.2])
    tx = np.array([2.6, -0.4, -2.9, 1.1])          # |tx / 2| > pi / 3 in layers 0 and 2
    assert (np.abs(np.cos(tx / 2)) < 0.5).sum() == 2
    sim = sim_for(w, precision)
    e, gzz, gx = sim.adjoint(tzz, tx, mode=mode)
    e_ref, rzz, rx = oracle.adjoint(n, w, tzz, tx)
    scale = max(np.abs(rzz).max(), np.abs(rx).max())
    err = max(np.abs(gzz - rzz).max(), np.abs(gx - rx).max()) / scale
    say(f"  {precision} {mode}: <C> rel {abs(e - e_ref) / e_ref:.2e}, gradient rel {err:.2e}")
    tol, etol = (1e-4, 1e-6) if precision == "c64" else (1e-10, 1e-12)
    assert abs(e - e_ref) <= etol * e_ref and err <= tol
    sim.close()


def test_adjoint_vs_finite_differences_then_forward_again():
    n, p = 15, 3
    w = workloads.complete_graph_tenths(n, 77)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(p, 0.8, 0.4))
    sim = sim_for(w, "c128")
    e, gzz, gx = sim.adjoint(tzz, tx)
    fzz, fx = oracle.fd_gradient(n, w, tzz, tx, h=1e-4)
    assert np.abs(gzz - fzz).max() <= 1e-6 * max(1, np.abs(fzz).max())
    assert np.abs(gx - fx).max() <= 1e-6 * max(1, np.abs(fx).max())
    # the reverse sweep overwrites the state; a new forward recomputes psi_p
    e2, _ = sim.forward(tzz, tx)
    assert abs(e2 - e) <= 1e-12 * e
    assert np.abs(host_state(sim) - oracle.simulate(n, w, tzz, tx)).max() <= 1e-12
    sim.close()


@pytest.mark.parametrize("n,mode", [(10, "uncompute"), (15, "store")])
def test_autograd_function(n, mode):
    from paper_2604_26423_amd import expect_c
    p = 3
    w = workloads.complete_graph_tenths(n, 3)
    sim = sim_for(w, "c128")
    gam = torch.tensor([0.1, 0.3, 0.5], dtype=torch.float64, requires_grad=True)
    bet = torch.tensor([0.5, 0.3, 0.1], dtype=torch.float64, requires_grad=True)
    e = expect_c(gam, bet, sim, "paper", mode)
    e.backward()
    tzz, tx = oracle.gate_angles(gam.detach().numpy(), bet.detach().numpy(), "paper")
    e_ref, rzz, rx = oracle.adjoint(n, w, tzz, tx)
    assert abs(e.item() - e_ref) < 1e-12
    assert np.allclose(gam.grad.numpy(), 2 * rzz, atol=1e-11)
    assert np.allclose(bet.grad.numpy(), -2 * rx, atol=1e-11)
    sim.close()
