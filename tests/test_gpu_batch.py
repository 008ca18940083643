"""Batched forward + adjoint (one persistent launch) vs the single-circuit GPU
path and the CPU oracle, on uneven circuits."""
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


SMALL = [(14, 1), (14, 3), (15, 2), (16, 3), (17, 5), (19, 2), (20, 3), (16, 1)]


def angles_for(p, seed):
    rng = np.random.default_rng(seed)
    dg, db = rng.uniform(0.2, 1.0, size=2)
    return oracle.gate_angles(*oracle.ramp_midpoint(p, dg, db))


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_batch_matches_single_and_oracle(precision):
    from paper_2604_26423_amd import Batch, Simulator
    inst = [(workloads.complete_graph_tenths(n, 300 + i), p) for i, (n, p) in enumerate(SMALL)]
    ang = [angles_for(p, i) for i, (n, p) in enumerate(SMALL)]
    say(f"batch of {len(SMALL)} circuits, {precision}")
    b = Batch(inst, precision)
    e, gzz, gx = b.forward_grad([a[0] for a in ang], [a[1] for a in ang])
    for i, ((n, p), (w, _)) in enumerate(zip(SMALL, inst)):
        sim = Simulator(w, precision)
        es, szz, sx = sim.adjoint(*ang[i])
        sim.close()
        assert b.w_total[i] == oracle.weight_total(w)
        scale = max(np.abs(szz).max(), np.abs(sx).max())
        tol = 1e-10 if precision == "c128" else 2e-5
        assert abs(e[i] - es) <= tol * abs(es), (i, e[i], es)
        assert np.abs(gzz[i] - szz).max() <= tol * scale and np.abs(gx[i] - sx).max() <= tol * scale
        if n <= 16:
            er, rzz, rx = oracle.adjoint(n, w, *ang[i])
            assert b.cmax[i] == oracle.cmax_direct(n, w)
            tol_o = 1e-10 if precision == "c128" else 1e-4
            sc = max(np.abs(rzz).max(), np.abs(rx).max())
            assert abs(e[i] - er) <= max(tol_o, 1e-6) * er
            assert np.abs(gzz[i] - rzz).max() <= tol_o * sc and np.abs(gx[i] - rx).max() <= tol_o * sc
    # a second run with other angles reuses the batch
    ang2 = [angles_for(p, 100 + i) for i, (n, p) in enumerate(SMALL)]
    e2, _, _ = b.forward_grad([a[0] for a in ang2], [a[1] for a in ang2])
    sim = Simulator(inst[3][0], precision)
    assert abs(e2[3] - sim.adjoint(*ang2[3])[0]) <= (1e-10 if precision == "c128" else 2e-5) * e2[3]
    sim.close()
    b.close()


def test_full_uneven_batch():
    """The 512-circuit workload: n ~ U{14..22}, p in {3,5,10}, slopes ~ U[0.2,1]."""
    import time
    from paper_2604_26423_amd import Batch, Simulator
    items = workloads.batch()
    inst = [(it.weights(), it.p) for it in items]
    ang = [oracle.gate_angles(*oracle.ramp_midpoint(it.p, it.delta_gamma, it.delta_beta)) for it in items]
    say(f"512-circuit batch: {sum(1 << it.n for it in items) / 1e6:.0f}M amplitudes")
    b = Batch(inst, "c64")
    t0 = time.perf_counter()
    e, gzz, gx = b.forward_grad([a[0] for a in ang], [a[1] for a in ang])
    say(f"  first run {time.perf_counter() - t0:.3f} s")
    e_again, gzz2, _ = b.forward_grad([a[0] for a in ang], [a[1] for a in ang])
    assert np.array_equal(e, e_again) and all(np.array_equal(a, c) for a, c in zip(gzz, gzz2))
    assert np.all(np.isfinite(e))
    for i in range(len(items)):
        assert 0 <= e[i] <= b.w_total[i] / 10
    # The batched kernel runs 512-thread tiles, the single-circuit forward
    # 256-thread ones: the same arithmetic in a different rounding order, so
    # the two complex64 results agree to the complex64 gradient accuracy
    # (1e-4 of the largest component, as against the FP64 oracle).
    rng = np.random.default_rng(0)
    for i in sorted(rng.choice(len(items), size=16, replace=False)):
        sim = Simulator(inst[i][0], "c64")
        es, szz, sx = sim.adjoint(*ang[i])
        sim.close()
        scale = max(np.abs(szz).max(), np.abs(sx).max())
        assert abs(e[i] - es) <= 2e-5 * es
        assert np.abs(gzz[i] - szz).max() <= 1e-4 * scale and np.abs(gx[i] - sx).max() <= 1e-4 * scale
    b.close()


def test_full_batch_c128_vs_oracle_and_c64_vs_c128():
    """The 512-circuit workload in both precisions.  The complex128 batch is
    pinned to the FP64 oracle on 36 circuits, four of each size n = 14..22
    (<C> from the oracle's state, the gradient from its gate-by-gate adjoint
    on the smallest-depth circuit of each size), which covers every pass
    geometry of the batch (8 down to 4 carrier bits).  Every complex64
    circuit is then held to the complex128 one: <C> within 5e-7 relative and
    the gradient within 3e-5 of its largest component (measured: 5.3e-8 and
    2.4e-6 at most, medians 1.5e-9 and 2.9e-7)."""
    from paper_2604_26423_amd import Batch
    items = workloads.batch()
    inst = [(it.weights(), it.p) for it in items]
    ang = [oracle.gate_angles(*oracle.ramp_midpoint(it.p, it.delta_gamma, it.delta_beta)) for it in items]
    out = {}
    for prec in ("c128", "c64"):
        say(f"512-circuit batch, {prec}")
        b = Batch(inst, prec)
        out[prec] = b.forward_grad([a[0] for a in ang], [a[1] for a in ang])
        cmax = list(b.cmax)
        b.close()
    e128, gzz128, gx128 = out["c128"]
    picked = []
    for n in range(14, 23):
        of_n = [i for i, it in enumerate(items) if it.n == n]
        assert len(of_n) >= 4, n
        picked += of_n[:4]
        i = min(of_n, key=lambda j: items[j].p)
        say(f"  oracle adjoint: circuit {i}, n={n}, p={items[i].p}")
        er, rzz, rx = oracle.adjoint(n, inst[i][0], *ang[i])
        sc = max(np.abs(rzz).max(), np.abs(rx).max())
        assert abs(e128[i] - er) <= 1e-12 * er
        assert np.abs(gzz128[i] - rzz).max() <= 1e-10 * sc and np.abs(gx128[i] - rx).max() <= 1e-10 * sc
    for i in picked:
        it = items[i]
        ref = oracle.simulate(it.n, inst[i][0], *ang[i], mode=1)
        er, _ = oracle.expect(ref, oracle.cost_diagonal(it.n, inst[i][0]))
        assert abs(e128[i] - er) <= 1e-12 * er, (i, it.n, e128[i], er)
        assert cmax[i] == oracle.cmax_direct(it.n, inst[i][0])
    e64, gzz64, gx64 = out["c64"]
    e_err = np.abs(np.asarray(e64) - np.asarray(e128)) / np.asarray(e128)
    g_err = np.array([max(np.abs(a - c).max(), np.abs(b - d).max()) / max(np.abs(c).max(), np.abs(d).max())
                      for a, b, c, d in zip(gzz64, gx64, gzz128, gx128)])
    say(f"  complex64 vs complex128 over 512 circuits: <C> max {e_err.max():.2e} median {np.median(e_err):.2e}; "
        f"gradient max {g_err.max():.2e} median {np.median(g_err):.2e}")
    for i in np.argsort(g_err)[-3:]:
        it = items[i]
        say(f"    circuit {i}: n={it.n} p={it.p} D=({it.delta_gamma:.3f}, {it.delta_beta:.3f}) gradient error "
            f"{g_err[i]:.2e}, largest component {max(np.abs(gzz128[i]).max(), np.abs(gx128[i]).max()):.3e}")
    assert e_err.max() <= 5e-7
    assert g_err.max() <= 3e-5
