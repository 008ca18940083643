"""GPU parity of the store mode of the adjoint (checkpointed psi,
qs_adjoint_grad_store) against the oracle's gate-by-gate adjoint and against
the uncompute mode.

Sizes span the single-workgroup path (no checkpoints), two tile passes per
circuit (the state buffer is the only checkpoint), several passes, the
complement-symmetric layout and a deep circuit where the uncompute mode's
undone passes could drift.  Tolerances as for the uncompute mode: complex128
gradients within 1e-10 of the largest component, complex64 within 1e-4.
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


def say(*a):
    print(*a, flush=True)


def rel_err(gzz, gx, rzz, rx):
    scale = max(np.abs(rzz).max(), np.abs(rx).max())
    return max(np.abs(gzz - rzz).max(), np.abs(gx - rx).max()) / scale


@pytest.mark.parametrize("precision,n,p", [("c128", 9, 3), ("c128", 14, 1), ("c128", 14, 3), ("c128", 16, 4),
                                           ("c128", 19, 2), ("c64", 14, 3), ("c64", 18, 5)])
def test_store_vs_oracle(precision, n, p):
    from paper_2604_26423_amd import Simulator
    say(f"store adjoint {precision} n={n} p={p}")
    w = workloads.complete_graph_tenths(n, 80 + n)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(p, 0.6, 0.6))
    sim = Simulator(w, precision)
    e, gzz, gx = sim.adjoint(tzz, tx, mode="store")
    e_ref, rzz, rx = oracle.adjoint(n, w, tzz, tx)
    err = rel_err(gzz, gx, rzz, rx)
    say(f"  <C> rel {abs(e - e_ref) / e_ref:.2e}, gradient rel {err:.2e}")
    tol, etol = (1e-10, 1e-12) if precision == "c128" else (1e-4, 1e-6)
    assert abs(e - e_ref) <= etol * e_ref
    assert err <= tol
    # the state buffer was not undone; a new forward recomputes psi_p
    e2, _ = sim.forward(tzz, tx)
    assert abs(e2 - e_ref) <= etol * e_ref
    sim.close()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_store_symmetric_layout_vs_oracle(precision):
    from paper_2604_26423_amd import Simulator
    n, p = 17, 3
    w = workloads.complete_graph_tenths(n, 91)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(p, 0.6, 0.6))
    s = Simulator(w, precision, symmetric=True)
    e, gzz, gx = s.adjoint(tzz, tx, mode="store")
    e_ref, rzz, rx = oracle.adjoint(n, w, tzz, tx)
    err = rel_err(gzz, gx, rzz, rx)
    say(f"store sym {precision}: gradient rel {err:.2e}")
    assert err <= (1e-10 if precision == "c128" else 1e-4)
    s.close()


def test_store_leaves_memory_past_the_checkpoints_alone():
    from paper_2604_26423_amd import Simulator
    from paper_2604_26423_amd import qs
    n, p = 20, 3
    w = workloads.complete_graph_tenths(n, 5)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(p, 0.6, 0.6))
    sim = Simulator(w, "c64")
    nb = qs.qs_adjoint_ckpt_bytes(sim.handle, p)
    sb = sim.psi.numel() * sim.psi.element_size()
    say(f"checkpoints: {nb} bytes = {nb / sb:.0f} states")
    assert nb == 2 * sb                       # 13 + 7 qubits: P = p + 1 passes, P - 2 checkpoints
    guard = 1 << 16
    buf = torch.full((nb + 2 * guard,), 0xA5, dtype=torch.uint8, device="cuda")
    lam = torch.empty_like(sim.psi)
    e, gzz, gx = qs.qs_adjoint_grad_store(sim.handle, sim.diag, sim.w_total, tzz, tx, buf[guard:guard + nb], nb,
                                          lam, sb)
    torch.cuda.synchronize()
    host = buf.cpu().numpy()
    assert (host[:guard] == 0xA5).all() and (host[guard + nb:] == 0xA5).all()
    e_u, uzz, ux = sim.adjoint(tzz, tx)
    assert rel_err(gzz, gx, uzz, ux) <= 1e-4
    sim.close()


def test_store_against_uncompute_deep_circuit():
    """p = 10 at n = 24 in complex64: both modes against each other (the
    uncompute mode undoes 20 passes on psi, the store mode none)."""
    from paper_2604_26423_amd import Simulator
    n, p = 24, 10
    w = workloads.complete_graph_tenths(n, 6)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(p, 0.6, 0.6))
    sim = Simulator(w, "c64")
    e_s, szz, sx = sim.adjoint(tzz, tx, mode="store")
    e_u, uzz, ux = sim.adjoint(tzz, tx)
    ref = Simulator(w, "c128")
    e_r, rzz, rx = ref.adjoint(tzz, tx, mode="store")
    d_store, d_unc = rel_err(szz, sx, rzz, rx), rel_err(uzz, ux, rzz, rx)
    say(f"n={n} p={p} complex64 vs complex128 store: store {d_store:.2e}, uncompute {d_unc:.2e}")
    assert abs(e_s - e_r) <= 1e-6 * e_r and abs(e_u - e_r) <= 1e-6 * e_r
    assert d_store <= 1e-4 and d_unc <= 1e-4
    sim.close()
    ref.close()
