"""The `run` subcommand of the package's command line on the GPU, against the oracle."""
import io
import json
from contextlib import redirect_stdout

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_run_prints_the_oracle_values():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_26423_amd import __main__ as cli
    buf = io.StringIO()
    with redirect_stdout(buf):
        rc = cli.main(["run", "--n", "12", "--seed", "0", "--p", "3", "--precision", "c128", "--shots", "1000",
                       "--adjoint", "store"])
    assert rc == 0
    out = json.loads(buf.getvalue().strip().splitlines()[-1])
    w = workloads.complete_graph_tenths(12, 0)
    tzz, tx = oracle.gate_angles(*oracle.ramp_midpoint(3, 0.6, 0.6))
    e_ref, rzz, rx = oracle.adjoint(12, w, tzz, tx)
    assert abs(out["exp_c"] - e_ref) <= 1e-12 * e_ref
    assert abs(out["r_exact"] - e_ref / (oracle.cmax_direct(12, w) / 10)) <= 1e-12
    # paper convention: theta_zz = 2 gamma, theta_x = -2 beta
    assert np.allclose(out["d_gamma"], 2 * rzz, atol=1e-10) and np.allclose(out["d_beta"], -2 * rx, atol=1e-10)
    assert set(out["ms"]) == {"setup_and_cost_diagonal", "forward", "sample", "forward_plus_adjoint"}
