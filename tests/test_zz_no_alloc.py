"""qs_cost_diagonal_noalloc (scratch in the library's static device array, no
device allocation) against qs_cost_diagonal, through the C ABI: identical
diagonals, W_t and C(x*), on two calls in a row, the second smaller."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_noalloc_cost_diagonal_matches_allocating_entry_point():
    from paper_2604_26423_amd import qs
    st = torch.cuda.current_stream()
    # the largest size first, then a smaller one: the second call must not
    # see anything the first one left in the shared array
    for n, seed in ((27, 5), (17, 6), (9, 7)):
        print(f"noalloc diagonal n={n}", flush=True)
        w = workloads.complete_graph_tenths(n, seed)
        a = torch.empty(1 << n, dtype=torch.int32, device="cuda")
        b = torch.full((1 << n,), -1, dtype=torch.int32, device="cuda")
        Wa, ca = qs.qs_cost_diagonal(n, w, a, st)
        Wb, cb = qs.qs_cost_diagonal_noalloc(n, w, b, st)
        assert (Wa, ca) == (Wb, cb)
        assert torch.equal(a, b)
        assert int(b.max()) == cb
    with pytest.raises(qs.QSError) as ei:
        qs.qs_cost_diagonal_noalloc(35, np.ones(35 * 34 // 2, dtype=np.int32), a, st)
    assert ei.value.status == qs.QS_ERR_ARG
