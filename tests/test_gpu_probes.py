"""The probe kernels of include/qs_probe.h do the work they claim: the
streaming kinds move the data unchanged, and the two mixer-window kernels
(butterflies and FP32 matrix cores) both compute K^m x for every group of 16
amplitudes, K the four-qubit tangent-form RX, against numpy."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def window_matrix(u, m):
    k1 = np.array([[1.0, -1j * u], [-1j * u, 1.0]])
    k = np.kron(np.kron(k1, k1), np.kron(k1, k1))
    return np.linalg.matrix_power(k, m)


@pytest.mark.parametrize("kind", ["window_valu", "window_mfma"])
@pytest.mark.parametrize("n,windows", [(12, 1), (12, 3), (14, 5)])
def test_window_probe_against_numpy(kind, n, windows):
    from paper_2604_26423_amd import qs
    rng = np.random.default_rng(n + windows)
    x0 = (rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)).astype(np.complex64) * 0.5
    y0 = (rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)).astype(np.complex64) * 0.5
    a = torch.as_tensor(x0).cuda()
    b = torch.as_tensor(y0).cuda()
    reps = 2
    ms, by = qs.qs_bandwidth_probe(qs.PROBE_KINDS[kind], a, b, 8 << n, reps=reps, n=n, windows=windows,
                                   stream=torch.cuda.current_stream())
    assert by == 4 * (8 << n) and ms > 0
    K = window_matrix(qs.PROBE_WINDOW_U, windows * (reps + 1))
    for got, x in ((a, x0), (b, y0)):
        want = (x.astype(np.complex128).reshape(-1, 16) @ K.T).reshape(-1)
        err = np.abs(got.cpu().numpy().astype(np.complex128) - want).max() / np.abs(want).max()
        print(f"{kind} n={n} windows={windows}: relative error {err:.2e}", flush=True)
        assert err <= 1e-5


def test_streaming_probes_move_data_unchanged():
    from paper_2604_26423_amd import qs
    nb = 64 << 20
    src = torch.arange(nb // 4, dtype=torch.int32, device="cuda").view(torch.complex64)
    dst = torch.zeros_like(src)
    st = torch.cuda.current_stream()
    for flags in (0, qs.QS_PROBE_NT_LOAD | qs.QS_PROBE_NT_STORE):
        dst.zero_()
        qs.qs_bandwidth_probe(qs.QS_PROBE_COPY, dst, src, nb, reps=1, flags=flags, stream=st)
        assert torch.equal(dst.view(torch.int32), src.view(torch.int32))
        vals = torch.randn(nb // 8, dtype=torch.complex64, device="cuda")
        upd = vals.clone()
        qs.qs_bandwidth_probe(qs.QS_PROBE_UPDATE, upd, None, nb, reps=1, flags=flags, stream=st)  # a = 1 * a
        assert torch.equal(upd, vals)
