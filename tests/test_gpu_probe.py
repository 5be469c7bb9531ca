"""The streaming measurement pass (fps_probe_stream) computes c = a + b
exactly, including ragged lengths, and rejects misaligned arrays."""
import pytest

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 1, 2, 3, 1023, 2048, 2049, 1 << 20, (1 << 20) + 5])
def test_probe_stream_sums(n):
    g = torch.Generator(device="cpu").manual_seed(n)
    a = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    b = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    c = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    print(f"probe_stream n={n}", flush=True)
    fps.probe_stream(a, b, c)
    torch.cuda.synchronize()
    assert torch.equal(c, a + b)


def test_probe_stream_rejects_misaligned():
    a = torch.zeros(17, dtype=torch.float64, device="cuda")
    with pytest.raises(fps.FpsError):
        fps.probe_stream(a[1:], a[1:], torch.empty(16, dtype=torch.float64, device="cuda"))
