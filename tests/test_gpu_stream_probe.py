"""bddmma_stream_probe: the in-place stream that bounds the updating sweep
writes a + 1 and b * 2 over every element, ragged sizes included, in both
precisions, and nothing outside the n elements it is given."""
import pytest

from paper_2111_10270_amd import binding as B

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("n", [1, 63, 64, 575, 576, 2305, 100_000])
def test_stream_probe_updates_every_element_in_place(dtype, n):
    import torch
    dt = getattr(torch, dtype)
    print(f"stream probe {dtype} n={n}", flush=True)
    # guard elements past n stay untouched
    a = torch.arange(n + 7, dtype=dt, device="cuda:0")
    b = torch.arange(n + 7, dtype=dt, device="cuda:0") - 3.5
    a0, b0 = a.clone(), b.clone()
    B.stream_probe(a[:n], b[:n])
    B.stream_probe(a[:n], b[:n])
    torch.cuda.synchronize()
    assert torch.equal(a[:n], a0[:n] + 2)
    assert torch.equal(b[:n], b0[:n] * 4)
    assert torch.equal(a[n:], a0[n:]) and torch.equal(b[n:], b0[n:])


def test_stream_probe_checks_tensors():
    import torch
    x = torch.zeros(10, dtype=torch.float32, device="cuda:0")
    with pytest.raises(ValueError):
        B.stream_probe(x, torch.zeros(10, dtype=torch.float64, device="cuda:0"))
    with pytest.raises(ValueError):
        B.stream_probe(x, torch.zeros(11, dtype=torch.float32, device="cuda:0"))
    B.stream_probe(x[:0], x[:0])   # n = 0 launches nothing
