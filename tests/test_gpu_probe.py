"""The streaming probe used to measure the practical bandwidth ceiling of
the step kernels' access mixes: its values on every built mix in both tile
orders (a ragged n, so the last block is partial) and its rejection of a
mix that is not built and of an unknown order."""
import pytest

pytestmark = pytest.mark.gpu

MIXES = [(19, 18), (19, 21), (23, 20), (39, 42), (44, 40)]


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("reads,writes", MIXES)
def test_stream_probe_values(reads, writes, order):
    import torch
    from paper_1908_03876_amd import abi
    n = 1000
    inp = torch.arange(1, reads + 1, dtype=torch.float32, device="cuda").repeat_interleave(n)
    out = torch.full((writes * n,), -1.0, dtype=torch.float32, device="cuda")
    abi.mrt_stream_probe(reads, writes, inp, out, n, order=order)
    torch.cuda.synchronize()
    want = reads * (reads + 1) / 2.0
    got = out.view(writes, n).cpu()
    for w in range(writes):
        assert torch.all(got[w] == want + w), w


def test_stream_probe_rejects_unbuilt_mix():
    import torch
    from paper_1908_03876_amd import abi
    a = torch.zeros(8, device="cuda")
    with pytest.raises(abi.MrtError):
        abi.mrt_stream_probe(3, 2, a, a, 2)
    with pytest.raises(abi.MrtError):
        abi.mrt_stream_probe(19, 18, a, a, 0, order=2)
