"""The read-only stream probe reads every 16-byte chunk exactly once: the XOR
of its sink equals the XOR of all 32-bit words of the buffer."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
sk = pytest.importorskip("paper_1808_10365_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("nbytes,wgs", [(16, 1), (4096 * 16, 3), (1 << 20, 64), ((1 << 22) + 48, 1000)])
def test_read_probe_reads_every_chunk_once(nbytes, wgs):
    rng = np.random.default_rng(nbytes + wgs)
    x = rng.integers(0, 256, size=nbytes, dtype=np.uint8)
    xd = torch.from_numpy(x).to(DEV)
    sink = torch.zeros(wgs * 256, dtype=torch.int32, device=DEV)
    sk.read_probe(xd, wgs, sink)
    torch.cuda.synchronize()
    got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))
    want = np.bitwise_xor.reduce(x.view(np.uint32))
    assert got == want


def test_read_probe_rejects_ragged_size():
    xd = torch.zeros(40, dtype=torch.uint8, device=DEV)
    sink = torch.zeros(256, dtype=torch.int32, device=DEV)
    with pytest.raises(sk.SKError):
        sk.read_probe(xd, 1, sink)
