"""The bandwidth probes behind the bench's context figures (through the C ABI):
the copy probe copies exactly, and the read probe's per-block XOR digests combine
to the XOR of every 16-byte word of the buffer (bit-exact integer work)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def asq():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1411_2223_amd as m

    m.load()
    return m


@pytest.mark.parametrize("nbytes", [16, 16 * 1000 + 16 * 7, 1 << 24, (1 << 26) + 48])
def test_copy_and_read_probes(asq, nbytes):
    import torch

    rng = np.random.default_rng(nbytes)
    host = rng.integers(0, 2**32, size=nbytes // 4, dtype=np.uint64).astype(np.uint32)
    src = torch.from_numpy(host.view(np.uint8).copy()).cuda()
    dst = torch.zeros_like(src)
    asq.check(asq.asq_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, 0), "asq_copy_probe")
    nblk = asq.asq_read_probe_blocks(nbytes)
    sink = torch.zeros(nblk * 16, dtype=torch.uint8, device="cuda")
    asq.check(asq.asq_read_probe(src.data_ptr(), nbytes, sink.data_ptr(), 0), "asq_read_probe")
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    words = host.reshape(-1, 4)
    want = np.bitwise_xor.reduce(words, axis=0)
    got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32).reshape(-1, 4), axis=0)
    assert np.array_equal(got, want)


def test_probes_reject_misaligned(asq):
    import torch

    src = torch.zeros(64, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(16, dtype=torch.uint8, device="cuda")
    assert asq.asq_read_probe(src.data_ptr(), 17, sink.data_ptr(), 0) == asq.ASQ_EINVAL
    assert asq.asq_read_probe(src.data_ptr() + 8, 16, sink.data_ptr(), 0) == asq.ASQ_EINVAL
    assert asq.asq_copy_probe(sink.data_ptr(), src.data_ptr(), 24, 0) == asq.ASQ_EINVAL
