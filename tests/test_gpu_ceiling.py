"""The measured-ceiling helpers compute nothing of the patterns, but the copy
that the bench's HBM ceiling comes from must move every byte: byte-exact
copies at sizes below one workgroup's block, across ragged block counts, and at
a size that spans many blocks; misaligned sizes are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


@pytest.mark.parametrize("nbytes", [16, 4096 - 16, 4096, 4096 + 48, 3 * 4096 + 16, 1 << 20, (1 << 24) + 4096 + 32])
def test_copy_moves_every_byte(rise, nbytes):
    import torch

    g = np.random.default_rng(nbytes)
    src_h = g.integers(0, 256, size=nbytes, dtype=np.uint8)
    src = torch.from_numpy(src_h).cuda()
    # the destination is larger than the copy and pre-filled: bytes past the end stay
    dst = torch.full((nbytes + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    rise.rise_ceiling_copy(dst[:nbytes], src)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    assert np.array_equal(out[:nbytes], src_h)
    assert np.all(out[nbytes:] == 0xA5)


def test_copy_rejects_ragged_sizes(rise):
    import torch

    src = torch.zeros(40, dtype=torch.uint8, device="cuda")
    dst = torch.zeros(40, dtype=torch.uint8, device="cuda")
    with pytest.raises(rise.RiseError, match="16-byte"):
        rise.rise_ceiling_copy(dst, src)
