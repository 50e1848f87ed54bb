"""The library's stream copy (the HBM ceiling the sweep passes are compared
with) copies exactly, for lengths that are not whole workgroups of vectors and for
one (4 GiB and up) that takes more than one round of the capped grid."""
import pytest

from paper_1206_6152_amd._lib import vp_stream_copy

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [0, 16, 48, 4096 + 16 * 37, (1 << 22) + 16 * 255, (1 << 32) + 16 * 3])
def test_stream_copy_is_exact(nbytes):
    import torch
    print("case", nbytes, flush=True)
    n = nbytes // 4
    gen = torch.Generator(device="cuda:0").manual_seed(nbytes % 1000003)
    src = torch.rand(n + 8, generator=gen, dtype=torch.float32, device="cuda:0")
    dst = torch.full((n + 8,), -1.0, dtype=torch.float32, device="cuda:0")
    vp_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src[:n])
    assert bool((dst[n:] == -1.0).all())      # nothing past the range is written
    del src, dst
    torch.cuda.empty_cache()
