"""The library's stream copy (the HBM ceiling the sweep passes are compared
with) copies exactly, for lengths that are not whole workgroups of vectors."""
import numpy as np
import pytest

from paper_1206_6152_amd._lib import vp_stream_copy

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [0, 16, 48, 4096 + 16 * 37, (1 << 22) + 16 * 255])
def test_stream_copy_is_exact(nbytes):
    import torch
    print("case", nbytes, flush=True)
    n = nbytes // 4
    src = torch.from_numpy(np.random.default_rng(nbytes).standard_normal(n + 8).astype(np.float32)).to("cuda:0")
    dst = torch.full((n + 8,), -1.0, dtype=torch.float32, device="cuda:0")
    vp_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out, ref = dst.cpu().numpy(), src.cpu().numpy()
    assert np.array_equal(out[:n], ref[:n])
    assert np.all(out[n:] == -1.0)            # nothing past the range is written
