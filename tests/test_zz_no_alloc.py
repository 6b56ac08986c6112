"""The allocation-free transform (fsd_fft3d_noalloc) against fsd_fft3d, through the C ABI.

Two calls in a row on the same GPU, the second with a smaller grid, each compared with the
allocating entry point on the same input; sizes past the fixed twiddle array are refused.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F(gpu):
    import paper_2607_25161_amd as F
    return F


def _noalloc(F, torch, a, sign):
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    stream = torch.cuda.current_stream()
    F.fft3d_noalloc(a.shape[0], sign, t.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("sign", [-1, 1])
def test_noalloc_matches_fft3d_twice(F, sign):
    import torch
    rng = np.random.default_rng(7 + sign)
    for n in (80, 24):  # the second call is smaller: the twiddles of the first must not leak in
        a = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
        ref = F.fft3d(a, sign)
        out = _noalloc(F, torch, a, sign)
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max(), n


def test_noalloc_refuses_sizes_past_its_array(F):
    import torch
    t = torch.zeros(2 * 8, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FsdError) as e:
        F.fft3d_noalloc(1024, -1, t.data_ptr())
    assert "512" in str(e.value)
    with pytest.raises(F.FsdError):
        F.fft3d_noalloc(7, -1, t.data_ptr())
