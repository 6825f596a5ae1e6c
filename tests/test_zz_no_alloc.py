"""The allocation-free forward of the warm-start network (hpr_mlp_forward_device) against the
allocating one (hpr_mlp_forward), through the C interface on torch-owned device arrays: equal
bit for bit on two calls in a row, the second with fewer rows, for a network whose rows span
several chunks of the fixed device scratch and for the warm-start network's shape."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2510_10891_amd import mlp  # noqa: E402
from paper_2510_10891_amd.hprlp import HPR_ERR_INVALID, HprError  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    # (layer widths, rows of the first call, rows of the second call)
    ([4096, 4096, 4096, 8], 3000, 1000),   # 1,360 rows per scratch chunk: 3 chunks, then 1
    ([12, 256, 256, 4], 5000, 37),         # the warm-start network's shape; a ragged second call
]


@pytest.mark.parametrize("sizes,n1,n2", CASES, ids=["wide-3-chunks", "warmstart-shape"])
def test_device_forward_equals_the_allocating_forward(sizes, n1, n2):
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    net = mlp.MLP(sizes, mlp.init_params(sizes, seed=3), stream=stream.cuda_stream)
    rng = np.random.default_rng(11)
    X1 = rng.standard_normal((n1, sizes[0])).astype(np.float32)
    X2 = rng.standard_normal((n2, sizes[0])).astype(np.float32)
    x1, x2 = torch.from_numpy(X1).to(dev), torch.from_numpy(X2).to(dev)
    y1 = torch.full((n1, sizes[-1]), np.nan, dtype=torch.float32, device=dev)
    y2 = torch.full((n2, sizes[-1]), np.nan, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    free_before, _ = torch.cuda.mem_get_info(dev)
    net.forward_device(x1.data_ptr(), n1, y1.data_ptr())
    net.forward_device(x2.data_ptr(), n2, y2.data_ptr())
    torch.cuda.synchronize()
    free_after, _ = torch.cuda.mem_get_info(dev)
    # the host-array forward allocates its own activation buffers (after the measurement)
    ref1, ref2 = net.forward(X1), net.forward(X2)
    got1, got2 = y1.cpu().numpy(), y2.cpu().numpy()
    assert np.isfinite(ref1).all() and np.isfinite(ref2).all()
    assert np.array_equal(got1, ref1), np.abs(got1 - ref1).max()
    assert np.array_equal(got2, ref2), np.abs(got2 - ref2).max()
    # no device memory was taken by the two calls (an allocation of the activations would
    # take n * (sizes[0] + 2 * 256..4096) * 2 bytes, megabytes here)
    assert free_before - free_after < (1 << 20), (free_before, free_after)


def test_device_forward_rejects_bad_arguments():
    net = mlp.MLP([4, 16, 2], mlp.init_params([4, 16, 2]))
    with pytest.raises(HprError) as e:
        net.forward_device(0, 5, 0)
    assert e.value.code == HPR_ERR_INVALID
    with pytest.raises(HprError):
        net.forward_device(0, -1, 0)
    net.forward_device(0, 0, 0)   # no rows: nothing to do
