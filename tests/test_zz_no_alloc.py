"""dem_get_contacts_device_noalloc, the variant of dem_get_contacts_device
for callers that cannot allocate: its workspace is a file-scope device array
of the library.  Two calls in a row, the second on a smaller context, each
against the allocating entry point's output (bitwise, same order)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_09576_amd import Dem
    return torch, Dem


def _fetch(torch, g, noalloc):
    m = g.count_contacts_device()
    pairs = torch.full((max(m, 1), 2), -1, dtype=torch.int64, device="cuda")
    dt = torch.full((max(m, 1), 3), np.nan, dtype=torch.float64, device="cuda")
    touch = torch.full((max(m, 1),), 7, dtype=torch.uint8, device="cuda")
    fn = g.get_contacts_device_noalloc if noalloc else g.get_contacts_device
    n = fn(max(m, 1), pairs.data_ptr(), dt.data_ptr(), touch.data_ptr())
    assert n == m
    return pairs[:m].cpu().numpy(), dt[:m].cpu().numpy(), touch[:m].cpu().numpy()


@pytest.mark.parametrize("n", [3000, 500])
def test_noalloc_contacts_equal_allocating_entry_point(torch_dem, n):
    torch, Dem = torch_dem
    g = Dem.from_scene(W.dense_snapshot(n=n, seed=n, polydisperse=0.3, K=7))
    g.step(9)
    a = _fetch(torch, g, noalloc=False)
    b = _fetch(torch, g, noalloc=True)
    assert len(a[0]) > n
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    g.close()
