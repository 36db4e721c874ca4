"""dem_get_contacts_device: the candidate pairs written to device buffers
equal those of dem_get_contacts (same pairs, tangential overlaps and touching
flags; only the order differs: spatial instead of gid order), on a dense
polydisperse bed after steps (histories non-zero), on one instance of a
batch, and with the capacity rule."""
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


def device_pairs(torch, g, instance=0):
    m = g.count_contacts_device(instance)
    pairs = torch.full((max(m, 1), 2), -1, dtype=torch.int64, device="cuda")
    dt = torch.full((max(m, 1), 3), np.nan, dtype=torch.float64, device="cuda")
    touch = torch.full((max(m, 1),), 7, dtype=torch.uint8, device="cuda")
    n = g.get_contacts_device(max(m, 1), pairs.data_ptr(), dt.data_ptr(), touch.data_ptr(),
                              instance=instance)
    assert n == m
    return pairs[:m].cpu().numpy(), dt[:m].cpu().numpy(), touch[:m].cpu().numpy().astype(bool)


def same_as_host(torch, g, instance=0):
    dp, dd, dtch = device_pairs(torch, g, instance)
    hp, hd, htch = g.get_contacts(instance)
    assert dp.shape == hp.shape
    order = np.lexsort((dp[:, 1], dp[:, 0]))
    assert np.array_equal(dp[order], hp)
    assert np.array_equal(dd[order], hd)  # bitwise: the same stored values
    assert np.array_equal(dtch[order], htch)
    return len(hp), int(np.count_nonzero(hd.any(axis=1)))


def test_device_pairs_equal_host_pairs(torch_dem):
    torch, Dem = torch_dem
    g = Dem.from_scene(W.dense_snapshot(n=3000, seed=3, polydisperse=0.05, overlap=0.03, K=7))
    g.step(12)
    n, with_hist = same_as_host(torch, g)
    print("pairs", n, "with history", with_hist, flush=True)
    assert n > 5000 and with_hist > 1000


def test_device_pairs_of_one_instance_of_a_batch(torch_dem):
    torch, Dem = torch_dem
    scenes = [W.dense_snapshot(n=n, seed=s, K=5) for n, s in ((700, 1), (1200, 2), (65, 3))]
    g = Dem.from_scenes(scenes)
    g.step(6)
    for b in range(3):
        n, _ = same_as_host(torch, g, b)
        assert n > 0


def test_device_pairs_capacity_rule(torch_dem):
    torch, Dem = torch_dem
    from paper_2106_09576_amd.dem import DemError
    g = Dem.from_scene(W.dense_snapshot(n=500, seed=4))
    m = g.count_contacts_device()
    assert m > 0
    pairs = torch.full((m, 2), -5, dtype=torch.int64, device="cuda")
    with pytest.raises(DemError):
        g.get_contacts_device(m - 1, pairs.data_ptr())
    assert bool((pairs == -5).all())  # nothing written
    assert g.get_contacts_device(m, pairs.data_ptr()) == m
