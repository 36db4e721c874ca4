"""Exact resume from a checkpoint (state, touching-pair and wall overlaps,
last forces, step count) taken right after a contact search: the resumed
context rebuilds the same sorted order and lists, so it repeats the saved
run bit for bit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Dem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_09576_amd import Dem as D
    return D


def resumed(Dem, sc, ck, precision):
    sc2 = dict(sc, particles=dict(sc["particles"], pos=ck["pos"], vel=ck["vel"],
                                  omega=ck["omega"]))
    b = Dem.from_scene(sc2, precision=precision)
    b.restore(ck)
    return b


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resume_after_search_is_bitwise_exact(Dem, precision):
    sc = W.dense_snapshot(n=2500, seed=61, polydisperse=0.2, n_types=2, K=10)
    a = Dem.from_scene(sc, precision=precision)
    a.step(100)  # ends right after the search of step 100
    ck = a.checkpoint()
    assert len(ck["pairs"]) > 100 and len(ck["wall_pairs"]) > 10
    assert np.any(ck["delta_t"] != 0) and np.any(ck["wall_delta_t"] != 0)
    b = resumed(Dem, sc, ck, precision)
    assert b.get_stats()["step"] == 100
    for chunk in (37, 113):
        a.step(chunk)
        b.step(chunk)
        sa, sb = a.get_state(), b.get_state()
        for k in ("pos", "vel", "omega"):
            assert np.array_equal(sa[k], sb[k]), k
        assert sa["time"] == sb["time"]
        Fa, Ta = a.get_forces()
        Fb, Tb = b.get_forces()
        assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb)
        pa, da, ta = a.get_contacts()
        pb, db, tb = b.get_contacts()
        assert np.array_equal(pa, pb) and np.array_equal(da, db) and np.array_equal(ta, tb)


def test_resume_on_a_rotating_drum_with_floating_wall(Dem):
    """Walls in motion and a wall that switches off later: the step count
    restores the time of the activity windows."""
    sc = W.drum_scene(n=3000, omega=2.0, seed=5, dt=1e-5, K=10)
    sc["walls"][1] = dict(sc["walls"][1], t_off=160 * 1e-5)  # one end plane opens at step 160
    a = Dem.from_scene(sc)
    a.step(120)
    ck = a.checkpoint()
    b = resumed(Dem, sc, ck, "fp64")
    a.step(100)
    b.step(100)
    assert np.array_equal(a.get_state()["pos"], b.get_state()["pos"])
    assert np.array_equal(a.get_wall_contacts()[1], b.get_wall_contacts()[1])


def test_restore_rejects_pairs_outside_the_lists(Dem):
    sc = W.dense_snapshot(n=500, seed=62, K=10)
    a = Dem.from_scene(sc)
    a.step(10)
    ck = a.checkpoint()
    bad = dict(ck, pairs=np.array([[0, 499]]), delta_t=np.zeros((1, 3)))
    b = Dem.from_scene(sc)
    with pytest.raises(Exception):
        b.restore(bad)
