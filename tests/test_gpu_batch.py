"""Batched instances: several independent simulations in one context.

Each instance of a batch must give exactly what it gives alone (the sorted
order inside an instance, hence every summation order, is the same), and
match the FP64 oracle run on that instance's scene.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_from_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Dem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_09576_amd import Dem as D
    return D


def small_drums(k=5, seed=11):
    return W.batched_drums(n_inst=k, n_min=300, n_max=3000, seed=seed, dt=1e-5, K=10)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_instances_equal_single_runs_bitwise(Dem, precision):
    scenes = small_drums()
    batch = Dem.from_scenes(scenes, precision=precision)
    batch.step(120)
    for k, sc in enumerate(scenes):
        one = Dem.from_scene(sc, precision=precision)
        one.step(120)
        a, b = batch.get_state(k), one.get_state()
        assert np.array_equal(a["pos"], b["pos"]), k
        assert np.array_equal(a["vel"], b["vel"]), k
        assert np.array_equal(a["omega"], b["omega"]), k
        pa, da, ta = batch.get_contacts(k)
        pb, db, tb = one.get_contacts()
        assert np.array_equal(pa, pb) and np.array_equal(da, db) and np.array_equal(ta, tb)
        wa, wda = batch.get_wall_contacts(k)
        wb, wdb = one.get_wall_contacts()
        assert np.array_equal(wa, wb) and np.array_equal(wda, wdb)
        Fa, Ta = batch.get_forces(k)
        Fb, Tb = one.get_forces()
        assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb)
        one.close()


def test_batch_instances_match_oracle(Dem):
    scenes = small_drums(k=4, seed=5)
    batch = Dem.from_scenes(scenes)
    batch.step(100)
    for k, sc in enumerate(scenes):
        o = oracle_from_scene(sc)
        o.step(100)
        gp, gd, gt = batch.get_contacts(k)
        op, od, ot = o.contacts()
        assert np.array_equal(gp, op) and np.array_equal(gt, ot), k
        assert np.max(np.abs(gd - od), initial=0.0) <= 1e-9 * (np.max(np.abs(od), initial=0) + 1e-300)
        gw, _ = batch.get_wall_contacts(k)
        ow, _ = o.wall_contacts()
        assert np.array_equal(gw, ow), k
        Fg, _ = batch.get_forces(k)
        Fo, _, S = o.forces()
        err = np.max(np.linalg.norm(Fg - Fo, axis=1) / (np.linalg.norm(Fo, axis=1) + S + 1e-300))
        assert err <= 1e-9, (k, err)
        dx = np.max(np.abs(batch.get_state(k)["pos"] - o.state()["pos"]))
        assert dx <= 1e-12, (k, dx)


def test_batch_with_empty_and_single_particle_instances(Dem):
    scenes = small_drums(k=3, seed=2)
    empty = dict(scenes[0])
    empty["particles"] = W._particles(np.zeros((0, 3)), np.zeros(0))
    single = dict(scenes[1])
    single["particles"] = {k: v[:1] for k, v in scenes[1]["particles"].items()}
    batch = Dem.from_scenes([empty, scenes[2], single])
    batch.step(50)
    assert batch.get_state(0)["pos"].shape == (0, 3)
    o = oracle_from_scene(scenes[2])
    o.step(50)
    assert np.max(np.abs(batch.get_state(1)["pos"] - o.state()["pos"])) <= 1e-12
    o1 = oracle_from_scene(single)
    o1.step(50)
    assert np.max(np.abs(batch.get_state(2)["pos"] - o1.state()["pos"])) <= 1e-15


def test_batch_of_256_uneven_drums_runs_and_sampled_instances_match(Dem):
    scenes = W.batched_drums(n_inst=256, n_min=200, n_max=5000, seed=4, dt=5e-6, K=20)
    batch = Dem.from_scenes(scenes, precision="fp32")
    batch.step(60)
    st = batch.get_stats()
    assert st["n_particles"] == sum(s["particles"]["pos"].shape[0] for s in scenes)
    for k in (0, 97, 255):
        o = oracle_from_scene(scenes[k])
        o.step(60)
        gp, _, gt = batch.get_contacts(k)
        op, _, ot = o.contacts()
        assert np.array_equal(gp, op) and np.array_equal(gt, ot), k
        d = 2 * scenes[k]["particles"]["radius"][0]
        assert np.max(np.abs(batch.get_state(k)["pos"] - o.state()["pos"])) <= 1e-6 * d


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_dynamic_search_with_different_skins(Dem, precision):
    """Dynamic search in a batch whose instances have different particle
    sizes, hence different skins: each instance still follows the oracle
    searching at every step, and equals its own single dynamic run."""
    scenes = [W.drum_scene(n=n, d=d, omega=om, seed=s, dt=1e-5, K=0)
              for n, d, om, s in ((900, 3e-3, 2.0, 1), (1500, 2e-3, 3.0, 2), (400, 4e-3, 1.0, 3))]
    rng = np.random.default_rng(8)
    for sc in scenes:  # random motion, so that spheres collide and searches are due
        sc["particles"]["vel"] = rng.normal(0.0, 0.2, sc["particles"]["pos"].shape)
    batch = Dem.from_scenes(scenes, precision=precision)
    batch.step(150)
    batch.step(90)
    assert batch.get_stats()["n_rebuilds"] < 240 / 4
    for k, sc in enumerate(scenes):
        one = Dem.from_scene(sc, precision=precision)
        one.step(150)
        one.step(90)
        a, b = batch.get_state(k), one.get_state()
        # the batch searches when its fastest instance needs it: contact sets,
        # hence trajectories, agree; summation orders may differ (re-sorts)
        d = 2 * sc["particles"]["radius"][0]
        assert np.max(np.abs(a["pos"] - b["pos"])) <= 1e-9 * d
        o = oracle_from_scene(dict(sc, config=dict(sc["config"], rebuild_interval=1)))
        o.step(240)
        gp, gd, gt = batch.get_contacts(k)
        op, od, ot = o.contacts()
        gtp = {tuple(p) for p, t in zip(gp, gt) if t}
        otp = {tuple(p) for p, t in zip(op, ot) if t}
        assert gtp == otp, k
        err = np.max(np.abs(a["pos"] - o.state()["pos"]))
        if precision == "fp64":
            assert err <= 1e-12, k
        else:
            # colliding spheres amplify the FP32 law's rounding; the search
            # schedule must add nothing to it: compare with searching every step
            k1 = Dem.from_scene(dict(sc, config=dict(sc["config"], rebuild_interval=1)),
                                precision=precision)
            k1.step(240)
            err1 = np.max(np.abs(k1.get_state()["pos"] - o.state()["pos"]))
            assert err <= 5 * err1 + 1e-15, (k, err, err1)
            k1.close()
        one.close()
