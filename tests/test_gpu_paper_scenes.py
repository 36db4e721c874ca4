"""GPU parity on two more scenes of the paper, through the C ABI against the
oracle: the case of the appendix parameter file (spheres dropped into a cube
whose floor translates at 0.15 m/s) and the dam break of the weak-scaling
study (spheres held in the left half of a box by a floating dam that is
removed).
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


def sets_equal(g, o):
    gp, gd, gt = g.get_contacts()
    op, od, ot = o.contacts()
    assert np.array_equal(gp, op) and np.array_equal(gt, ot)
    gw, _ = g.get_wall_contacts()
    ow, _ = o.wall_contacts()
    assert np.array_equal(gw, ow)
    return int(gt.sum()), len(gw)


def force_err(g, o, radius):
    Fg, Tg = g.get_forces()
    Fo, To, S = o.forces()
    ef = np.max(np.linalg.norm(Fg - Fo, axis=1) / (np.linalg.norm(Fo, axis=1) + S + 1e-300))
    et = np.max(np.linalg.norm(Tg - To, axis=1) /
                (np.linalg.norm(To, axis=1) + S * radius + 1e-300))
    return ef, et


def test_sliding_floor_of_the_appendix(Dem):
    """0.4 s (40,000 steps): the spheres land, are dragged by the floor,
    reach the belt speed and pile against the far wall.  A 1e-15 relative
    perturbation of the start moves the oracle's own end state by about
    2e-10 m, which bounds what parity can show at the end."""
    sc = W.sliding_floor_scene()
    g, o = Dem.from_scene(sc), oracle_from_scene(sc)
    for chunk in (10_000, 10_000):
        g.step(chunk)
        o.step(chunk)
        nt, nw = sets_equal(g, o)
        dx = np.max(np.abs(g.get_state()["pos"] - o.state()["pos"]))
        print("sliding floor", g.get_state()["time"], "touching", nt, "wall", nw, "dx", dx,
              flush=True)
        assert dx <= 1e-10
    g.step(20_000)
    o.step(20_000)
    sg, so = g.get_state(), o.state()
    assert np.max(np.abs(sg["pos"] - so["pos"])) <= 1e-8
    assert np.max(np.abs(sg["vel"] - so["vel"])) <= 1e-6
    # most spheres have been brought to the floor's speed
    assert np.median(sg["vel"][:, 0]) == pytest.approx(0.15, abs=0.01)


def small_dam(spacing=0.97, t_dam_steps=20):
    return W.dam_break_scene(n=3000, depth=0.005, length=0.1, spacing=spacing,
                             t_dam=t_dam_steps * 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dam_break_parity(Dem, precision):
    """Overlapping start (spacing 0.97 d) so that contacts exist from the first
    step; the dam is removed at step 20, inside the compared window."""
    sc = small_dam()
    R = sc["particles"]["radius"]
    g = Dem.from_scene(sc, precision=precision)
    o = oracle_from_scene(sc)
    tol = 1e-11 if precision == "fp64" else 1e-5
    g.step(1)
    o.step(1)
    nt, nw = sets_equal(g, o)
    dam = len(sc["walls"]) - 1
    on_dam = np.sum(g.get_wall_contacts()[0][:, 1] == dam)
    ef, et = force_err(g, o, R)
    print(precision, "step 1: touching", nt, "wall", nw, "on the dam", on_dam, "err", ef, et,
          flush=True)
    assert nt > 1000 and on_dam > 20 and ef <= tol and et <= tol
    for chunk in (19, 20):  # the dam is gone from step 20 on
        g.step(chunk)
        o.step(chunk)
        ef, et = force_err(g, o, R)
        dx = np.max(np.abs(g.get_state()["pos"] - o.state()["pos"]))
        print(precision, "step", g.get_stats()["step"], "err", ef, et, "dx", dx, flush=True)
        assert ef <= max(10 * tol, 1e-9) and et <= max(10 * tol, 1e-9)
        assert dx <= (1e-12 if precision == "fp64" else 1e-6 * 1e-3)
    if precision == "fp64":
        g.step(60)
        o.step(60)
        sets_equal(g, o)


def test_dam_break_flows_once_the_dam_is_removed(Dem):
    """Without parity (the collapse of a lattice is chaotic): nothing crosses
    the dam while it stands, the front advances once it is gone."""
    sc = small_dam(spacing=1.02, t_dam_steps=400)
    L = sc["geometry"]["length"]
    R = sc["particles"]["radius"][0]
    g = Dem.from_scene(sc)
    g.step(400)
    assert np.max(g.get_state()["pos"][:, 0]) < L / 2 - R + 0.1 * R
    g.step(9600)  # 0.1 s: the front has left the dam's line by millimetres
    x = g.get_state()["pos"][:, 0]
    assert np.max(x) > L / 2 + 2e-3
    assert g.get_stats()["n_active"] == 3000
