"""GPU parity of the second contact model and the second rolling model.

The linear spring-dashpot law (Sec. 2.1, Eqs. linearkn and linearetan) and the
viscous rolling torque (second row of the table of rolling models) run in the
same force kernel as the Hertz-Mindlin law.  Bars as for the default models:
contact sets bit-exact, forces within 1e-11 (FP64 law) and 1e-5 (FP32 law),
non-chaotic trajectories within 1e-6 d after 1,000 steps.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_from_scene

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 1e-5}
VARIANTS = [("linear", "constant"), ("nonlinear", "viscous"), ("linear", "viscous"),
            ("linear", "none")]


@pytest.fixture(scope="module")
def Dem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_09576_amd import Dem as D
    return D


def force_err(g, o, radius):
    Fg, Tg = g.get_forces()
    Fo, To, S = o.forces()
    ef = np.max(np.linalg.norm(Fg - Fo, axis=1) / (np.linalg.norm(Fo, axis=1) + S + 1e-300))
    et = np.max(np.linalg.norm(Tg - To, axis=1) /
                (np.linalg.norm(To, axis=1) + S * radius + 1e-300))
    return ef, et


def same_sets(g, o):
    gp, gd, gt = g.get_contacts()
    op, od, ot = o.contacts()
    assert np.array_equal(gp, op) and np.array_equal(gt, ot)
    gw, _ = g.get_wall_contacts()
    ow, _ = o.wall_contacts()
    assert np.array_equal(gw, ow)


@pytest.mark.parametrize("model,rolling", VARIANTS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_model_forces_one_step_and_after_twenty(Dem, model, rolling, precision):
    sc = W.dense_snapshot(n=2500, seed=41, polydisperse=0.25, n_types=2, K=10,
                          model=model, V=0.5, rolling=rolling)
    g = Dem.from_scene(sc, precision=precision)
    o = oracle_from_scene(sc)
    R = sc["particles"]["radius"]
    g.step(1)
    o.step(1)
    same_sets(g, o)
    ef, et = force_err(g, o, R)
    print(model, rolling, precision, "one step", ef, et, flush=True)
    assert ef <= TOL[precision] and et <= TOL[precision]
    g.step(19)
    o.step(19)
    if precision == "fp64":
        same_sets(g, o)
    ef, et = force_err(g, o, R)
    print(model, rolling, precision, "20 steps", ef, et, flush=True)
    assert ef <= 10 * max(TOL[precision], 1e-10) and et <= 10 * max(TOL[precision], 1e-10)


def _case(case, model, rolling, V=0.5):
    R = 1.5e-3
    d = 2 * R
    mat = dict(W.BOX_MATERIAL)
    lo, hi = (-0.1, -0.1, -0.1), (0.1, 0.1, 0.1)
    g = (0, 0, -9.81)
    walls = []
    if case == "head_on":
        pos, vel, om, g = [[0, 0, 0], [0, 0, d + 1e-4]], [[0, 0, 0.3], [0, 0, -0.3]], None, (0, 0, 0)
        rad = [R, R]
    elif case == "wall_bounce":
        pos, vel, om, rad = [[0, 0, R + 2e-4]], [[0, 0, -0.5]], None, [R]
        walls = [W.plane((0, 0, 0), (0, 0, 1))]
    elif case == "oblique_sliding":
        pos = [[0, 0, 0], [0.8 * d, 0, 0.6 * d + 1e-4]]
        vel, om = [[0.2, 0.05, 0.3], [-0.2, 0, -0.3]], [[0, 30, 0], [5, 0, 0]]
        rad, g = [R, R], (0, 0, 0)
    else:  # rolling sphere on a plane
        mat = dict(mat, rolling_friction=0.3)
        pos, vel, om, rad = [[0, 0, R - 5e-6]], [[0.2, 0, 0]], None, [R]
        walls = [W.plane((0, 0, 0), (0, 0, 1))]
    cfg = W._cfg(1e-5, lo, hi, K=20, rolling=rolling, gravity=g, model=model, V=V)
    part = W._particles(np.array(pos, float), np.array(rad, float), np.array(vel, float),
                        None if om is None else np.array(om, float))
    return dict(name=case, config=cfg, materials=[mat], walls=walls, particles=part)


@pytest.mark.parametrize("case,model,rolling", [
    ("head_on", "linear", "constant"), ("wall_bounce", "linear", "constant"),
    ("oblique_sliding", "linear", "viscous"), ("rolling_sphere", "nonlinear", "viscous"),
    ("rolling_sphere", "linear", "viscous")])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_model_trajectory_1000_steps(Dem, case, model, rolling, precision):
    sc = _case(case, model, rolling)
    g = Dem.from_scene(sc, precision=precision)
    o = oracle_from_scene(sc)
    g.step(1000)
    o.step(1000)
    err = np.max(np.abs(g.get_state()["pos"] - o.state()["pos"]))
    print(case, model, rolling, precision, "max |dx| / d =", err / 3e-3, flush=True)
    assert err <= 1e-6 * 3e-3


def test_linear_model_needs_characteristic_velocity(Dem):
    with pytest.raises(Exception):
        Dem(dt=1e-5, contact_model="linear", characteristic_velocity=0.0)
