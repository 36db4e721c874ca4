"""GPU parity with translating walls (Sec. 3.7: boundaries move by rotation or
translation), through the C ABI against the oracle.

Scenes: a box whose lid presses down while its floor runs as a belt and a
side wall moves obliquely; a rotating drum that also translates across its
axis, rising into its charge; the small hopper silo with its cone, cylinder and plug rising.  Contact
sets (particle pairs and particle-wall candidates) are compared bit for bit,
also at searches long after the start, where the walls have moved; forces
within the law's tolerance.  The dynamic schedule is checked on a piston that
starts beyond the search radius of spheres at rest: only the wall's own
motion can make the library search again.
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
    return int(gt.sum()), gw


def force_err(g, o, radius):
    Fg, Tg = g.get_forces()
    Fo, To, S = o.forces()
    ef = np.max(np.linalg.norm(Fg - Fo, axis=1) / (np.linalg.norm(Fo, axis=1) + S + 1e-300))
    et = np.max(np.linalg.norm(Tg - To, axis=1) /
                (np.linalg.norm(To, axis=1) + S * radius + 1e-300))
    return ef, et


def moving_box():
    """Dense snapshot in a box of six planes: the lid moves down at 0.2 m/s,
    the floor slides in its own plane (a belt), the wall of normal +x moves
    obliquely."""
    sc = W.dense_snapshot(n=2500, seed=29, polydisperse=0.1, n_types=2, K=10)
    walls = []
    for w in sc["walls"]:
        n = np.array(w["normal"])
        v = None
        if n[2] < -0.5:
            v = (0.0, 0.0, -0.2)
        elif n[2] > 0.5:
            v = (0.3, 0.1, 0.0)
        elif n[0] > 0.5:
            v = (0.05, 0.02, -0.03)
        walls.append(dict(w, velocity=v))
    return dict(sc, walls=walls)


def moving_drum():
    """Spinning drum (slightly overlapping start) rising into its charge
    while drifting sideways."""
    sc = W.drum_scene(n=3000, omega=2.0, seed=13, dt=1e-5, K=10, spacing=0.97)
    V = (0.02, 0.05, 0.3)
    return dict(sc, walls=[dict(w, velocity=V) for w in sc["walls"]])


def moving_hopper():
    sc = W.hopper_silo_scene(n=3000, spacing=0.8, clearance=1.0, t_open=300 * 2e-6, K=10)
    rng = np.random.default_rng(17)
    sc["particles"]["omega"] = rng.uniform(-20.0, 20.0, sc["particles"]["pos"].shape)
    return dict(sc, walls=[dict(w, velocity=(0.0, 0.0, 0.05)) for w in sc["walls"]])


SCENES = {"box": moving_box, "drum": moving_drum, "hopper": moving_hopper}


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_translating_walls_parity(Dem, name, precision):
    sc = SCENES[name]()
    R = sc["particles"]["radius"]
    print(name, precision, flush=True)
    g = Dem.from_scene(sc, precision=precision)
    o = oracle_from_scene(sc)
    tol = 1e-11 if precision == "fp64" else 1e-5
    g.step(1)
    o.step(1)
    nt, gw = sets_equal(g, o)
    ef, et = force_err(g, o, R)
    print(name, precision, "step 1: touching", nt, "wall candidates", len(gw), "err", ef, et,
          flush=True)
    assert nt > 100 and len(gw) > 20 and ef <= tol and et <= tol
    g.step(19)
    o.step(19)
    ef, et = force_err(g, o, R)
    dx = np.max(np.abs(g.get_state()["pos"] - o.state()["pos"]))
    print(name, precision, "step 20: err", ef, et, "max |dx|", dx, flush=True)
    assert ef <= max(10 * tol, 1e-9) and et <= max(10 * tol, 1e-9)
    assert dx <= (1e-12 if precision == "fp64" else 1e-6 * 2e-3)
    if precision == "fp64":
        # searches at steps 30 ... 400, with the walls far from where they began
        for chunk in (110, 170, 100):
            g.step(chunk)
            o.step(chunk)
            sets_equal(g, o)
        assert g.get_state()["time"] == o.state()["time"]


def test_static_and_zero_velocity_walls_agree_bitwise(Dem):
    """A zero velocity leaves every result bit-identical to a fixed wall."""
    sc = W.drum_scene(n=2000, omega=2.0, seed=3, dt=1e-5, K=10)
    sc0 = dict(sc, walls=[dict(w, velocity=(0.0, 0.0, 0.0)) for w in sc["walls"]])
    a, b = Dem.from_scene(sc), Dem.from_scene(sc0)
    a.step(137)
    b.step(137)
    sa, sb = a.get_state(), b.get_state()
    for k in ("pos", "vel", "omega"):
        assert np.array_equal(sa[k], sb[k])


def piston_scene(V, dt, K, gap=3e-3):
    """Spheres at rest in a 4 x 4 x 2 block, no gravity; a plane of normal +x
    moving at V along +x starts `gap` from the nearest spheres, beyond the
    search radius."""
    R = 1.5e-3
    ys, zs, xs = np.meshgrid(np.arange(4) * 2.2 * R, np.arange(4) * 2.2 * R,
                             np.arange(2) * 2.2 * R, indexing="ij")
    pos = np.stack([xs.ravel() + R + gap, ys.ravel(), zs.ravel()], 1) + 0.01
    mat = dict(W.BOX_MATERIAL, restitution=0.8, friction=0.2)
    cfg = W._cfg(dt, (0.0, 0.0, 0.0), (0.06, 0.03, 0.03), K=K, gravity=(0.0, 0.0, 0.0))
    walls = [W.plane((0.01, 0.0, 0.0), (1.0, 0.0, 0.0), velocity=(V, 0.0, 0.0))]
    return dict(name="piston", config=cfg, materials=[mat], walls=walls,
                particles=W._particles(pos, R))


@pytest.mark.parametrize("integrator", ["verlet", "euler"])
def test_dynamic_schedule_follows_a_piston(Dem, integrator):
    """Spheres at rest never drift, so only the piston's own motion can
    trigger the searches that find it; the dynamic run equals the oracle
    searching at every step."""
    sc = piston_scene(V=2.0, dt=1e-6, K=1)
    sc["config"]["integrator"] = integrator
    o = oracle_from_scene(sc)
    g = Dem.from_scene(dict(sc, config=dict(sc["config"], rebuild_interval=0)))
    for chunk in (500, 1000, 1500):
        g.step(chunk)
        o.step(chunk)
    sg, so = g.get_state(), o.state()
    assert np.max(sg["vel"][:, 0]) > 2.0  # the front spheres were hit
    assert np.max(np.abs(sg["pos"] - so["pos"])) <= 1e-12
    assert np.max(np.abs(sg["vel"] - so["vel"])) <= 1e-9
    st = g.get_stats()
    assert 5 < st["n_rebuilds"] < 3000 / 4, st


def test_fixed_schedule_piston(Dem):
    sc = piston_scene(V=2.0, dt=1e-6, K=50)
    o, g = oracle_from_scene(sc), Dem.from_scene(sc)
    for chunk in (777, 2223):
        g.step(chunk)
        o.step(chunk)
        sets_equal(g, o)
    sg, so = g.get_state(), o.state()
    assert np.max(sg["vel"][:, 0]) > 2.0
    assert np.max(np.abs(sg["pos"] - so["pos"])) <= 1e-12


def test_wall_too_fast_for_the_schedule_is_rejected(Dem):
    # skin = 0.3 d = 0.9 mm; 2 m/s x 250 steps x 1 us = 0.5 mm > 0.45 mm
    sc = piston_scene(V=2.0, dt=1e-6, K=250)
    with pytest.raises(Exception, match="half the skin"):
        Dem.from_scene(sc)
    sc = piston_scene(V=2.0, dt=1e-6, K=220)  # 0.44 mm: allowed
    Dem.from_scene(sc).step(10)
    sc = piston_scene(V=500.0, dt=1e-6, K=0)  # 0.5 mm in one step
    with pytest.raises(Exception, match="half the skin"):
        Dem.from_scene(sc)


def test_wall_motion_argument_checks(Dem):
    sim = Dem(dt=1e-5)
    sim.set_material(0, 2500.0, 1e6, 0.3, 0.9, 0.3, 0.1)
    w = sim.add_planar_wall((0, 0, 0), (0, 0, 1))
    with pytest.raises(Exception):
        sim.set_wall_motion(w + 1, (0.0, 0.0, 1.0))
    with pytest.raises(Exception):
        sim.set_wall_motion(w, (0.0, float("nan"), 1.0))
    sim.set_wall_motion(w, (0.0, 0.0, 0.001))
    sim.set_particles([[0.0, 0.0, 0.01]], [1e-3])
    with pytest.raises(Exception):
        sim.set_wall_motion(w, (0.0, 0.0, 0.0))  # after the particles


def test_resume_with_translating_walls_is_bitwise_exact(Dem):
    """The resumed context searches again with the walls at the restored
    time, so it repeats the saved run bit for bit."""
    sc = moving_box()
    a = Dem.from_scene(sc)
    a.step(100)
    ck = a.checkpoint()
    assert len(ck["wall_pairs"]) > 10 and np.any(ck["wall_delta_t"] != 0)
    sc2 = dict(sc, particles=dict(sc["particles"], pos=ck["pos"], vel=ck["vel"],
                                  omega=ck["omega"]))
    b = Dem.from_scene(sc2)
    b.restore(ck)
    for chunk in (37, 113):
        a.step(chunk)
        b.step(chunk)
        sa, sb = a.get_state(), b.get_state()
        for k in ("pos", "vel", "omega"):
            assert np.array_equal(sa[k], sb[k]), k
        wa, da = a.get_wall_contacts()
        wb, db = b.get_wall_contacts()
        assert np.array_equal(wa, wb) and np.array_equal(da, db)


def test_autotune_skips_intervals_a_wall_outruns(Dem):
    """K = 40 and 80 would let the piston cover more than half the skin
    between searches: the tuner does not try them.  (The piston starts far
    enough away not to reach the spheres while the tuner runs.)"""
    sc = piston_scene(V=3.0, dt=5e-6, K=10, gap=0.012)  # 15 um per step: K <= 30
    g = Dem.from_scene(sc)
    t = g.autotune(trial_steps=40)
    sched = t["schedule_ms"]
    assert np.max(g.get_state()["vel"]) == 0.0
    assert sched[40] == -1.0 and sched[80] == -1.0
    assert sched[20] > 0
    assert t["rebuild_interval"] not in (40, 80)
