"""GPU parity with mesh walls (Sec. 3.7: particle-face, particle-line and
particle-point contacts), through the C ABI against the oracle.

Scenes: a dense snapshot inside a triangulated box (concave edges and
corners); the 3,000-sphere hopper silo with its cone replaced by a spinning
triangulated frustum (faces, and the convex rim of the outlet); spheres
thrown onto a roof and a pyramid (convex ridge, edges and apex); a spinning
drum with a triangulated cylinder; a translating triangulated plate.  Particle-triangle candidate triples are
compared bit for bit, forces within the law's tolerance.
"""
import math

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
    gm, _ = g.get_mesh_contacts()
    om, _ = o.mesh_contacts()
    assert np.array_equal(gm, om)
    return int(gt.sum()), len(gm)


def force_err(g, o, radius):
    Fg, Tg = g.get_forces()
    Fo, To, S = o.forces()
    ef = np.max(np.linalg.norm(Fg - Fo, axis=1) / (np.linalg.norm(Fo, axis=1) + S + 1e-300))
    et = np.max(np.linalg.norm(Tg - To, axis=1) /
                (np.linalg.norm(To, axis=1) + S * radius + 1e-300))
    return ef, et


def meshed_box():
    sc = W.dense_snapshot(n=2500, seed=31, polydisperse=0.1, n_types=2, K=10)
    n = [np.array(w["normal"]) for w in sc["walls"]]
    lo = [w["point"] for w, nn in zip(sc["walls"], n) if nn.sum() > 0][0]
    hi = [w["point"] for w, nn in zip(sc["walls"], n) if nn.sum() < 0][0]
    return dict(sc, walls=[W.box_mesh(lo, hi, divisions=4)])


def meshed_hopper():
    # spheres start slightly into the cone, so that its faces act at once
    sc = W.hopper_silo_scene(n=3000, spacing=0.8, clearance=0.7, t_open=300 * 2e-6, K=10)
    rng = np.random.default_rng(17)
    sc["particles"]["omega"] = rng.uniform(-20.0, 20.0, sc["particles"]["pos"].shape)
    cone = sc["walls"][0]
    frustum = W.frustum_mesh(cone["axis_point"], cone["radius0"], cone["slope"], cone["s_min"],
                             cone["s_max"], segments=48, rings=20, omega=1.5)
    return dict(sc, walls=[frustum] + sc["walls"][1:])


def roof_and_pyramid(n_side=24, seed=5):
    """A roof (ridge along y) and a pyramid side by side on a floor, spheres
    raining onto them from a lattice just above, with random velocities and
    spins; the pyramid switches off at step 80."""
    rng = np.random.default_rng(seed)
    R = 1.5e-3
    a = math.radians(30.0)
    L = 0.04
    dx, dz = L * math.cos(a), -L * math.sin(a)
    V1 = np.array([(0, -L, 0), (0, L, 0), (-dx, -L, dz), (-dx, L, dz), (dx, -L, dz), (dx, L, dz)])
    T1 = np.array([(0, 1, 3), (0, 3, 2), (0, 5, 1), (0, 4, 5)])
    c = np.array([0.1, 0.0, 0.0])
    V2 = np.array([(0, 0, 0), (-L, -L, -0.02), (L, -L, -0.02), (L, L, -0.02), (-L, L, -0.02)]) + c
    T2 = np.array([(0, 1, 2), (0, 2, 3), (0, 3, 4), (0, 4, 1)])
    xs = np.linspace(-0.03, 0.13, n_side)
    ys = np.linspace(-0.03, 0.03, n_side // 2)
    pts = []
    for x in xs:
        for y in ys:
            # height of the surface below (roof or pyramid), then just above it
            zr = -abs(x) * math.tan(a) if abs(x) < dx else -0.03
            zp = (-max(abs(x - c[0]), abs(y)) * 0.02 / L) if max(abs(x - c[0]), abs(y)) < L else -0.03
            z = max(zr, zp, -0.03)
            pts.append((x, y, z + R * 1.2 + 2e-4 * rng.random()))
    pts = np.array(pts)
    vel = np.column_stack([rng.normal(0, 0.05, len(pts)), rng.normal(0, 0.05, len(pts)),
                           -0.3 - 0.1 * rng.random(len(pts))])
    om = rng.uniform(-30, 30, (len(pts), 3))
    cfg = W._cfg(1e-5, (-0.06, -0.06, -0.06), (0.16, 0.06, 0.06), K=10)
    # the pyramid is a floating wall: it disappears at step 80
    walls = [W.mesh(V1, T1), W.mesh(V2, T2, t_off=80e-5), W.plane((0, 0, -0.03), (0, 0, 1))]
    return dict(name="roof_pyramid", config=cfg, materials=[dict(W.BOX_MATERIAL)], walls=walls,
                particles=W._particles(pts, R, vel, om))


def meshed_drum():
    """The spinning drum with a triangulated cylinder (48 x 8 squares), made
    0.3 radii narrower than the analytic one so that the outer spheres press
    on it from the start."""
    sc = W.drum_scene(n=3000, omega=2.0, seed=13, dt=1e-5, K=10, spacing=0.97)
    g = sc["geometry"]
    r = sc["particles"]["radius"][0]
    m = W.drum_mesh(g["R"] - 0.3 * r, -g["L"] / 2, g["L"] / 2, 48, 8, omega=g["omega"])
    return dict(sc, walls=[m] + sc["walls"][1:])


SCENES = {"box": meshed_box, "hopper": meshed_hopper, "roof": roof_and_pyramid,
          "drum": meshed_drum}


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mesh_walls_parity(Dem, name, precision):
    sc = SCENES[name]()
    R = sc["particles"]["radius"]
    g = Dem.from_scene(sc, precision=precision)
    o = oracle_from_scene(sc)
    tol = 1e-11 if precision == "fp64" else 1e-5
    g.step(1)
    o.step(1)
    nt, nm = sets_equal(g, o)
    ef, et = force_err(g, o, R)
    print(name, precision, "step 1: touching", nt, "triangle candidates", nm, "err", ef, et,
          flush=True)
    assert nm > 20 and ef <= tol and et <= tol
    # FP32: 20 steps (later on, the constant rolling torque of spheres coming
    # to rest takes the direction of a relative spin at the rounding level)
    for chunk in ((19, 30) if precision == "fp64" else (19,)):
        g.step(chunk)
        o.step(chunk)
        nt, nm = sets_equal(g, o)
        ef, et = force_err(g, o, R)
        dx = np.max(np.abs(g.get_state()["pos"] - o.state()["pos"]))
        print(name, precision, "step", g.get_stats()["step"], "err", ef, et, "dx", dx,
              "triangle candidates", nm, flush=True)
        assert ef <= max(10 * tol, 1e-9) and et <= max(10 * tol, 1e-9)
        assert dx <= (1e-12 if precision == "fp64" else 1e-9)
    # tangential overlaps kept in the candidates' slots
    _, dto = o.mesh_contacts()
    _, dtg = g.get_mesh_contacts()
    assert np.max(np.abs(dtg - dto)) <= (1e-9 if precision == "fp64" else 1e-3) * \
        (np.max(np.abs(dto)) + 1e-300)
    if precision == "fp64":
        assert np.count_nonzero(np.any(dto != 0, axis=1)) >= 5  # at step 50
        for chunk in (100, 150):
            g.step(chunk)
            o.step(chunk)
            sets_equal(g, o)


def test_translating_mesh_plate(Dem):
    """A triangulated plate moving at 0.3 m/s sweeps spheres at rest."""
    rng = np.random.default_rng(2)
    R = 1.5e-3
    pts = W.rsa_box(200, R, (0.005, -0.02, -0.02), (0.03, 0.02, 0.02), rng)
    Vx = np.array([(0, -0.03, -0.03), (0, 0.03, -0.03), (0, 0.03, 0.03), (0, -0.03, 0.03)])
    plate = W.mesh(Vx, np.array([(0, 1, 2), (0, 2, 3)]), velocity=(0.3, 0.0, 0.0))
    cfg = W._cfg(1e-5, (-0.01, -0.05, -0.05), (0.1, 0.05, 0.05), K=10, gravity=(0, 0, 0))
    sc = dict(name="plate", config=cfg, materials=[dict(W.BOX_MATERIAL)], walls=[plate],
              particles=W._particles(pts, R))
    g, o = Dem.from_scene(sc), oracle_from_scene(sc)
    for chunk in (1000, 1000):
        g.step(chunk)
        o.step(chunk)
        nt, nm = sets_equal(g, o)
        print("plate", g.get_state()["time"], "touching", nt, "triangle candidates", nm,
              flush=True)
    assert nm > 10
    assert np.max(np.abs(g.get_state()["pos"] - o.state()["pos"])) <= 1e-9
    assert np.max(g.get_state()["vel"][:, 0]) > 0.3


def test_too_many_triangle_candidates_is_reported(Dem):
    """A fine mesh (triangles much smaller than the sphere) overflows the 8
    candidate slots: a capacity error, not a silent miss."""
    m = 40
    xs = np.linspace(-0.01, 0.01, m + 1)
    V = np.array([(x, y, 0.0) for y in xs for x in xs])
    T = []
    for j in range(m):
        for i in range(m):
            a, b = j * (m + 1) + i, j * (m + 1) + i + 1
            T += [(a, b, b + m + 1), (a, b + m + 1, a + m + 1)]
    cfg = W._cfg(1e-5, (-0.05,) * 3, (0.05,) * 3, K=10)
    sc = dict(name="fine", config=cfg, materials=[dict(W.BOX_MATERIAL)],
              walls=[W.mesh(V, np.array(T))], particles=W._particles([[0.0, 0.0, 1.6e-3]], 1.5e-3))
    with pytest.raises(Exception, match="capacity"):
        g = Dem.from_scene(sc)
        g.step(1)


def test_mesh_wall_argument_checks(Dem):
    sim = Dem(dt=1e-5)
    sim.set_material(0, 2500.0, 1e6, 0.3, 0.9, 0.3, 0.1)
    with pytest.raises(Exception):
        sim.add_mesh_wall([[0, 0, 0], [1, 0, 0], [2, 0, 0]], [[0, 1, 2]])  # degenerate
    with pytest.raises(Exception):
        sim.add_mesh_wall([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 1, 3]])  # bad index
    sim.add_mesh_wall([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 1, 2]])
    sim.set_particles([[0.2, 0.2, 0.01]], [1e-3])
    ck = sim.checkpoint()
    sim.restore(ck)
    ck["mesh_triples"] = np.array([[0, 0, 1]])  # no triangle 1
    ck["mesh_delta_t"] = np.zeros((1, 3))
    with pytest.raises(Exception, match="mesh contact"):
        sim.restore(ck)


def test_resume_with_mesh_walls_is_bitwise_exact(Dem):
    """Checkpoint right after a search (step 100), rebuild a context from the
    saved state and restore: the two runs agree bit for bit."""
    sc = meshed_box()
    a = Dem.from_scene(sc)
    a.step(100)
    ck = a.checkpoint()
    assert len(ck["mesh_triples"]) > 10
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
        ma, da = a.get_mesh_contacts()
        mb, db = b.get_mesh_contacts()
        assert np.array_equal(ma, mb) and np.array_equal(da, db)


def test_meshes_in_a_batch(Dem):
    """Three instances with different meshes (a box, a roof and pyramid, a
    drum) in one context: each follows its own oracle, with its own wall and
    triangle numbering."""
    scenes = [meshed_box(), roof_and_pyramid(), meshed_drum()]
    b = Dem.from_scenes(scenes)
    orc = [oracle_from_scene(sc) for sc in scenes]
    for chunk in (1, 29):
        b.step(chunk)
        for k, o in enumerate(orc):
            o.step(chunk)
            gm, gd = b.get_mesh_contacts(k)
            om, od = o.mesh_contacts()
            assert np.array_equal(gm, om), k
            Fg, _ = b.get_forces(k)
            Fo, _, S = o.forces()
            ef = np.max(np.linalg.norm(Fg - Fo, axis=1) /
                        (np.linalg.norm(Fo, axis=1) + S + 1e-300))
            assert ef <= 1e-9, (k, ef)


def test_euler_integrator_with_meshes(Dem):
    sc = meshed_box()
    sc = dict(sc, config=dict(sc["config"], integrator="euler"))
    g, o = Dem.from_scene(sc), oracle_from_scene(sc)
    R = sc["particles"]["radius"]
    for chunk in (1, 19, 30):
        g.step(chunk)
        o.step(chunk)
        sets_equal(g, o)
        ef, et = force_err(g, o, R)
        assert ef <= 1e-9 and et <= 1e-9
    assert np.max(np.abs(g.get_state()["pos"] - o.state()["pos"])) <= 1e-12


def test_dynamic_schedule_with_a_translating_mesh(Dem):
    """Spheres at rest and a triangulated piston that starts beyond the
    search radius: only the mesh's motion triggers the searches that find
    it; equal to the oracle searching every step."""
    R = 1.5e-3
    ys, zs = np.meshgrid(np.arange(4) * 2.2 * R, np.arange(4) * 2.2 * R, indexing="ij")
    pos = np.stack([np.full(16, 0.01 + R + 3e-3), ys.ravel(), zs.ravel()], 1)
    Vx = np.array([(0.01, -0.02, -0.02), (0.01, 0.03, -0.02), (0.01, 0.03, 0.03),
                   (0.01, -0.02, 0.03)])
    plate = W.mesh(Vx, np.array([(0, 1, 2), (0, 2, 3)]), velocity=(2.0, 0.0, 0.0))
    cfg = W._cfg(1e-6, (0.0, -0.05, -0.05), (0.06, 0.05, 0.05), K=1, gravity=(0, 0, 0))
    sc = dict(name="mesh_piston", config=cfg, materials=[dict(W.BOX_MATERIAL)], walls=[plate],
              particles=W._particles(pos, R))
    o = oracle_from_scene(sc)
    g = Dem.from_scene(dict(sc, config=dict(cfg, rebuild_interval=0)))
    for chunk in (1000, 2000):
        g.step(chunk)
        o.step(chunk)
    sg, so = g.get_state(), o.state()
    assert np.max(sg["vel"][:, 0]) > 2.0
    assert np.max(np.abs(sg["pos"] - so["pos"])) <= 1e-12
    assert 5 < g.get_stats()["n_rebuilds"] < 750
