"""Pins of the oracle's cone wall (conical hopper of the large-silo workload).

Walls are analytic surfaces standing in for the paper's meshed boundaries
(Sec. 2.1, last paragraph: a wall acts as a body of infinite mass and radius).
The cone's surface lies at r(s) = r0 + slope s from its axis.  The expected
values below come from the geometry of the surface (the normal as the
normalised gradient of rho - r(s), the distance by numerical minimisation)
and from mechanics (Hertz's static force, sliding down a frictionless
incline), and the cone with slope 0 must reproduce the already pinned
cylinder.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import OracleSim

MAT = dict(density=2500.0, youngs=1.0e6, poisson=0.3, restitution=0.9, friction=0.3,
           rolling_friction=0.1)
R = 1.5e-3


def sim(mat=MAT, dt=1e-6, gravity=(0, 0, 0), K=1, rolling="none", threshold=1.3):
    s = OracleSim(dt=dt, gravity=gravity, domain_lo=(-1, -1, -1), domain_hi=(1, 1, 1),
                  neighbor_threshold=threshold, rebuild_interval=K, rolling_model=rolling)
    s.set_material(0, **mat)
    return s


def ye(mat=MAT):
    return 1.0 / (2.0 * (1.0 - mat["poisson"] ** 2) / mat["youngs"])


def outward_normal(x, slope):
    """Unit gradient of F(x) = sqrt(x^2 + y^2) - slope z (cone about the z axis)."""
    rho = math.hypot(x[0], x[1])
    g = np.array([x[0] / rho, x[1] / rho, -slope])
    return g / np.linalg.norm(g)


@pytest.mark.parametrize("inside", [True, False])
def test_cone_static_force_is_hertz_along_surface_normal(oracle_built, inside):
    r0, slope = 0.02, 1.0 / math.tan(math.radians(60.0))
    s = sim()
    s.add_cone((0, 0, 0), (0, 0, 1), r0, slope, 0.0, 0.4, inside=inside)
    # a surface point at height 0.1 on the meridian at 30 degrees
    zc = 0.1
    rc = r0 + slope * zc
    phi = math.radians(30.0)
    xc = np.array([rc * math.cos(phi), rc * math.sin(phi), zc])
    m = outward_normal(xc, slope)
    delta = 2e-5
    # centre on the particle's side of the surface, overlapping by delta
    side = -1.0 if inside else 1.0
    x = xc + side * (R - delta) * m
    s.set_particles([x], [R])
    s.step(1)
    F, _, _ = s.forces()
    Fh = 4.0 / 3.0 * ye() * math.sqrt(R) * delta ** 1.5
    np.testing.assert_allclose(F[0], side * Fh * m, rtol=1e-8, atol=1e-15)


def test_cone_frictionless_slide_down_generator(oracle_built):
    """On the outside of an upright cone of surface inclination theta (a
    conical heap, slope < 0), a frictionless sphere released at its resting
    overlap slides down its meridian with acceleration g sin(theta)."""
    theta = math.radians(35.0)
    slope = -1.0 / math.tan(theta)
    r0 = 0.2
    mat = dict(MAT, friction=0.0, rolling_friction=0.0, restitution=0.5)
    dt = 2e-6
    s = sim(mat=mat, dt=dt, gravity=(0, 0, -9.81), K=20)
    s.add_cone((0, 0, 0), (0, 0, 1), r0, slope, 0.0, 0.9 * r0 / -slope, inside=False)
    zc = 0.1
    rc = r0 + slope * zc
    xc = np.array([rc, 0.0, zc])
    m = outward_normal(xc, slope)
    mass = MAT["density"] * 4 / 3 * math.pi * R ** 3
    deq = (3 * mass * 9.81 * math.cos(theta) / (4 * ye() * math.sqrt(R))) ** (2 / 3)
    x0 = xc + (R - deq) * m
    s.set_particles([x0], [R])
    n = 10000
    s.step(n)
    x1 = s.state()["pos"][0]
    down = np.array([math.cos(theta), 0.0, -math.sin(theta)])  # along the generator
    travel = np.dot(x1 - x0, down)
    T = n * dt
    assert travel == pytest.approx(0.5 * 9.81 * math.sin(theta) * T * T, rel=2e-3)
    assert abs(x1[1]) < 1e-12  # stays on its meridian


@pytest.mark.parametrize("inside", [True, False])
def test_cone_with_zero_slope_is_the_cylinder(oracle_built, inside):
    """A rotating cone of slope 0 reproduces the rotating cylinder."""
    Rd = 0.04
    rng = np.random.default_rng(5)
    n = 40
    ang = np.linspace(0, 2 * math.pi, n, endpoint=False) + rng.uniform(-0.02, 0.02, n)
    rad = Rd - R + rng.uniform(-2e-5, 4e-4, n) if inside else Rd + R + rng.uniform(-4e-4, 2e-5, n)
    pos = np.stack([rng.uniform(-0.015, 0.015, n), rad * np.cos(ang), rad * np.sin(ang)], 1)
    vel = rng.normal(0, 0.05, (n, 3))
    out = []
    for kind in ("cyl", "cone"):
        s = sim(dt=1e-5, gravity=(0, 0, -9.81), K=10, rolling="constant")
        if kind == "cyl":
            s.add_cylinder((0, 0, 0), (1, 0, 0), Rd, -0.02, 0.02, inside=inside, omega=2.0)
        else:
            s.add_cone((0, 0, 0), (1, 0, 0), Rd, 0.0, -0.02, 0.02, inside=inside, omega=2.0)
        s.set_particles(pos, [R] * n, vel=vel)
        s.step(300)
        out.append((s.state()["pos"], s.wall_contacts()[0]))
    assert np.array_equal(out[0][1], out[1][1])
    assert np.max(np.abs(out[0][0] - out[1][0])) < 1e-12


def test_cone_candidates_match_numerical_distance(oracle_built):
    """A particle is a wall candidate when its distance to the cone surface,
    found here by minimising over the meridian's generator line, lies in
    (-R, R + skin)."""
    r0, slope = 0.02, 0.6
    s = sim()
    s.add_cone((0, 0, 0), (0, 0, 1), r0, slope, 0.0, 0.3, inside=True)
    rng = np.random.default_rng(11)
    n = 400
    z = rng.uniform(0.01, 0.29, n)
    ang = rng.uniform(0, 2 * math.pi, n)
    rr = r0 + slope * z + rng.uniform(-4 * R, 2 * R, n)
    pos = np.stack([rr * np.cos(ang), rr * np.sin(ang), z], 1)
    # keep particles at least 3 R apart so that only walls matter
    keep = [0]
    for i in range(1, n):
        if np.min(np.linalg.norm(pos[keep] - pos[i], axis=1)) > 3 * R:
            keep.append(i)
    pos = pos[keep]
    s.set_particles(pos, [R] * len(pos))
    skin = s.search_params()["skin"]
    got = set(int(i) for i, _ in s.wall_contacts()[0])
    expect, near = set(), 0
    for i, p in enumerate(pos):
        rho, zz = math.hypot(p[0], p[1]), p[2]
        f = lambda t: (rho - (r0 + slope * t)) ** 2 + (zz - t) ** 2  # noqa: E731
        d = math.sqrt(minimize_scalar(f, bounds=(-0.1, 0.4), method="bounded",
                                      options={"xatol": 1e-12}).fun)
        d = d if rho < r0 + slope * zz else -d  # positive on the inside
        if min(abs(d + R), abs(d - R - skin)) < 1e-8:
            near += 1
            continue
        if -R < d < R + skin:
            expect.add(i)
    assert near < 3
    assert len(expect) > 50
    assert expect <= got and len(got - expect) <= near
