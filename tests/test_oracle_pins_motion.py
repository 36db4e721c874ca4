"""Pins of the oracle's translating walls (Sec. 3.7: boundaries move by
rotation or translation).  A wall with translational velocity V has its
point and rotation axis at p + V t and its surface moving at V + Omega x r.

Expected values from mechanics: a sphere put on a moving belt ends up rolling
at 2 V / 7 (rigid body); a piston of infinite mass hitting a resting sphere
sends it off at (1 + e) V; and Galilean invariance: a translating drum or
hopper with co-moving spheres reproduces the static one shifted by V t.
"""
import math

import numpy as np
import pytest

from oracle import OracleSim

MAT = dict(density=2500.0, youngs=1.0e6, poisson=0.3, restitution=0.9, friction=0.3,
           rolling_friction=0.1)
R = 1.5e-3


def sim(mat=MAT, dt=2e-6, gravity=(0, 0, -9.81), K=10, rolling="none", lo=-1.0, hi=1.0):
    s = OracleSim(dt=dt, gravity=gravity, domain_lo=(lo,) * 3, domain_hi=(hi,) * 3,
                  neighbor_threshold=1.3, rebuild_interval=K, rolling_model=rolling)
    s.set_material(0, **mat)
    return s


def ye(mat=MAT):
    return 1.0 / (2.0 * (1.0 - mat["poisson"] ** 2) / mat["youngs"])


def test_sphere_on_moving_belt_rolls_at_two_sevenths(oracle_built):
    mu, V = 0.3, 0.2
    mat = dict(MAT, friction=mu, rolling_friction=0.0, restitution=0.3)
    s = sim(mat=mat)
    w = s.add_plane((0, 0, 0), (0, 0, 1))
    s.set_wall_velocity(w, (V, 0.0, 0.0))
    m = MAT["density"] * 4 / 3 * math.pi * R ** 3
    deq = (3 * m * 9.81 / (4 * ye() * math.sqrt(R))) ** (2 / 3)
    s.set_particles([[0, 0, R - deq]], [R])
    t_star = 2 * V / (7 * mu * 9.81)
    s.step(int(1.5 * t_star / 2e-6))
    st = s.state()
    assert st["vel"][0, 0] == pytest.approx(2 * V / 7, rel=1e-2)
    # rolling without slip on the belt: v - R omega_y = V
    assert st["vel"][0, 0] - R * st["omega"][0, 1] == pytest.approx(V, rel=1e-2)


@pytest.mark.parametrize("e", [1.0, 0.8])
def test_piston_sends_sphere_off_at_one_plus_e_times_its_speed(oracle_built, e):
    V = 0.2
    mat = dict(MAT, restitution=e, friction=0.0, rolling_friction=0.0)
    dt = 2e-7
    s = sim(mat=mat, dt=dt, gravity=(0, 0, 0), K=1)
    w = s.add_plane((0, 0, 0), (1, 0, 0))
    s.set_wall_velocity(w, (V, 0.0, 0.0))
    # the piston starts 3 mm away, beyond the search radius: it must be found
    # where it has moved to
    s.set_particles([[R + 3e-3, 0, 0]], [R])
    hit = False
    for _ in range(2000):
        s.step(100)
        st = s.state()
        gap = st["pos"][0, 0] - V * st["time"] - R
        hit = hit or gap < 0
        if hit and gap > 0:  # the piston has let go
            break
    assert hit
    v = s.state()["vel"][0, 0]
    assert v == pytest.approx((1 + e) * V, rel=2e-3)


def _drum(s, moving, V, axis_dir, omega):
    w = s.add_cylinder((0, 0, 0), axis_dir, 0.02, -0.02, 0.02, True, 0, omega)
    if moving:
        s.set_wall_velocity(w, V)


@pytest.mark.parametrize("V", [(0.05, 0.0, 0.0), (0.0, 0.05, 0.02)])
def test_translating_rotating_drum_is_galilean(oracle_built, V):
    """Drum (axis x, spinning) translating along its axis or across it, with
    spheres given the same velocity: positions equal the static drum's plus
    V t (gravity along -z is the same in both frames)."""
    rng = np.random.default_rng(4)
    n = 30
    ang = np.linspace(0, 2 * np.pi, n, endpoint=False)
    rad = 0.02 - R + rng.uniform(0, 2e-5, n)  # all pressed against the wall
    pos = np.stack([rng.uniform(-0.01, 0.01, n), rad * np.cos(ang), rad * np.sin(ang)], 1)
    vel = rng.normal(0, 0.02, (n, 3))
    V = np.array(V)
    out = []
    for moving in (False, True):
        s = sim(dt=1e-5, K=10, rolling="constant", lo=-0.5, hi=0.5)
        _drum(s, moving, V, (1, 0, 0), 3.0)
        s.set_particles(pos, [R] * n, vel=vel + (V if moving else 0.0))
        s.step(500)
        st = s.state()
        out.append((st["pos"], st["vel"], st["time"]))
    shift = V * out[1][2]
    assert np.max(np.abs(out[1][0] - (out[0][0] + shift))) < 1e-12
    assert np.max(np.abs(out[1][1] - (out[0][1] + V))) < 1e-9


def test_translating_hopper_cone_is_galilean(oracle_built):
    rng = np.random.default_rng(6)
    n = 25
    z = rng.uniform(0.01, 0.03, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    slope = 0.6
    rr = 0.01 + slope * z - R * 1.2
    pos = np.stack([rr * np.cos(ang), rr * np.sin(ang), z], 1)
    keep = [0]
    for i in range(1, n):
        if np.min(np.linalg.norm(pos[keep] - pos[i], axis=1)) > 2.2 * R:
            keep.append(i)
    pos = pos[keep]
    V = np.array([0.0, 0.0, 0.03])
    out = []
    for moving in (False, True):
        s = sim(dt=1e-5, K=10, lo=-0.5, hi=0.5)
        w = s.add_cone((0, 0, 0), (0, 0, 1), 0.01, slope, 0.0, 0.05, True, 0, 1.5)
        if moving:
            s.set_wall_velocity(w, V)
        s.set_particles(pos, [R] * len(pos), vel=np.zeros_like(pos) + (V if moving else 0.0))
        s.step(400)
        st = s.state()
        out.append((st["pos"], st["time"]))
    assert np.max(np.abs(out[1][0] - (out[0][0] + V * out[1][1]))) < 1e-12


def test_wall_faster_than_half_skin_per_search_is_rejected(oracle_built):
    s = sim(dt=1e-5, K=100)
    w = s.add_plane((0, 0, 0), (0, 0, 1))
    s.set_wall_velocity(w, (0.0, 0.0, 1.0))  # 1 mm per search > half the skin (0.45 mm)
    with pytest.raises(Exception):
        s.set_particles([[0, 0, 0.01]], [R])
