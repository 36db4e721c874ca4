"""Pins of the effective mass and radius with unequal spheres.

The table of effective parameters of Sec. 2.1 combines the two bodies of a
contact as 1/m_e = 1/m_i + 1/m_j and 1/R_e = 1/R_i + 1/R_j, and Young's
moduli and Poisson ratios of two materials into Y_e.  With equal spheres many
wrong combinations agree with these (a geometric or arithmetic mean gives
m_e = m at equal masses, only half as large as the right m / 2, and the
equal-sphere pins scale their expectations from m / 2 themselves), so these
pins collide spheres that differ in radius, density and material, and check
the oracle against closed forms of mechanics computed here:
* the undamped Hertz contact time 2.868 (m_e^2 / (R_e Y_e^2 v))^(1/5) and
  maximum overlap (15 m_e v^2 / (16 Y_e sqrt(R_e)))^(2/5) (these pin R_e and
  Y_e: without damping the Hertz law itself does not contain m_e);
* the restitution of a damped Hertz impact: the relative motion of the two
  spheres is that of one body of mass m_e, so the damping coefficient of
  Eqs. (nonlinearetan), built with the same m_e, returns exactly the input
  e (the continuous-time value, reached as dt shrinks); any other m_e in the
  damping changes the damping ratio and with it the rebound;
* for the linear law the oscillator of stiffness k = m_e V^2 / delta_H(V)^2
  (the stiffness that reaches Hertz's maximum overlap at the characteristic
  velocity V): contact time pi sqrt(m_e / k) and maximum overlap
  v sqrt(m_e / k).
Momentum conservation across the impact fixes the mass ratio independently.
"""
import math

import pytest

from oracle import OracleSim

# two materials: a light, soft sphere and a heavy, stiff one
MAT_A = dict(density=2000.0, youngs=1.0e6, poisson=0.30, restitution=1.0, friction=0.0,
             rolling_friction=0.0)
MAT_B = dict(density=7850.0, youngs=5.0e6, poisson=0.25, restitution=1.0, friction=0.0,
             rolling_friction=0.0)
RA, RB = 0.75e-3, 1.5e-3


def _mass(mat, r):
    return mat["density"] * 4.0 / 3.0 * math.pi * r ** 3


def _effective():
    ma, mb = _mass(MAT_A, RA), _mass(MAT_B, RB)
    me = ma * mb / (ma + mb)
    Re = RA * RB / (RA + RB)
    Ye = 1.0 / ((1.0 - MAT_A["poisson"] ** 2) / MAT_A["youngs"]
                + (1.0 - MAT_B["poisson"] ** 2) / MAT_B["youngs"])
    return ma, mb, me, Re, Ye


def _impact(model, v0, dt, V=0.0, e=1.0):
    """Head-on impact along z at relative speed v0 in the centre-of-mass
    frame (both materials with restitution e); returns (contact time, max
    overlap, final velocities)."""
    s = OracleSim(dt=dt, gravity=(0, 0, 0), domain_lo=(-1, -1, -1), domain_hi=(1, 1, 1),
                  neighbor_threshold=1.3, rebuild_interval=1, rolling_model="none",
                  contact_model=model, characteristic_velocity=V)
    s.set_material(0, **dict(MAT_A, restitution=e))
    s.set_material(1, **dict(MAT_B, restitution=e))
    ma, mb = _mass(MAT_A, RA), _mass(MAT_B, RB)
    va, vb = v0 * mb / (ma + mb), -v0 * ma / (ma + mb)
    s.set_particles([[0, 0, 0], [0, 0, RA + RB + 1e-9]], [RA, RB],
                    vel=[[0, 0, va], [0, 0, vb]], types=[0, 1])
    n_in, best, was = 0, 0.0, False
    for _ in range(400000):
        s.step(1)
        st = s.state()
        ov = RA + RB - (st["pos"][1, 2] - st["pos"][0, 2])
        if ov > 0:
            was = True
            n_in += 1
            best = max(best, ov)
        elif was:
            return n_in * dt, best, st["vel"]
    raise AssertionError("collision did not end")


def test_hertz_contact_time_and_overlap_unequal_spheres(oracle_built):
    ma, mb, me, Re, Ye = _effective()
    v0 = 0.5
    dt = 5e-8
    tc = 2.868265699 * (me ** 2 / (Re * Ye ** 2 * v0)) ** 0.2
    dmax = (15.0 * me * v0 ** 2 / (16.0 * Ye * math.sqrt(Re))) ** 0.4
    t, best, vel = _impact("nonlinear", v0, dt)
    assert abs(t - tc) / tc < 2e-3, (t, tc)
    assert abs(best - dmax) / dmax < 1e-3, (best, dmax)
    # elastic: each sphere leaves with its velocity reversed, momentum zero
    va, vb = v0 * mb / (ma + mb), -v0 * ma / (ma + mb)
    assert abs(vel[0, 2] + va) / abs(va) < 1e-4
    assert abs(vel[1, 2] + vb) / abs(vb) < 1e-4
    assert abs(ma * vel[0, 2] + mb * vel[1, 2]) <= 1e-12 * ma * abs(va)


@pytest.mark.parametrize("e", [0.5, 0.8])
def test_hertz_restitution_unequal_spheres(oracle_built, e):
    ma, mb, me, Re, Ye = _effective()
    v0 = 0.5
    errs = []
    for dt in (1e-7, 5e-8):
        _, _, vel = _impact("nonlinear", v0, dt, e=e)
        errs.append(abs((vel[1, 2] - vel[0, 2]) / v0 - e))
        assert abs(ma * vel[0, 2] + mb * vel[1, 2]) <= 1e-12 * ma * v0
    assert errs[-1] < 1e-3, errs
    assert errs[-1] <= errs[0] + 1e-6, errs  # converges as dt shrinks


def test_wrong_effective_masses_would_be_caught(oracle_built):
    """The contact-time pin above separates the harmonic combination from the
    geometric and arithmetic means and the sum by more than ten times its
    tolerance."""
    ma, mb, me, Re, Ye = _effective()
    v0 = 0.5
    tc = lambda m: 2.868265699 * (m ** 2 / (Re * Ye ** 2 * v0)) ** 0.2  # noqa: E731
    for wrong in (math.sqrt(ma * mb), 0.5 * (ma + mb), ma + mb):
        assert abs(tc(wrong) - tc(me)) / tc(me) > 10 * 2e-3


@pytest.mark.parametrize("V", [0.5, 1.0])
def test_linear_law_contact_time_and_overlap_unequal_spheres(oracle_built, V):
    ma, mb, me, Re, Ye = _effective()
    dH = (15.0 * me * V ** 2 / (16.0 * Ye * math.sqrt(Re))) ** 0.4
    k = me * V ** 2 / dH ** 2
    v0 = 0.3
    dt = 5e-8
    t, best, _ = _impact("linear", v0, dt, V=V)
    assert abs(t - math.pi * math.sqrt(me / k)) / (math.pi * math.sqrt(me / k)) < 2e-3
    assert abs(best - v0 * math.sqrt(me / k)) / (v0 * math.sqrt(me / k)) < 1e-3
