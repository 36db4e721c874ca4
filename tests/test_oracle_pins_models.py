"""Pins of the oracle's second contact model and second rolling model.

Linear spring-dashpot (Sec. 2.1, Eqs. linearkn and linearetan, the same
constants in the tangential direction) and the viscous rolling torque (second
row of the table of rolling models).  The expected values come from closed
forms of mechanics, not from the oracle's formulas: the linear oscillator's
contact time and restitution, the energy equivalence with Hertz's maximum
overlap that the linear stiffness is built on, rigid-body rolling, and special
spin configurations in which the rolling velocity vanishes.
"""
import math

import numpy as np
import pytest

from oracle import OracleSim

MAT = dict(density=2500.0, youngs=1.0e6, poisson=0.3, restitution=0.9, friction=0.3,
           rolling_friction=0.1)
R = 1.5e-3


def sim(mat=MAT, dt=1e-6, gravity=(0, 0, 0), K=1, rolling="none", model="linear", V=1.0):
    s = OracleSim(dt=dt, gravity=gravity, domain_lo=(-1, -1, -1), domain_hi=(1, 1, 1),
                  neighbor_threshold=1.3, rebuild_interval=K, rolling_model=rolling,
                  contact_model=model, characteristic_velocity=V)
    s.set_material(0, **mat)
    s.dt = dt
    return s


def mass(r=R, rho=MAT["density"]):
    return rho * 4.0 / 3.0 * math.pi * r ** 3


def ye(mat=MAT):
    return 1.0 / (2.0 * (1.0 - mat["poisson"] ** 2) / mat["youngs"])


def hertz_dmax(me, Re, Ye, v):
    """Maximum overlap of an undamped Hertz impact at speed v (textbook)."""
    return (15.0 * me * v * v / (16.0 * Ye * math.sqrt(Re))) ** 0.4


def head_on(s, v0, wall=False):
    """Run a head-on impact; returns (restitution, contact time, max overlap)."""
    dt = s.dt
    if wall:
        s.add_plane((0, 0, 0), (0, 0, 1), 0)
        s.set_particles([[0.0, 0.0, R + 1e-9]], [R], vel=[[0, 0, -v0]])
    else:
        s.set_particles([[0, 0, 0], [0, 0, 2 * R + 1e-9]], [R, R],
                        vel=[[0, 0, v0 / 2], [0, 0, -v0 / 2]])
    n_in, best, was = 0, 0.0, False
    for _ in range(400000):
        s.step(1)
        st = s.state()
        if wall:
            gap = st["pos"][0, 2] - R
            vrel = st["vel"][0, 2]
        else:
            gap = st["pos"][1, 2] - st["pos"][0, 2] - 2 * R
            vrel = st["vel"][1, 2] - st["vel"][0, 2]
        if gap < 0:
            was = True
            n_in += 1
            best = max(best, -gap)
        elif was:
            return vrel / v0, n_in * dt, best
    raise AssertionError("collision did not end")


# ------------------------------------------------------- linear spring-dashpot

def test_linear_undamped_matches_hertz_energy_at_characteristic_velocity(oracle_built):
    """Eq. (linearkn) picks the stiffness whose undamped impact at the
    characteristic velocity V reaches Hertz's maximum overlap: then
    k = m_e V^2 / delta_H^2, the contact lasts pi sqrt(m_e / k) = pi delta_H / V,
    and the overlap peaks at delta_H."""
    me, Re, Ye = mass() / 2, R / 2, ye()
    V = 0.8
    s = sim(mat=dict(MAT, restitution=1.0, friction=0.0), dt=2e-7, V=V)
    e, tc, dmax = head_on(s, V)
    dH = hertz_dmax(me, Re, Ye, V)
    assert dmax == pytest.approx(dH, rel=1e-3)
    assert tc == pytest.approx(math.pi * dH / V, rel=2e-3)
    assert e == pytest.approx(1.0, abs=1e-4)


def test_linear_spring_is_linear_in_impact_speed(oracle_built):
    """A linear spring: the maximum overlap scales with the impact speed and
    the contact time does not depend on it."""
    mat = dict(MAT, restitution=1.0, friction=0.0)
    out = {}
    for v in (0.25, 1.0):
        s = sim(mat=mat, dt=2e-7, V=1.0)
        out[v] = head_on(s, v)
    assert out[0.25][2] / out[1.0][2] == pytest.approx(0.25, rel=1e-3)
    assert out[0.25][1] == pytest.approx(out[1.0][1], rel=2e-3)


@pytest.mark.parametrize("e", [0.3, 0.7])
@pytest.mark.parametrize("wall", [False, True])
def test_linear_restitution_and_damped_contact_time(oracle_built, e, wall):
    """Eq. (linearetan) makes the linear oscillator's restitution equal to e at
    any impact speed (damping ratio zeta = |ln e| / sqrt(ln^2 e + pi^2)), and
    the damped contact lasts sqrt(1 + (ln e / pi)^2) times the undamped one."""
    mat = dict(MAT, restitution=e, friction=0.0)
    res = []
    for v in (0.2, 1.0):
        s = sim(mat=mat, dt=2e-7, V=0.5)
        res.append(head_on(s, v, wall=wall))
    s1 = sim(mat=dict(mat, restitution=1.0), dt=2e-7, V=0.5)
    _, tc1, _ = head_on(s1, 1.0, wall=wall)
    for e_num, tc, _ in res:
        assert e_num == pytest.approx(e, abs=2e-3)
        assert tc == pytest.approx(tc1 * math.sqrt(1 + (math.log(e) / math.pi) ** 2), rel=3e-3)


def test_linear_tangential_constants_equal_normal(oracle_built):
    """The tangential spring and damping constants of the linear model are the
    normal ones (Sec. 2.1, sentence after Eq. linearetan); the normal stiffness
    is m_e V^2 / delta_H^2 (energy equivalence with Hertz at V)."""
    V = 0.6
    s = sim(mat=dict(MAT, friction=10.0), V=V)
    me, Re, Ye = mass() / 2, R / 2, ye()
    k_expect = me * V * V / hertz_dmax(me, Re, Ye, V) ** 2
    n = np.array([0.0, 0.0, 1.0])
    t = np.array([1.0, 0.0, 0.0])
    dn = 2e-5
    xi, xj = np.zeros(3), (2 * R - dn) * n
    z = np.zeros(3)
    a = s.pair_force(xi, xj, z, z, z, z, R, R)
    kn = -a["F"][2] / dn
    assert kn == pytest.approx(k_expect, rel=1e-9)
    # tangential spring: a stored overlap at rest
    d0 = 1e-7 * t
    b = s.pair_force(xi, xj, z, z, z, z, R, R, delta_t=d0)
    assert -b["F"][0] / 1e-7 == pytest.approx(kn, rel=1e-9)
    # damping: the same relative speed u along n and along t
    u = 0.01
    c = s.pair_force(xi, xj, u * n, z, z, z, R, R)
    eta_n = (-c["F"][2] - kn * dn) / u
    assert eta_n > 0
    d = s.pair_force(xi, xj, u * t, z, z, z, R, R)
    # F^t = -k_t (u dt) - eta_t u, the overlap being incremented first
    assert -d["F"][0] == pytest.approx(kn * u * s.dt + eta_n * u, rel=1e-9)


def test_linear_model_needs_characteristic_velocity(oracle_built):
    with pytest.raises(Exception):
        sim(V=0.0)


# ---------------------------------------------------------- viscous rolling

def test_viscous_rolling_torque_special_spins(oracle_built):
    """Viscous rolling torque -mu_r R_e |F^n| |V_omega| w_hat with V_omega =
    (R_i w_i + R_j w_j) x n: with w_j = 0 and w_i normal to n, |V_omega| =
    R_i |w_i|; gear-like spins R_i w_i = -R_j w_j roll without slip (V_omega =
    0, no torque although w_i != w_j); spins along n give no torque either.
    Friction 0 removes the tangential force, so the torque is the rolling one;
    the normal force is Hertz's static force."""
    mur = 0.2
    s = sim(mat=dict(MAT, friction=0.0, rolling_friction=mur), rolling="viscous",
            model="nonlinear", dt=1e-5)
    Ri, Rj = 1.5e-3, 1.0e-3
    n = np.array([0.0, 0.0, 1.0])
    dn = 1e-5
    xi, xj = np.zeros(3), (Ri + Rj - dn) * n
    z = np.zeros(3)
    Re = Ri * Rj / (Ri + Rj)
    Fn = 4.0 / 3.0 * ye() * math.sqrt(Re) * dn ** 1.5
    w = np.array([30.0, -40.0, 0.0])
    a = s.pair_force(xi, xj, z, z, w, z, Ri, Rj)
    Mr = -mur * Re * Fn * (Ri * 50.0) * w / 50.0
    np.testing.assert_allclose(a["Mi"], Mr, rtol=1e-9)
    np.testing.assert_allclose(a["Mj"], -Mr, rtol=1e-9)
    # the torque grows with the spin (unlike the constant model)
    b = s.pair_force(xi, xj, z, z, 3 * w, z, Ri, Rj)
    np.testing.assert_allclose(b["Mi"], 3 * Mr, rtol=1e-9)
    g = s.pair_force(xi, xj, z, z, w, -(Ri / Rj) * w, Ri, Rj)
    assert np.max(np.abs(g["Mi"])) <= 1e-12 * np.max(np.abs(Mr))
    tw = s.pair_force(xi, xj, z, z, 40.0 * n, z, Ri, Rj)
    assert np.max(np.abs(tw["Mi"])) <= 1e-12 * np.max(np.abs(Mr))


def test_viscous_rolling_decays_exponentially_on_plane(oracle_built):
    """On a static plane the rolling velocity is |V_omega| = R |w| = v, so the
    torque mu_r R m g v decelerates the rolling sphere at (5/7) mu_r g v:
    v(t) = v0 exp(-(5/7) mu_r g t) (rigid-body rolling)."""
    mur = 0.5
    mat = dict(MAT, friction=0.5, rolling_friction=mur, restitution=0.3)
    dt = 2e-6
    s = sim(mat=mat, dt=dt, gravity=(0, 0, -9.81), K=20, rolling="viscous",
            model="nonlinear")
    s.add_plane((0, 0, 0), (0, 0, 1))
    m = mass()
    deq = (3 * m * 9.81 / (4 * ye() * math.sqrt(R))) ** (2 / 3)
    v0 = 0.1
    s.set_particles([[0, 0, R - deq]], [R], vel=[[v0, 0, 0]], omega=[[0, v0 / R, 0]])
    s.step(2000)
    v1 = s.state()["vel"][0, 0]
    s.step(20000)
    v2 = s.state()["vel"][0, 0]
    rate = math.log(v1 / v2) / (20000 * dt)
    assert rate == pytest.approx(5 / 7 * mur * 9.81, rel=2e-2)


def test_viscous_rolling_against_rotating_wall_uses_relative_spin(oracle_built):
    """Against a rotating wall V_omega uses the spin relative to the wall's: a
    sphere spinning with the wall feels no rolling torque; one at rest feels
    mu_r R |F^n| R |Omega| towards the wall's spin (contacts on the rotation
    axis, where the surface does not move; friction 0)."""
    mur = 0.3
    s = sim(mat=dict(MAT, friction=0.0, rolling_friction=mur), rolling="viscous",
            model="nonlinear", dt=1e-6, gravity=(0, 0, -9.81))
    Om = np.array([0.0, 2.0, 0.0])
    s.add_plane((0, 0, 0), (0, 0, 1), 0, axis_point=(0, 0, 0), omega=Om)
    s.set_particles([[0, 0, R - 1e-6], [0, 0.1, R - 1e-6]], [R, R], omega=[Om, [0, 0, 0]])
    s.step(1)
    F, T, _ = s.forces()
    assert np.all(T[0] == 0)
    fn = np.linalg.norm(F[1])
    assert fn > 0
    np.testing.assert_allclose(T[1], [0.0, mur * R * fn * R * 2.0, 0.0], rtol=1e-9, atol=1e-18)
