"""Pins of the oracle's two force scales (test infrastructure for the error
measures): the net contact-force scale sum |F^n + F^t| and the term scale,
the sum of the magnitudes of the spring and dashpot terms of Eqs.
(normal_force) and (tangential_force) before the Coulomb limit.

The term scale never falls below the net scale (triangle inequality); for an
approaching head-on pair the spring and dashpot push the same way, so the two
scales agree; for the same pair separating, the dashpot pulls against the
spring: the term scale keeps its value and the net scale becomes the
difference of the two terms, whose spring part a static pair of the same
geometry gives on its own.
"""
import numpy as np

import workloads as W
from oracle import OracleSim, oracle_from_scene

MAT = dict(density=2500.0, youngs=1.0e6, poisson=0.3, restitution=0.5, friction=0.3,
           rolling_friction=0.0)
R = 1.5e-3
DT = 1e-6
OVERLAP = 2e-5


def pair_after_one_step(v, restitution):
    """Two spheres along z, their overlap OVERLAP after the first drift, closing
    speed 2 v (v > 0 approaching, v < 0 separating), no gravity; one step."""
    s = OracleSim(dt=DT, gravity=(0, 0, 0), domain_lo=(-1, -1, -1), domain_hi=(1, 1, 1),
                  rebuild_interval=1, rolling_model="none")
    s.set_material(0, **dict(MAT, restitution=restitution))
    gap = 2 * R - OVERLAP + 2 * v * DT  # undone by the drift of the first step
    s.set_particles([[0.0, 0.0, 0.0], [0.0, 0.0, gap]], [R, R],
                    vel=[[0.0, 0.0, v], [0.0, 0.0, -v]])
    s.step(1)
    F, T, S = s.forces()
    return F, S, s.term_scale()


def test_term_scale_is_never_below_the_net_scale(oracle_built):
    sc = W.dense_snapshot(n=2500, seed=29, polydisperse=0.1, n_types=2, K=10)
    o = oracle_from_scene(sc)
    o.step(20)
    _, _, S = o.forces()
    S2 = o.term_scale()
    assert np.count_nonzero(S) > 1000
    assert np.all(S2 >= S * (1.0 - 1e-12))
    assert np.array_equal(S == 0, S2 == 0)  # both zero exactly without contacts
    assert np.any(S2 > 1.5 * S)  # dashpots oppose springs somewhere in a dense bed


def test_term_scale_of_a_head_on_pair(oracle_built):
    # static, undamped: the spring alone; both scales equal |F|
    F0, S0, T0 = pair_after_one_step(0.0, 1.0)
    spring = np.linalg.norm(F0[0])
    assert spring > 0
    np.testing.assert_allclose([S0[0], T0[0], T0[1]], spring, rtol=1e-14)
    # approaching, damped: spring and dashpot add up
    Fa, Sa, Ta = pair_after_one_step(0.05, 0.5)
    np.testing.assert_allclose(Ta[0], Sa[0], rtol=1e-13)
    assert Ta[0] > spring * (1 + 1e-3)
    # separating at the same speed: same terms, net force their difference
    Fs, Ss, Ts = pair_after_one_step(-0.05, 0.5)
    np.testing.assert_allclose(Ts[0], Ta[0], rtol=1e-9)
    dashpot = Ta[0] - spring
    np.testing.assert_allclose(Ss[0], abs(spring - dashpot), rtol=1e-6)
    assert Ts[0] > Ss[0]
