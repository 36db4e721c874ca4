"""Pins of the FP64 oracle against what the paper and mechanics fix.

Each test checks the oracle against a value that does not come from the
oracle's own formulas: closed forms (free fall, Hertz contact, rigid-body
rolling), an independent high-accuracy ODE integration of the contact law,
conservation laws, exact symmetries, brute force, and the convergence orders
the paper prints for its two integrators.  A plausible mistake in the oracle
(a dropped term, a wrong sign, a swapped operand) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import OracleSim, oracle_from_scene
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MAT = dict(density=2500.0, youngs=1.0e6, poisson=0.3, restitution=0.9, friction=0.3,
           rolling_friction=0.1)


def sim_with(mat=MAT, dt=1e-5, gravity=(0, 0, -9.81), lo=(-1, -1, -1), hi=(1, 1, 1), K=20,
             integrator="verlet", rolling="constant", threshold=1.3, mats=None):
    s = OracleSim(dt=dt, gravity=gravity, domain_lo=lo, domain_hi=hi,
                  neighbor_threshold=threshold, rebuild_interval=K, integrator=integrator,
                  rolling_model=rolling)
    for t, m in enumerate(mats or [mat]):
        s.set_material(t, **m)
    return s


def eff(mat_a, mat_b):
    Ye = 1.0 / ((1 - mat_a["poisson"] ** 2) / mat_a["youngs"] + (1 - mat_b["poisson"] ** 2) / mat_b["youngs"])
    return Ye


# ----------------------------------------------------------------- P1 free fall

def test_free_fall_velocity_verlet_exact(oracle_built):
    """Velocity Verlet is exact for constant acceleration (free-fall part of the
    wall-collision verification, Sec. 4.1.1, first equation)."""
    s = sim_with(dt=1e-4, K=10**9)  # single particle: no search needed
    z0 = 0.5
    s.set_particles([[0.0, 0.0, z0]], [1e-3])
    done = 0
    for n in (1, 10, 100, 1000):
        s.step(n - done)
        done = n
        t = n * 1e-4
        st = s.state()
        assert abs(st["pos"][0, 2] - (z0 - 9.81 * t * t / 2)) < 1e-12
        assert abs(st["vel"][0, 2] - (-9.81 * t)) < 1e-12
        assert st["time"] == pytest.approx(t, rel=1e-15)


def test_free_fall_explicit_euler_discrete_closed_form(oracle_built):
    """Explicit Euler (Eq. integ_EE): z_n = z0 - g dt^2 n(n-1)/2, v_n = -g n dt."""
    dt = 1e-4
    s = sim_with(dt=dt, integrator="euler", K=10**9)
    s.set_particles([[0.0, 0.0, 0.5]], [1e-3])
    s.step(500)
    st = s.state()
    n = 500
    assert abs(st["pos"][0, 2] - (0.5 - 9.81 * dt * dt * n * (n - 1) / 2)) < 1e-12
    assert abs(st["vel"][0, 2] + 9.81 * n * dt) < 1e-12


# ------------------------------------------------------------ P2 Hertz contact

def _ode_restitution(e, v0, me, Re, Ye):
    """Independent continuous-time integration of the head-on normal law."""
    beta = math.log(e) / math.sqrt(math.log(e) ** 2 + math.pi ** 2)

    def rhs(t, y):
        d, dd = y
        d = max(d, 0.0)
        a = math.sqrt(Re * d)
        damp = -2.0 * math.sqrt(5.0 / 6.0) * beta * math.sqrt(2.0 * Ye * a * me)
        return [dd, -((4.0 / 3.0) * Ye * a * d + damp * dd) / me]

    ev = lambda t, y: y[0]  # noqa: E731
    ev.terminal = True
    ev.direction = -1
    sol = solve_ivp(rhs, [0, 1.0], [0.0, v0], method="DOP853", rtol=1e-12, atol=1e-18,
                    events=ev, first_step=1e-9)
    return -sol.y_events[0][0][1] / v0


def _head_on(e, v0, dt, wall=False):
    mat = dict(MAT, restitution=e, friction=0.3, rolling_friction=0.0)
    R = 1.5e-3
    s = sim_with(mat=mat, dt=dt, gravity=(0, 0, 0), K=1)
    if wall:
        s.add_plane((0, 0, 0), (0, 0, 1), 0)
        s.set_particles([[0.0, 0.0, R + 1e-6]], [R], vel=[[0, 0, -v0]])
    else:
        s.set_particles([[0, 0, 0], [0, 0, 2 * R + 1e-6]], [R, R],
                        vel=[[0, 0, v0 / 2], [0, 0, -v0 / 2]])
    steps_in_contact = 0
    was = False
    for _ in range(200000):
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
            steps_in_contact += 1
        elif was:
            return vrel / v0, steps_in_contact
    raise AssertionError("collision did not end")


@pytest.mark.parametrize("e", [0.3, 0.5, 0.9])
def test_restitution_particle_particle(oracle_built, e):
    """Head-on binary collisions recover the input restitution coefficient: the
    damping coefficient of Eqs. (nonlinearetan) with beta of the parameter
    table makes the continuous-time restitution equal to e (independent ODE),
    and the oracle converges to it as dt shrinks."""
    R = 1.5e-3
    m = MAT["density"] * 4 / 3 * math.pi * R ** 3
    Ye = eff(MAT, MAT)
    e_ode = _ode_restitution(e, 1.0, m / 2, R / 2, Ye)
    assert abs(e_ode - e) < 1e-8
    errs = []
    for dt in (4e-6, 2e-6, 1e-6):
        e_num, steps = _head_on(e, 1.0, dt)
        errs.append(abs(e_num - e_ode))
    assert steps > 500
    # first-order error of Verlet with a velocity-dependent force, ~1/(steps)
    assert max(errs) < 2e-3, errs
    assert errs[-1] < 5e-4, errs


@pytest.mark.parametrize("e", [0.5, 0.8])
def test_restitution_particle_wall(oracle_built, e):
    """Same pin for a sphere hitting a plane (wall = body of infinite mass and
    radius, Sec. 2.1 last paragraph)."""
    R = 1.5e-3
    m = MAT["density"] * 4 / 3 * math.pi * R ** 3
    Ye = eff(MAT, MAT)
    e_ode = _ode_restitution(e, 0.5, m, R, Ye)
    e_num, steps = _head_on(e, 0.5, 1e-6, wall=True)
    assert steps > 300
    assert abs(e_num - e_ode) < 1e-3


def test_hertz_undamped_contact_time_and_max_overlap(oracle_built):
    """Undamped Hertz impact (e = 1): contact time 2.868 (m_e^2/(R_e Y_e^2 v))^(1/5)
    and maximum overlap (15 m_e v^2 / (16 Y_e sqrt(R_e)))^(2/5) (textbook Hertz)."""
    mat = dict(MAT, restitution=1.0, friction=0.0, rolling_friction=0.0)
    R = 1.5e-3
    v0 = 1.0
    dt = 2e-7
    s = sim_with(mat=mat, dt=dt, gravity=(0, 0, 0), K=1)
    s.set_particles([[0, 0, 0], [0, 0, 2 * R]], [R, R], vel=[[0, 0, v0 / 2], [0, 0, -v0 / 2]])
    m = mat["density"] * 4 / 3 * math.pi * R ** 3
    me, Re, Ye = m / 2, R / 2, eff(mat, mat)
    tc = 2.868265699 * (me ** 2 / (Re * Ye ** 2 * v0)) ** 0.2
    dmax = (15 * me * v0 ** 2 / (16 * Ye * math.sqrt(Re))) ** 0.4
    n_contact = 0
    best = 0.0
    started = False
    for _ in range(20000):
        s.step(1)
        p = s.state()["pos"]
        ov = 2 * R - (p[1, 2] - p[0, 2])
        if ov > 0:
            started = True
            n_contact += 1
            best = max(best, ov)
        elif started:
            break
    assert abs(n_contact * dt - tc) / tc < 2e-3
    assert abs(best - dmax) / dmax < 1e-3
    v = s.state()["vel"]
    assert abs((v[1, 2] - v[0, 2]) / v0 - 1.0) < 1e-4  # elastic


def test_static_hertz_force_and_mindlin_stiffness(oracle_built):
    """At rest the normal force is Hertz's (4/3) Y_e sqrt(R_e) delta^(3/2) along
    -n on i; a tangential overlap below the Coulomb limit gives Mindlin's
    no-slip force -8 G_e sqrt(R_e delta) delta_t."""
    mats = [MAT, dict(MAT, youngs=5e6, poisson=0.25, density=3000.0)]
    s = sim_with(mats=mats)
    Ri, Rj, delta = 1.5e-3, 1.0e-3, 2e-5
    xi = np.array([0.01, 0.02, 0.03])
    n = np.array([1.0, 2.0, -2.0]) / 3.0
    xj = xi + (Ri + Rj - delta) * n
    z = np.zeros(3)
    out = s.pair_force(xi, xj, z, z, z, z, Ri, Rj, 0, 1)
    Ye = eff(mats[0], mats[1])
    Re = Ri * Rj / (Ri + Rj)
    Fh = 4.0 / 3.0 * Ye * math.sqrt(Re) * delta ** 1.5
    np.testing.assert_allclose(out["F"], -Fh * n, rtol=1e-9, atol=1e-18)
    np.testing.assert_allclose(out["Mi"], 0, atol=1e-18)
    # tangential: a small tangential overlap perpendicular to n, zero velocity
    t = np.cross(n, [0.0, 0.0, 1.0])
    t /= np.linalg.norm(t)
    dt0 = 1e-7 * t
    out = s.pair_force(xi, xj, z, z, z, z, Ri, Rj, 0, 1, delta_t=dt0)
    Ge = 1.0 / sum(2 * (2 - m["poisson"]) * (1 + m["poisson"]) / m["youngs"] for m in mats)
    Ft_expect = -8 * Ge * math.sqrt(Re * delta) * dt0
    Fn_expect = -Fh * n
    np.testing.assert_allclose(out["F"], Fn_expect + Ft_expect, rtol=1e-9, atol=1e-15)
    # torque on i is R_i n x F^t, on j R_j n x F^t (same sense, action-reaction)
    np.testing.assert_allclose(out["Mi"], Ri * np.cross(n, Ft_expect), rtol=1e-9, atol=1e-20)
    np.testing.assert_allclose(out["Mj"], Rj * np.cross(n, Ft_expect), rtol=1e-9, atol=1e-20)
    np.testing.assert_allclose(out["delta_t"], dt0, rtol=0, atol=0)


def test_pair_not_touching_resets_history(oracle_built):
    s = sim_with()
    z = np.zeros(3)
    out = s.pair_force([0, 0, 0], [0, 0, 3.0001e-3], z, z, z, z, 1.5e-3, 1.5e-3,
                       delta_t=(1e-6, 2e-6, 0))
    assert not out["touching"]
    assert np.all(out["delta_t"] == 0) and np.all(out["F"] == 0)


# --------------------------------------------------------------- P13 symmetry

def test_exact_antisymmetry_and_frame_invariance(oracle_built):
    """Evaluating a pair from j's side gives exactly -F and -delta_t and swaps the
    torques; rotating the whole configuration rotates every output; adding a
    common translational velocity changes nothing."""
    mats = [MAT, dict(MAT, youngs=5e6, poisson=0.25, density=3000.0, restitution=0.5,
                      friction=0.1, rolling_friction=0.05)]
    s = sim_with(mats=mats)
    rng = np.random.default_rng(3)
    for trial in range(200):
        Ri, Rj = rng.uniform(0.8e-3, 1.6e-3, 2)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        xi = rng.uniform(0, 0.1, 3)
        xj = xi + (Ri + Rj) * (1 - rng.uniform(1e-4, 3e-2)) * n
        vi, vj = rng.normal(0, 0.3, (2, 3))
        wi, wj = rng.normal(0, 50, (2, 3))
        dt0 = rng.normal(0, 2e-6, 3)
        ti, tj = rng.integers(0, 2, 2)
        a = s.pair_force(xi, xj, vi, vj, wi, wj, Ri, Rj, ti, tj, dt0)
        b = s.pair_force(xj, xi, vj, vi, wj, wi, Rj, Ri, tj, ti, -dt0)
        assert a["touching"] and b["touching"]
        assert np.array_equal(a["F"], -b["F"])
        assert np.array_equal(a["delta_t"], -b["delta_t"])
        assert np.array_equal(a["Mi"], b["Mj"])
        assert np.array_equal(a["Mj"], b["Mi"])
        # frame rotation
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        c = s.pair_force(q @ xi, q @ xj, q @ vi, q @ vj, q @ wi, q @ wj, Ri, Rj, ti, tj, q @ dt0)
        scale = np.linalg.norm(a["F"]) + 1e-30
        assert np.linalg.norm(c["F"] - q @ a["F"]) <= 1e-9 * scale
        tscale = np.linalg.norm(a["Mi"]) + np.linalg.norm(a["Mj"]) + 1e-30
        assert np.linalg.norm(c["Mi"] - q @ a["Mi"]) <= 1e-8 * tscale
        # Galilean invariance
        u = rng.normal(0, 1.0, 3)
        d = s.pair_force(xi, xj, vi + u, vj + u, wi, wj, Ri, Rj, ti, tj, dt0)
        assert np.linalg.norm(d["F"] - a["F"]) <= 1e-9 * scale


def test_coulomb_limit_holds_and_truncates_overlap(oracle_built):
    """After truncation |F^t| = mu |F^n| and the stored overlap reproduces the
    limited elastic force: -k_t delta_t = F_hat + eta_t v_rt (continuity)."""
    mat = dict(MAT, friction=0.2)
    s = sim_with(mat=mat)
    R = 1.5e-3
    n = np.array([0.0, 0.0, 1.0])
    xi, xj = np.zeros(3), (2 * R - 1e-5) * n
    z = np.zeros(3)
    big = np.array([5e-5, 0, 0])  # far beyond the limit
    out = s.pair_force(xi, xj, z, z, z, z, R, R, delta_t=big)
    F = out["F"]
    Fn = np.dot(F, n) * n
    Ft = F - Fn
    assert np.linalg.norm(Ft) == pytest.approx(0.2 * np.linalg.norm(Fn), rel=1e-12)
    # with zero velocity the limited overlap is F_hat / (-k_t)
    Ge = 1.0 / (2 * 2 * (2 - 0.3) * (1 + 0.3) / 1e6)
    kt = 8 * Ge * math.sqrt(R / 2 * 1e-5)
    np.testing.assert_allclose(out["delta_t"], -Ft / kt, rtol=1e-12)
    # zero friction: tangential force vanishes (no 0/0)
    s0 = sim_with(mat=dict(MAT, friction=0.0))
    out0 = s0.pair_force(xi, xj, z, [0.1, 0, 0], z, z, R, R, delta_t=big)
    assert abs(out0["F"][0]) == 0.0 and np.all(np.isfinite(out0["delta_t"]))


def test_rolling_torque_constant_model(oracle_built):
    """Constant rolling torque: -mu_r R_e |F^n| (w_i - w_j)/|w_i - w_j| on i and
    the opposite on j (first row of the rolling-model table), independent of |w|;
    zero when the angular velocities are equal."""
    s = sim_with(mat=dict(MAT, friction=0.0))
    R = 1.5e-3
    n = np.array([0.0, 0.0, 1.0])
    xi, xj = np.zeros(3), (2 * R - 1e-5) * n
    z = np.zeros(3)
    w = np.array([3.0, -4.0, 0.0])
    a = s.pair_force(xi, xj, z, z, w, z, R, R)
    b = s.pair_force(xi, xj, z, z, 7 * w, z, R, R)
    Ye = eff(MAT, MAT)
    Fn = 4 / 3 * Ye * math.sqrt(R / 2) * 1e-5 ** 1.5
    Mr = -0.1 * (R / 2) * Fn * w / 5.0
    # friction 0 -> no tangential force, so torque is the rolling torque alone
    np.testing.assert_allclose(a["Mi"], Mr, rtol=1e-9)
    np.testing.assert_allclose(a["Mj"], -Mr, rtol=1e-9)
    np.testing.assert_allclose(b["Mi"], a["Mi"], rtol=1e-12)
    c = s.pair_force(xi, xj, z, z, w, w, R, R)
    assert np.all(c["Mi"] == 0)


# ----------------------------------------------------------- P3/P10 invariants

def test_energy_conserved_without_dissipation(oracle_built):
    """e = 1, mu = 0, mu_r = 0: kinetic + gravitational + Hertz potential energy
    (8/15) Y_e sqrt(R_e) delta^(5/2) per contact stays bounded with no drift."""
    mat = dict(MAT, restitution=1.0, friction=0.0, rolling_friction=0.0)
    sc = W.box_scene(n=60, L=0.015, seed=5)
    sc["materials"] = [mat]
    sc["config"]["dt"] = 2e-6
    rng = np.random.default_rng(1)
    sc["particles"]["vel"] = rng.normal(0, 0.3, (60, 3))
    s = oracle_from_scene(sc)
    R = 1.5e-3
    m = mat["density"] * 4 / 3 * math.pi * R ** 3
    Ye = eff(mat, mat)
    L = 0.015

    def energy():
        st = s.state()
        x, v = st["pos"], st["vel"]
        ke = 0.5 * m * np.sum(v * v)
        pe = m * 9.81 * np.sum(x[:, 2])
        d = np.linalg.norm(x[:, None, :] - x[None, :, :], axis=-1)
        iu = np.triu_indices(len(x), 1)
        ov = np.clip(2 * R - d[iu], 0, None)
        he = np.sum(8 / 15 * Ye * math.sqrt(R / 2) * ov ** 2.5)
        wo = np.concatenate([R - x, R - (L - x)], axis=1).clip(0, None)
        we = np.sum(8 / 15 * Ye * math.sqrt(R) * wo ** 2.5)
        return ke + pe + he + we, ke

    e0, ke0 = energy()
    es = []
    for _ in range(40):
        s.step(500)
        es.append(energy()[0])
    es = np.array(es)
    assert np.max(np.abs(es - e0)) < 2e-3 * ke0
    # no drift: the last quarter is no farther from e0 than the spread
    assert abs(np.mean(es[-10:]) - e0) < 1e-3 * ke0


def test_momentum_conserved_pair_antisymmetry(oracle_built):
    """No walls, no gravity: total linear momentum is conserved to rounding."""
    sc = W.dense_snapshot(n=400, seed=11, walls=False, n_types=3, polydisperse=0.01)
    sc["config"]["gravity"] = (0.0, 0.0, 0.0)
    s = oracle_from_scene(sc)
    t = sc["particles"]["types"]
    R = sc["particles"]["radius"]
    rho = np.array([m["density"] for m in sc["materials"]])[t]
    m = rho * 4 / 3 * math.pi * R ** 3
    p0 = (m[:, None] * s.state()["vel"]).sum(0)
    s.step(300)
    F, _, S = s.forces()
    assert np.sum(S > 0) > 100  # contacts were active
    p1 = (m[:, None] * s.state()["vel"]).sum(0)
    scale = np.sum(m[:, None] * np.abs(s.state()["vel"]))
    assert np.all(np.abs(p1 - p0) < 1e-12 * scale)


# ----------------------------------------------------------------- P4 search

@pytest.mark.parametrize("seed", [0, 1])
def test_cell_search_equals_bruteforce(oracle_built, seed):
    sc = W.dense_snapshot(n=1500, seed=seed, polydisperse=0.4)
    s = oracle_from_scene(sc)
    pairs, _, _ = s.contacts()
    bf = s.bruteforce_candidates()
    assert len(pairs) > 3000
    assert np.array_equal(pairs, bf)


def test_search_threshold_is_strict_and_exact(oracle_built):
    """Pairs at exactly r_s are excluded, one ulp inside are included."""
    d = 3e-3
    s = sim_with(threshold=1.3)
    rs = 1.3 * d
    xs = [0.0, np.nextafter(rs, 0), 0.5, 0.5 + rs, 0.9, 0.9 + np.nextafter(rs, 1)]
    pos = np.array([[x, 0.1, 0.1] for x in xs])
    s.set_particles(pos, np.full(6, d / 2))
    pairs, _, _ = s.contacts()
    d2 = lambda i, j: (pos[j, 0] - pos[i, 0]) ** 2  # noqa: E731
    expect = [(i, j) for i in range(6) for j in range(i + 1, 6) if d2(i, j) < rs * rs]
    assert [tuple(p) for p in pairs] == expect
    assert (0, 1) in expect


def test_rebuild_interval_invariance(oracle_built):
    """With no missed contact, searching every step or every 10 steps gives the
    same trajectory (history carried for persisting pairs, Sec. 3.2)."""
    outs = []
    for K in (1, 10):
        sc = W.dense_snapshot(n=300, seed=4, K=K)
        s = oracle_from_scene(sc)
        s.step(100)
        outs.append(s.state()["pos"])
        c = s.contacts()
        outs.append(c[1][c[2]])
    assert np.array_equal(outs[0], outs[2])
    assert np.array_equal(outs[1], outs[3])


# --------------------------------------------------------- P5 integrator order

def _bounce_error(integrator, dt, T=1.2e-3):
    """Sphere touching a plane (delta = 0, so the zero initial force is exact)
    moving into it at 5 cm/s, undamped and frictionless; position at T (still
    in contact) against a DOP853 solution of the same Hertz ODE."""
    mat = dict(MAT, restitution=1.0, friction=0.0, rolling_friction=0.0)
    R = 1.5e-3
    m = mat["density"] * 4 / 3 * math.pi * R ** 3
    Ye = eff(mat, mat)
    s = sim_with(mat=mat, dt=dt, integrator=integrator, K=1)
    s.add_plane((0, 0, 0), (0, 0, 1))
    s.set_particles([[0, 0, R]], [R], vel=[[0, 0, -0.05]])
    n = int(round(T / dt))
    s.step(n)
    z = s.state()["pos"][0, 2]

    def rhs(t, y):
        d = max(R - y[0], 0.0)
        return [y[1], -9.81 + 4 / 3 * Ye * math.sqrt(R) * d ** 1.5 / m]

    sol = solve_ivp(rhs, [0, n * dt], [R, -0.05], method="DOP853", rtol=1e-13, atol=1e-16)
    return abs(z - sol.y[0, -1])


def test_integrator_orders_match_paper_table(oracle_built):
    """Error ratios per halving of dt give order ~1 (explicit Euler) and ~2
    (velocity Verlet), as the paper's convergence table does."""
    g = json.load(open(os.path.join(GOLDEN, "integration_order.json")))
    ee_paper = np.log2(np.array(g["explicit_euler_error"][:-1]) / np.array(g["explicit_euler_error"][1:]))
    vv_paper = np.log2(np.array(g["velocity_verlet_error"][:-1]) / np.array(g["velocity_verlet_error"][1:]))
    dts = [4e-6, 2e-6, 1e-6]
    ee = [_bounce_error("euler", dt) for dt in dts]
    vv = [_bounce_error("verlet", dt) for dt in dts]
    ee_order = np.log2(np.array(ee[:-1]) / np.array(ee[1:]))
    vv_order = np.log2(np.array(vv[:-1]) / np.array(vv[1:]))
    assert np.all(np.abs(ee_order - ee_paper.mean()) < 0.2), ee_order
    assert np.all(np.abs(vv_order - vv_paper.mean()) < 0.25), vv_order


# ------------------------------------------------------- P6-P8 rigid body pins

def test_resting_sphere_equilibrium_overlap(oracle_built):
    """A damped sphere settles on a plane at delta = (3 m g / (4 Y_e sqrt R))^(2/3)."""
    mat = dict(MAT, restitution=0.3)
    R = 1.5e-3
    s = sim_with(mat=mat, dt=1e-5)
    s.add_plane((0, 0, 0), (0, 0, 1))
    s.set_particles([[0, 0, R + 1e-4]], [R])
    s.step(40000)
    m = mat["density"] * 4 / 3 * math.pi * R ** 3
    Ye = eff(mat, mat)
    deq = (3 * m * 9.81 / (4 * Ye * math.sqrt(R))) ** (2 / 3)
    assert deq == pytest.approx(5.305e-6, rel=1e-3)
    d = R - s.state()["pos"][0, 2]
    assert d == pytest.approx(deq, rel=1e-6)


def test_sliding_to_rolling_transition(oracle_built):
    """A sphere launched without spin slides, then rolls at 5 v0/7 after
    t = 2 v0/(7 mu g) (rigid-body mechanics); the tangential spring, Coulomb
    cap, torque and rotation update all take part."""
    mu = 0.3
    mat = dict(MAT, friction=mu, rolling_friction=0.0, restitution=0.3)
    R = 1.5e-3
    dt = 2e-6
    s = sim_with(mat=mat, dt=dt, rolling="none")
    s.add_plane((0, 0, 0), (0, 0, 1))
    m = mat["density"] * 4 / 3 * math.pi * R ** 3
    deq = (3 * m * 9.81 / (4 * eff(mat, mat) * math.sqrt(R))) ** (2 / 3)
    v0 = 0.2
    s.set_particles([[0, 0, R - deq]], [R], vel=[[v0, 0, 0]])
    t_roll = 2 * v0 / (7 * mu * 9.81)
    s.step(int(1.5 * t_roll / dt))
    st = s.state()
    assert st["vel"][0, 0] == pytest.approx(5 * v0 / 7, rel=1e-2)
    assert st["omega"][0, 1] * R == pytest.approx(st["vel"][0, 0], rel=1e-2)
    # during the sliding phase the speed decreases at mu g
    s2 = sim_with(mat=mat, dt=dt, rolling="none")
    s2.add_plane((0, 0, 0), (0, 0, 1))
    s2.set_particles([[0, 0, R - deq]], [R], vel=[[v0, 0, 0]])
    s2.step(int(0.5 * t_roll / dt))
    v_half = s2.state()["vel"][0, 0]
    assert v_half == pytest.approx(v0 - mu * 9.81 * 0.5 * t_roll, rel=1e-2)


def test_rolling_resistance_deceleration(oracle_built):
    """Constant rolling torque mu_r R m g decelerates a rolling sphere at
    (5/7) mu_r g."""
    mur = 0.1
    mat = dict(MAT, friction=0.5, rolling_friction=mur, restitution=0.3)
    R = 1.5e-3
    dt = 2e-6
    s = sim_with(mat=mat, dt=dt)
    s.add_plane((0, 0, 0), (0, 0, 1))
    m = mat["density"] * 4 / 3 * math.pi * R ** 3
    deq = (3 * m * 9.81 / (4 * eff(mat, mat) * math.sqrt(R))) ** (2 / 3)
    v0 = 0.1
    s.set_particles([[0, 0, R - deq]], [R], vel=[[v0, 0, 0]], omega=[[0, v0 / R, 0]])
    s.step(2000)
    v1 = s.state()["vel"][0, 0]
    s.step(20000)
    v2 = s.state()["vel"][0, 0]
    a = (v1 - v2) / (20000 * dt)
    assert a == pytest.approx(5 / 7 * mur * 9.81, rel=2e-2)


def test_coulomb_regime_by_contact_angle(oracle_built):
    """Oblique sphere-wall impacts with the parameters of the paper's force
    comparison (d = 2 mm steel, mu = 0.3): at 25 and 65 degrees (incidence
    measured from the wall normal) the tangential force reaches the Coulomb
    limit; at 5 degrees it stays below it while the normal force is large."""
    g = json.load(open(os.path.join(GOLDEN, "contact_properties.json")))
    mat = dict(density=g["density_kg_m3"], youngs=g["youngs_pa"], poisson=g["poisson"],
               restitution=0.7, friction=g["friction"], rolling_friction=0.0)
    R = g["diameter_m"] / 2
    limited = {}
    for ang in g["contact_angles_deg"]:
        s = sim_with(mat=mat, dt=2e-9, gravity=(0, 0, 0), K=1, rolling="none")
        s.add_plane((0, 0, 0), (0, 0, 1))
        v = 1.0
        th = math.radians(ang)
        s.set_particles([[0, 0, R + 1e-9]], [R], vel=[[v * math.sin(th), 0, -v * math.cos(th)]])
        frac = []
        fmax = 0.0
        rec = []
        for _ in range(4000):
            s.step(1)
            F, _, _ = s.forces()
            fn, ft = abs(F[0, 2]), math.hypot(F[0, 0], F[0, 1])
            rec.append((fn, ft))
            fmax = max(fmax, fn)
        for fn, ft in rec:
            if fn > 0.2 * fmax:
                frac.append(ft >= g["friction"] * fn * (1 - 1e-9))
        limited[ang] = np.mean(frac)
    assert limited[25] > 0.05 and limited[65] > 0.9
    assert limited[5] == 0.0


# ------------------------------------------------------------- guards, walls

def test_guard_trips_on_fast_particle(oracle_built):
    """A particle that moves more than half the skin between two searches makes
    the step fail (a contact could have been missed)."""
    s = sim_with(dt=1e-4, K=10, gravity=(0, 0, 0))
    s.set_particles([[0, 0, 0], [0.5, 0.5, 0.5]], [1e-3, 1e-3], vel=[[10.0, 0, 0], [0, 0, 0]])
    assert s.step_rc(10) == -5


def test_particle_leaving_domain_becomes_inactive(oracle_built):
    s = sim_with(dt=1e-4, K=5, lo=(-0.1, -0.1, -0.1), hi=(0.1, 0.1, 0.1), gravity=(0, 0, 0))
    s.set_particles([[0.0, 0.0, 0.0997], [0.0, 0.0, 0.0]], [1e-4, 1e-4],
                    vel=[[0, 0, 0.05], [0, 0, 0.0]])
    s.step(40)
    assert s.state()["active"][0]
    s.step(40)
    st = s.state()
    assert not st["active"][0] and st["active"][1]
    p = st["pos"][0].copy()
    s.step(5)
    assert np.array_equal(s.state()["pos"][0], p)


def test_cylinder_drum_particle_rests_and_is_carried(oracle_built):
    """A single sphere at the bottom of a cylinder spinning at Omega about +x
    (surface velocity Omega x r, +y at the bottom) ends up rolling without slip
    on the moving surface: v_y + omega_x R = Omega R_drum, still in contact."""
    mat = dict(MAT, friction=0.5, rolling_friction=0.0, restitution=0.5)
    Rd = 0.05
    R = 1.5e-3
    s = sim_with(mat=mat, dt=1e-5)
    s.add_cylinder((0, 0, 0), (1, 0, 0), Rd, -0.05, 0.05, True, 0, omega=1.0)
    s.set_particles([[0, 0, -Rd + R]], [R])
    s.step(20000)
    x = s.state()["pos"][0]
    # rotation +x carries the bottom point towards -y ... (omega x r with r = -z)
    rho = math.hypot(x[1], x[2])
    assert rho > Rd - R - 1e-4
    st = s.state()
    w, v = st["omega"][0], st["vel"][0]
    assert abs(v[1]) > 1e-3  # it swings like a pendulum about the bottom
    assert v[1] + w[0] * R == pytest.approx(1.0 * Rd, rel=1e-2)
    pairs, _ = s.wall_contacts()
    assert len(pairs) == 1 and pairs[0, 1] == 0


def test_floating_wall_window(oracle_built):
    """A floating wall acts only inside [t_on, t_off): the sphere rests on it,
    then falls when it is switched off."""
    s = sim_with(dt=1e-5, K=10)
    s.add_plane((0, 0, 0), (0, 0, 1), 0, t_on=0.0, t_off=0.05)
    R = 1.5e-3
    s.set_particles([[0, 0, R]], [R])
    s.step(4000)
    assert s.state()["pos"][0, 2] > R - 1e-4
    s.step(6000)
    assert s.state()["pos"][0, 2] < -0.01


def test_invalid_arguments(oracle_built):
    s = sim_with()
    from oracle.binding import OracleError
    with pytest.raises(OracleError):
        s.set_particles([[0, 0, 0]], [-1.0])
    with pytest.raises(OracleError):
        s.add_plane((0, 0, 0), (0, 0, 0))
    with pytest.raises(OracleError):
        s.set_material(0, density=-1, youngs=1, poisson=0.3, restitution=0.5, friction=0.1,
                       rolling_friction=0.0)


def test_friction_opposes_contact_point_slip_particle_pair(oracle_built):
    """A spinning sphere pressed on a static one: the contact point of i moves
    with omega_i x (R_i n); the tangential force on i opposes that motion and
    its torque opposes the spin (relative velocity of Sec. 2.1)."""
    s = sim_with(mat=dict(MAT, rolling_friction=0.0, friction=0.5))
    R = 1.5e-3
    rng = np.random.default_rng(8)
    z = np.zeros(3)
    for _ in range(20):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        w = rng.normal(0, 30, 3)
        out = s.pair_force(z, (2 * R - 1e-5) * n, z, z, w, z, R, R)
        slip = np.cross(w, R * n)
        Ft = out["F"] - np.dot(out["F"], n) * n
        assert np.dot(Ft, slip) < -0.99 * np.linalg.norm(Ft) * np.linalg.norm(slip)
        assert np.dot(out["Mi"], w - np.dot(w, n) * n) < 0


def test_coulomb_truncation_keeps_force_continuous(oracle_built):
    """Eqs. (coulomb_overlap)-(coulomb_overlap3): the truncated overlap is the
    limited force *plus* the damping part, so that re-evaluating at a lower
    sliding speed drops below the limit (sticks) instead of staying pinned at
    it; without the damping part the force would jump."""
    mat = dict(MAT, friction=0.2, restitution=0.3)
    dt = 1e-5
    s = sim_with(mat=mat, dt=dt)
    R = 1.5e-3
    n = np.array([0.0, 0.0, 1.0])
    xi, xj = np.zeros(3), (2 * R - 1e-5) * n
    z = np.zeros(3)
    v = np.array([1e-3, 0.0, 0.0])  # slow sliding: damping below the limit
    a = s.pair_force(xi, xj, v, z, z, z, R, R, delta_t=(2e-5, 0, 0))
    Fa = a["F"] - np.dot(a["F"], n) * n
    fn = abs(np.dot(a["F"], n))
    assert np.linalg.norm(Fa) == pytest.approx(0.2 * fn, rel=1e-12)
    # re-evaluate at half the sliding speed, cancelling the history increment
    b = s.pair_force(xi, xj, v / 2, z, z, z, R, R, delta_t=a["delta_t"] - v / 2 * dt)
    Fb = b["F"] - np.dot(b["F"], n) * n
    assert np.linalg.norm(Fb) < 0.2 * fn * (1 - 1e-3)
    assert Fb[0] < 0  # still opposes the sliding


def test_tangential_oscillation_of_resting_sphere(oracle_built):
    """A sphere resting on a plane, kicked tangentially with mu large: the
    contact-point displacement u obeys the linear oscillator
    (2m/7) u'' = -k_t u - eta_t u' (translation and rotation both respond), with
    Mindlin's k_t = 8 G_e sqrt(R delta_eq).  The measured frequency pins k_t, the
    lever arm and the moment of inertia; the measured decay rate pins eta_t."""
    e = 0.9
    mat = dict(MAT, friction=5.0, rolling_friction=0.0, restitution=e)
    R = 1.5e-3
    dt = 1e-6
    s = sim_with(mat=mat, dt=dt, K=10**9)
    s.add_plane((0, 0, 0), (0, 0, 1))
    m = mat["density"] * 4 / 3 * math.pi * R ** 3
    Ye = eff(mat, mat)
    Ge = 1.0 / (2 * 2 * (2 - 0.3) * (1 + 0.3) / mat["youngs"])
    deq = (3 * m * 9.81 / (4 * Ye * math.sqrt(R))) ** (2 / 3)
    s.set_particles([[0, 0, R - deq]], [R], vel=[[1e-4, 0, 0]])
    ts, us = [], []
    for k in range(12000):
        s.step(1)
        st = s.state()
        us.append(st["vel"][0, 0] - R * st["omega"][0, 1])
        ts.append((k + 1) * dt)
    us = np.array(us)
    ts = np.array(ts)
    kt = 8 * Ge * math.sqrt(R * deq)
    w0 = math.sqrt(7 * kt / (2 * m))
    beta = math.log(e) / math.sqrt(math.log(e) ** 2 + math.pi ** 2)
    zeta_expect = 7 * (-2 * math.sqrt(5 / 6) * beta * math.sqrt(kt * m)) / (4 * m * w0)
    # zero crossings of u' give the damped period, peaks the decay
    sgn = np.sign(us)
    cross = np.where(np.diff(sgn) != 0)[0]
    tc = ts[cross] - us[cross] * (ts[cross + 1] - ts[cross]) / (us[cross + 1] - us[cross])
    period = 2 * np.mean(np.diff(tc[:6]))
    wd = 2 * math.pi / period
    assert wd == pytest.approx(w0 * math.sqrt(1 - zeta_expect ** 2), rel=5e-3)
    peaks = [np.max(np.abs(us[cross[i]:cross[i + 1] + 1])) for i in range(5)]
    decay = np.log(peaks[0] / peaks[4]) / (4 * period / 2)
    assert decay == pytest.approx(zeta_expect * w0, rel=3e-2)
