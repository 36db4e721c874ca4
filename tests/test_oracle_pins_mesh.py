"""Pins of the oracle's mesh walls (Sec. 3.7: particles collide with boundary
faces, lines and points of a meshed boundary).

Expected values come from outside the mesh code: the closest point of a
triangle from a constrained minimisation; and the analytic walls, already
pinned, which a mesh must reproduce wherever the geometry is the same — a
flat mesh is a plane, whichever triangle, edge or vertex the sphere lands on
(one contact, never two); a sphere dropped on a convex ridge or apex feels a
single line or point contact whose overlap is R minus the distance, i.e. the
same head-on impact as on a plane; the inside of a triangulated box is six
planes; a concave groove is two planes; a translating mesh plate is a
translating plane.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import workloads as W
from oracle import OracleSim, triangle_closest

MAT = dict(density=2500.0, youngs=1.0e6, poisson=0.3, restitution=0.8, friction=0.3,
           rolling_friction=0.1)
R = 1.5e-3


def sim(mat=MAT, dt=1e-5, gravity=(0, 0, -9.81), K=10, rolling="constant", lo=-0.2, hi=0.2):
    s = OracleSim(dt=dt, gravity=gravity, domain_lo=(lo,) * 3, domain_hi=(hi,) * 3,
                  neighbor_threshold=1.3, rebuild_interval=K, rolling_model=rolling)
    s.set_material(0, **mat)
    return s


def add(s, m):
    return s.add_mesh(m["vertices"], m["triangles"], m["material"], m.get("axis_point"),
                      m.get("omega"), m["t_on"], m["t_off"])


def run(s, n, every):
    out = []
    for _ in range(n // every):
        s.step(every)
        st = s.state()
        out.append(np.concatenate([st["pos"].ravel(), st["vel"].ravel(), st["omega"].ravel()]))
    return np.array(out)


# ------------------------------------------------------------ closest point

def test_closest_point_matches_constrained_minimisation(oracle_built):
    rng = np.random.default_rng(1)
    kinds = set()
    for _ in range(300):
        P = rng.normal(size=(3, 3))
        x = rng.normal(size=3) * 1.5
        feat, s, d2, q = triangle_closest(P, x)
        e1, e2 = P[1] - P[0], P[2] - P[0]

        def f(uv):
            r = x - (P[0] + uv[0] * e1 + uv[1] * e2)
            return r @ r

        best = None
        for start in ((0.2, 0.2), (0.8, 0.1), (0.1, 0.8), (0.0, 0.0)):
            res = minimize(f, start, method="SLSQP", bounds=[(0, 1), (0, 1)],
                           constraints=[{"type": "ineq", "fun": lambda uv: 1 - uv[0] - uv[1]}],
                           options={"ftol": 1e-15, "maxiter": 500})
            if best is None or res.fun < best.fun:
                best = res
        assert d2 == pytest.approx(best.fun, rel=1e-7, abs=1e-12)
        assert np.sum((x - q) ** 2) == pytest.approx(d2, rel=1e-12, abs=1e-15)
        n = np.cross(e1, e2)
        n /= np.linalg.norm(n)
        assert s == pytest.approx((x - P[0]) @ n, rel=1e-12, abs=1e-14)
        u, v = best.x
        assert q == pytest.approx(P[0] + u * e1 + v * e2, abs=1e-6)
        assert (q - P[0]) @ n == pytest.approx(0.0, abs=1e-12)
        inside = u > 1e-6 and v > 1e-6 and u + v < 1 - 1e-6
        if inside:
            assert feat == "face"
        kinds.add(feat if feat == "face" else feat[0])
    assert kinds == {"face", "edge", "vertex"}


# ---------------------------------------------------------- flat mesh = plane

def flat_square(z=0.0, half=0.05, m=4):
    """The square [-half, half]^2 at height z, m x m squares of two triangles,
    normals +z."""
    xs = np.linspace(-half, half, m + 1)
    V = np.array([(x, y, z) for y in xs for x in xs])
    T = []
    for j in range(m):
        for i in range(m):
            a, b = j * (m + 1) + i, j * (m + 1) + i + 1
            c, d = a + m + 1, b + m + 1
            T += [(a, b, d), (a, d, c)]
    return W.mesh(V, np.array(T))


@pytest.mark.parametrize("where", ["face", "diagonal", "grid_edge", "vertex", "near_vertex"])
def test_drop_on_flat_mesh_equals_plane(oracle_built, where):
    """A sphere dropped anywhere on a flat mesh bounces as on a plane: one
    contact on a face, on an edge shared by two triangles and on a vertex
    shared by six.  (No rolling torque: the constant torque takes the
    direction of the relative spin, which is rounding noise here.)"""
    xy = {"face": (0.011, 0.004), "diagonal": (0.006, 0.006), "grid_edge": (0.0, 0.007),
          "vertex": (0.0, 0.0), "near_vertex": (1e-4, 3e-5)}[where]
    out = []
    for wall in ("plane", "mesh"):
        s = sim(K=5, rolling="none")
        if wall == "plane":
            s.add_plane((0, 0, 0), (0, 0, 1))
        else:
            add(s, flat_square())
        s.set_particles([[xy[0], xy[1], R + 2e-4]], [R], vel=[[0, 0, -0.3]])
        out.append(run(s, 600, 20))
    assert np.max(np.abs(out[1] - out[0])) <= 1e-12
    assert np.max(out[0][:, 5]) > 0.2  # it bounced


def test_centre_behind_a_mesh_face_equals_plane(oracle_built):
    """A sphere whose centre starts below the surface (overlap above R) is
    pushed out as by a plane."""
    out = []
    for wall in ("plane", "mesh"):
        s = sim(K=5, rolling="none", gravity=(0, 0, 0))
        if wall == "plane":
            s.add_plane((0, 0, 0), (0, 0, 1))
        else:
            add(s, flat_square())
        s.set_particles([[0.011, 0.004, -0.2 * R]], [R])
        out.append(run(s, 300, 10))
    assert np.max(np.abs(out[1] - out[0])) <= 1e-12
    assert out[0][-1, 5] > 0.1


def test_triangles_meeting_at_one_vertex_equal_plane(oracle_built):
    """Two coplanar triangles that share only a vertex (a bow tie): near the
    vertex, inside one triangle, the face alone acts; the other triangle's
    closest point is the shared vertex, which does not count."""
    V = np.array([(0, 0, 0), (0.02, -0.01, 0), (0.02, 0.01, 0), (-0.02, 0.01, 0),
                  (-0.02, -0.01, 0)])
    T = np.array([(0, 1, 2), (0, 3, 4)])
    out = []
    for wall in ("plane", "mesh"):
        s = sim(K=5, rolling="none")
        if wall == "plane":
            s.add_plane((0, 0, 0), (0, 0, 1))
        else:
            add(s, W.mesh(V, T))
        s.set_particles([[2e-4, 1e-5, R + 1e-4]], [R], vel=[[0, 0, -0.3]])
        out.append(run(s, 400, 10))
    assert np.max(np.abs(out[1] - out[0])) <= 1e-12


def test_rolling_on_a_flat_mesh_face_equals_plane(oracle_built):
    """With friction, spin and sliding, inside one triangle."""
    out = []
    for wall in ("plane", "mesh"):
        s = sim(K=5)
        if wall == "plane":
            s.add_plane((0, 0, 0), (0, 0, 1))
        else:
            add(s, flat_square(m=1, half=0.2))
        s.set_particles([[0.05, -0.1, R - 1e-6]], [R], vel=[[0.2, 0.0, 0.0]],
                        omega=[[0.0, 30.0, 5.0]])
        out.append(run(s, 3000, 100))
    assert np.max(np.abs(out[1] - out[0])) <= 1e-11


# ------------------------------------------------------- convex edges, apex

def roof(angle_deg=30.0, L=0.05):
    """Two rectangles meeting at a ridge along y at height 0, sloping down
    at angle_deg on both sides (normals upwards)."""
    a = math.radians(angle_deg)
    dx, dz = L * math.cos(a), -L * math.sin(a)
    V = np.array([(0, -L, 0), (0, L, 0), (-dx, -L, dz), (-dx, L, dz), (dx, -L, dz), (dx, L, dz)])
    T = np.array([(0, 1, 3), (0, 3, 2), (0, 5, 1), (0, 4, 5)])
    for t in T:
        p0, p1, p2 = V[t]
        assert np.cross(p1 - p0, p2 - p0)[2] > 0
    return W.mesh(V, T)


def pyramid(h=0.02, b=0.05):
    V = np.array([(0, 0, 0), (-b, -b, -h), (b, -b, -h), (b, b, -h), (-b, b, -h)])
    T = np.array([(0, 1, 2), (0, 2, 3), (0, 3, 4), (0, 4, 1)])
    for t in T:
        p0, p1, p2 = V[t]
        assert np.cross(p1 - p0, p2 - p0)[2] > 0
    return W.mesh(V, T)


@pytest.mark.parametrize("e", [1.0, 0.8])
@pytest.mark.parametrize("shape", ["ridge", "apex"])
def test_head_on_impact_on_ridge_or_apex_equals_plane(oracle_built, shape, e):
    """Dropped exactly above a convex ridge or apex: a single line or point
    contact with overlap R - distance, i.e. the plane's head-on impact (same
    rebound speed e v and contact time)."""
    mat = dict(MAT, restitution=e)
    out = []
    for wall in ("plane", "mesh"):
        s = sim(mat=mat, K=5, gravity=(0, 0, 0), rolling="none")
        if wall == "plane":
            s.add_plane((0, 0, 0), (0, 0, 1))
        else:
            add(s, roof() if shape == "ridge" else pyramid())
        s.set_particles([[0.0, 0.003 if shape == "ridge" else 0.0, R + 2e-4]], [R],
                        vel=[[0, 0, -0.3]])
        out.append(run(s, 600, 10))
    assert np.max(np.abs(out[1] - out[0])) <= 1e-12
    assert out[1][-1, 5] == pytest.approx(0.3 * e, rel=2e-3)


def test_drop_on_a_roof_face_near_the_ridge_equals_the_inclined_plane(oracle_built):
    """Inside one face's prism near the ridge the face contact alone acts (the
    ridge, farther away, is not counted)."""
    a = math.radians(30.0)
    n = np.array([-math.sin(a), 0.0, math.cos(a)])  # the left face's normal
    x0 = np.array([-0.6e-3, 0.0, 0.0]) + (R + 1e-4) * n
    out = []
    for wall in ("plane", "mesh"):
        s = sim(K=5, gravity=(0, 0, 0), mat=dict(MAT, friction=0.0, rolling_friction=0.0))
        if wall == "plane":
            s.add_plane((0, 0, 0), tuple(n))
        else:
            add(s, roof())
        s.set_particles([x0], [R], vel=[-0.3 * n])
        out.append(run(s, 400, 10))
    assert np.max(np.abs(out[1] - out[0])) <= 1e-12


def test_oblique_ridge_impact_pushes_along_the_line_to_the_centre(oracle_built):
    """A frictionless sphere hitting the ridge off-centre, in the ridge's own
    region: the impulse lies in the plane normal to the ridge, along the
    line from the ridge to the centre."""
    s = sim(K=5, gravity=(0, 0, 0), mat=dict(MAT, friction=0.0, rolling_friction=0.0))
    add(s, roof())
    x0 = np.array([0.4e-3, 0.0, R + 2e-4])
    v0 = np.array([0.0, 0.1, -0.3])
    s.set_particles([x0], [R], vel=[v0])
    touching_dir = None
    for _ in range(200):
        s.step(2)
        st = s.state()
        F, _, _ = s.forces()
        if np.linalg.norm(F[0]) > 0 and touching_dir is None:
            x = st["pos"][0]
            touching_dir = np.array([x[0], 0.0, x[2]])
            touching_dir /= np.linalg.norm(touching_dir)
            f = F[0] / np.linalg.norm(F[0])
            assert f[1] == pytest.approx(0.0, abs=1e-12)
            assert f == pytest.approx(touching_dir, abs=1e-9)
    assert touching_dir is not None
    v = s.state()["vel"][0]
    assert v[1] == pytest.approx(0.1, rel=1e-12)  # no impulse along the ridge


# ----------------------------------------------------------- concave shapes

def test_inside_of_a_triangulated_box_equals_six_planes(oracle_built):
    """Concave edges and corners: spheres thrown into the box's edges and
    corners, one at a time (no sphere-sphere contacts)."""
    L = 0.03
    rng = np.random.default_rng(3)
    for k in range(6):
        target = np.array([rng.choice([R * 1.01, L - R * 1.01]) for _ in range(3)])
        if k % 2:
            target[k % 3] = L / 2  # an edge instead of a corner
        x0 = np.array([L / 2] * 3)
        v0 = (target - x0) / np.linalg.norm(target - x0) * 0.5
        out = []
        for wall in ("planes", "mesh"):
            s = sim(K=5, lo=-0.01, hi=0.05)
            if wall == "planes":
                for w in W.box_walls((0, 0, 0), (L, L, L)):
                    s.add_plane(w["point"], w["normal"])
            else:
                add(s, W.box_mesh((0, 0, 0), (L, L, L), divisions=2))
            s.set_particles([x0], [R], vel=[v0], omega=[[10.0, -5.0, 3.0]])
            out.append(run(s, 3000, 100))
        assert np.max(np.abs(out[1] - out[0])) <= 1e-10, k


def test_sphere_in_a_groove_equals_two_planes(oracle_built):
    """A 90-degree V-groove (two triangulated planes meeting at a concave
    edge): the sphere settles on both faces."""
    L = 0.05
    V = np.array([(-L, -L, L), (-L, L, L), (0, -L, 0), (0, L, 0), (L, -L, L), (L, L, L)])
    T = np.array([(0, 2, 3), (0, 3, 1), (2, 4, 5), (2, 5, 3)])
    for t in T:
        p0, p1, p2 = V[t]
        assert np.cross(p1 - p0, p2 - p0)[2] > 0
    out = []
    for wall in ("planes", "mesh"):
        s = sim(K=5)
        if wall == "planes":
            s.add_plane((0, 0, 0), (1 / math.sqrt(2), 0, 1 / math.sqrt(2)))
            s.add_plane((0, 0, 0), (-1 / math.sqrt(2), 0, 1 / math.sqrt(2)))
        else:
            add(s, W.mesh(V, T))
        s.set_particles([[0.05e-3, 0.001, R * math.sqrt(2) + 2e-5]], [R])
        out.append(run(s, 20000, 500))
    # the normals of the triangles and of the planes are rounded differently
    d = np.abs(out[1] - out[0])
    assert np.max(d[:, :3]) <= 1e-12 and np.max(d[:, 3:6]) <= 1e-11
    assert np.max(d[:, 6:]) <= 1e-9 * np.max(np.abs(out[0][:, 6:]))
    # at rest on both faces: the contact forces balance gravity
    F, _, _ = s.forces()
    m = MAT["density"] * 4 / 3 * math.pi * R ** 3
    assert F[0] == pytest.approx([0.0, 0.0, m * 9.81], abs=1e-3 * m * 9.81)


# ------------------------------------------------------------- candidates

def test_candidates_front_side_and_skin(oracle_built):
    s = sim(K=5, gravity=(0, 0, 0))
    add(s, flat_square(m=1, half=0.01))
    skin = 0.3 * 2 * R
    pos = [[0.0, 0.0, R + 0.99 * skin],       # above the face, inside R + skin
           [0.0, 0.0, R + 1.01 * skin],       # above, beyond
           [0.0, 0.0, -0.99 * R],             # behind, less than R
           [0.0, 0.0, -1.01 * R],             # behind, more than R
           [0.01 + 0.7 * (R + skin), 0.0, 0.7 * (R + skin)],   # beyond the edge x = 0.01
           [0.01 + 0.72 * (R + skin), 0.0, 0.72 * (R + skin)]]  # distance 1.018 (R + skin)
    s.set_particles(pos, [R] * 6)
    tr, _ = s.mesh_contacts()
    assert sorted(set(tr[:, 0].tolist())) == [0, 2, 4]


# --------------------------------------------------------------- motion

def test_translating_mesh_plate_equals_translating_plane(oracle_built):
    V = 0.2
    out = []
    for wall in ("plane", "mesh"):
        s = sim(K=1, dt=2e-7, gravity=(0, 0, 0), mat=dict(MAT, friction=0.0))
        if wall == "plane":
            w = s.add_plane((0, 0, 0), (1, 0, 0))
        else:
            Vx = np.array([(0, -0.05, -0.05), (0, 0.05, -0.05), (0, 0.05, 0.05), (0, -0.05, 0.05)])
            w = add(s, W.mesh(Vx, np.array([(0, 1, 2), (0, 2, 3)])))
        s.set_wall_velocity(w, (V, 0.0, 0.0))
        s.set_particles([[R + 1e-3, 0.001, 0.002]], [R])
        out.append(run(s, 40000, 1000))
    assert np.max(np.abs(out[1] - out[0])) <= 1e-12
    assert out[1][-1, 3] == pytest.approx(1.8 * V, rel=2e-3)


def test_spinning_mesh_floor_equals_spinning_plane(oracle_built):
    out = []
    for wall in ("plane", "mesh"):
        s = sim(K=5)
        if wall == "plane":
            s.add_plane((0, 0, 0), (0, 0, 1), axis_point=(0, 0, 0), omega=(0, 0, 4.0))
        else:
            m = flat_square(m=1, half=0.2)
            m = dict(m, axis_point=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 4.0))
            add(s, m)
        s.set_particles([[0.03, 0.011, R - 1e-6]], [R])
        out.append(run(s, 3000, 100))
    assert np.max(np.abs(out[1] - out[0])) <= 1e-11
    assert np.linalg.norm(out[1][-1, 3:5]) > 0.01  # dragged along


def test_mesh_argument_checks(oracle_built):
    s = sim()
    with pytest.raises(Exception):
        s.add_mesh([[0, 0, 0], [1, 0, 0], [2, 0, 0]], [[0, 1, 2]])  # degenerate
    with pytest.raises(Exception):
        s.add_mesh([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 1, 3]])  # index out of range
    s.add_mesh([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 1, 2]])
