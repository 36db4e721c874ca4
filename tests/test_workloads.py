"""The seeded scene generators (host only): mesh orientation and closure, and
the placement rules of the dam break and the appendix case."""
import math

import numpy as np
from scipy.spatial import cKDTree

import workloads as W


def _normals_and_centres(m):
    V, T = m["vertices"], m["triangles"]
    p0, p1, p2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    return np.cross(p1 - p0, p2 - p0), (p0 + p1 + p2) / 3


def _edges_closed_and_consistent(T):
    """Every edge is shared by exactly two triangles that run along it in
    opposite directions (a closed, consistently oriented surface)."""
    directed = {}
    for t in T:
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            directed[(int(a), int(b))] = directed.get((int(a), int(b)), 0) + 1
    for (a, b), k in directed.items():
        assert k == 1 and directed.get((b, a)) == 1


def test_box_mesh_is_closed_with_normals_inwards():
    for div in (1, 3):
        m = W.box_mesh((0.0, -1.0, 2.0), (1.0, 2.0, 5.0), divisions=div)
        assert len(m["triangles"]) == 12 * div * div
        N, c = _normals_and_centres(m)
        inside = np.array([0.5, 0.5, 3.5])
        assert np.all(np.einsum("ij,ij->i", N, inside - c) > 0)
        _edges_closed_and_consistent(m["triangles"])
        # the triangles tile the six faces: total area 2 (ab + bc + ca)
        area = 0.5 * np.linalg.norm(N, axis=1).sum()
        assert math.isclose(area, 2 * (1 * 3 + 3 * 3 + 3 * 1), rel_tol=1e-12)


def test_frustum_and_drum_meshes_face_the_axis():
    f = W.frustum_mesh((0.0, 0.0, 0.0), 0.02, 0.5, 0.0, 0.1, segments=24, rings=3)
    N, c = _normals_and_centres(f)
    to_axis = -np.column_stack([c[:, 0], c[:, 1], np.zeros(len(c))])
    assert np.all(np.einsum("ij,ij->i", N, to_axis) > 0)
    d = W.drum_mesh(0.1, -0.05, 0.05, segments=32, rings=4, omega=2.0)
    N, c = _normals_and_centres(d)
    to_axis = -np.column_stack([np.zeros(len(c)), c[:, 1], c[:, 2]])
    assert np.all(np.einsum("ij,ij->i", N, to_axis) > 0)
    assert d["omega"] == (2.0, 0.0, 0.0)
    # corners on the cylinder
    V = d["vertices"]
    assert np.allclose(np.hypot(V[:, 1], V[:, 2]), 0.1)


def test_dam_break_scene_placement():
    sc = W.dam_break_scene(n=20_000, t_dam=0.25)
    p = sc["particles"]["pos"]
    r = sc["particles"]["radius"][0]
    L, depth = sc["geometry"]["length"], sc["geometry"]["depth"]
    assert math.isclose(depth, 0.01 * 20_000 / 160_000)
    assert np.all(p[:, 0] <= L / 2 - r) and np.all(p[:, 0] >= r)
    assert np.all(p[:, 2] >= r) and np.all(p[:, 2] <= depth - r)
    assert np.all(p[:, 1] >= r)
    dmin = cKDTree(p).query(p, k=2)[0][:, 1].min()
    assert dmin >= 2 * r * (1.02 - 2 * 0.01 * math.sqrt(3))
    dam = sc["walls"][-1]
    assert dam["t_off"] == 0.25 and dam["point"][0] == L / 2 and dam["normal"] == (-1.0, 0.0, 0.0)
    assert sc["config"]["gravity"] == (0.0, -9.81, 0.0)


def test_sliding_floor_scene_of_the_appendix():
    sc = W.sliding_floor_scene()
    p = sc["particles"]["pos"]
    r = sc["particles"]["radius"][0]
    assert p.shape == (20, 3) and r == 0.0025
    assert np.all(np.abs(p[:, :2]) <= 0.05 - r) and np.all(p[:, 2] <= -r) and np.all(p[:, 2] >= -0.06 + r)
    assert cKDTree(p).query(p, k=2)[0][:, 1].min() >= 2 * r
    floor = [w for w in sc["walls"] if w["normal"] == (0.0, 0.0, 1.0)][0]
    assert floor["velocity"] == (0.15, 0.0, 0.0) and floor["point"][2] == -0.07
    assert sum(w.get("velocity") is not None for w in sc["walls"]) == 1
    m = sc["materials"][0]
    assert (m["density"], m["restitution"], m["friction"], m["rolling_friction"]) == \
        (2000.0, 0.3, 0.1, 0.05)
