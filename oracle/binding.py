"""ctypes binding of the C oracle (test infrastructure only).

The C source is ``oracle_dem.c``; this file only marshals arguments.  The
library is compiled with ``-ffp-contract=off`` so that no multiply-add is fused
and every expression is rounded exactly as written in the source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_dem.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# timing build for the benchmark's CPU baseline: the same source with the
# pair loop, kicks and drifts spread over OpenMP threads (deterministic
# per-particle sums); the tests use the serial library only
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

ORA_ERRORS = {-1: "EINVAL", -3: "ENOMEM", -5: "EUNSTABLE", -6: "ESTATE"}


def oracle_lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, FP64, no contraction), and its
    OpenMP timing build."""
    builds = ((_LIB, ["-O2"]),
              (_LIB_OMP, ["-O3", "-march=x86-64-v2", "-fopenmp", "-DORA_PARALLEL"]))
    for lib, extra in builds:
        if force or not os.path.exists(lib):
            tmp = lib + ".tmp"
            cmd = ["gcc", "-std=c99", *extra, "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                   "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, lib)
    return _LIB


class _Config(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double * 3),
                ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3),
                ("neighbor_threshold", C.c_double), ("cell_factor", C.c_double),
                ("rebuild_interval", C.c_int32), ("integrator", C.c_int32),
                ("rolling_model", C.c_int32), ("contact_model", C.c_int32),
                ("characteristic_velocity", C.c_double)]


class _Material(C.Structure):
    _fields_ = [("density", C.c_double), ("youngs", C.c_double), ("poisson", C.c_double),
                ("restitution", C.c_double), ("friction", C.c_double),
                ("rolling_friction", C.c_double)]


_lib = None
_lib_omp = None


def _load(parallel=False):
    global _lib, _lib_omp
    if parallel:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP):
                build_oracle()
            _lib_omp = _declare(C.CDLL(_LIB_OMP))
        return _lib_omp
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        _lib = _declare(C.CDLL(_LIB))
    return _lib


def _declare(lib):
    """Argument types of the oracle's C interface."""
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    lib.ora_create.argtypes = [C.POINTER(_Config), C.POINTER(P)]
    lib.ora_destroy.argtypes = [P]
    lib.ora_destroy.restype = None
    lib.ora_set_material.argtypes = [P, C.c_int32, C.POINTER(_Material)]
    lib.ora_set_particles.argtypes = [P, C.c_int64, D, D, D, D, C.POINTER(C.c_int32)]
    lib.ora_add_plane.argtypes = [P, D, D, D, C.c_int32, D, D, C.c_double, C.c_double,
                                  C.POINTER(C.c_int32)]
    lib.ora_add_cylinder.argtypes = [P, D, D, C.c_double, C.c_double, C.c_double,
                                     C.c_int32, C.c_int32, C.c_double, C.c_double,
                                     C.c_double, C.POINTER(C.c_int32)]
    lib.ora_add_cone.argtypes = [P, D, D, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                                 C.POINTER(C.c_int32)]
    lib.ora_add_mesh.argtypes = [P, C.c_int64, D, C.c_int64, C.POINTER(C.c_int32),
                                 C.c_int32, D, D, C.c_double, C.c_double,
                                 C.POINTER(C.c_int32)]
    lib.ora_get_mesh_contacts.argtypes = [P, C.c_int64, C.POINTER(C.c_int64), D,
                                          C.POINTER(C.c_int64)]
    lib.ora_triangle_closest.argtypes = [D, D, D]
    lib.ora_step.argtypes = [P, C.c_int64]
    lib.ora_set_wall_velocity.argtypes = [P, C.c_int32, D]
    lib.ora_get_state.argtypes = [P, D, D, D, C.POINTER(C.c_uint8), D]
    lib.ora_get_forces.argtypes = [P, D, D]
    lib.ora_get_force_scale.argtypes = [P, D]
    lib.ora_get_term_scale.argtypes = [P, D]
    lib.ora_num_contacts.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.ora_get_contacts.argtypes = [P, C.c_int64, C.POINTER(C.c_int64), D,
                                     C.POINTER(C.c_uint8), C.POINTER(C.c_int64)]
    lib.ora_get_wall_contacts.argtypes = [P, C.c_int64, C.POINTER(C.c_int64), D,
                                          C.POINTER(C.c_int64)]
    lib.ora_get_contact_forces.argtypes = [P, C.c_int64, C.POINTER(C.c_int64), D,
                                           C.POINTER(C.c_int64)]
    lib.ora_search_params.argtypes = [P, D]
    lib.ora_bruteforce_candidates.argtypes = [P, C.c_int64, C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int64)]
    lib.ora_pair_force.argtypes = [P, D, D, D, D, D, D, C.c_double, C.c_double,
                                   C.c_int32, C.c_int32, D, D, D, D,
                                   C.POINTER(C.c_int32)]
    return lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(v, n=3):
    if v is None:
        return None
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n))
    return a


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed: {ORA_ERRORS.get(rc, rc)}")


class OracleSim:
    """One oracle simulation (FP64, single-threaded, particle-input order)."""

    def __init__(self, dt, gravity=(0.0, 0.0, -9.81), domain_lo=(0, 0, 0),
                 domain_hi=(1, 1, 1), neighbor_threshold=1.3, cell_factor=None,
                 rebuild_interval=20, integrator="verlet", rolling_model="constant",
                 contact_model="nonlinear", characteristic_velocity=0.0, parallel=False):
        lib = _load(parallel)
        cfg = _Config()
        cfg.dt = dt
        cfg.gravity = (C.c_double * 3)(*gravity)
        cfg.domain_lo = (C.c_double * 3)(*domain_lo)
        cfg.domain_hi = (C.c_double * 3)(*domain_hi)
        cfg.neighbor_threshold = neighbor_threshold
        cfg.cell_factor = neighbor_threshold if cell_factor is None else cell_factor
        cfg.rebuild_interval = rebuild_interval
        cfg.integrator = {"verlet": 0, "euler": 1}[integrator]
        cfg.rolling_model = {"none": 0, "constant": 1, "viscous": 2}[rolling_model]
        cfg.contact_model = {"nonlinear": 0, "linear": 1}[contact_model]
        cfg.characteristic_velocity = characteristic_velocity
        self._lib = lib
        self._h = C.c_void_p()
        _check(lib.ora_create(C.byref(cfg), C.byref(self._h)), "ora_create")
        self.n = 0

    def close(self):
        if self._h:
            self._lib.ora_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material(self, type_id, density, youngs, poisson, restitution, friction,
                     rolling_friction):
        m = _Material(density, youngs, poisson, restitution, friction, rolling_friction)
        _check(self._lib.ora_set_material(self._h, type_id, C.byref(m)), "ora_set_material")

    def add_plane(self, point, normal, material=0, extent=None, axis_point=None,
                  omega=None, t_on=-np.inf, t_off=np.inf):
        wid = C.c_int32()
        p, nrm = _vec(point), _vec(normal)
        ext = None if extent is None else _vec(extent, 5)
        ap = _vec(axis_point)
        om = _vec(omega)
        _check(self._lib.ora_add_plane(self._h, _dp(p), _dp(nrm), _dp(ext), material,
                                       _dp(ap), _dp(om), t_on, t_off, C.byref(wid)),
               "ora_add_plane")
        return wid.value

    def add_cylinder(self, axis_point, axis_dir, radius, s_min, s_max, inside=True,
                     material=0, omega=0.0, t_on=-np.inf, t_off=np.inf):
        wid = C.c_int32()
        ap, ad = _vec(axis_point), _vec(axis_dir)
        _check(self._lib.ora_add_cylinder(self._h, _dp(ap), _dp(ad), radius, s_min, s_max,
                                          1 if inside else 0, material, omega, t_on, t_off,
                                          C.byref(wid)), "ora_add_cylinder")
        return wid.value

    def add_cone(self, axis_point, axis_dir, radius0, slope, s_min, s_max, inside=True,
                 material=0, omega=0.0, t_on=-np.inf, t_off=np.inf):
        wid = C.c_int32()
        ap, ad = _vec(axis_point), _vec(axis_dir)
        _check(self._lib.ora_add_cone(self._h, _dp(ap), _dp(ad), radius0, slope, s_min, s_max,
                                      1 if inside else 0, material, omega, t_on, t_off,
                                      C.byref(wid)), "ora_add_cone")
        return wid.value

    def add_mesh(self, vertices, triangles, material=0, axis_point=None, omega=None,
                 t_on=-np.inf, t_off=np.inf):
        V = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1, 3)
        T = np.ascontiguousarray(triangles, dtype=np.int32).reshape(-1, 3)
        wid = C.c_int32()
        ap, om = _vec(axis_point), _vec(omega)
        _check(self._lib.ora_add_mesh(self._h, V.shape[0], _dp(V), T.shape[0],
                                      T.ctypes.data_as(C.POINTER(C.c_int32)), material,
                                      _dp(ap), _dp(om), t_on, t_off, C.byref(wid)),
               "ora_add_mesh")
        return wid.value

    def mesh_contacts(self):
        """(particle, wall, triangle) candidate triples and their overlaps."""
        cnt = C.c_int64()
        self._lib.ora_get_mesh_contacts(self._h, 0, None, None, C.byref(cnt))
        m = cnt.value
        tr = np.empty((max(m, 1), 3), dtype=np.int64)
        dt = np.empty((max(m, 1), 3))
        _check(self._lib.ora_get_mesh_contacts(self._h, max(m, 1),
                                               tr.ctypes.data_as(C.POINTER(C.c_int64)),
                                               _dp(dt), C.byref(cnt)), "ora_get_mesh_contacts")
        return tr[:m], dt[:m]

    def set_wall_velocity(self, wall_id, vel):
        v = _vec(vel)
        _check(self._lib.ora_set_wall_velocity(self._h, wall_id, _dp(v)), "ora_set_wall_velocity")

    def set_particles(self, pos, radius, vel=None, omega=None, types=None):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        n = pos.shape[0]
        radius = np.ascontiguousarray(radius, dtype=np.float64).reshape(n)
        vel = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64).reshape(n, 3)
        omega = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64).reshape(n, 3)
        tp = None
        if types is not None:
            tp = np.ascontiguousarray(types, dtype=np.int32).reshape(n)
        _check(self._lib.ora_set_particles(
            self._h, n, _dp(pos), _dp(vel), _dp(omega), _dp(radius),
            None if tp is None else tp.ctypes.data_as(C.POINTER(C.c_int32))),
            "ora_set_particles")
        self.n = n

    def step(self, n_steps=1):
        rc = self._lib.ora_step(self._h, n_steps)
        _check(rc, "ora_step")

    def step_rc(self, n_steps=1):
        return self._lib.ora_step(self._h, n_steps)

    def state(self):
        n = self.n
        x = np.empty((n, 3)); v = np.empty((n, 3)); w = np.empty((n, 3))
        act = np.empty(n, dtype=np.uint8)
        t = C.c_double()
        _check(self._lib.ora_get_state(self._h, _dp(x), _dp(v), _dp(w),
                                       act.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(t)),
               "ora_get_state")
        return {"pos": x, "vel": v, "omega": w, "active": act.astype(bool), "time": t.value}

    def forces(self):
        n = self.n
        F = np.empty((n, 3)); T = np.empty((n, 3)); S = np.empty(n)
        _check(self._lib.ora_get_forces(self._h, _dp(F), _dp(T)), "ora_get_forces")
        _check(self._lib.ora_get_force_scale(self._h, _dp(S)), "ora_get_force_scale")
        return F, T, S

    def term_scale(self):
        """Per particle: sum over its contacts of the magnitudes of the spring
        and dashpot terms of the last evaluation (before the Coulomb limit)."""
        S2 = np.empty(self.n)
        _check(self._lib.ora_get_term_scale(self._h, _dp(S2)), "ora_get_term_scale")
        return S2

    def contacts(self):
        npairs = C.c_int64(); nw = C.c_int64()
        _check(self._lib.ora_num_contacts(self._h, C.byref(npairs), C.byref(nw)), "num")
        m = npairs.value
        pairs = np.empty((max(m, 1), 2), dtype=np.int64)
        dt = np.empty((max(m, 1), 3))
        touch = np.empty(max(m, 1), dtype=np.uint8)
        nout = C.c_int64()
        _check(self._lib.ora_get_contacts(self._h, max(m, 1),
                                          pairs.ctypes.data_as(C.POINTER(C.c_int64)), _dp(dt),
                                          touch.ctypes.data_as(C.POINTER(C.c_uint8)),
                                          C.byref(nout)), "ora_get_contacts")
        return pairs[:m], dt[:m], touch[:m].astype(bool)

    def contact_forces(self):
        """Candidate pairs (the order of contacts()) and F^n + F^t on the
        pair's first particle at the last evaluation (zero if not touching)."""
        npairs = C.c_int64(); nw = C.c_int64()
        _check(self._lib.ora_num_contacts(self._h, C.byref(npairs), C.byref(nw)), "num")
        m = npairs.value
        pairs = np.empty((max(m, 1), 2), dtype=np.int64)
        f = np.empty((max(m, 1), 3))
        nout = C.c_int64()
        _check(self._lib.ora_get_contact_forces(self._h, max(m, 1),
                                                pairs.ctypes.data_as(C.POINTER(C.c_int64)),
                                                _dp(f), C.byref(nout)), "ora_get_contact_forces")
        return pairs[:m], f[:m]

    def wall_contacts(self):
        npairs = C.c_int64(); nw = C.c_int64()
        _check(self._lib.ora_num_contacts(self._h, C.byref(npairs), C.byref(nw)), "num")
        m = nw.value
        pairs = np.empty((max(m, 1), 2), dtype=np.int64)
        dt = np.empty((max(m, 1), 3))
        nout = C.c_int64()
        _check(self._lib.ora_get_wall_contacts(self._h, max(m, 1),
                                               pairs.ctypes.data_as(C.POINTER(C.c_int64)),
                                               _dp(dt), C.byref(nout)), "ora_get_wall_contacts")
        return pairs[:m], dt[:m]

    def search_params(self):
        out = np.empty(4)
        _check(self._lib.ora_search_params(self._h, _dp(out)), "ora_search_params")
        return {"d_max": out[0], "r_s": out[1], "h": out[2], "skin": out[3]}

    def bruteforce_candidates(self):
        cnt = C.c_int64()
        self._lib.ora_bruteforce_candidates(self._h, 0, None, C.byref(cnt))
        m = cnt.value
        pairs = np.empty((max(m, 1), 2), dtype=np.int64)
        _check(self._lib.ora_bruteforce_candidates(
            self._h, max(m, 1), pairs.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(cnt)),
            "ora_bruteforce_candidates")
        return pairs[:m]

    def pair_force(self, xi, xj, vi, vj, wi, wj, Ri, Rj, ti=0, tj=0, delta_t=(0, 0, 0)):
        a = [_vec(q) for q in (xi, xj, vi, vj, wi, wj)]
        dt = _vec(delta_t).copy()
        F = np.zeros(3); Mi = np.zeros(3); Mj = np.zeros(3)
        touch = C.c_int32()
        _check(self._lib.ora_pair_force(self._h, *[_dp(q) for q in a], Ri, Rj, ti, tj,
                                        _dp(dt), _dp(F), _dp(Mi), _dp(Mj), C.byref(touch)),
               "ora_pair_force")
        return {"F": F, "Mi": Mi, "Mj": Mj, "delta_t": dt, "touching": bool(touch.value)}


def triangle_closest(corners, x):
    """The oracle's closest point of a triangle to x: (feature, signed plane
    distance, squared distance, point); feature 'face', ('edge', a) for the
    edge from corner a to a + 1, ('vertex', a)."""
    lib = _load()
    c = np.ascontiguousarray(corners, dtype=np.float64).reshape(9)
    xx = _vec(x)
    out = np.empty(6)
    _check(lib.ora_triangle_closest(_dp(c), _dp(xx), _dp(out)), "ora_triangle_closest")
    f = int(out[0])
    feat = "face" if f == 0 else (("edge", f - 1) if f < 4 else ("vertex", f - 4))
    return feat, out[1], out[2], out[3:6].copy()


def oracle_from_scene(scene: dict, parallel: bool = False) -> OracleSim:
    """Build an oracle simulation from a scene dictionary (see ``workloads``);
    parallel=True uses the OpenMP timing build."""
    c = scene["config"]
    sim = OracleSim(dt=c["dt"], gravity=c["gravity"], domain_lo=c["domain_lo"],
                    domain_hi=c["domain_hi"], neighbor_threshold=c["neighbor_threshold"],
                    cell_factor=c["cell_factor"], rebuild_interval=c["rebuild_interval"],
                    integrator=c["integrator"], rolling_model=c["rolling_model"],
                    contact_model=c.get("contact_model", "nonlinear"),
                    characteristic_velocity=c.get("characteristic_velocity", 0.0),
                    parallel=parallel)
    for t, m in enumerate(scene["materials"]):
        sim.set_material(t, m["density"], m["youngs"], m["poisson"], m["restitution"],
                         m["friction"], m["rolling_friction"])
    for w in scene["walls"]:
        if w["kind"] == "plane":
            sim.add_plane(w["point"], w["normal"], w["material"], w.get("extent"),
                          w.get("axis_point"), w.get("omega"), w["t_on"], w["t_off"])
        elif w["kind"] == "cylinder":
            sim.add_cylinder(w["axis_point"], w["axis_dir"], w["radius"], w["s_min"],
                             w["s_max"], w["inside"], w["material"], w["omega"], w["t_on"],
                             w["t_off"])
        elif w["kind"] == "mesh":
            sim.add_mesh(w["vertices"], w["triangles"], w["material"], w.get("axis_point"),
                         w.get("omega"), w["t_on"], w["t_off"])
        else:
            sim.add_cone(w["axis_point"], w["axis_dir"], w["radius0"], w["slope"], w["s_min"],
                         w["s_max"], w["inside"], w["material"], w["omega"], w["t_on"],
                         w["t_off"])
    for k, w in enumerate(scene["walls"]):
        if w.get("velocity") is not None:
            sim.set_wall_velocity(k, w["velocity"])
    p = scene["particles"]
    sim.set_particles(p["pos"], p["radius"], p["vel"], p["omega"], p["types"])
    return sim
