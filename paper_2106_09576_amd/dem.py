"""Thin ctypes binding of libdem.so (the C ABI in include/dem.h).

Only argument marshalling lives here: every step of the simulation runs in the
HIP kernels of the library.  If the library is missing this module raises; it
never falls back to any other implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdem.so")

DEM_OK = 0
DEM_EINVAL = -1
DEM_EHIP = -2
DEM_ENOMEM = -3
DEM_ECAPACITY = -4
DEM_EUNSTABLE = -5
DEM_ESTATE = -6
DEM_ENODEV = -7
ERROR_NAMES = {DEM_EINVAL: "DEM_EINVAL", DEM_EHIP: "DEM_EHIP", DEM_ENOMEM: "DEM_ENOMEM",
               DEM_ECAPACITY: "DEM_ECAPACITY", DEM_EUNSTABLE: "DEM_EUNSTABLE",
               DEM_ESTATE: "DEM_ESTATE", DEM_ENODEV: "DEM_ENODEV"}


class dem_material(C.Structure):
    _fields_ = [("density", C.c_double), ("youngs", C.c_double), ("poisson", C.c_double),
                ("restitution", C.c_double), ("friction", C.c_double),
                ("rolling_friction", C.c_double)]


class dem_tuning(C.Structure):
    _fields_ = [("force_block", C.c_int32), ("rebuild_interval", C.c_int32),
                ("cell_factor", C.c_double), ("ms_per_step", C.c_double),
                ("steps", C.c_int64), ("block_ms", C.c_double * 3),
                ("cell_factors", C.c_double * 4), ("search_ms", C.c_double * 4),
                ("schedules", C.c_int32 * 8), ("schedule_ms", C.c_double * 8)]


class dem_config(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double * 3),
                ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3),
                ("neighbor_threshold", C.c_double), ("cell_factor", C.c_double),
                ("rebuild_interval", C.c_int32), ("integrator", C.c_int32),
                ("rolling_model", C.c_int32), ("precision", C.c_int32),
                ("n_instances", C.c_int32), ("max_neighbors", C.c_int32),
                ("hip_stream", C.c_void_p), ("contact_model", C.c_int32),
                ("reserved", C.c_int32), ("characteristic_velocity", C.c_double),
                ("force_block", C.c_int32), ("reserved2", C.c_int32)]


class dem_stats(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("n_active", C.c_int64),
                ("n_list_entries", C.c_int64), ("n_touching", C.c_int64),
                ("n_wall_candidates", C.c_int64), ("step", C.c_int64),
                ("n_rebuilds", C.c_int64), ("max_neighbors", C.c_int32),
                ("precision", C.c_int32), ("r_s", C.c_double), ("cell_size", C.c_double),
                ("skin", C.c_double), ("d_max", C.c_double), ("n_cells", C.c_int64),
                ("device_bytes", C.c_int64)]


class DemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

P = C.c_void_p
DP = C.POINTER(C.c_double)
I64P = C.POINTER(C.c_int64)
I32P = C.POINTER(C.c_int32)
U8P = C.POINTER(C.c_uint8)

# name -> (restype, argtypes); mirrors include/dem.h
SIGNATURES = {
    "dem_create": (C.c_int, [C.POINTER(dem_config), C.POINTER(P)]),
    "dem_destroy": (None, [P]),
    "dem_last_error": (C.c_char_p, [P]),
    "dem_set_material": (C.c_int, [P, C.c_int32, C.c_int32, C.POINTER(dem_material)]),
    "dem_add_planar_wall": (C.c_int, [P, C.c_int32, DP, DP, DP, C.c_int32, DP, DP, C.c_double,
                                      C.c_double, I32P]),
    "dem_add_cylinder_wall": (C.c_int, [P, C.c_int32, DP, DP, C.c_double, C.c_double,
                                        C.c_double, C.c_int32, C.c_int32, C.c_double,
                                        C.c_double, C.c_double, I32P]),
    "dem_add_cone_wall": (C.c_int, [P, C.c_int32, DP, DP, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                    C.c_double, I32P]),
    "dem_set_wall_motion": (C.c_int, [P, C.c_int32, C.c_int32, DP]),
    "dem_set_particles": (C.c_int, [P, C.c_int32, C.c_int64, DP, DP, DP, DP, I32P]),
    "dem_set_particles_device": (C.c_int, [P, C.c_int32, C.c_int64, P, P, P, P, P]),
    "dem_commit": (C.c_int, [P]),
    "dem_set_instance_domain": (C.c_int, [P, C.c_int32, DP, DP]),
    "dem_step": (C.c_int, [P, C.c_int64]),
    "dem_get_state": (C.c_int, [P, C.c_int32, DP, DP, DP, U8P, DP]),
    "dem_get_state_device": (C.c_int, [P, C.c_int32, P, P, P, P]),
    "dem_get_forces": (C.c_int, [P, C.c_int32, DP, DP]),
    "dem_get_contacts": (C.c_int, [P, C.c_int32, C.c_int64, I64P, DP, U8P, I64P]),
    "dem_get_wall_contacts": (C.c_int, [P, C.c_int32, C.c_int64, I64P, DP, I64P]),
    "dem_record_contact_forces": (C.c_int, [P, C.c_int32]),
    "dem_get_contacts_device": (C.c_int, [P, C.c_int32, C.c_int64, P, P, P, I64P]),
    "dem_get_contacts_device_noalloc": (C.c_int, [P, C.c_int32, C.c_int64, P, P, P, I64P]),
    "dem_get_contact_forces": (C.c_int, [P, C.c_int32, C.c_int64, I64P, DP, I64P]),
    "dem_add_mesh_wall": (C.c_int, [P, C.c_int32, C.c_int64, DP, C.c_int64, I32P, C.c_int32, DP,
                                    DP, C.c_double, C.c_double, I32P]),
    "dem_get_mesh_contacts": (C.c_int, [P, C.c_int32, C.c_int64, I64P, DP, I64P]),
    "dem_restore_mesh_contacts": (C.c_int, [P, C.c_int32, C.c_int64, I64P, DP]),
    "dem_resort": (C.c_int, [P]),
    "dem_get_stats": (C.c_int, [P, C.POINTER(dem_stats)]),
    "dem_stream": (C.c_void_p, [P]),
    "dem_set_timing": (C.c_int, [P, C.c_int32]),
    "dem_autotune": (C.c_int, [P, C.c_int32, C.POINTER(dem_tuning)]),
    "dem_restore": (C.c_int, [P, C.c_int32, C.c_int64, I64P, DP, C.c_int64, I64P, DP, DP, DP,
                              C.c_int64]),
    "dem_get_timing": (C.c_int, [P, DP]),
}


def load_library(path: str | None = None):
    """Load libdem.so (built by ``paper_2106_09576_amd.build``); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libdem.so not built at {p}; run __graft_entry__.build() or "
                          f"python -m paper_2106_09576_amd.build")
    lib = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _d(a):
    return None if a is None else a.ctypes.data_as(DP)


def _v3(v):
    if v is None:
        return None
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))


class Dem:
    """One simulation context (a ``dem_ctx``)."""

    def __init__(self, dt, gravity=(0.0, 0.0, -9.81), domain_lo=(0, 0, 0), domain_hi=(1, 1, 1),
                 neighbor_threshold=1.3, cell_factor=None, rebuild_interval=20,
                 integrator="verlet", rolling_model="constant", precision="fp64",
                 max_neighbors=0, hip_stream=None, n_instances=1, contact_model="nonlinear",
                 characteristic_velocity=0.0, force_block=0):
        self._lib = load_library()
        cfg = dem_config()
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
        cfg.force_block = force_block
        cfg.precision = {"fp64": 0, "fp32": 1}[precision]
        cfg.n_instances = n_instances
        cfg.max_neighbors = max_neighbors
        cfg.hip_stream = hip_stream
        self._h = P()
        self._check(self._lib.dem_create(C.byref(cfg), C.byref(self._h)))
        self.n_instances = n_instances
        self.counts = [0] * n_instances
        self.precision = precision

    # ------------------------------------------------------------ plumbing
    def _check(self, rc):
        if rc != DEM_OK:
            msg = self._lib.dem_last_error(None)
            raise DemError(rc, msg.decode() if msg else "")

    def close(self):
        if self._h:
            self._lib.dem_destroy(self._h)
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- ABI
    @property
    def n(self):
        return self.counts[0]

    def set_material(self, type_id, density, youngs, poisson, restitution, friction,
                     rolling_friction, instance=0):
        m = dem_material(density, youngs, poisson, restitution, friction, rolling_friction)
        self._check(self._lib.dem_set_material(self._h, instance, type_id, C.byref(m)))

    def add_planar_wall(self, point, normal, material=0, extent=None, axis_point=None,
                        omega=None, t_on=-np.inf, t_off=np.inf, instance=0):
        wid = C.c_int32()
        p, nr = _v3(point), _v3(normal)
        ext = None if extent is None else np.ascontiguousarray(extent, dtype=np.float64).reshape(5)
        ap, om = _v3(axis_point), _v3(omega)
        self._check(self._lib.dem_add_planar_wall(self._h, instance, _d(p), _d(nr), _d(ext), material,
                                                  _d(ap), _d(om), t_on, t_off, C.byref(wid)))
        return wid.value

    def add_cylinder_wall(self, axis_point, axis_dir, radius, s_min, s_max, inside=True,
                          material=0, omega=0.0, t_on=-np.inf, t_off=np.inf, instance=0):
        wid = C.c_int32()
        ap, ad = _v3(axis_point), _v3(axis_dir)
        self._check(self._lib.dem_add_cylinder_wall(self._h, instance, _d(ap), _d(ad), radius, s_min,
                                                    s_max, 1 if inside else 0, material, omega,
                                                    t_on, t_off, C.byref(wid)))
        return wid.value

    def add_cone_wall(self, axis_point, axis_dir, radius0, slope, s_min, s_max, inside=True,
                      material=0, omega=0.0, t_on=-np.inf, t_off=np.inf, instance=0):
        wid = C.c_int32()
        ap, ad = _v3(axis_point), _v3(axis_dir)
        self._check(self._lib.dem_add_cone_wall(self._h, instance, _d(ap), _d(ad), radius0, slope,
                                                s_min, s_max, 1 if inside else 0, material, omega,
                                                t_on, t_off, C.byref(wid)))
        return wid.value

    def add_mesh_wall(self, vertices, triangles, material=0, axis_point=None, omega=None,
                      t_on=-np.inf, t_off=np.inf, instance=0):
        """Triangle-mesh wall; each triangle's corners ordered so that
        (p1 - p0) x (p2 - p0) points to the particles' side."""
        V = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1, 3)
        T = np.ascontiguousarray(triangles, dtype=np.int32).reshape(-1, 3)
        wid = C.c_int32()
        ap, om = _v3(axis_point), _v3(omega)
        self._check(self._lib.dem_add_mesh_wall(self._h, instance, V.shape[0], _d(V), T.shape[0],
                                                T.ctypes.data_as(I32P), material, _d(ap),
                                                _d(om), t_on, t_off, C.byref(wid)))
        return wid.value

    def set_wall_motion(self, wall_id, velocity, instance=0):
        """Translate wall ``wall_id`` at constant ``velocity`` (before set_particles)."""
        v = _v3(velocity)
        self._check(self._lib.dem_set_wall_motion(self._h, instance, wall_id, _d(v)))

    def set_particles(self, pos, radius, vel=None, omega=None, types=None, instance=0):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        n = pos.shape[0]
        radius = np.ascontiguousarray(radius, dtype=np.float64).reshape(n)
        vel = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64).reshape(n, 3)
        omega = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64).reshape(n, 3)
        tp = None if types is None else np.ascontiguousarray(types, dtype=np.int32).reshape(n)
        self._check(self._lib.dem_set_particles(
            self._h, instance, n, _d(pos), _d(vel), _d(omega), _d(radius),
            None if tp is None else tp.ctypes.data_as(I32P)))
        self.counts[instance] = n

    def set_particles_device(self, n, pos_ptr, radius_ptr, vel_ptr=None, omega_ptr=None,
                             type_ptr=None, instance=0):
        self._check(self._lib.dem_set_particles_device(self._h, instance, n, pos_ptr, vel_ptr,
                                                       omega_ptr, radius_ptr, type_ptr))
        self.counts[instance] = n

    def commit(self):
        self._check(self._lib.dem_commit(self._h))

    def step(self, n_steps=1):
        self._check(self._lib.dem_step(self._h, n_steps))

    def step_rc(self, n_steps=1):
        return self._lib.dem_step(self._h, n_steps)

    def get_state(self, instance=0):
        n = self.counts[instance]
        x = np.empty((n, 3)); v = np.empty((n, 3)); w = np.empty((n, 3))
        a = np.empty(n, dtype=np.uint8)
        t = C.c_double()
        self._check(self._lib.dem_get_state(self._h, instance, _d(x), _d(v), _d(w),
                                            a.ctypes.data_as(U8P), C.byref(t)))
        return {"pos": x, "vel": v, "omega": w, "active": a.astype(bool), "time": t.value}

    state = get_state

    def get_forces(self, instance=0):
        n = self.counts[instance]
        F = np.empty((n, 3)); T = np.empty((n, 3))
        self._check(self._lib.dem_get_forces(self._h, instance, _d(F), _d(T)))
        return F, T

    def get_contacts(self, instance=0):
        cnt = C.c_int64()
        rc = self._lib.dem_get_contacts(self._h, instance, 0, None, None, None, C.byref(cnt))
        if rc not in (DEM_OK, DEM_EINVAL):
            self._check(rc)
        m = cnt.value
        pairs = np.empty((max(m, 1), 2), dtype=np.int64)
        dt = np.empty((max(m, 1), 3))
        touch = np.empty(max(m, 1), dtype=np.uint8)
        self._check(self._lib.dem_get_contacts(self._h, instance, max(m, 1), pairs.ctypes.data_as(I64P),
                                               _d(dt), touch.ctypes.data_as(U8P), C.byref(cnt)))
        return pairs[:m], dt[:m], touch[:m].astype(bool)

    def get_contacts_device(self, cap, pairs_ptr=None, delta_t_ptr=None, touching_ptr=None,
                            instance=0):
        """Candidate pairs into device buffers given by address (e.g. a
        tensor's data_ptr(); int64 [cap, 2], float64 [cap, 3], uint8 [cap]),
        in the library's spatial order; returns the count.  Raises DemError
        (DEM_EINVAL) when the count exceeds cap."""
        cnt = C.c_int64()
        self._check(self._lib.dem_get_contacts_device(self._h, instance, int(cap), pairs_ptr,
                                                      delta_t_ptr, touching_ptr,
                                                      C.byref(cnt)))
        return cnt.value

    def get_contacts_device_noalloc(self, cap, pairs_ptr=None, delta_t_ptr=None,
                                    touching_ptr=None, instance=0):
        """As get_contacts_device, through the entry point that allocates
        nothing (its workspace is a device array of the library)."""
        cnt = C.c_int64()
        self._check(self._lib.dem_get_contacts_device_noalloc(
            self._h, instance, int(cap), pairs_ptr, delta_t_ptr, touching_ptr, C.byref(cnt)))
        return cnt.value

    def count_contacts_device(self, instance=0):
        """Number of candidate pairs (a dem_get_contacts_device call with cap 0)."""
        cnt = C.c_int64()
        rc = self._lib.dem_get_contacts_device(self._h, instance, 0, None, None, None,
                                               C.byref(cnt))
        if rc not in (DEM_OK, DEM_EINVAL):
            self._check(rc)
        return cnt.value

    def record_contact_forces(self, enable=True):
        self._check(self._lib.dem_record_contact_forces(self._h, 1 if enable else 0))

    def get_contact_forces(self, instance=0):
        """Candidate pairs (the order of get_contacts) and the force of the
        last evaluation on each pair's first particle (zero if not touching)."""
        cnt = C.c_int64()
        rc = self._lib.dem_get_contact_forces(self._h, instance, 0, None, None, C.byref(cnt))
        if rc not in (DEM_OK, DEM_EINVAL):
            self._check(rc)
        m = cnt.value
        pairs = np.empty((max(m, 1), 2), dtype=np.int64)
        f = np.empty((max(m, 1), 3))
        self._check(self._lib.dem_get_contact_forces(self._h, instance, max(m, 1),
                                                     pairs.ctypes.data_as(I64P), _d(f),
                                                     C.byref(cnt)))
        return pairs[:m], f[:m]

    def get_wall_contacts(self, instance=0):
        cnt = C.c_int64()
        rc = self._lib.dem_get_wall_contacts(self._h, instance, 0, None, None, C.byref(cnt))
        if rc not in (DEM_OK, DEM_EINVAL):
            self._check(rc)
        m = cnt.value
        pairs = np.empty((max(m, 1), 2), dtype=np.int64)
        dt = np.empty((max(m, 1), 3))
        self._check(self._lib.dem_get_wall_contacts(self._h, instance, max(m, 1),
                                                    pairs.ctypes.data_as(I64P), _d(dt),
                                                    C.byref(cnt)))
        return pairs[:m], dt[:m]

    def get_mesh_contacts(self, instance=0):
        """(particle, wall, triangle) candidates of mesh walls and their
        tangential overlaps, sorted."""
        cnt = C.c_int64()
        rc = self._lib.dem_get_mesh_contacts(self._h, instance, 0, None, None, C.byref(cnt))
        if rc not in (DEM_OK, DEM_EINVAL):
            self._check(rc)
        m = cnt.value
        tr = np.empty((max(m, 1), 3), dtype=np.int64)
        dt = np.empty((max(m, 1), 3))
        self._check(self._lib.dem_get_mesh_contacts(self._h, instance, max(m, 1),
                                                    tr.ctypes.data_as(I64P), _d(dt),
                                                    C.byref(cnt)))
        return tr[:m], dt[:m]

    def resort(self):
        self._check(self._lib.dem_resort(self._h))

    def get_stats(self):
        s = dem_stats()
        self._check(self._lib.dem_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in dem_stats._fields_}

    def stream(self):
        return self._lib.dem_stream(self._h)

    def checkpoint(self, instance=0):
        """Everything an exact resume needs (see restore)."""
        st = self.get_state(instance)
        pairs, dt, touching = self.get_contacts(instance)
        wpairs, wdt = self.get_wall_contacts(instance)
        mtri, mdt = self.get_mesh_contacts(instance)
        F, T = self.get_forces(instance)
        t = touching.astype(bool)
        keep = np.any(mdt != 0, axis=1)
        return {"pos": st["pos"], "vel": st["vel"], "omega": st["omega"],
                "pairs": pairs[t], "delta_t": dt[t], "wall_pairs": wpairs,
                "wall_delta_t": wdt, "mesh_triples": mtri[keep], "mesh_delta_t": mdt[keep],
                "force": F, "torque": T, "step": self.get_stats()["step"]}

    def restore(self, ck, instance=0):
        """Restore histories, forces and step count of a checkpoint into an
        instance whose particles were set from the checkpoint's state."""
        pairs = np.ascontiguousarray(ck["pairs"], dtype=np.int64).reshape(-1, 2)
        dt = np.ascontiguousarray(ck["delta_t"], dtype=np.float64).reshape(-1, 3)
        wp = np.ascontiguousarray(ck["wall_pairs"], dtype=np.int64).reshape(-1, 2)
        wdt = np.ascontiguousarray(ck["wall_delta_t"], dtype=np.float64).reshape(-1, 3)
        F = np.ascontiguousarray(ck["force"], dtype=np.float64)
        T = np.ascontiguousarray(ck["torque"], dtype=np.float64)
        self._check(self._lib.dem_restore(self._h, instance, pairs.shape[0],
                                          pairs.ctypes.data_as(I64P), _d(dt), wp.shape[0],
                                          wp.ctypes.data_as(I64P), _d(wdt), _d(F), _d(T),
                                          int(ck["step"])))
        mt = np.ascontiguousarray(ck.get("mesh_triples", np.zeros((0, 3))),
                                  dtype=np.int64).reshape(-1, 3)
        mdt = np.ascontiguousarray(ck.get("mesh_delta_t", np.zeros((0, 3))),
                                   dtype=np.float64).reshape(-1, 3)
        if mt.shape[0]:
            self._check(self._lib.dem_restore_mesh_contacts(self._h, instance, mt.shape[0],
                                                            mt.ctypes.data_as(I64P), _d(mdt)))

    def autotune(self, trial_steps=200):
        """Tune force block size, cell edge and search schedule on the running
        simulation (advances it by the trial steps); returns the report."""
        t = dem_tuning()
        self._check(self._lib.dem_autotune(self._h, trial_steps, C.byref(t)))
        sched = [int(k) for k in t.schedules if k >= 0]
        return {"force_block": t.force_block, "rebuild_interval": t.rebuild_interval,
                "cell_factor": t.cell_factor, "ms_per_step": t.ms_per_step, "steps": t.steps,
                "block_ms": dict(zip((64, 128, 256), list(t.block_ms))),
                "search_ms": dict(zip(list(t.cell_factors), list(t.search_ms))),
                "schedule_ms": dict(zip(sched, list(t.schedule_ms)[:len(sched)]))}

    def set_timing(self, enable=True):
        self._check(self._lib.dem_set_timing(self._h, 1 if enable else 0))

    def get_timing(self):
        out = np.zeros(4)
        self._check(self._lib.dem_get_timing(self._h, _d(out)))
        return {"force_ms": out[0], "force_launches": int(out[1]), "search_ms": out[2],
                "searches": int(out[3])}

    # ------------------------------------------------------------- scenes
    def set_instance_domain(self, lo, hi, instance=0):
        lo, hi = _v3(lo), _v3(hi)
        self._check(self._lib.dem_set_instance_domain(self._h, instance, _d(lo), _d(hi)))

    def _add_scene(self, scene, instance, own_domain=False):
        if own_domain:
            self.set_instance_domain(scene["config"]["domain_lo"], scene["config"]["domain_hi"],
                                     instance=instance)
        for t, m in enumerate(scene["materials"]):
            self.set_material(t, m["density"], m["youngs"], m["poisson"], m["restitution"],
                              m["friction"], m["rolling_friction"], instance=instance)
        for w in scene["walls"]:
            if w["kind"] == "plane":
                wid = self.add_planar_wall(w["point"], w["normal"], w["material"],
                                           w.get("extent"), w.get("axis_point"), w.get("omega"),
                                           w["t_on"], w["t_off"], instance=instance)
            elif w["kind"] == "mesh":
                wid = self.add_mesh_wall(w["vertices"], w["triangles"], w["material"],
                                         w.get("axis_point"), w.get("omega"), w["t_on"],
                                         w["t_off"], instance=instance)
            elif w["kind"] == "cylinder":
                wid = self.add_cylinder_wall(w["axis_point"], w["axis_dir"], w["radius"],
                                             w["s_min"], w["s_max"], w["inside"], w["material"],
                                             w["omega"], w["t_on"], w["t_off"], instance=instance)
            else:
                wid = self.add_cone_wall(w["axis_point"], w["axis_dir"], w["radius0"], w["slope"],
                                         w["s_min"], w["s_max"], w["inside"], w["material"],
                                         w["omega"], w["t_on"], w["t_off"], instance=instance)
            if w.get("velocity") is not None:
                self.set_wall_motion(wid, w["velocity"], instance=instance)
        p = scene["particles"]
        self.set_particles(p["pos"], p["radius"], p["vel"], p["omega"], p["types"],
                           instance=instance)

    @classmethod
    def from_scene(cls, scene, precision="fp64", max_neighbors=0, hip_stream=None,
                   force_block=0):
        """Build a context from a scene dictionary (see ``workloads``)."""
        return cls.from_scenes([scene], precision, max_neighbors, hip_stream, force_block)

    @classmethod
    def from_scenes(cls, scenes, precision="fp64", max_neighbors=0, hip_stream=None,
                    force_block=0):
        """Build one batched context holding one instance per scene.  The scenes
        must share dt, gravity, search settings and integrator; each keeps its
        own domain box."""
        c = scenes[0]["config"]

        def shared(cfg):
            return {k: v for k, v in cfg.items() if k not in ("domain_lo", "domain_hi")}
        for s in scenes[1:]:
            if shared(s["config"]) != shared(c):
                raise ValueError("batched scenes must share their run configuration")
        sim = cls(dt=c["dt"], gravity=c["gravity"], domain_lo=c["domain_lo"],
                  domain_hi=c["domain_hi"], neighbor_threshold=c["neighbor_threshold"],
                  cell_factor=c["cell_factor"], rebuild_interval=c["rebuild_interval"],
                  integrator=c["integrator"], rolling_model=c["rolling_model"],
                  precision=precision, max_neighbors=max_neighbors, hip_stream=hip_stream,
                  n_instances=len(scenes), contact_model=c.get("contact_model", "nonlinear"),
                  characteristic_velocity=c.get("characteristic_velocity", 0.0),
                  force_block=force_block)
        for k, s in enumerate(scenes):
            sim._add_scene(s, k, own_domain=len(scenes) > 1)
        if len(scenes) > 1:
            sim.commit()
        return sim
