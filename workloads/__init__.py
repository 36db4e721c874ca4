"""Seeded synthetic inputs for the DEM hot path.

This module only places particles and describes walls, materials and run
settings as plain dictionaries of numbers and numpy arrays.  It holds none of
the method's arithmetic (no contact law, no search, no integration) and is the
one thing that both the oracle and the GPU library consume.  Every generator is
deterministic given its seed (numpy PCG64).

Scene dictionary layout::

    {"name": str,
     "config": {dt, gravity, domain_lo, domain_hi, neighbor_threshold,
                cell_factor, rebuild_interval, integrator, rolling_model,
                contact_model, characteristic_velocity},
     "materials": [dict(density, youngs, poisson, restitution, friction,
                        rolling_friction), ...],        # index = type id
     "walls": [dict(kind="plane", point, normal, material, extent=None,
                    axis_point=None, omega=None, t_on, t_off) |
               dict(kind="cylinder", axis_point, axis_dir, radius, s_min, s_max,
                    inside, material, omega, t_on, t_off) |
               dict(kind="cone", axis_point, axis_dir, radius0, slope, s_min, s_max,
                    inside, material, omega, t_on, t_off) |
               dict(kind="mesh", vertices (m,3), triangles (k,3), material,
                    axis_point=None, omega=None, t_on, t_off), ...],
     every wall may carry velocity=(vx, vy, vz) (translation, None = fixed)
     "particles": {pos (n,3), radius (n,), vel (n,3), omega (n,3), types (n,)}}
"""
from __future__ import annotations

import math

import numpy as np

INF = float("inf")

# Material of the 1,000-sphere box (d = 3 mm glass-like beads, soft modulus).
BOX_MATERIAL = dict(density=2500.0, youngs=1.0e6, poisson=0.3, restitution=0.9,
                    friction=0.3, rolling_friction=0.1)


def _cfg(dt, lo, hi, threshold=1.3, cell_factor=None, K=20, integrator="verlet",
         rolling="constant", gravity=(0.0, 0.0, -9.81), model="nonlinear", V=0.0):
    return dict(dt=float(dt), gravity=tuple(float(g) for g in gravity),
                domain_lo=tuple(float(v) for v in lo), domain_hi=tuple(float(v) for v in hi),
                neighbor_threshold=float(threshold),
                cell_factor=float(threshold if cell_factor is None else cell_factor),
                rebuild_interval=int(K), integrator=integrator, rolling_model=rolling,
                contact_model=model, characteristic_velocity=float(V))


def _particles(pos, radius, vel=None, omega=None, types=None):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    radius = np.ascontiguousarray(np.broadcast_to(np.asarray(radius, dtype=np.float64), (n,)))
    vel = np.zeros((n, 3)) if vel is None else np.ascontiguousarray(vel, dtype=np.float64).reshape(n, 3)
    omega = np.zeros((n, 3)) if omega is None else np.ascontiguousarray(omega, dtype=np.float64).reshape(n, 3)
    types = np.zeros(n, dtype=np.int32) if types is None else np.ascontiguousarray(types, dtype=np.int32)
    return dict(pos=pos, radius=radius, vel=vel, omega=omega, types=types)


def _vel(velocity):
    return None if velocity is None else tuple(float(v) for v in velocity)


def plane(point, normal, material=0, extent=None, axis_point=None, omega=None,
          t_on=-INF, t_off=INF, velocity=None):
    """Plane wall; ``velocity`` translates it (None: fixed)."""
    return dict(kind="plane", point=tuple(point), normal=tuple(normal), material=material,
                extent=None if extent is None else tuple(extent),
                axis_point=None if axis_point is None else tuple(axis_point),
                omega=None if omega is None else tuple(omega), t_on=t_on, t_off=t_off,
                velocity=_vel(velocity))


def cylinder(axis_point, axis_dir, radius, s_min, s_max, inside=True, material=0,
             omega=0.0, t_on=-INF, t_off=INF, velocity=None):
    return dict(kind="cylinder", axis_point=tuple(axis_point), axis_dir=tuple(axis_dir),
                radius=float(radius), s_min=float(s_min), s_max=float(s_max),
                inside=bool(inside), material=material, omega=float(omega), t_on=t_on,
                t_off=t_off, velocity=_vel(velocity))


def cone(axis_point, axis_dir, radius0, slope, s_min, s_max, inside=True, material=0,
         omega=0.0, t_on=-INF, t_off=INF, velocity=None):
    """Cone (frustum) whose surface lies at radius0 + slope * s from the axis."""
    return dict(kind="cone", axis_point=tuple(axis_point), axis_dir=tuple(axis_dir),
                radius0=float(radius0), slope=float(slope), s_min=float(s_min),
                s_max=float(s_max), inside=bool(inside), material=material,
                omega=float(omega), t_on=t_on, t_off=t_off, velocity=_vel(velocity))


def mesh(vertices, triangles, material=0, axis_point=None, omega=None, t_on=-INF, t_off=INF,
         velocity=None):
    """Triangle-mesh wall: corners (m, 3) and corner indices (k, 3), each
    triangle ordered so that (p1 - p0) x (p2 - p0) points to the particles."""
    return dict(kind="mesh", vertices=np.ascontiguousarray(vertices, dtype=np.float64),
                triangles=np.ascontiguousarray(triangles, dtype=np.int32), material=material,
                axis_point=None if axis_point is None else tuple(axis_point),
                omega=None if omega is None else tuple(omega), t_on=t_on, t_off=t_off,
                velocity=_vel(velocity))


def box_mesh(lo, hi, material=0, divisions=1):
    """The inside of the box [lo, hi] as a closed triangle mesh (normals
    inwards), each face split into divisions x divisions squares of two
    triangles."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    verts, index, tris = [], {}, []

    def vid(p):
        key = tuple(np.round(p, 15))
        if key not in index:
            index[key] = len(verts)
            verts.append(p)
        return index[key]

    m = divisions
    for ax in range(3):
        a, b = (ax + 1) % 3, (ax + 2) % 3
        for side, val in ((0, lo[ax]), (1, hi[ax])):
            grid = {}
            for i in range(m + 1):
                for j in range(m + 1):
                    p = np.empty(3)
                    p[ax] = val
                    p[a] = lo[a] + (hi[a] - lo[a]) * i / m
                    p[b] = lo[b] + (hi[b] - lo[b]) * j / m
                    grid[i, j] = vid(p)
            for i in range(m):
                for j in range(m):
                    q = [grid[i, j], grid[i + 1, j], grid[i + 1, j + 1], grid[i, j + 1]]
                    # e_a x e_b = e_ax: counter-clockwise faces +ax, the low side
                    t1, t2 = (q[0], q[1], q[2]), (q[0], q[2], q[3])
                    if side == 1:
                        t1, t2 = t1[::-1], t2[::-1]
                    tris += [t1, t2]
    return mesh(np.array(verts), np.array(tris), material)


def frustum_mesh(axis_point, radius0, slope, s_min, s_max, segments=48, rings=4, material=0,
                 omega=0.0):
    """Inside of a cone frustum around the z axis through axis_point
    (radius radius0 + slope s at height s in [s_min, s_max]) as a triangle
    mesh: `segments` corners around, `rings` + 1 rings, normals towards the
    axis.  The polygonal surface lies inside the analytic one between its
    corners."""
    c = np.asarray(axis_point, dtype=np.float64)
    verts, tris = [], []
    for r in range(rings + 1):
        sz = s_min + (s_max - s_min) * r / rings
        rad = radius0 + slope * sz
        for k in range(segments):
            a = 2 * math.pi * k / segments
            verts.append(c + np.array([rad * math.cos(a), rad * math.sin(a), sz]))
    for r in range(rings):
        for k in range(segments):
            a0 = r * segments + k
            a1 = r * segments + (k + 1) % segments
            b0, b1 = a0 + segments, a1 + segments
            # counter-clockwise seen from the axis
            tris += [(a0, b0, a1), (a1, b0, b1)]
    return mesh(np.array(verts), np.array(tris), material,
                axis_point=tuple(c), omega=(0.0, 0.0, float(omega)))


def drum_mesh(radius, x0, x1, segments=256, rings=64, material=0, omega=0.0):
    """Inside of the cylinder of the given radius around the x axis, x in
    [x0, x1], as a triangle mesh (`segments` corners around, `rings` + 1
    rings, normals towards the axis), spinning at omega about the x axis."""
    verts, tris = [], []
    for r in range(rings + 1):
        x = x0 + (x1 - x0) * r / rings
        for k in range(segments):
            a = 2 * math.pi * k / segments
            verts.append((x, radius * math.cos(a), radius * math.sin(a)))
    for r in range(rings):
        for k in range(segments):
            a0 = r * segments + k
            a1 = r * segments + (k + 1) % segments
            b0, b1 = a0 + segments, a1 + segments
            tris += [(a0, b1, a1), (a0, b0, b1)]
    return mesh(np.array(verts), np.array(tris), material, axis_point=(0.0, 0.0, 0.0),
                omega=(float(omega), 0.0, 0.0))


def meshed_drum_scene(n=1_000_000, segments=256, rings=64, **kw):
    """The rotating drum with its cylinder replaced by a spinning triangle
    mesh (the end planes stay analytic)."""
    sc = drum_scene(n=n, **kw)
    g = sc["geometry"]
    m = drum_mesh(g["R"], -g["L"] / 2, g["L"] / 2, segments, rings, omega=g["omega"])
    return dict(sc, name=f"meshed_drum_{n}", walls=[m] + sc["walls"][1:])


def box_walls(lo, hi, material=0):
    """Six planes bounding [lo, hi], normals pointing inwards."""
    walls = []
    for k in range(3):
        n = [0.0, 0.0, 0.0]
        n[k] = 1.0
        walls.append(plane(tuple(lo), tuple(n), material))
        n = [0.0, 0.0, 0.0]
        n[k] = -1.0
        walls.append(plane(tuple(hi), tuple(n), material))
    return walls


# --------------------------------------------------------------- placement

def rsa_box(n, radius, lo, hi, rng, max_tries=200000):
    """Random sequential addition of n equal spheres with centres in [lo, hi].

    Rejection uses a hash grid of edge 2*radius; raises if it cannot place n.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = 2.0 * radius
    dims = np.maximum(1, np.ceil((hi - lo) / d).astype(np.int64))
    grid = {}
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries + 50 * n:
            raise RuntimeError(f"rsa_box: placed only {len(pts)} of {n}")
        p = lo + rng.random(3) * (hi - lo)
        c = np.minimum(((p - lo) / d).astype(np.int64), dims - 1)
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    for q in grid.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                        if np.sum((pts[q] - p) ** 2) < d * d:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            grid.setdefault((c[0], c[1], c[2]), []).append(len(pts))
            pts.append(p)
    return np.array(pts)


def jittered_lattice(lo, hi, spacing, jitter, rng):
    """Cubic lattice points in [lo, hi] with uniform jitter of +-jitter per axis."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    axes = [np.arange(lo[k], hi[k] + 1e-12, spacing) for k in range(3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    g = g + rng.uniform(-jitter, jitter, size=g.shape)
    return g


# ------------------------------------------------------------------ scenes

def box_scene(n=1000, d=3.0e-3, L=0.05, seed=0, steps_dt=1.0e-5, K=20):
    """1,000 monodisperse spheres at seeded random non-overlapping positions in
    a closed cube with six planar walls, gravity -z, dt = 1e-5, cell 1.2 d."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = d / 2
    pos = rsa_box(n, R, (R, R, R), (L - R, L - R, L - R), rng)
    lo = (-d, -d, -d)
    hi = (L + d, L + d, L + d)
    return dict(name=f"box_{n}", config=_cfg(steps_dt, lo, hi, threshold=1.3, cell_factor=1.2, K=K),
                materials=[dict(BOX_MATERIAL)], walls=box_walls((0, 0, 0), (L, L, L)),
                particles=_particles(pos, R))


DRUM_MATERIAL = dict(density=2500.0, youngs=1.0e6, poisson=0.3, restitution=0.8,
                     friction=0.5, rolling_friction=0.2)


def drum_geometry_for(n, d, bulk_fill=0.35, packing=0.6, aspect=2.0):
    """Drum radius R and length L = aspect*R holding n spheres of diameter d as
    a bed of packing fraction `packing` that fills `bulk_fill` of the volume."""
    vs = n * math.pi * d ** 3 / 6.0
    vol = vs / packing / bulk_fill
    R = (vol / (math.pi * aspect)) ** (1.0 / 3.0)
    return R, aspect * R


def drum_scene(n=1_000_000, d=3.0e-3, R_drum=None, L=None, omega=1.0, seed=2,
               dt=5.0e-6, K=20, material=None, threshold=1.3, spacing=1.05, jitter=0.02):
    """Rotating drum: n monodisperse spheres in a horizontal cylinder (axis x)
    spinning at `omega` rad/s with two co-rotating end planes.  Particles start
    at rest on a jittered cubic lattice (spacing 1.05 d, jitter +-0.02 d per
    axis, so no two spheres overlap) filling the lowest part of the drum."""
    mat = dict(DRUM_MATERIAL if material is None else material)
    if R_drum is None or L is None:
        R_drum, L = drum_geometry_for(n, d)
    rng = np.random.Generator(np.random.PCG64(seed))
    r = d / 2
    a = spacing * d
    # generate lattice points in the box hull with a margin, keep those inside
    lo = (-L / 2 + r * 1.2, -R_drum + r * 1.2, -R_drum + r * 1.2)
    hi = (L / 2 - r * 1.2, R_drum - r * 1.2, R_drum - r * 1.2)
    # only the lower part is needed: estimate the height to keep memory small
    g = jittered_lattice(lo, hi, a, jitter * d, rng)
    rho = np.sqrt(g[:, 1] ** 2 + g[:, 2] ** 2)
    keep = (rho < R_drum - 1.2 * r) & (np.abs(g[:, 0]) < L / 2 - 1.2 * r)
    g = g[keep]
    if g.shape[0] < n:
        raise RuntimeError(f"drum too small: {g.shape[0]} lattice sites < {n}")
    order = np.lexsort((g[:, 0], g[:, 1], g[:, 2]))  # lowest z first
    g = g[order[:n]]
    # shuffle so that the input order carries no spatial structure
    g = g[rng.permutation(n)]
    m = 2 * d
    dlo = (-L / 2 - m, -R_drum - m, -R_drum - m)
    dhi = (L / 2 + m, R_drum + m, R_drum + m)
    walls = [
        cylinder((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), R_drum, -L / 2, L / 2, True, 0, omega),
        plane((-L / 2, 0.0, 0.0), (1.0, 0.0, 0.0), 0, None, (0.0, 0.0, 0.0), (omega, 0.0, 0.0)),
        plane((L / 2, 0.0, 0.0), (-1.0, 0.0, 0.0), 0, None, (0.0, 0.0, 0.0), (omega, 0.0, 0.0)),
    ]
    return dict(name=f"drum_{n}", config=_cfg(dt, dlo, dhi, threshold=threshold, K=K),
                materials=[mat], walls=walls, particles=_particles(g, r),
                geometry=dict(R=R_drum, L=L, omega=omega))


def _fill_from_bottom(lo, hi, spacing, jitter, clearance_ok, n, rng, what):
    """The n lowest points of a jittered lattice over [lo, hi] that pass
    clearance_ok (a vectorised test on an (m, 3) array), shuffled."""
    g = jittered_lattice(lo, hi, spacing, jitter, rng)
    g = g[clearance_ok(g)]
    if g.shape[0] < n:
        raise RuntimeError(f"{what}: only {g.shape[0]} lattice sites for {n} spheres")
    order = np.lexsort((g[:, 0], g[:, 1], g[:, 2]))
    g = g[order[:n]]
    return g[rng.permutation(n)]


SILO_MATERIAL = dict(BOX_MATERIAL)


def wedge_silo_scene(n=200_000, d_min=2.0e-3, d_max=3.0e-3, width=0.2, depth=0.04,
                     height=0.9, outlet=0.012, angle_deg=30.0, t_open=INF, seed=1,
                     dt=5.0e-6, K=20, spacing=1.02, clearance=1.02, threshold=1.3,
                     material=None):
    """Wedge-shaped silo: a box (x across, y through the depth, z up) whose
    floor is two planes inclined at angle_deg from the horizontal meeting a
    slot outlet of width `outlet` at z = 0, plugged by a floating plane that
    disappears at t_open.  Diameters uniform in [d_min, d_max]; spheres start
    at rest on a jittered lattice of spacing `spacing` d_max filling the silo
    from the bottom, at least `clearance` radii from every wall.  The domain
    box ends 2 d_max below the outlet: spheres that leave become inactive."""
    mat = dict(SILO_MATERIAL if material is None else material)
    rng = np.random.Generator(np.random.PCG64(seed))
    a = math.radians(angle_deg)
    sa, ca = math.sin(a), math.cos(a)
    ho = outlet / 2
    run = width / 2 - ho                  # horizontal extent of one wedge plane
    rise = run * math.tan(a)
    hl = 0.5 * run / ca                   # half length along the slope
    hv = depth / 2 + d_max
    nL, nR = (sa, 0.0, ca), (-sa, 0.0, ca)
    pL = (-ho - run / 2, 0.0, rise / 2)
    pR = (ho + run / 2, 0.0, rise / 2)
    walls = [
        plane(pL, nL, 0, (-ca, 0.0, sa, hl, hv)),
        plane(pR, nR, 0, (ca, 0.0, sa, hl, hv)),
        plane((-width / 2, 0.0, 0.0), (1.0, 0.0, 0.0)),
        plane((width / 2, 0.0, 0.0), (-1.0, 0.0, 0.0)),
        plane((0.0, -depth / 2, 0.0), (0.0, 1.0, 0.0)),
        plane((0.0, depth / 2, 0.0), (0.0, -1.0, 0.0)),
        plane((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 0, (1.0, 0.0, 0.0, ho + 0.25 * d_max, hv),
              t_off=t_open),
    ]
    c = clearance * d_max / 2

    def ok(g):
        dl = (g[:, 0] - pL[0]) * nL[0] + (g[:, 2] - pL[2]) * nL[2]
        dr = (g[:, 0] - pR[0]) * nR[0] + (g[:, 2] - pR[2]) * nR[2]
        return ((dl >= c) & (dr >= c) & (g[:, 2] >= c) & (np.abs(g[:, 0]) <= width / 2 - c)
                & (np.abs(g[:, 1]) <= depth / 2 - c) & (g[:, 2] <= height - c))

    g = _fill_from_bottom((-width / 2, -depth / 2, 0.0), (width / 2, depth / 2, height),
                          spacing * d_max, 0.01 * d_max, ok, n, rng, "wedge silo")
    radius = rng.uniform(d_min, d_max, n) / 2
    m = 2 * d_max
    lo = (-width / 2 - m, -depth / 2 - m, -2 * d_max)
    hi = (width / 2 + m, depth / 2 + m, height + m)
    return dict(name=f"wedge_silo_{n}", config=_cfg(dt, lo, hi, threshold=threshold, K=K),
                materials=[mat], walls=walls, particles=_particles(g, radius),
                geometry=dict(width=width, depth=depth, height=height, outlet=outlet,
                              angle_deg=angle_deg))


HOPPER_MATERIAL = dict(BOX_MATERIAL, youngs=1.0e7, friction=0.4)


def lognormal_diameters(n, mean, sigma, lo, hi, rng):
    """Log-normal diameters with mean `mean` and standard deviation `sigma` of
    ln d, clamped to [lo, hi]."""
    mu = math.log(mean) - sigma * sigma / 2
    return np.clip(np.exp(rng.normal(mu, sigma, n)), lo, hi)


def hopper_silo_scene(n=4_300_000, d_mean=2.5e-3, sigma=0.1, d_lo=2.0e-3, d_hi=3.5e-3,
                      R=0.25, H=1.0, outlet=0.04, angle_deg=60.0, t_open=INF, seed=3,
                      dt=2.0e-6, K=20, spacing=1.02, clearance=1.02, threshold=1.3,
                      material=None):
    """Cylindrical silo with a conical hopper: a cone around the vertical axis
    from the outlet radius at z = 0, inclined at angle_deg from the horizontal,
    up to radius R, then a cylinder of radius R and height H (taller when the
    spheres need it to start on the lattice).  The outlet is plugged by a
    floating plane until t_open.  Log-normal diameters; spheres start at rest
    on a jittered lattice filling the silo from the bottom."""
    mat = dict(HOPPER_MATERIAL if material is None else material)
    rng = np.random.Generator(np.random.PCG64(seed))
    d = lognormal_diameters(n, d_mean, sigma, d_lo, d_hi, rng)
    dmax = float(d.max()) if n else d_hi
    r0 = outlet / 2
    slope = 1.0 / math.tan(math.radians(angle_deg))
    s_top = (R - r0) / slope
    q = math.sqrt(1.0 + slope * slope)
    c = clearance * dmax / 2
    a = spacing * dmax
    # the lattice holds about (pi R^2 / a^2) spheres per layer of height a
    per_layer = math.pi * (R - c) ** 2 / (a * a)
    need = s_top + 1.3 * a * n / max(per_layer, 1.0) + a
    top = s_top + max(H, need)

    def ok(g):
        rho = np.sqrt(g[:, 0] ** 2 + g[:, 1] ** 2)
        z = g[:, 2]
        in_cone = (z < s_top) & (rho <= r0 + slope * z - c * q)
        in_cyl = (z >= s_top) & (rho <= R - c)
        return (in_cone | in_cyl) & (z >= c) & (z <= top - c)

    g = _fill_from_bottom((-R, -R, 0.0), (R, R, top), a, 0.01 * dmax, ok, n, rng, "hopper silo")
    walls = [
        cone((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), r0, slope, 0.0, s_top, True),
        cylinder((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), R, s_top, top, True),
        plane((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 0,
              (1.0, 0.0, 0.0, r0 + 0.5 * dmax, r0 + 0.5 * dmax), t_off=t_open),
    ]
    m = 2 * dmax
    lo = (-R - m, -R - m, -2 * dmax)
    hi = (R + m, R + m, top + m)
    return dict(name=f"hopper_silo_{n}", config=_cfg(dt, lo, hi, threshold=threshold, K=K),
                materials=[mat], walls=walls, particles=_particles(g, d / 2),
                geometry=dict(R=R, H=top - s_top, outlet=outlet, angle_deg=angle_deg,
                              cone_top=s_top))


def dense_snapshot(n=3000, d=3.0e-3, seed=7, overlap=0.01, vmax=0.05, wmax=20.0,
                   polydisperse=0.0, n_types=1, dt=1.0e-5, K=5, walls=True,
                   rolling="constant", integrator="verlet", friction=None,
                   model="nonlinear", V=0.0,
                   threshold=1.3):
    """A jammed-like random snapshot that exercises every branch of the law:
    jittered lattice with spacing slightly below d (so many pairs overlap),
    random translational and angular velocities, optional size spread and
    several materials, inside a box of six walls some of which touch spheres."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side = int(math.ceil(n ** (1 / 3)))
    a = d * (1.0 - overlap)
    pts = np.stack(np.meshgrid(*[np.arange(side) * a] * 3, indexing="ij"), -1).reshape(-1, 3)
    pts = pts[:n] + rng.uniform(-0.003 * d, 0.003 * d, size=(n, 3))
    radius = np.full(n, d / 2)
    if polydisperse > 0:
        radius = radius * (1.0 - polydisperse * rng.random(n))
    pts = pts - pts.min(axis=0) + d
    vel = rng.uniform(-vmax, vmax, size=(n, 3))
    om = rng.uniform(-wmax, wmax, size=(n, 3))
    types = rng.integers(0, n_types, size=n).astype(np.int32)
    mats = []
    for t in range(n_types):
        m = dict(BOX_MATERIAL)
        m["restitution"] = [0.9, 0.5, 0.7, 0.3][t % 4]
        m["friction"] = [0.3, 0.1, 0.5, 0.05][t % 4] if friction is None else friction
        m["youngs"] = [1.0e6, 5.0e6, 2.0e6, 1.0e7][t % 4]
        m["poisson"] = [0.3, 0.25, 0.35, 0.2][t % 4]
        m["density"] = [2500.0, 3000.0, 2000.0, 7850.0][t % 4]
        mats.append(m)
    hi_box = pts.max(axis=0) + d
    wl = []
    if walls:
        # walls placed so that the outermost spheres slightly overlap them
        lo_w = pts.min(axis=0) - 0.45 * d
        hi_w = pts.max(axis=0) + 0.45 * d
        wl = box_walls(tuple(lo_w), tuple(hi_w), material=0)
    lo = (0.0, 0.0, 0.0)
    hi = tuple(hi_box + d)
    return dict(name=f"dense_{n}", config=_cfg(dt, lo, hi, threshold=threshold, K=K,
                                                 rolling=rolling, integrator=integrator,
                                                 model=model, V=V),
                materials=mats, walls=wl,
                particles=_particles(pts, radius, vel, om, types))


def batched_drums(n_inst=256, n_min=2000, n_max=50000, d=3.0e-3, seed=4, dt=5.0e-6, K=20,
                  threshold=1.3):
    """Independent rotating drums of uneven size: per instance k (seeded by
    SeedSequence(seed).spawn(n_inst)[k]) the particle count is log-uniform in
    [n_min, n_max], the friction coefficient uniform in [0.1, 0.5], the drum
    speed uniform in [0.5, 3] rad/s; the drum holds its spheres as a 35 % bulk
    fill with length = 2 R.  Other material values are the drum material's."""
    seqs = np.random.SeedSequence(seed).spawn(n_inst)
    scenes = []
    for k, ss in enumerate(seqs):
        rng = np.random.Generator(np.random.PCG64(ss))
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        mu = float(rng.uniform(0.1, 0.5))
        om = float(rng.uniform(0.5, 3.0))
        lattice_seed = int(rng.integers(0, 2 ** 31 - 1))
        mat = dict(DRUM_MATERIAL, friction=mu)
        sc = drum_scene(n=n, d=d, omega=om, seed=lattice_seed, dt=dt, K=K, material=mat,
                        threshold=threshold)
        sc["name"] = f"drum{k}_{n}"
        scenes.append(sc)
    return scenes


# Material of the parameter file printed in the paper's appendix (particles
# and walls alike): d = 5 mm, rho 2000, E 1 MPa, nu 0.3, e 0.3, mu 0.1,
# mu_r 0.05.
APPENDIX_MATERIAL = dict(density=2000.0, youngs=1.0e6, poisson=0.3, restitution=0.3,
                         friction=0.1, rolling_friction=0.05)


def sliding_floor_scene(n=20, d=5.0e-3, half=0.07, floor_speed=0.15, seed=19, dt=1.0e-5,
                        K=20):
    """The case of the appendix parameter file: a cube [-0.07, 0.07]^3 whose
    floor (boundary z = -0.07) translates at 0.15 m/s along x, 20 spheres of
    5 mm dropped from the insertion box [-0.05, 0.05]^2 x [-0.06, 0] (placed
    at seeded random non-overlapping positions, at rest, instead of being
    inserted during the run), dt 1e-5 s, a search every 20 steps, threshold
    1.3, constant rolling resistance, velocity Verlet, gravity -z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = d / 2
    pos = rsa_box(n, R, (-0.05 + R, -0.05 + R, -0.06 + R), (0.05 - R, 0.05 - R, 0.0 - R), rng)
    lo, hi = (-half,) * 3, (half,) * 3
    walls = box_walls(lo, hi)
    walls[4] = dict(walls[4], velocity=(float(floor_speed), 0.0, 0.0))  # the floor
    m = 2 * d
    return dict(name=f"sliding_floor_{n}",
                config=_cfg(dt, tuple(v - m for v in lo), tuple(v + m for v in hi), K=K),
                materials=[dict(APPENDIX_MATERIAL)], walls=walls, particles=_particles(pos, R))


def dam_break_scene(n=1_280_000, d=1.0e-3, length=0.4, height=0.2, t_dam=0.5, seed=5,
                    dt=1.0e-5, K=20, spacing=1.02, jitter=0.01, threshold=1.3,
                    material=None, depth=None):
    """Dam break (the paper's weak-scaling scene): spheres at rest in the left
    half of a box of length 0.4 m (x) and height 0.2 m (y, gravity -y), held
    by a floating dam (a plane at x = length / 2) that is removed at t_dam;
    then they spread over the whole length.  The depth (z) grows with n at
    the table's ratio of 0.01 m per 160,000 spheres unless given (small test
    cases).  Spheres of 1 mm on a jittered lattice (spacing 1.02 d, jitter
    +-0.01 d, its first column 1.02 radii from the dam) filling the left half
    from the bottom; the appendix material."""
    mat = dict(APPENDIX_MATERIAL if material is None else material)
    rng = np.random.Generator(np.random.PCG64(seed))
    r = d / 2
    depth = 0.01 * n / 160_000 if depth is None else float(depth)
    a = spacing * d
    c = 1.02 * r
    # enough layers for n spheres (at least one row of cells across the depth)
    per_layer = max(1, int((length / 2 - 2 * c) / a + 1)) * max(1, int((depth - 2 * c) / a + 1))
    layers = n / per_layer + 2
    while True:
        top = min(height - c, c + a * layers)
        jd = jitter * d  # lattice inset by the jitter so that no site is pushed out
        g = jittered_lattice((c + jd, c + jd, c + jd), (length / 2 - c - jd, top, depth - c - jd),
                             a, jd, rng)
        keep = ((g[:, 0] >= c) & (g[:, 0] <= length / 2 - c) & (g[:, 1] >= c) &
                (g[:, 2] >= c) & (g[:, 2] <= depth - c))
        g = g[keep]
        if g.shape[0] >= n:
            break
        if top >= height - c:
            raise RuntimeError(f"dam break: only {g.shape[0]} lattice sites for {n} spheres")
        layers += 2
    g[:, 0] = length / 2 - g[:, 0]  # columns counted from the dam
    g = g[np.lexsort((g[:, 2], g[:, 0], g[:, 1]))[:n]]  # lowest y first
    g = g[rng.permutation(n)]
    lo, hi = (0.0, 0.0, 0.0), (length, height, depth)
    walls = [plane((0.0, 0.0, 0.0), (1.0, 0.0, 0.0)), plane((length, 0.0, 0.0), (-1.0, 0.0, 0.0)),
             plane((0.0, 0.0, 0.0), (0.0, 1.0, 0.0)),
             plane((0.0, 0.0, 0.0), (0.0, 0.0, 1.0)), plane((0.0, 0.0, depth), (0.0, 0.0, -1.0)),
             plane((length / 2, 0.0, 0.0), (-1.0, 0.0, 0.0), t_off=float(t_dam))]
    m = 2 * d
    cfg = _cfg(dt, (-m, -m, -m), (length + m, height + m, depth + m), threshold=threshold, K=K,
               gravity=(0.0, -9.81, 0.0))
    return dict(name=f"dam_break_{n}", config=cfg, materials=[mat], walls=walls,
                particles=_particles(g, r), geometry=dict(length=length, depth=depth))
