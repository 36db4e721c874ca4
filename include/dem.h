/*
 * dem.h - C ABI of the MI355X (gfx950) soft-sphere DEM library (libdem.so).
 *
 * The library runs the data-parallel hot path of the soft-sphere discrete
 * element method of Golshan et al., "Lethe-DEM: an open-source parallel
 * discrete element solver with load balancing" (arXiv 2106.09576):
 *   - contact search every K steps ("constant" detection, Sec. 3.1): particles
 *     sorted into a uniform cell grid, broad search over neighbouring cells,
 *     fine search keeping pairs closer than r_s = threshold * d_max;
 *   - nonlinear Hertz-Mindlin particle-particle and particle-wall contact
 *     forces with tangential-overlap history, Coulomb limit with overlap
 *     truncation and constant-torque rolling resistance (Sec. 2.1);
 *   - velocity Verlet or explicit Euler integration of translation and
 *     rotation (Sec. 2.2).
 *
 * Conventions for every function:
 *   - returns 0 (DEM_OK) on success or a negative DEM_E* code; dem_last_error()
 *     gives a message for the calling thread;
 *   - host arrays passed in are copied before the call returns; output host
 *     arrays are caller-owned and filled in particle-input order ("gid" =
 *     index in the array given to dem_set_particles);
 *   - "*_device" variants take device pointers (e.g. PyTorch tensors'
 *     data_ptr()) that stay owned by the caller; they are read or written on
 *     the library's stream, which waits for the configured hip_stream first;
 *   - vectors are 3 doubles (x, y, z), arrays of vectors are n x 3 row-major;
 *   - a context is not thread-safe; separate contexts are independent;
 *   - call order: dem_create -> dem_set_material -> dem_add_*_wall ->
 *     dem_set_particles -> dem_step / dem_get_*.  Calling dem_set_particles
 *     again restarts the simulation (time 0, all contact history cleared).
 *   - a context holds n_instances >= 1 independent simulations ("instances")
 *     that share dt, gravity, domain box, search settings and precision and
 *     advance together: one dem_step launches each kernel once for all of
 *     them.  Materials, walls and particles are per instance; particle and
 *     wall ids are local to their instance.
 */
#ifndef DEM_H
#define DEM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dem_ctx dem_ctx; /* opaque context */

enum {
  DEM_OK = 0,
  DEM_EINVAL = -1,     /* invalid argument (message says which)               */
  DEM_EHIP = -2,       /* a HIP runtime call failed                           */
  DEM_ENOMEM = -3,     /* device or host allocation failed                    */
  DEM_ECAPACITY = -4,  /* more neighbours or wall contacts than the capacity  */
  DEM_EUNSTABLE = -5,  /* non-finite state, or a particle moved more than half
                          the search skin between two searches (a contact may
                          have been missed); the state stops at that search  */
  DEM_ESTATE = -6,     /* call order violated, or a previous error is sticky  */
  DEM_ENODEV = -7      /* no usable gfx950 device                              */
};

/* Material of a particle type or of a wall (physical-properties section of the
   paper's parameter file): density [kg/m^3], Young's modulus Y [Pa], Poisson
   ratio nu, restitution coefficient e in (0, 1], Coulomb friction mu >= 0,
   rolling friction mu_r >= 0. */
typedef struct {
  double density, youngs, poisson, restitution, friction, rolling_friction;
} dem_material;

typedef struct {
  double dt;                 /* time step [s] */
  double gravity[3];         /* [m/s^2] */
  double domain_lo[3];       /* domain box: the cell grid covers [lo, hi); a   */
  double domain_hi[3];       /* particle outside becomes inactive at a search  */
  double neighbor_threshold; /* r_s / d_max (paper default 1.3, Sec. 3.2) */
  double cell_factor;        /* cell edge h / d_max; r_s = min(threshold,
                                cell_factor) * d_max, so h >= r_s always */
  int32_t rebuild_interval;  /* K >= 1: contact search every K steps
                                (Sec. 3.1); 0 = dynamic: search when a
                                particle may have moved half the skin
                                r_s - d_max since the last search */
  int32_t integrator;        /* 0 velocity Verlet (Eqs. halfstep/newvv),
                                1 explicit Euler (Eq. integ_EE) */
  int32_t rolling_model;     /* 0 none, 1 constant torque, 2 viscous torque
                                (Sec. 2.1, table of rolling models) */
  int32_t precision;         /* 0 plain FP64; 1 contact law in FP32 with
                                positions, velocities, tangential history and
                                force sums in FP64 */
  int32_t n_instances;       /* independent simulations in the batch, 1..2048 */
  int32_t max_neighbors;     /* candidate neighbours kept per particle;
                                0 = derived from r_s and the smallest radius */
  void* hip_stream;          /* optional hipStream_t the library orders its
                                work after (and that waits for the library);
                                NULL = none */
  int32_t contact_model;     /* 0 nonlinear Hertz-Mindlin (Eqs. nonlinearkn-
                                nonlinearetat), 1 linear spring-dashpot (Eqs.
                                linearkn, linearetan; tangential constants
                                equal to the normal ones) */
  int32_t reserved;          /* must be 0 */
  double characteristic_velocity; /* V of Eq. (linearkn) [m/s], > 0 for the
                                     linear model, ignored otherwise */
  int32_t force_block;       /* threads per force workgroup: 64, 128 or 256;
                                0 = 256 (results do not depend on it) */
  int32_t reserved2;         /* must be 0 */
} dem_config;

typedef struct {
  int64_t n_particles;     /* particles of all instances                    */
  int64_t n_active;        /* not deactivated by leaving the domain box     */
  int64_t n_list_entries;  /* directed candidate entries (2 per pair)       */
  int64_t n_touching;      /* directed entries whose spheres overlap        */
  int64_t n_wall_candidates;
  int64_t step;            /* steps completed since dem_set_particles       */
  int64_t n_rebuilds;      /* contact searches run, including the first     */
  int32_t max_neighbors;   /* capacity per particle in use                  */
  int32_t precision;
  double r_s, cell_size, skin, d_max;  /* of instance 0 */
  int64_t n_cells;         /* cells of the grids (one key per cell)          */
  int64_t device_bytes;    /* device memory held by the context             */
} dem_stats;

/* Create a context on the current HIP device.  cfg is copied.  Fails with
   DEM_EINVAL for dt <= 0, an empty domain, rebuild_interval < 0, threshold or
   cell_factor < 1, an unknown integrator/rolling model/precision or
   n_instances outside [1, 2048]; DEM_ENODEV if the device is not gfx950. */
int dem_create(const dem_config* cfg, dem_ctx** out_ctx);
/* Release every device buffer of the context.  NULL is ignored. */
void dem_destroy(dem_ctx* ctx);
/* Message of the last error on the calling thread ("" if none). */
const char* dem_last_error(dem_ctx* ctx);

/* Material of particle type / wall material id `type` (0 <= type < 16) of
   instance `instance` (0 <= instance < n_instances). */
int dem_set_material(dem_ctx* ctx, int32_t instance, int32_t type, const dem_material* m);

/* Planar wall through `point` with unit `normal` pointing into the domain
   (normalised here; a zero vector is DEM_EINVAL).  extent: NULL = infinite,
   else 5 doubles {u_x, u_y, u_z, half_u, half_v}: u is projected into the
   plane, v = normal x u, and the wall acts only where the particle centre
   projects inside the rectangle (no edge contacts).  The wall's surface
   moves with velocity omega x (x_c - axis_point) at the contact point x_c
   (NULL omega = static; NULL axis_point = point); the geometry itself does
   not move, so omega should be parallel to the normal.  The wall acts for
   t_on <= t < t_off (floating walls, Sec. 3.7).  Writes its id to *wall_id
   (may be NULL).  Walls are added before dem_set_particles (else
   DEM_ESTATE); at most 32 walls. */
int dem_add_planar_wall(dem_ctx* ctx, int32_t instance, const double point[3],
                        const double normal[3], const double* extent, int32_t material,
                        const double axis_point[3], const double omega[3], double t_on,
                        double t_off, int32_t* wall_id);

/* Cylindrical wall of radius `radius` around the axis through axis_point
   along axis_dir (normalised), acting where the axial coordinate
   s = (x - axis_point).axis_dir lies in [s_min, s_max]; inside != 0 keeps
   particles inside the cylinder, 0 outside.  The wall spins at `omega` rad/s
   about the axis (surface velocity omega axis_dir x (x_c - axis_point)).
   Same activity window and ordering rules as the planar wall. */
int dem_add_cylinder_wall(dem_ctx* ctx, int32_t instance, const double axis_point[3],
                          const double axis_dir[3], double radius, double s_min, double s_max,
                          int32_t inside, int32_t material, double omega, double t_on,
                          double t_off, int32_t* wall_id);

/* Conical wall (frustum) around the axis through axis_point along axis_dir
   (normalised): at axial coordinate s = (x - axis_point).axis_dir the
   surface lies at radius0 + slope s from the axis (slope = cot of the
   surface's angle to the axis-normal plane, negative when the cone narrows
   with s), acting where s of the particle centre lies in [s_min, s_max]; the
   radius must stay > 0 there (DEM_EINVAL otherwise).  A particle at distance
   rho from the axis is at (r(s) - rho) / sqrt(1 + slope^2) from the surface
   of its meridian (inside != 0; the opposite sign outside), and is pushed
   along that meridian's surface normal.  Walls are analytic surfaces here,
   standing in for the paper's meshed boundaries (Sec. 2.1, last paragraph:
   the wall acts as a body of infinite mass and radius); a cone closes the
   hopper of a cylindrical silo.  Spins at `omega` rad/s about the axis;
   activity window and ordering rules as for the planar wall. */
int dem_add_cone_wall(dem_ctx* ctx, int32_t instance, const double axis_point[3],
                      const double axis_dir[3], double radius0, double slope, double s_min,
                      double s_max, int32_t inside, int32_t material, double omega, double t_on,
                      double t_off, int32_t* wall_id);

/* Mesh wall: a rigid surface of n_triangles triangles over n_vertices
   corners (vertices: n_vertices x 3 doubles; triangles: n_triangles x 3
   corner indices, each triangle ordered so that (p1 - p0) x (p2 - p0) points
   to the particles' side).  Sec. 3.7: particles collide with the boundary's
   faces, lines (edges) and points (vertices).  Every triangle whose plane
   the centre is less than R behind and which is closer than R + skin at a
   contact search is a candidate (at most 8 per particle, else DEM_ECAPACITY:
   triangles should not be much smaller than the spheres).  At each step a
   face touches when the centre projects strictly inside it and is less
   than R above its plane; an edge or a vertex touches when it is the
   closest point of every candidate triangle around it (a local minimum of
   the distance over the surface) and closer than R; each contact acts once,
   with the law of Sec. 2.1 and the wall as a body of infinite mass and
   radius.  Surface velocity omega x (x_c - axis_point) (NULL omega = none;
   NULL axis_point = the first vertex); translation with dem_set_wall_motion;
   active for t_on <= t < t_off.  At most 2^24 triangles per instance;
   DEM_EINVAL for out-of-range corner indices, degenerate triangles or
   non-finite corners.  The arrays are copied.  Walls are added before
   dem_set_particles (else DEM_ESTATE). */
int dem_add_mesh_wall(dem_ctx* ctx, int32_t instance, int64_t n_vertices,
                      const double* vertices, int64_t n_triangles, const int32_t* triangles,
                      int32_t material, const double axis_point[3], const double omega[3],
                      double t_on, double t_off, int32_t* wall_id);

/* Translational motion of wall `wall_id` of an instance (Sec. 3.7, boundary
   motion: boundaries may rotate or translate): the wall moves with constant
   velocity `velocity` (3 doubles, m/s), so that at time t its point and its
   rotation axis lie at their given positions + velocity t, and the velocity
   of its surface at a contact point x_c is velocity + Omega x (x_c - axis(t)).
   Every contact search places the walls where they are at the step it runs
   at.  Between two searches a translating wall may move at most half the
   skin (r_s - d_max): |velocity| K dt <= skin / 2 for rebuild_interval K, or
   |velocity| dt <= skin / 2 with the dynamic schedule, which then also
   searches before any wall has covered half the skin since the last search;
   the call that builds the batch returns DEM_EINVAL otherwise.  Called
   before dem_set_particles for that instance (else DEM_ESTATE); DEM_EINVAL
   for an unknown wall id or a non-finite velocity.  The default is 0. */
int dem_set_wall_motion(dem_ctx* ctx, int32_t instance, int32_t wall_id,
                        const double velocity[3]);

/* Set n >= 0 particles of one instance: positions (n x 3), velocities and
   angular velocities (n x 3, NULL = zero), radii (n, > 0) and material types
   (n, NULL = type 0; each type's material must be set).  Masses are
   rho (4/3) pi R^3 and moments of inertia (2/5) m R^2.  The inputs are
   copied; the batch is built on the device (first contact search at these
   positions with all tangential overlaps zero, stored forces zero so the
   first velocity-Verlet half kick sees gravity only) immediately when
   n_instances == 1, otherwise by dem_commit or the first dem_step/dem_get_*
   once every instance has particles.  Setting particles again restarts the
   whole batch from the inputs last given for each instance.  DEM_ECAPACITY
   (from the call that builds the batch) if a particle already has more
   neighbours than max_neighbors; DEM_EINVAL if n or the batch's total
   exceeds 2^29 particles. */
int dem_set_particles(dem_ctx* ctx, int32_t instance, int64_t n, const double* pos,
                      const double* vel, const double* omega, const double* radius,
                      const int32_t* type);
/* Same with device pointers (caller-owned, read on the library's stream and
   staged through host memory for validation). */
int dem_set_particles_device(dem_ctx* ctx, int32_t instance, int64_t n, const double* pos,
                             const double* vel, const double* omega, const double* radius,
                             const int32_t* type);

/* Domain box of one instance, replacing the config's domain_lo/domain_hi for
   it (cell grid and deactivation box).  Called before dem_set_particles for
   that instance. */
int dem_set_instance_domain(dem_ctx* ctx, int32_t instance, const double lo[3],
                            const double hi[3]);

/* Build the batch on the device now (all instances must have particles).
   Returns the errors described for dem_set_particles. */
int dem_commit(dem_ctx* ctx);

/* Advance every instance by n_steps >= 0 steps.  Synchronous: returns after the work finished.
   With rebuild_interval K >= 1, contact searches run at every step number
   that is a multiple of K.  With K = 0 the library reads back, every few
   steps, the largest per-step displacement |v| dt of any particle and
   searches before the summed bound could reach half the skin; a missed
   bound still trips the displacement check of the next search
   (DEM_EUNSTABLE).  dem_commit with K = 0 fails with DEM_EINVAL when an
   instance has no skin (neighbor_threshold = 1).  Errors (DEM_EUNSTABLE, DEM_ECAPACITY) are sticky: the
   state is frozen at the step where they were detected and later dem_step
   calls return DEM_ESTATE until dem_set_particles is called again. */
int dem_step(dem_ctx* ctx, int64_t n_steps);

/* Current state in input order (Sec. 2.2: the integrated translational and
   angular state; for velocity Verlet the full-step velocities of Eq. newvv):
   positions, velocities, angular velocities (n x 3 each), active flags (n;
   0 once a particle left the domain box, Sec. 3.1) and time; any pointer may
   be NULL.  Host arrays are caller-owned; DEM_EINVAL for a bad instance,
   DEM_ESTATE before the particles are set. */
int dem_get_state(dem_ctx* ctx, int32_t instance, double* pos, double* vel, double* omega,
                  uint8_t* active, double* time_out);
/* Same into device buffers (caller-owned; written on the library's stream,
   complete when the call returns).  Same errors. */
int dem_get_state_device(dem_ctx* ctx, int32_t instance, double* pos, double* vel,
                         double* omega, uint8_t* active);

/* Exact resume: restore into a freshly set instance what dem_set_particles
   does not carry, as read from the saved context (instance-local gids):
   n_pairs particle pairs (n_pairs x 2, gid_i < gid_j) that touched at the
   last force evaluation with their tangential overlap (n_pairs x 3, i -> j;
   j -> i gets the exact negative), n_wall particle-wall contacts (gid, wall
   id) with their overlaps, the force and torque of the last evaluation
   (n x 3 each, input order; NULL keeps the current ones), and the step
   count (-1 keeps it; it sets the time used by wall activity windows).  The
   pairs and walls must be candidates of the current lists: true when the
   positions were saved right after a contact search (a multiple of K under
   the constant schedule), which is also when the resumed run repeats the
   saved one bit for bit.  Histories of the instance not listed are zeroed.
   Host arrays are read and copied; DEM_EINVAL for a pair or wall contact that
   is not in the lists (nothing is changed on the device then, except, with
   translating walls, the step count and the contact search at the restored
   time that precede the check). */
int dem_restore(dem_ctx* ctx, int32_t instance, int64_t n_pairs, const int64_t* pairs,
                const double* delta_t, int64_t n_wall, const int64_t* wall_pairs,
                const double* wall_delta_t, const double* force, const double* torque,
                int64_t step);

/* Exact resume, mesh walls: after dem_restore, the tangential overlaps of
   n_tri particle-triangle candidates given as (gid, wall id, triangle index
   within the wall) triples (n_tri x 3) with their overlaps (n_tri x 3), as
   dem_get_mesh_contacts returned them in the saved context; the overlaps of
   the instance's other triangle candidates are zeroed.  DEM_EINVAL for a
   triple that is not a candidate of the current lists (nothing is changed
   on the device then). */
int dem_restore_mesh_contacts(dem_ctx* ctx, int32_t instance, int64_t n_tri,
                              const int64_t* triples, const double* delta_t);

/* Total contact force and torque on every particle from the last force
   evaluation of the last dem_step call (zero before the first step): the sum
   over its contacts of F^n + F^t (Eqs. normal_force, tangential_force after
   the Coulomb limit of Eqs. coulomb_overlap) and of the tangential and
   rolling torques (Eq. torque_t and the rolling-model table), walls
   included, gravity excluded (Sec. 2.1).  n x 3 each, input order,
   caller-owned host arrays (either may be NULL).  Same errors as
   dem_get_state. */
int dem_get_forces(dem_ctx* ctx, int32_t instance, double* force, double* torque);

/* Candidate particle pairs of the current contact list (the fine search of
   Sec. 3.2: pairs closer than the neighbour threshold at the last search),
   each once as (gid_i, gid_j) with gid_i < gid_j, sorted; delta_t =
   tangential overlap of Eq. delta_t of the pair oriented from i to j (3 per
   pair, zero for pairs that did not touch at the last force evaluation);
   touching = 1 if the spheres overlap at the current positions (Eq.
   deltan > 0).  *n_out receives the count; if it exceeds cap nothing else is
   written and DEM_EINVAL is returned.  Host arrays, caller-owned; any of
   pairs, delta_t, touching may be NULL. */
int dem_get_contacts(dem_ctx* ctx, int32_t instance, int64_t cap, int64_t* pairs,
                     double* delta_t, uint8_t* touching, int64_t* n_out);
/* The candidate pairs of dem_get_contacts written to device buffers
   (caller-owned, on the device of the context; written on the library's
   stream, complete when the call returns): pairs (2 int64 per pair, gid_i <
   gid_j), delta_t (3 doubles per pair), touching (1 byte per pair); any of
   them may be NULL.  Same pairs and values as dem_get_contacts, but in the
   library's spatial order (the sorted order of gid_i, then the order of its
   neighbour row) instead of gid order.  *n_out (host) receives the count; if
   it exceeds cap nothing else is written and DEM_EINVAL is returned.  Uses a
   device workspace of about 8 bytes per 256 particles, allocated and freed
   by the call (DEM_EHIP if that fails); DEM_EINVAL when the neighbour list
   has 2^31 entries or more. */
int dem_get_contacts_device(dem_ctx* ctx, int32_t instance, int64_t cap, int64_t* pairs,
                            double* delta_t, uint8_t* touching, int64_t* n_out);
/* dem_get_contacts_device for callers that cannot allocate device memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): the same pairs in the same order, but the workspace is a
   file-scope device array of the library (512 KiB per GPU, held until the
   process ends; its address is looked up once per device, on the first call
   with that device current) instead of a per-call allocation.  Contexts of
   at most 2^24 particles (DEM_EINVAL beyond, and when the context's device
   is not the current one).  Every call on a GPU shares that GPU's workspace:
   calls that overlap on one GPU (several host threads, or contexts on other
   streams) race and must be serialised by the caller.  Allocates nothing,
   host or device. */
int dem_get_contacts_device_noalloc(dem_ctx* ctx, int32_t instance, int64_t cap,
                                    int64_t* pairs, double* delta_t, uint8_t* touching,
                                    int64_t* n_out);
/* Per-contact force record, for error measures per contact.  While enabled
   (enable != 0; off by default), every force evaluation also writes the force
   F^n + F^t (Eqs. normal_force and tangential_force after the Coulomb limit of
   Eqs. coulomb_overlap) of each touching pair on the particle whose row holds
   it, into a device buffer of 24 bytes per neighbour-list entry that the
   context owns (allocated here or at the next dem_set_particles commit, freed
   when disabled or destroyed).  DEM_ENOMEM if it cannot be allocated. */
int dem_record_contact_forces(dem_ctx* ctx, int32_t enable);
/* The record of the last force evaluation: the candidate pairs of
   dem_get_contacts in the same order, each with the force on gid_i (3 per
   pair, zero for a pair that did not touch then).  Same capacity rule and
   ownership as dem_get_contacts.  DEM_ESTATE when the record is off, or when
   a constant-interval explicit-Euler run ended with a contact search (the
   record then belongs to the previous list). */
int dem_get_contact_forces(dem_ctx* ctx, int32_t instance, int64_t cap, int64_t* pairs,
                           double* force, int64_t* n_out);
/* Particle-wall candidates of the analytic walls (Sec. 2.1 last paragraph,
   walls as bodies of infinite mass and radius) as (gid, wall_id), sorted,
   with their tangential overlaps (Eq. delta_t).  Same capacity rule and
   ownership. */
int dem_get_wall_contacts(dem_ctx* ctx, int32_t instance, int64_t cap, int64_t* pairs,
                          double* delta_t, int64_t* n_out);
/* Particle-triangle candidates of the mesh walls (Sec. 3.7: contacts with
   boundary faces, lines and points) as (gid, wall_id, triangle index within
   the wall) triples, sorted, with the tangential overlap (Eq. delta_t) kept
   in each candidate's slot.  Same capacity rule and ownership. */
int dem_get_mesh_contacts(dem_ctx* ctx, int32_t instance, int64_t cap, int64_t* triples,
                          double* delta_t, int64_t* n_out);

/* Re-sort particles into cells and rebuild the contact lists at the current
   positions without moving them (the tangential overlaps are carried over);
   for testing the history carry-over and for restarts. */
int dem_resort(dem_ctx* ctx);

/* Counters of the current state (runs a small reduction on the device):
   active particles, candidate list entries and touching entries (Sec. 3.2),
   wall candidates, steps, searches, search geometry (r_s, cell edge, skin,
   d_max of Sec. 3.2) and device memory.  out is caller-owned. */
int dem_get_stats(dem_ctx* ctx, dem_stats* out);

/* Stream the library launches on (hipStream_t), for timing with events. */
void* dem_stream(dem_ctx* ctx);

/* Result of dem_autotune. */
typedef struct {
  int32_t force_block;       /* chosen threads per force workgroup            */
  int32_t rebuild_interval;  /* chosen search schedule: K >= 1, 0 = dynamic   */
  double cell_factor;        /* chosen cell edge / d_max                      */
  double ms_per_step;        /* whole step with the chosen settings           */
  int64_t steps;             /* simulation steps the trials advanced          */
  double block_ms[3];        /* force kernel ms with 64, 128, 256 threads     */
  double cell_factors[4];    /* cell edges / d_max tried                      */
  double search_ms[4];       /* ms per contact search with each of them       */
  int32_t schedules[8];      /* schedules tried (K, 0 = dynamic, -1 unused)   */
  double schedule_ms[8];     /* ms per step with each (-1: not tried, a
                                constant K too long for the measured drift)   */
} dem_tuning;

/* Pick, by measurement on the running simulation, the threads per workgroup
   of the force kernel (64, 128, 256: force-kernel time), the cell edge (from
   r_s / d_max up to 1.5 times that: time of a contact search) and the search
   schedule (dynamic and K = 5..80: whole steps per second), and keep them.
   Contact searches are the constant/dynamic approaches of Sec. 3.1; the cell
   edge and block size change no result beyond summation order.  Every trial
   is trial_steps (10..100000) ordinary steps of the simulation, so the call
   advances it (out->steps steps, plus forced re-sorts); constant K are tried
   only while K times the largest per-step drift measured in the dynamic
   trial stays below a quarter of half the skin.  The choice depends on
   timings, so runs that must be bitwise reproducible fix their settings
   instead.  Errors of the steps (DEM_EUNSTABLE ...) are returned as from
   dem_step. */
int dem_autotune(dem_ctx* ctx, int32_t trial_steps, dem_tuning* out);

/* Benchmark instrumentation.  While enabled, dem_step launches every kernel
   directly (no graphs) and records HIP events around each force launch and
   each contact search; dem_get_timing writes {force ms total, force launches,
   search ms total, searches} accumulated since dem_set_timing was called. */
int dem_set_timing(dem_ctx* ctx, int32_t enable);
int dem_get_timing(dem_ctx* ctx, double* out4);

#ifdef __cplusplus
}
#endif
#endif /* DEM_H */
