/*
 * Plain FP64 CPU oracle of the soft-sphere DEM time step (Lethe-DEM,
 * arXiv 2106.09576, Sections 2 and 3.2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the GPU library; the two are independent
 * implementations of the same method and are compared by the tests.
 *
 * Every function returns 0 on success and a negative code on error:
 *   ORA_EINVAL -1   invalid argument
 *   ORA_ENOMEM -3   allocation failed
 *   ORA_EUNSTABLE -5 non-finite state or a particle moved more than half the
 *                    search skin between two contact searches
 *   ORA_ESTATE -6   wrong call order (particles not set yet)
 * All arrays are host arrays in particle-input order (gid = input index).
 */
#ifndef ORACLE_DEM_H
#define ORACLE_DEM_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ENOMEM (-3)
#define ORA_EUNSTABLE (-5)
#define ORA_ESTATE (-6)

#define ORA_MAX_TYPES 16
#define ORA_MAX_WALLS 32

typedef struct {
  double dt;
  double gravity[3];
  double domain_lo[3];
  double domain_hi[3];
  double neighbor_threshold; /* r_s / d_max (paper default 1.3)            */
  double cell_factor;        /* h / d_max, >= neighbor_threshold if given  */
  int32_t rebuild_interval;  /* contact search every K steps ("constant")  */
  int32_t integrator;        /* 0 velocity Verlet, 1 explicit Euler        */
  int32_t rolling_model;     /* 0 none, 1 constant torque, 2 viscous torque */
  int32_t contact_model;     /* 0 nonlinear (Hertz-Mindlin), 1 linear      */
  double characteristic_velocity; /* V of the linear model [m/s]           */
} ora_config;

typedef struct {
  double density, youngs, poisson, restitution, friction, rolling_friction;
} ora_material;

typedef struct ora_sim ora_sim;

int ora_create(const ora_config* cfg, ora_sim** out);
void ora_destroy(ora_sim* s);
int ora_set_material(ora_sim* s, int32_t type, const ora_material* m);
int ora_set_particles(ora_sim* s, int64_t n, const double* pos, const double* vel,
                      const double* omega, const double* radius, const int32_t* type);
/* extent: NULL = infinite plane, else {u_x,u_y,u_z, half_u, half_v}; the
   in-plane axes are u and normal x u. */
int ora_add_plane(ora_sim* s, const double point[3], const double normal[3],
                  const double* extent, int32_t material, const double axis_point[3],
                  const double omega[3], double t_on, double t_off, int32_t* wall_id);
int ora_add_cylinder(ora_sim* s, const double axis_point[3], const double axis_dir[3],
                     double radius, double s_min, double s_max, int32_t inside,
                     int32_t material, double omega, double t_on, double t_off,
                     int32_t* wall_id);
/* Cone around the axis: surface radius radius0 + slope s at axial coordinate
   s in [s_min, s_max] (s measured from axis_point along axis_dir). */
int ora_add_cone(ora_sim* s, const double axis_point[3], const double axis_dir[3],
                 double radius0, double slope, double s_min, double s_max, int32_t inside,
                 int32_t material, double omega, double t_on, double t_off, int32_t* wall_id);
/* Mesh wall: n_triangles triangles over n_vertices corners (x, y, z each);
   triangles holds three corner indices per triangle, ordered so that
   (p1 - p0) x (p2 - p0) points to the particles' side.  Surface velocity
   omega x (x_c - axis_point) (NULL = none; axis_point NULL = first vertex).
   Particle-face, particle-edge and particle-vertex contacts. */
int ora_add_mesh(ora_sim* s, int64_t n_vertices, const double* vertices, int64_t n_triangles,
                 const int32_t* triangles, int32_t material, const double axis_point[3],
                 const double omega[3], double t_on, double t_off, int32_t* wall_id);
/* Constant translational velocity of a wall (before the particles are set):
   its point and rotation axis move with it. */
int ora_set_wall_velocity(ora_sim* s, int32_t wall_id, const double vel[3]);
int ora_step(ora_sim* s, int64_t n_steps);
int ora_get_state(ora_sim* s, double* pos, double* vel, double* omega, uint8_t* active,
                  double* time_out);
int ora_get_forces(ora_sim* s, double* force, double* torque);
/* sum over the particle's contacts of |F^n + F^t| of the last evaluation */
int ora_get_force_scale(ora_sim* s, double* scale);
/* sum over the particle's contacts of the magnitudes of the spring and
   dashpot terms of the normal and tangential forces (before the Coulomb
   limit): a scale that does not shrink where spring and dashpot cancel */
int ora_get_term_scale(ora_sim* s, double* scale);
int ora_num_contacts(ora_sim* s, int64_t* n_pairs, int64_t* n_wall);
int ora_get_contacts(ora_sim* s, int64_t cap, int64_t* pairs, double* delta_t,
                     uint8_t* touching, int64_t* n_out);
/* per candidate pair (the order of ora_get_contacts): F^n + F^t on the pair's
   first particle at the last force evaluation, zero for a pair that did not
   touch then (a record for per-contact error measures; changes nothing) */
int ora_get_contact_forces(ora_sim* s, int64_t cap, int64_t* pairs, double* force,
                           int64_t* n_out);
int ora_get_wall_contacts(ora_sim* s, int64_t cap, int64_t* pairs, double* delta_t,
                          int64_t* n_out);
/* particle-triangle candidates of mesh walls: (gid, wall id, triangle index
   within the wall) triples and their tangential overlaps, sorted */
int ora_get_mesh_contacts(ora_sim* s, int64_t cap, int64_t* triples, double* delta_t,
                          int64_t* n_out);
int ora_search_params(ora_sim* s, double* out4 /* d_max, r_s, h, skin */);
/* Closest point of the triangle corners[0..2] to x (unit pin): out[0] = 0
   face, 1 + a edge (a, a + 1), 4 + a corner a; out[1] signed distance from
   the plane; out[2] squared distance; out[3..5] the point. */
int ora_triangle_closest(const double corners[9], const double x[3], double out[6]);

/* O(n^2) reference of the candidate set: all active pairs gid_i < gid_j with
   |x_j - x_i|^2 < r_s^2, sorted.  For the brute-force pin only. */
int ora_bruteforce_candidates(ora_sim* s, int64_t cap, int64_t* pairs, int64_t* n_out);

/* One particle-particle contact evaluated in isolation (unit pin).  Material
   indices refer to ora_set_material.  delta_t is read and updated.  Outputs the
   force on i, the torques on i and j and whether the pair touches. */
int ora_pair_force(ora_sim* s, const double xi[3], const double xj[3],
                   const double vi[3], const double vj[3], const double wi[3],
                   const double wj[3], double Ri, double Rj, int32_t ti, int32_t tj,
                   double delta_t[3], double F_i[3], double M_i[3], double M_j[3],
                   int32_t* touching);

#ifdef __cplusplus
}
#endif
#endif
