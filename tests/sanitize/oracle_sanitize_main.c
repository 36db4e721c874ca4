/* Host driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of
   the oracle: runs a small scene through every kind of wall, both contact
   models, both integrators and the three rolling options, with searches,
   resets and error paths, so that out-of-bounds accesses, use after free and
   undefined arithmetic in the oracle abort the run.  Exit code 0 = clean. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle_dem.h"

#define CHECK(x)                                                       \
  do {                                                                 \
    int rc_ = (x);                                                     \
    if (rc_ != 0) {                                                    \
      fprintf(stderr, "%s:%d: %s returned %d\n", __FILE__, __LINE__, #x, rc_); \
      return 1;                                                        \
    }                                                                  \
  } while (0)

static int run(int integrator, int rolling, int model, int K) {
  ora_config cfg = {0};
  cfg.dt = 1e-5;
  cfg.gravity[2] = -9.81;
  for (int k = 0; k < 3; ++k) {
    cfg.domain_lo[k] = -0.01;
    cfg.domain_hi[k] = 0.04;
  }
  cfg.neighbor_threshold = 1.3;
  cfg.cell_factor = 1.3;
  cfg.rebuild_interval = K;
  cfg.integrator = integrator;
  cfg.rolling_model = rolling;
  cfg.contact_model = model;
  cfg.characteristic_velocity = 0.5;
  ora_sim* s = NULL;
  CHECK(ora_create(&cfg, &s));
  ora_material m0 = {2500.0, 1e6, 0.3, 0.9, 0.3, 0.1};
  ora_material m1 = {7850.0, 5e6, 0.25, 0.6, 0.5, 0.05};
  CHECK(ora_set_material(s, 0, &m0));
  CHECK(ora_set_material(s, 1, &m1));
  /* walls: floor (rotating), bounded plane, cylinder, cone, a two-triangle mesh */
  int32_t w;
  const double p0[3] = {0, 0, 0}, nz[3] = {0, 0, 1}, om[3] = {0, 0, 2.0};
  CHECK(ora_add_plane(s, p0, nz, NULL, 0, p0, om, -INFINITY, INFINITY, &w));
  const double pb[3] = {0.015, 0.015, 0.004}, nb[3] = {0, 0.3, 1};
  const double ext[5] = {1, 0, 0, 0.004, 0.004};
  CHECK(ora_add_plane(s, pb, nb, ext, 1, NULL, NULL, -INFINITY, 0.001, &w));
  const double ax[3] = {0.015, 0.015, 0}, az[3] = {0, 0, 1};
  CHECK(ora_add_cylinder(s, ax, az, 0.014, 0.0, 0.03, 1, 0, 1.5, -INFINITY, INFINITY, &w));
  CHECK(ora_add_cone(s, ax, az, 0.004, 0.8, 0.0, 0.01, 1, 1, 0.0, -INFINITY, INFINITY, &w));
  const double vel[3] = {0.01, 0, 0};
  CHECK(ora_set_wall_velocity(s, w, vel));
  const double verts[12] = {0.005, 0.005, 0.002, 0.025, 0.005, 0.002,
                            0.025, 0.025, 0.003, 0.005, 0.025, 0.002};
  const int32_t tris[6] = {0, 1, 2, 0, 2, 3};
  CHECK(ora_add_mesh(s, 4, verts, 2, tris, 0, NULL, NULL, -INFINITY, INFINITY, &w));
  /* a dense jittered lattice, two sizes and materials, moving and spinning */
  const int side = 7, n = side * side * side;
  double* x = malloc(sizeof(double) * 3 * n);
  double* v = malloc(sizeof(double) * 3 * n);
  double* o = malloc(sizeof(double) * 3 * n);
  double* r = malloc(sizeof(double) * n);
  int32_t* t = malloc(sizeof(int32_t) * n);
  unsigned long long st = 12345;
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      const double u = (double)(st >> 11) / 9007199254740992.0;
      const int c = k == 0 ? i % side : (k == 1 ? (i / side) % side : i / (side * side));
      x[3 * i + k] = 0.0055 + 0.00298 * c + 1e-5 * (u - 0.5);
      v[3 * i + k] = 0.05 * (u - 0.5);
      o[3 * i + k] = 20.0 * (u - 0.5);
    }
    r[i] = i % 3 ? 1.5e-3 : 1.2e-3;
    t[i] = i % 2;
  }
  CHECK(ora_set_particles(s, n, x, v, o, r, t));
  for (int k = 0; k < 6; ++k) CHECK(ora_step(s, 25));
  int64_t np = 0, nw = 0, cnt = 0;
  CHECK(ora_num_contacts(s, &np, &nw));
  int64_t* pairs = malloc(sizeof(int64_t) * 2 * (np + 1));
  int64_t* trip = malloc(sizeof(int64_t) * 3 * (np + 1) * 4);
  double* dt = malloc(sizeof(double) * 3 * (np + 1) * 4);
  uint8_t* touch = malloc(np + 1);
  CHECK(ora_get_contacts(s, np, pairs, dt, touch, &cnt));
  CHECK(ora_get_contact_forces(s, np, pairs, dt, &cnt));
  CHECK(ora_get_wall_contacts(s, nw, pairs, dt, &cnt));
  if (ora_get_mesh_contacts(s, 0, NULL, NULL, &cnt) != ORA_EINVAL && cnt > 0) return 1;
  CHECK(ora_get_mesh_contacts(s, 4 * (np + 1), trip, dt, &cnt));
  double* f3 = malloc(sizeof(double) * 3 * n);
  double* t3 = malloc(sizeof(double) * 3 * n);
  double* sc = malloc(sizeof(double) * n);
  uint8_t* act = malloc(n);
  double time = 0.0;
  CHECK(ora_get_forces(s, f3, t3));
  CHECK(ora_get_force_scale(s, sc));
  CHECK(ora_get_term_scale(s, sc));
  CHECK(ora_get_state(s, x, v, o, act, &time));
  CHECK(ora_bruteforce_candidates(s, np, pairs, &cnt));
  free(f3);
  free(t3);
  free(sc);
  free(act);
  /* resetting the particles frees and rebuilds every list */
  CHECK(ora_set_particles(s, n, x, v, o, r, t));
  CHECK(ora_step(s, 3));
  /* error paths */
  if (ora_get_contacts(s, 0, pairs, dt, touch, &cnt) != ORA_EINVAL && cnt > 0) return 1;
  if (ora_set_material(s, 99, &m0) != ORA_EINVAL) return 1;
  free(x);
  free(v);
  free(o);
  free(r);
  free(t);
  free(pairs);
  free(trip);
  free(dt);
  free(touch);
  ora_destroy(s);
  return 0;
}

int main(void) {
  for (int integrator = 0; integrator < 2; ++integrator)
    for (int rolling = 0; rolling < 3; ++rolling)
      for (int model = 0; model < 2; ++model) {
        const int rc = run(integrator, rolling, model, model ? 3 : 1);
        if (rc) fprintf(stderr, "integrator %d rolling %d model %d\n", integrator, rolling, model);
        if (rc) return rc;
      }
  printf("oracle sanitizer run clean\n");
  return 0;
}
