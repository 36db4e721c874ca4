// Host driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of
// the library's host code: every entry point on its argument-checking and
// error paths (null context, invalid configuration values, no device), the
// paths that run without a GPU.  Exit code 0 = clean.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "dem.h"

static int fails = 0;
#define EXPECT(cond)                                                     \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                           \
    }                                                                    \
  } while (0)

static dem_config base() {
  dem_config c;
  std::memset(&c, 0, sizeof(c));
  c.dt = 1e-5;
  c.gravity[2] = -9.81;
  for (int k = 0; k < 3; ++k) {
    c.domain_lo[k] = 0.0;
    c.domain_hi[k] = 0.05;
  }
  c.neighbor_threshold = 1.3;
  c.cell_factor = 1.3;
  c.rebuild_interval = 20;
  c.n_instances = 1;
  return c;
}

int main() {
  dem_ctx* ctx = nullptr;
  EXPECT(dem_create(nullptr, &ctx) == DEM_EINVAL);
  dem_config c = base();
  EXPECT(dem_create(&c, nullptr) == DEM_EINVAL);
  const struct {
    void (*mutate)(dem_config&);
  } bad[] = {
      {[](dem_config& x) { x.dt = 0.0; }},
      {[](dem_config& x) { x.dt = NAN; }},
      {[](dem_config& x) { x.domain_hi[1] = x.domain_lo[1]; }},
      {[](dem_config& x) { x.rebuild_interval = -1; }},
      {[](dem_config& x) { x.neighbor_threshold = 0.9; }},
      {[](dem_config& x) { x.cell_factor = 0.5; }},
      {[](dem_config& x) { x.integrator = 2; }},
      {[](dem_config& x) { x.rolling_model = 3; }},
      {[](dem_config& x) { x.contact_model = 2; }},
      {[](dem_config& x) { x.contact_model = 1; x.characteristic_velocity = 0.0; }},
      {[](dem_config& x) { x.precision = 2; }},
      {[](dem_config& x) { x.force_block = 96; }},
      {[](dem_config& x) { x.n_instances = 0; }},
      {[](dem_config& x) { x.max_neighbors = -3; }},
  };
  for (const auto& b : bad) {
    dem_config x = base();
    b.mutate(x);
    ctx = reinterpret_cast<dem_ctx*>(0x1);
    EXPECT(dem_create(&x, &ctx) == DEM_EINVAL);
    EXPECT(ctx == nullptr);
    EXPECT(std::strlen(dem_last_error(nullptr)) > 0);
  }
  // a valid configuration: a context on a GPU, DEM_ENODEV without one
  const int rc = dem_create(&c, &ctx);
  EXPECT(rc == DEM_OK || rc == DEM_ENODEV);
  if (rc == DEM_OK) dem_destroy(ctx);
  // every entry point refuses a null context
  double v3[3] = {0, 0, 1};
  int32_t wid = 0;
  int64_t n = 0;
  dem_material m = {2500.0, 1e6, 0.3, 0.9, 0.3, 0.1};
  EXPECT(dem_set_material(nullptr, 0, 0, &m) != DEM_OK);
  EXPECT(dem_add_planar_wall(nullptr, 0, v3, v3, nullptr, 0, nullptr, nullptr, -INFINITY,
                             INFINITY, &wid) != DEM_OK);
  EXPECT(dem_step(nullptr, 1) != DEM_OK);
  EXPECT(dem_get_state(nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr) != DEM_OK);
  EXPECT(dem_get_contacts(nullptr, 0, 0, nullptr, nullptr, nullptr, &n) != DEM_OK);
  EXPECT(dem_get_contacts_device(nullptr, 0, 0, nullptr, nullptr, nullptr, &n) != DEM_OK);
  EXPECT(dem_get_contacts_device_noalloc(nullptr, 0, 0, nullptr, nullptr, nullptr, &n) !=
         DEM_OK);
  EXPECT(dem_record_contact_forces(nullptr, 1) != DEM_OK);
  EXPECT(dem_commit(nullptr) != DEM_OK);
  dem_destroy(nullptr);
  if (fails) return 1;
  std::printf("host sanitizer run clean\n");
  return 0;
}
