// Host runtime of the MI355X DEM library: the C ABI declared in include/dem.h.
//
// A context owns all device buffers of a batch of independent simulations
// ("instances", one or more), one HIP stream (default priority) and up to four
// instantiated HIP graphs, one per parity of the ping-pong buffers, each
// holding one K-step chunk: the contact search (Sec. 3.2, every K steps as in
// the "constant" detection of Sec. 3.1) followed by K force+integration
// launches and a clock tick.  The particles of all instances live in one
// array (each tagged with its instance), so every kernel launch covers the
// whole batch and uneven instance sizes need no load balancing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "dem.h"
#include "dem_device.hpp"

using namespace demgpu;

namespace {

thread_local std::string g_err;

constexpr double kPi = 3.14159265358979323846;
// dynamic search: steps per chunk between two host decisions
constexpr int kDynChunk = 16;

int set_err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

// Host-side description of one instance: materials, walls, the particles
// given to dem_set_particles (kept until the batch is built on the device)
// and the search geometry derived from them.
// One triangle of a mesh wall as given: corners and the mesh's corner
// indices; `wall` is the wall's index within its instance.
struct HostTri {
  double p[3][3];
  int v[3];
  int wall;
};

struct Instance {
  dem_material mat[kMaxTypes]{};
  bool mat_set[kMaxTypes]{};
  std::vector<WallDev> walls;
  std::vector<HostTri> tris;  // triangles of the mesh walls, in wall order
  bool staged = false;
  bool own_domain = false;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int64_t n = 0;
  std::vector<double> pos, vel, omg, rad;
  std::vector<int32_t> type;
  // derived when the batch is built
  double dmax = 0, rs = 0, h = 0, skin = 0;
  int64_t p_begin = 0;
  int w_begin = 0;
  GridDev grid{};
  uint32_t key_base = 0;
};

struct dem_ctx {
  dem_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev_user = nullptr;
  std::vector<Instance> inst;

  // particle state of the whole batch
  int n = 0;
  bool ready = false;
  bool failed = false;
  int fail_code = 0;
  int max_nb = 0;
  int64_t cap = 0;
  StepParams sp{};
  int64_t n_keys = 0;

  std::vector<void*> allocs;
  std::vector<size_t> alloc_bytes;
  size_t dev_bytes = 0;
  int force_block = kBlock;  // threads per force workgroup (64, 128, 256)
  double cell_factor = 0.0;  // cell edge / d_max of the grids in use
  uint32_t* d_ckey = nullptr;  // cell keys of every grid (GridDev::ckey)
  uint32_t* d_key_cell = nullptr;  // inverse: the cell (key_base + position) of each key
  int2* d_cse = nullptr;  // (start, end) of each cell at its position, written by the scan
  double4 *pos[2]{}, *vel[2]{}, *omg[2]{};
  int *gid[2]{}, *info[2]{};
  double4 *F[2]{}, *T[2]{};
  double4* xref = nullptr;
  int* wid[2]{};
  double* whist[2]{};
  // mesh walls (all null without any): triangle table, grids, candidates
  bool has_mesh = false;
  TriDev* d_tri = nullptr;
  int* d_mcell = nullptr;
  int* d_mcell_tri = nullptr;
  int* mtri[2]{};
  double* mhist[2]{};
  double4 *Fm = nullptr, *Tm = nullptr;
  // per-contact force record (tests): three planes of cap doubles, or null
  bool record_pf = false;
  int pair_mode = 0;  // 1: one instance, every particle of type 0; 2: every particle of type 0
  double* pair_force = nullptr;
  std::vector<int> tri_wall, tri_local;  // per global triangle: instance wall, index in it
  int* nbr[2]{};
  double* hist[2]{};
  int* rowlen[2]{};
  int* rowcut[2]{};  // per particle: the row cuts of each list
  // displacement bound of the row cuts (StepParams::bacc, brec)
  double* d_bacc = nullptr;
  unsigned long long* d_brec = nullptr;
  uint32_t* keys = nullptr;
  int *rank = nullptr, *count = nullptr, *start = nullptr, *tile_sums = nullptr;
  int *perm0 = nullptr, *perm = nullptr, *inv = nullptr;
  PairCoef *d_pp = nullptr, *d_pw = nullptr;
  WallDev* d_walls = nullptr;
  InstDev* d_inst = nullptr;
  int* d_flags = nullptr;
  int64_t* d_clock = nullptr;
  unsigned long long* d_stats = nullptr;

  int cur = 0;   // parity of pos/vel/omg (flips at every force launch and reorder)
  int pcur = 0;  // parity of gid/info/F/T/wall slots/neighbour list (flips at reorder)
  int64_t step = 0;
  int64_t host_base = 0;  // value of the device clock
  int64_t n_rebuilds = 0;
  hipGraphExec_t graph[2][2]{};

  // dynamic search trigger (rebuild_interval == 0): every force launch raises
  // drift[slot] to its largest drift in half skins; the host keeps a bound on
  // the largest displacement since the last search and the last step rate
  bool dynamic = false;
  unsigned long long* d_drift = nullptr;  // kDynChunk + 1 records of kDriftSpread words
  unsigned long long* h_drift = nullptr;  // pinned host copy
  double dyn_acc = 0.0;
  double dyn_rate = 0.0;
  double dyn_grav = 0.0;  // |g| dt^2 (2/skin)max: growth of the rate per step
  double dyn_wrate = 0.0;  // largest step of a translating wall, in half skins
  double dyn_wacc = 0.0;   // distance walls moved since the last search, in half skins
  hipGraphExec_t dyn_graph[2][2][2]{};  // [cur][pcur][chunk starts with a search]

  // optional per-kernel timing (benchmarks): events around force launches
  bool timing = false;
  std::vector<hipEvent_t> tev;
  std::vector<int> tkind;  // 0 force, 1 search chunk
  double t_force_ms = 0, t_search_ms = 0;
  int64_t n_force = 0, n_search = 0;
};

namespace {

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_err(DEM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

int dalloc(dem_ctx* c, void** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return set_err(DEM_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  c->allocs.push_back(*p);
  c->alloc_bytes.push_back(bytes);
  c->dev_bytes += bytes;
  return DEM_OK;
}

// Free one allocation made by dalloc (after the stream has drained).
void dfree(dem_ctx* c, void* p) {
  if (!p) return;
  for (size_t k = 0; k < c->allocs.size(); ++k)
    if (c->allocs[k] == p) {
      (void)hipFree(p);
      c->dev_bytes -= c->alloc_bytes[k];
      c->allocs.erase(c->allocs.begin() + (long)k);
      c->alloc_bytes.erase(c->alloc_bytes.begin() + (long)k);
      return;
    }
}

template <typename T>
int dalloc_t(dem_ctx* c, T** p, size_t count) {
  return dalloc(c, (void**)p, count * sizeof(T));
}

void destroy_graphs(dem_ctx* c) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      if (c->graph[a][b]) {
        (void)hipGraphExecDestroy(c->graph[a][b]);
        c->graph[a][b] = nullptr;
      }
      for (int r = 0; r < 2; ++r)
        if (c->dyn_graph[a][b][r]) {
          (void)hipGraphExecDestroy(c->dyn_graph[a][b][r]);
          c->dyn_graph[a][b][r] = nullptr;
        }
    }
}

void free_particles(dem_ctx* c) {
  destroy_graphs(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->h_drift) {
    (void)hipHostFree(c->h_drift);
    c->h_drift = nullptr;
  }
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  c->alloc_bytes.clear();
  c->dev_bytes = 0;
  c->d_ckey = nullptr;
  c->d_key_cell = nullptr;
  c->d_cse = nullptr;
  c->has_mesh = false;
  c->d_tri = nullptr;
  c->d_mcell = c->d_mcell_tri = nullptr;
  c->mtri[0] = c->mtri[1] = nullptr;
  c->mhist[0] = c->mhist[1] = nullptr;
  c->Fm = c->Tm = nullptr;
  c->pair_force = nullptr;
  c->ready = false;
  c->n = 0;
}

int check_instance(const dem_ctx* c, int32_t instance) {
  if (instance < 0 || instance >= (int32_t)c->inst.size())
    return set_err(DEM_EINVAL, "instance %d out of [0, %d)", instance, (int)c->inst.size());
  return DEM_OK;
}

int wait_user(dem_ctx* c) {
  if (c->cfg.hip_stream) {
    HIPCHK(hipEventRecord(c->ev_user, (hipStream_t)c->cfg.hip_stream));
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev_user, 0));
  }
  return DEM_OK;
}

int finish(dem_ctx* c) {
  HIPCHK(hipStreamSynchronize(c->stream));
  return DEM_OK;
}

bool unit3(const double* a, double* out) {
  double nn = sqrt((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]);
  if (!(nn > 0.0) || !std::isfinite(nn)) return false;
  for (int k = 0; k < 3; ++k) out[k] = a[k] / nn;
  return true;
}

// Effective parameters (Sec. 2.1 table) per material pair.
double eff_youngs(const dem_material& a, const dem_material& b) {
  return 1.0 / ((1.0 - a.poisson * a.poisson) / a.youngs +
                (1.0 - b.poisson * b.poisson) / b.youngs);
}
double eff_shear(const dem_material& a, const dem_material& b) {
  return 1.0 / (2.0 * (2.0 - a.poisson) * (1.0 + a.poisson) / a.youngs +
                2.0 * (2.0 - b.poisson) * (1.0 + b.poisson) / b.youngs);
}
double damping_factor(double e) {
  double le = log(e);
  double beta = le / sqrt(le * le + kPi * kPi);
  return -2.0 * sqrt(5.0 / 6.0) * beta;
}

PairCoef make_coef(const dem_config& cfg, double Ye, double Ge, double e, double mu,
                   double mur) {
  PairCoef q;
  memset(&q, 0, sizeof(q));
  if (cfg.contact_model == 0) {
    const double ceta = damping_factor(e);
    q.kn = 4.0 / 3.0 * Ye;
    q.kt = 8.0 * Ge;
    q.en = ceta * sqrt(2.0 * Ye);
    q.et = ceta * sqrt(8.0 * Ge);
  } else {
    // linear model: k = kn (R_e^2 m_e)^(1/5), eta = en sqrt(m_e k)
    const double V = cfg.characteristic_velocity;
    q.kn = 16.0 / 15.0 * Ye * pow(15.0 * V * V / (16.0 * Ye), 0.2);
    q.kt = q.kn;
    const double le = log(e);
    q.en = le == 0.0 ? 0.0 : 2.0 / sqrt(1.0 + (kPi / le) * (kPi / le));
    q.et = q.en;
  }
  q.mu = mu;
  q.mur = mur;
  return q;
}

// ------------------------------------------------------------ kernel groups

ParticleBufs pbufs(dem_ctx* c, int k) { return ParticleBufs{c->pos[k], c->vel[k], c->omg[k]}; }
NbrList nlist(dem_ctx* c, int k) {
  return NbrList{c->nbr[k], c->hist[k], c->rowlen[k], c->cap, c->rowcut[k]};
}

// Step offset (from the device clock) of the next force evaluation after
// the current state: velocity Verlet first kicks and drifts to step + 1,
// explicit Euler evaluates the current positions.  A search between dem_step
// calls restarts the row cuts' displacement bound there.
int64_t next_eval_rel(const dem_ctx* c) {
  return (c->cfg.integrator == 0 ? c->step + 1 : c->step) - c->host_base;
}
WallSlots wslots(dem_ctx* c, int k) { return WallSlots{c->wid[k], c->whist[k]}; }
MeshSlots mslots(dem_ctx* c, int k) { return MeshSlots{c->mtri[k], c->mhist[k]}; }
MeshTables mtables(dem_ctx* c) { return MeshTables{c->d_tri, c->d_mcell, c->d_mcell_tri}; }

// Contact search: counting sort into cells, reorder, particle-wall search and
// particle-pair search with history carry-over.  Flips both parities.  The
// search takes place at time (clock + step_rel) dt, where moving walls are,
// and restarts the displacement bound of the row cuts for the force
// evaluation at step clock + bound_step_rel (the next one at these
// positions; < 0: the same as step_rel, as for a search inside a step).
int enqueue_rebuild(dem_ctx* c, int check_guard, int move_forces, int64_t step_rel,
                    int64_t bound_step_rel = -1) {
  if (bound_step_rel < 0) bound_step_rel = step_rel;
  hipStream_t s = c->stream;
  const int a = c->cur, p = c->pcur;
  HIPCHK(launch_fill_i32(c->count, 0, c->n_keys + 1, s));
  HIPCHK(launch_keys(c->d_inst, c->sp, c->pos[a], c->vel[a], c->info[p], c->xref, check_guard,
                     c->keys, c->rank, c->count, c->d_flags, s));
  HIPCHK(launch_scan(c->count, c->start, c->n_keys + 1, c->tile_sums, s, c->d_key_cell, c->d_cse,
                     c->n_keys));
  HIPCHK(launch_scatter(c->n, c->keys, c->rank, c->start, c->perm0, s));
  HIPCHK(launch_cell_rank(c->n, c->n_keys, c->perm0, c->keys, c->start, c->gid[p],
                          c->perm, s));
  HIPCHK(launch_reorder(c->sp, c->d_inst, c->perm, c->inv, pbufs(c, a), pbufs(c, a ^ 1),
                        c->gid[p],
                        c->gid[p ^ 1],
                        c->info[p], c->info[p ^ 1], c->xref, wslots(c, p), wslots(c, p ^ 1),
                        c->d_walls, mtables(c), mslots(c, p), mslots(c, p ^ 1),
                        move_forces ? c->F[p] : nullptr,
                        move_forces ? c->T[p] : nullptr, c->F[p ^ 1], c->T[p ^ 1],
                        c->d_clock, step_rel, bound_step_rel, c->d_flags, s));
  HIPCHK(launch_search(c->d_inst, (int)c->inst.size(), c->sp, c->pos[a ^ 1], c->info[p ^ 1],
                       c->d_cse, c->perm, c->inv, nlist(c, p), nlist(c, p ^ 1), c->d_flags, s));
  c->cur ^= 1;
  c->pcur ^= 1;
  c->n_rebuilds += 1;
  return DEM_OK;
}

int enqueue_force(dem_ctx* c, int mode, int64_t step_rel, unsigned long long* drift = nullptr) {
  const int a = c->cur, p = c->pcur;
  if (c->has_mesh)
    HIPCHK(launch_mesh(c->cfg.precision, c->sp, c->d_pw, c->d_walls, mtables(c), pbufs(c, a),
                       c->info[p], mslots(c, p), c->Fm, c->Tm, c->d_clock, step_rel,
                       c->d_flags, c->stream));
  HIPCHK(launch_force(mode, c->cfg.precision, c->sp, c->d_inst, c->d_pp, c->d_pw, c->d_walls,
                      pbufs(c, a),
                      pbufs(c, a ^ 1), c->info[p], nlist(c, p), wslots(c, p), c->F[p], c->T[p],
                      c->d_clock, step_rel, c->d_flags, drift, c->has_mesh ? c->mtri[p] : nullptr,
                      c->Fm, c->Tm, c->pair_force, c->force_block, c->pair_mode, c->stream));
  c->cur ^= 1;
  return DEM_OK;
}

int timed_begin(dem_ctx* c, int kind) {
  if (!c->timing) return DEM_OK;
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  HIPCHK(hipEventRecord(e, c->stream));
  c->tev.push_back(e);
  c->tkind.push_back(kind);
  return DEM_OK;
}

int timed_end(dem_ctx* c) {
  if (!c->timing) return DEM_OK;
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  HIPCHK(hipEventRecord(e, c->stream));
  c->tev.push_back(e);
  c->tkind.push_back(-1);
  return DEM_OK;
}

int collect_timing(dem_ctx* c) {
  if (!c->timing) return DEM_OK;
  for (size_t k = 0; k + 1 < c->tev.size(); k += 2) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->tev[k], c->tev[k + 1]));
    if (c->tkind[k] == 0) {
      c->t_force_ms += ms;
      c->n_force += 1;
    } else {
      c->t_search_ms += ms;
      c->n_search += 1;
    }
  }
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  c->tev.clear();
  c->tkind.clear();
  return DEM_OK;
}

// Explicit Euler searches after the force evaluation of the same step, so the
// stored forces move with the particles to stay readable by dem_get_forces.
int move_forces_at_search(const dem_ctx* c) { return c->cfg.integrator == 1 ? 1 : 0; }

int eager_rebuild(dem_ctx* c, int64_t step_rel) {
  int rc = timed_begin(c, 1);
  if (rc) return rc;
  rc = enqueue_rebuild(c, 1, move_forces_at_search(c), step_rel);
  if (rc) return rc;
  return timed_end(c);
}

int eager_force(dem_ctx* c, int mode, int64_t step_rel, unsigned long long* drift = nullptr) {
  int rc = timed_begin(c, 0);
  if (rc) return rc;
  rc = enqueue_force(c, mode, step_rel, drift);
  if (rc) return rc;
  return timed_end(c);
}

int set_clock(dem_ctx* c, int64_t value) {
  if (c->host_base != value) {
    HIPCHK(launch_tick(c->d_clock, value - c->host_base, c->stream));
    c->host_base = value;
  }
  return DEM_OK;
}

// One K-step chunk captured in a graph, for the current parities.
int get_chunk_graph(dem_ctx* c, hipGraphExec_t* out) {
  hipGraphExec_t& g = c->graph[c->cur][c->pcur];
  if (g) {
    *out = g;
    return DEM_OK;
  }
  const int K = c->cfg.rebuild_interval;
  const int save_cur = c->cur, save_pcur = c->pcur;
  const int64_t save_rb = c->n_rebuilds;
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = DEM_OK;
  if (c->cfg.integrator == 0) {
    rc = enqueue_rebuild(c, 1, 0, 0);
    for (int j = 0; j < K && rc == DEM_OK; ++j) rc = enqueue_force(c, 0, j);
  } else {
    // Euler: the search follows the K updates, at the time of the last
    for (int j = 0; j < K && rc == DEM_OK; ++j) rc = enqueue_force(c, 2, j);
    if (rc == DEM_OK) rc = enqueue_rebuild(c, 1, move_forces_at_search(c), K);
  }
  if (rc == DEM_OK) {
    hipError_t e = launch_tick(c->d_clock, K, c->stream);
    if (e != hipSuccess) rc = set_err(DEM_EHIP, "tick launch: %s", hipGetErrorString(e));
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  c->cur = save_cur;
  c->pcur = save_pcur;
  c->n_rebuilds = save_rb;
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return set_err(DEM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g = nullptr;
    return set_err(DEM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *out = g;
  return DEM_OK;
}

// Capture and instantiate the chunk graphs of all four buffer parities before
// the first chunk runs, so that no capture or instantiation happens in the
// middle of a run (the parity a chunk starts with depends on how many
// searches came before it).
int prepare_chunk_graphs(dem_ctx* c) {
  const int save_cur = c->cur, save_pcur = c->pcur;
  int rc = DEM_OK;
  for (int a = 0; a < 2 && rc == DEM_OK; ++a)
    for (int p = 0; p < 2 && rc == DEM_OK; ++p) {
      c->cur = a;
      c->pcur = p;
      hipGraphExec_t g = nullptr;
      rc = get_chunk_graph(c, &g);
    }
  c->cur = save_cur;
  c->pcur = save_pcur;
  return rc;
}

int launch_chunk(dem_ctx* c, int64_t clock_at_start) {
  int rc = set_clock(c, clock_at_start);
  if (rc) return rc;
  hipGraphExec_t g = nullptr;
  rc = get_chunk_graph(c, &g);
  if (rc) return rc;
  HIPCHK(hipGraphLaunch(g, c->stream));
  const int K = c->cfg.rebuild_interval;
  c->cur ^= (K + 1) & 1;
  c->pcur ^= 1;
  c->n_rebuilds += 1;
  c->host_base += K;
  return DEM_OK;
}

// ------------------------------------------------- dynamic search trigger
//
// "dynamic" contact detection (Sec. 3.1): search when particles may have
// moved far enough to miss a contact.  Steps run in chunks of at most
// kDynChunk.  Before a chunk the host knows acc, a bound on the largest
// displacement since the last search (sum over steps of the largest drift),
// and rate, the largest drift of one step in the last chunk, both in units of
// half the skin.  The chunk starts with a search when acc + 2 L rate' could
// reach 1 (rate' = rate plus what gravity adds over the chunk); after it the
// per-step maxima are read back.  The displacement guard of every search
// still checks the true displacement.

int enqueue_dyn_chunk(dem_ctx* c, int L, bool search, bool last_is_call_end) {
  const int vv = c->cfg.integrator == 0;
  HIPCHK(launch_fill_i32((int*)(c->d_drift + kDriftSpread), 0, 2 * kDriftSpread * (int64_t)L,
                         c->stream));
  if (search) {
    int rc = enqueue_rebuild(c, 1, move_forces_at_search(c), 0);
    if (rc) return rc;
  }
  for (int j = 0; j < L; ++j) {
    const int mode = vv ? ((last_is_call_end && j == L - 1) ? 1 : 0) : 2;
    int rc = enqueue_force(c, mode, j, c->d_drift + (size_t)kDriftSpread * (1 + j));
    if (rc) return rc;
  }
  return DEM_OK;
}

int get_dyn_graph(dem_ctx* c, bool search, hipGraphExec_t* out) {
  hipGraphExec_t& g = c->dyn_graph[c->cur][c->pcur][search ? 1 : 0];
  if (g) {
    *out = g;
    return DEM_OK;
  }
  const int save_cur = c->cur, save_pcur = c->pcur;
  const int64_t save_rb = c->n_rebuilds;
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_dyn_chunk(c, kDynChunk, search, false);
  if (rc == DEM_OK) {
    hipError_t e = launch_tick(c->d_clock, kDynChunk, c->stream);
    if (e != hipSuccess) rc = set_err(DEM_EHIP, "tick launch: %s", hipGetErrorString(e));
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  c->cur = save_cur;
  c->pcur = save_pcur;
  c->n_rebuilds = save_rb;
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return set_err(DEM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g = nullptr;
    return set_err(DEM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *out = g;
  return DEM_OK;
}

// The dynamic chunk graphs of all buffer parities, with and without a
// search at their start, instantiated up front (see prepare_chunk_graphs).
int prepare_dyn_graphs(dem_ctx* c) {
  const int save_cur = c->cur, save_pcur = c->pcur;
  int rc = DEM_OK;
  for (int a = 0; a < 2 && rc == DEM_OK; ++a)
    for (int p = 0; p < 2 && rc == DEM_OK; ++p)
      for (int r = 0; r < 2 && rc == DEM_OK; ++r) {
        c->cur = a;
        c->pcur = p;
        hipGraphExec_t g = nullptr;
        rc = get_dyn_graph(c, r != 0, &g);
      }
  c->cur = save_cur;
  c->pcur = save_pcur;
  return rc;
}

// read back drift records [first, first + count) and fold them into the bound
int fold_drift(dem_ctx* c, int first, int count) {
  const size_t w0 = (size_t)kDriftSpread * first, nw = (size_t)kDriftSpread * count;
  HIPCHK(hipMemcpyAsync(c->h_drift + w0, c->d_drift + w0, sizeof(unsigned long long) * nw,
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double rate = 0.0;
  for (int k = first; k < first + count; ++k) {
    double v2 = 0.0;  // the device keeps the largest square, spread over words
    for (int w = 0; w < kDriftSpread; ++w) {
      double x;
      memcpy(&x, &c->h_drift[(size_t)kDriftSpread * k + w], sizeof(double));
      v2 = std::max(v2, x);
    }
    const double v = std::sqrt(v2);
    c->dyn_acc += v;
    rate = std::max(rate, v);
  }
  if (count > 0) c->dyn_rate = rate;
  return DEM_OK;
}

int step_dynamic(dem_ctx* c, int64_t n_steps) {
  const bool vv = c->cfg.integrator == 0;
  const int64_t s0 = c->step, s_end = s0 + n_steps;
  const bool graphs = !c->timing;
  int rc = DEM_OK;
  if (graphs && n_steps > kDynChunk && (rc = prepare_dyn_graphs(c))) return rc;
  if (vv) {
    HIPCHK(launch_fill_i32((int*)c->d_drift, 0, 2 * kDriftSpread, c->stream));
    HIPCHK(launch_kick_drift(c->sp, c->d_inst, pbufs(c, c->cur), c->info[c->pcur],
                             c->F[c->pcur], c->T[c->pcur], c->d_drift, c->d_clock,
                             s0 + 1 - c->host_base, c->stream));
    if ((rc = fold_drift(c, 0, 1))) return rc;
  }
  int64_t s = s0 + 1;
  while (s <= s_end) {
    int L = (int)std::min<int64_t>(kDynChunk, s_end - s + 1);
    // keep one chunk's worth of predicted drift below half a skin
    const double rate = c->dyn_rate + c->dyn_grav * L;
    while (L > 1 && 2.0 * L * rate >= 0.5) --L;
    // translating walls cover at most half a skin between two searches
    while (L > 1 && L * c->dyn_wrate > 1.0) --L;
    const double pred = 2.0 * L * (c->dyn_rate + c->dyn_grav * L);
    const bool search = c->dyn_acc + pred >= 1.0 || c->dyn_wacc + L * c->dyn_wrate > 1.0;
    if (search) {
      c->dyn_acc = 0.0;
      c->dyn_wacc = 0.0;
    }
    const bool call_end = s + L - 1 == s_end;
    if (graphs && L == kDynChunk && !call_end) {
      if ((rc = set_clock(c, s - (vv ? 0 : 1)))) return rc;
      hipGraphExec_t g = nullptr;
      if ((rc = get_dyn_graph(c, search, &g))) return rc;
      HIPCHK(hipGraphLaunch(g, c->stream));
      c->cur ^= (kDynChunk + (search ? 1 : 0)) & 1;
      if (search) {
        c->pcur ^= 1;
        c->n_rebuilds += 1;
      }
      c->host_base += kDynChunk;
    } else {
      // eager: the clock stays, the step offset is explicit
      const int64_t base = (vv ? s : s - 1) - c->host_base;
      HIPCHK(launch_fill_i32((int*)(c->d_drift + kDriftSpread), 0,
                             2 * kDriftSpread * (int64_t)L, c->stream));
      if (search && (rc = eager_rebuild(c, base))) return rc;
      for (int j = 0; j < L; ++j) {
        const int mode = vv ? ((call_end && j == L - 1) ? 1 : 0) : 2;
        unsigned long long* rec = c->d_drift + (size_t)kDriftSpread * (1 + j);
        if ((rc = eager_force(c, mode, base + j, rec))) return rc;
      }
    }
    // the last force launch of a Verlet call does not drift
    if ((rc = fold_drift(c, 1, vv && call_end ? L - 1 : L))) return rc;
    c->dyn_wacc += L * c->dyn_wrate;
    s += L;
  }
  return DEM_OK;
}

int read_flags(dem_ctx* c, int* flags) {
  HIPCHK(hipMemcpyAsync(flags, c->d_flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DEM_OK;
}

int flags_to_error(dem_ctx* c, int flags) {
  if (flags == 0) return DEM_OK;
  c->failed = true;
  if (flags & (kFlagNbrOverflow | kFlagWallOverflow | kFlagMeshOverflow)) {
    c->fail_code = DEM_ECAPACITY;
    return set_err(DEM_ECAPACITY,
                   "capacity exceeded (flags 0x%x): more than %d neighbours, %d wall "
                   "contacts or %d triangle candidates for a particle; raise max_neighbors "
                   "or use larger mesh triangles",
                   flags, c->max_nb, kWallSlots, kMeshSlots);
  }
  c->fail_code = DEM_EUNSTABLE;
  if (flags & kFlagNonFinite)
    return set_err(DEM_EUNSTABLE, "non-finite particle state (flags 0x%x)", flags);
  return set_err(DEM_EUNSTABLE,
                 "a particle moved more than half the skin between two contact "
                 "searches; lower rebuild_interval or dt (flags 0x%x)",
                 flags);
}

// host copy of the current particle arrays in sorted order
struct HostSnapshot {
  std::vector<double4> pos, vel, omg;
  std::vector<int> gid, info;
};

int snapshot(dem_ctx* c, HostSnapshot& h, bool want_pos, bool want_vel, bool want_omg) {
  const size_t n = (size_t)c->n;
  h.gid.resize(n);
  h.info.resize(n);
  HIPCHK(hipMemcpyAsync(h.gid.data(), c->gid[c->pcur], n * sizeof(int), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipMemcpyAsync(h.info.data(), c->info[c->pcur], n * sizeof(int),
                        hipMemcpyDeviceToHost, c->stream));
  if (want_pos) {
    h.pos.resize(n);
    HIPCHK(hipMemcpyAsync(h.pos.data(), c->pos[c->cur], n * sizeof(double4),
                          hipMemcpyDeviceToHost, c->stream));
  }
  if (want_vel) {
    h.vel.resize(n);
    HIPCHK(hipMemcpyAsync(h.vel.data(), c->vel[c->cur], n * sizeof(double4),
                          hipMemcpyDeviceToHost, c->stream));
  }
  if (want_omg) {
    h.omg.resize(n);
    HIPCHK(hipMemcpyAsync(h.omg.data(), c->omg[c->cur], n * sizeof(double4),
                          hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return DEM_OK;
}

int commit(dem_ctx* c);

// Triangle table and grids of the mesh walls of every instance.  Each mesh
// gets a uniform grid over its bounding box at time 0 grown by the largest
// reach of a candidate (largest radius + skin), every triangle listed in
// the cells its own grown box overlaps (ascending triangle order), so that
// the cell of a particle centre lists every triangle that can be its
// candidate.  Sets the mesh fields of the instances' walls.
int build_meshes(dem_ctx* c, std::vector<TriDev>* htri, std::vector<int>* hcell,
                 std::vector<int>* hcell_tri) {
  c->tri_wall.clear();
  c->tri_local.clear();
  for (Instance& I : c->inst) {
    const double reach = (0.5 * I.dmax + I.skin) * (1.0 + 1e-9);
    int64_t t0 = 0;
    for (size_t wl = 0; wl < I.walls.size(); ++wl) {
      WallDev& W = I.walls[wl];
      if (W.kind != 3) continue;
      const int gw = I.w_begin + (int)wl;
      W.tri_begin = (int)htri->size();
      double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
      double ext = 0.0;
      int cnt = 0;
      while (t0 < (int64_t)I.tris.size() && I.tris[(size_t)t0].wall == (int)wl) {
        const HostTri& h = I.tris[(size_t)t0];
        TriDev T;
        memset(&T, 0, sizeof(T));
        for (int cc = 0; cc < 3; ++cc) {
          const int c1 = cc == 2 ? 0 : cc + 1;
          for (int k = 0; k < 3; ++k) {
            T.p[cc][k] = h.p[cc][k];
            T.e[cc][k] = h.p[c1][k] - h.p[cc][k];
          }
          T.v[cc] = h.v[cc];
        }
        const double e01[3] = {h.p[1][0] - h.p[0][0], h.p[1][1] - h.p[0][1], h.p[1][2] - h.p[0][2]};
        const double e02[3] = {h.p[2][0] - h.p[0][0], h.p[2][1] - h.p[0][1], h.p[2][2] - h.p[0][2]};
        const double N[3] = {e01[1] * e02[2] - e01[2] * e02[1], e01[2] * e02[0] - e01[0] * e02[2],
                             e01[0] * e02[1] - e01[1] * e02[0]};
        const double len = sqrt((N[0] * N[0] + N[1] * N[1]) + N[2] * N[2]);
        for (int k = 0; k < 3; ++k) T.n[k] = N[k] / len;
        T.wall = gw;
        double tlo[3], thi[3];
        for (int k = 0; k < 3; ++k) {
          tlo[k] = std::min(h.p[0][k], std::min(h.p[1][k], h.p[2][k]));
          thi[k] = std::max(h.p[0][k], std::max(h.p[1][k], h.p[2][k]));
          lo[k] = std::min(lo[k], tlo[k]);
          hi[k] = std::max(hi[k], thi[k]);
          ext = std::max(ext, thi[k] - tlo[k]);
        }
        c->tri_wall.push_back((int)wl);
        c->tri_local.push_back(cnt);
        htri->push_back(T);
        ++cnt;
        ++t0;
      }
      W.tri_count = cnt;
      // grid: cells no smaller than the reach nor than the largest triangle,
      // at most about four per triangle
      double mh = std::max(reach, ext);
      if (!(mh > 0.0)) mh = 1.0;
      int64_t nc[3];
      for (;;) {
        int64_t tot = 1;
        for (int k = 0; k < 3; ++k) {
          W.mlo[k] = lo[k] - reach;
          nc[k] = std::max<int64_t>(1, (int64_t)ceil((hi[k] + reach - W.mlo[k]) / mh));
          tot *= nc[k];
        }
        if (tot <= 4 * (int64_t)cnt + 1024) break;
        mh *= 1.5;
      }
      W.mh = mh;
      for (int k = 0; k < 3; ++k) W.mnc[k] = (int)nc[k];
      const int64_t ncell = nc[0] * nc[1] * nc[2];
      std::vector<std::vector<int>> lists((size_t)ncell);
      for (int f = W.tri_begin; f < W.tri_begin + cnt; ++f) {
        const TriDev& T = (*htri)[(size_t)f];
        int64_t a[3], b[3];
        for (int k = 0; k < 3; ++k) {
          const double tl = std::min(T.p[0][k], std::min(T.p[1][k], T.p[2][k])) - reach;
          const double th = std::max(T.p[0][k], std::max(T.p[1][k], T.p[2][k])) + reach;
          a[k] = std::max<int64_t>(0, (int64_t)floor((tl - W.mlo[k]) / mh) - 1);
          b[k] = std::min<int64_t>(nc[k] - 1, (int64_t)floor((th - W.mlo[k]) / mh) + 1);
        }
        for (int64_t z = a[2]; z <= b[2]; ++z)
          for (int64_t y = a[1]; y <= b[1]; ++y)
            for (int64_t x = a[0]; x <= b[0]; ++x)
              lists[(size_t)(x + nc[0] * (y + nc[1] * z))].push_back(f);
      }
      size_t entries = hcell_tri->size();
      for (const std::vector<int>& li : lists) entries += li.size();
      if (entries > ((size_t)1 << 30))
        return set_err(DEM_EINVAL, "mesh grids too large (%zu cell entries)", entries);
      W.cell_base = (int)hcell->size();
      for (int64_t q = 0; q < ncell; ++q) {
        hcell->push_back((int)hcell_tri->size());
        for (int f : lists[(size_t)q]) hcell_tri->push_back(f);
      }
      hcell->push_back((int)hcell_tri->size());
    }
  }
  return DEM_OK;
}

// Translating walls: a wall may move at most half the skin between two
// searches, the particles' displacement guard taking the other half, so that
// no particle-wall contact is missed.  walls_fit tells whether K steps of
// every translating wall stay within that; wall_rate is the largest distance
// one step of a translating wall covers, in half skins of its instance.
double wall_speed(const WallDev& w) {
  return sqrt((w.vel[0] * w.vel[0] + w.vel[1] * w.vel[1]) + w.vel[2] * w.vel[2]);
}

bool walls_fit(const dem_ctx* c, int64_t K) {
  for (const Instance& I : c->inst) {
    if (I.n == 0) continue;
    for (const WallDev& w : I.walls) {
      const double v = wall_speed(w);
      if (v > 0.0 && !(v * (double)K * c->cfg.dt <= 0.5 * I.skin)) return false;
    }
  }
  return true;
}

double wall_rate(const dem_ctx* c) {
  double r = 0.0;
  for (const Instance& I : c->inst) {
    if (I.n == 0) continue;
    for (const WallDev& w : I.walls) {
      const double v = wall_speed(w);
      if (v > 0.0) r = std::max(r, I.skin > 0.0 ? v * c->cfg.dt * 2.0 / I.skin : HUGE_VAL);
    }
  }
  return r;
}

// Cell grid of every instance for the cell edge h = cf d_max (1 + 1e-9),
// never below the search radius r_s: cell counts and one key range per
// instance.  The instances keep their previous grids when the new ones would
// not fit.
int plan_grids(dem_ctx* c, double cf, int64_t* total_keys_out, size_t* ckey_total_out) {
  const int B = (int)c->inst.size();
  std::vector<GridDev> grids((size_t)B);
  std::vector<uint32_t> bases((size_t)B);
  std::vector<double> hs((size_t)B);
  int64_t total_keys = 0;
  for (int b = 0; b < B; ++b) {
    const Instance& I = c->inst[(size_t)b];
    const double h = std::max(cf * I.dmax * (1.0 + 1e-9), I.rs);
    GridDev g;
    memset(&g, 0, sizeof(g));
    int64_t cells = 1;
    for (int k = 0; k < 3; ++k) {
      g.lo[k] = I.own_domain ? I.lo[k] : c->cfg.domain_lo[k];
      g.hi[k] = I.own_domain ? I.hi[k] : c->cfg.domain_hi[k];
      const double span = g.hi[k] - g.lo[k];
      const double cc = I.n > 0 ? ceil(span / h) : 1.0;
      if (!(cc < 1e6)) return set_err(DEM_EINVAL, "domain too large for the cell grid");
      g.nc[k] = std::max(1, (int)cc);
      cells *= g.nc[k];
    }
    if (cells >= ((int64_t)1 << 30))
      return set_err(DEM_EINVAL, "instance %d: cell grid %dx%dx%d is too large; shrink the domain",
                     b, g.nc[0], g.nc[1], g.nc[2]);
    g.h = I.n > 0 ? h : 1.0;
    g.n_keys = cells;
    grids[(size_t)b] = g;
    hs[(size_t)b] = h;
    bases[(size_t)b] = (uint32_t)total_keys;
    total_keys += g.n_keys;
    if (total_keys >= ((int64_t)1 << 30))
      return set_err(DEM_EINVAL, "the cell grids of the batch need more than 2^30 cells");
  }
  for (int b = 0; b < B; ++b) {
    Instance& I = c->inst[(size_t)b];
    I.grid = grids[(size_t)b];
    I.h = hs[(size_t)b];
    I.key_base = bases[(size_t)b];
  }
  c->cell_factor = cf;
  *total_keys_out = total_keys;
  *ckey_total_out = (size_t)total_keys;
  return DEM_OK;
}

// Cell-key tables of the instance grids and the instance table.  A cell's
// Morton code interleaves the bits of its coordinates (bit l of axis a goes
// to the next free code bit, levels l = 0, 1, ... and axes x, y, z in turn,
// an axis dropping out once its bits are used up); its key is its rank by
// that code among the grid's cells.  The tables live at c->d_ckey; hkeycell
// (at c->d_key_cell) is the inverse, key -> cell, both over all instances.
void grid_tables(dem_ctx* c, std::vector<uint32_t>* hckey, std::vector<uint32_t>* hkeycell,
                 std::vector<InstDev>* hinst) {
  const int B = (int)c->inst.size();
  hckey->clear();
  hkeycell->clear();
  hinst->assign((size_t)B, InstDev{});
  std::vector<std::pair<uint64_t, uint32_t>> code;
  for (int b = 0; b < B; ++b) {
    Instance& I = c->inst[(size_t)b];
    GridDev& g = I.grid;
    int bits[3];
    for (int a = 0; a < 3; ++a) {
      bits[a] = 0;
      while ((1 << bits[a]) < g.nc[a]) ++bits[a];
    }
    int pos_of[3][32];
    int next = 0;
    const int maxb = std::max(bits[0], std::max(bits[1], bits[2]));
    for (int lvl = 0; lvl < maxb; ++lvl)
      for (int a = 0; a < 3; ++a)
        if (lvl < bits[a]) pos_of[a][lvl] = next++;
    std::vector<uint64_t> spread[3];
    for (int a = 0; a < 3; ++a) {
      spread[a].resize((size_t)g.nc[a]);
      for (int ci = 0; ci < g.nc[a]; ++ci) {
        uint64_t m = 0;
        for (int lvl = 0; lvl < bits[a]; ++lvl)
          if ((ci >> lvl) & 1) m |= uint64_t(1) << pos_of[a][lvl];
        spread[a][(size_t)ci] = m;
      }
    }
    // (code, linear index) of every cell, x fastest; sorted by code they are
    // in Morton order
    const size_t base = hckey->size(), cells = (size_t)g.n_keys;
    code.resize(cells);
    size_t lin = 0;
    for (int z = 0; z < g.nc[2]; ++z)
      for (int y = 0; y < g.nc[1]; ++y)
        for (int x = 0; x < g.nc[0]; ++x, ++lin)
          code[lin] = {spread[0][(size_t)x] | spread[1][(size_t)y] | spread[2][(size_t)z],
                       (uint32_t)lin};
    std::sort(code.begin(), code.end());
    hckey->resize(base + cells);
    hkeycell->resize(base + cells);
    for (size_t r = 0; r < cells; ++r) {
      (*hckey)[base + code[r].second] = (uint32_t)r;
      (*hkeycell)[base + r] = (uint32_t)(base + code[r].second);
    }
    g.ckey = c->d_ckey + base;
    InstDev& D = (*hinst)[(size_t)b];
    D.grid = g;
    D.key_base = I.key_base;
    D.wall_begin = I.w_begin;
    D.wall_end = I.w_begin + (int)I.walls.size();
    D.coef_base = b * kMaxTypes * kMaxTypes;
    D.rs2 = I.rs * I.rs;
    D.guard2 = (0.5 * I.skin) * (0.5 * I.skin);
    D.skin = I.skin;
    D.ihs = I.skin > 0.0 ? 2.0 / I.skin : 0.0;
  }
}

// Change the cell edge of a built batch to cf d_max.  The neighbour lists do
// not depend on the grid, so the next contact search simply uses the new
// cells (histories are carried as at every search).
int regrid(dem_ctx* c, double cf) {
  int64_t total_keys = 0;
  size_t ckey_total = 0;
  int rc = plan_grids(c, cf, &total_keys, &ckey_total);
  if (rc) return rc;
  destroy_graphs(c);
  HIPCHK(hipStreamSynchronize(c->stream));
  dfree(c, c->count);
  dfree(c, c->start);
  dfree(c, c->tile_sums);
  dfree(c, c->d_ckey);
  dfree(c, c->d_key_cell);
  dfree(c, c->d_cse);
  c->count = c->start = c->tile_sums = nullptr;
  c->d_ckey = c->d_key_cell = nullptr;
  c->d_cse = nullptr;
  rc = rc ? rc : dalloc_t(c, &c->count, (size_t)total_keys + 1);
  rc = rc ? rc : dalloc_t(c, &c->start, (size_t)total_keys + 2);
  rc = rc ? rc : dalloc_t(c, &c->tile_sums, (size_t)((total_keys + 1 + 1023) / 1024 + 1));
  rc = rc ? rc : dalloc_t(c, &c->d_ckey, std::max<size_t>(ckey_total, 1));
  rc = rc ? rc : dalloc_t(c, &c->d_key_cell, std::max<size_t>(ckey_total, 1));
  rc = rc ? rc : dalloc_t(c, &c->d_cse, std::max<size_t>(ckey_total, 1));
  if (rc) {
    c->failed = true;
    return rc;
  }
  std::vector<uint32_t> hckey, hkeycell;
  std::vector<InstDev> hinst;
  grid_tables(c, &hckey, &hkeycell, &hinst);
  if (!hckey.empty()) {
    HIPCHK(hipMemcpyAsync(c->d_ckey, hckey.data(), hckey.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_key_cell, hkeycell.data(), hkeycell.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(hipMemcpyAsync(c->d_inst, hinst.data(), hinst.size() * sizeof(InstDev),
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->n_keys = total_keys;
  c->sp.n_keys = (uint32_t)total_keys;
  return DEM_OK;
}

// The batch is built on the device at the first call that needs it.
int require_ready(dem_ctx* c) {
  if (!c) return set_err(DEM_EINVAL, "null context");
  if (!c->ready) {
    for (const Instance& I : c->inst)
      if (!I.staged) return set_err(DEM_ESTATE, "particles not set (call dem_set_particles)");
    if (c->failed) return set_err(DEM_ESTATE, "a previous error is sticky");
    return commit(c);
  }
  return DEM_OK;
}

// Build the whole batch on the device from the staged instances: search
// geometry per instance, one key range per instance grid, concatenated walls
// and material-pair tables, packed particle state, then the first contact
// search at the initial positions with all histories zero.
int commit(dem_ctx* c) {
  free_particles(c);
  const int B = (int)c->inst.size();
  int64_t N = 0;
  for (const Instance& I : c->inst) N += I.n;
  if (N > kMaxParticles)
    return set_err(DEM_EINVAL, "too many particles in the batch (at most 2^29)");
  const double f = std::min(c->cfg.neighbor_threshold, c->cfg.cell_factor);
  int64_t total_keys = 0;
  double bound_nb = 16.0;
  size_t ckey_total = 0;
  int n_walls = 0;
  for (int b = 0; b < B; ++b) {
    Instance& I = c->inst[(size_t)b];
    double rmin = INFINITY, rmax = 0.0;
    for (double r : I.rad) {
      rmin = std::min(rmin, r);
      rmax = std::max(rmax, r);
    }
    // search geometry: r_s = min(threshold, cell_factor) d_max, h >= r_s
    I.dmax = 2.0 * rmax;
    I.rs = f * I.dmax;
    I.skin = I.rs - I.dmax;
    if (I.n > 0) {
      // spheres of radius rmin whose centres lie within r_s of a centre fit in a
      // ball of radius r_s + rmin (packing density <= 0.7405), 25% margin
      const double ratio = (I.rs + rmin) / rmin;
      bound_nb = std::max(bound_nb, 0.7405 * ratio * ratio * ratio * 1.25);
    }
    I.w_begin = n_walls;
    n_walls += (int)I.walls.size();
  }
  {
    int rc = plan_grids(c, c->cfg.cell_factor, &total_keys, &ckey_total);
    if (rc) return rc;
  }
  std::vector<TriDev> htri;
  std::vector<int> hcell, hcell_tri;
  if (int rc = build_meshes(c, &htri, &hcell, &hcell_tri)) return rc;
  c->dynamic = c->cfg.rebuild_interval == 0;
  double ihs_max = 0.0, rate0 = 0.0, ihs_min = HUGE_VAL;
  bool all_skins = true;
  for (int b = 0; b < B; ++b)
    if (c->inst[(size_t)b].n > 0 && !(c->inst[(size_t)b].skin > 0.0)) all_skins = false;
  if (c->dynamic && !all_skins)
    return set_err(DEM_EINVAL,
                   "dynamic search (rebuild_interval 0) needs a skin: neighbor_threshold "
                   "and cell_factor must exceed 1");
  if (all_skins) {
    for (int b = 0; b < B; ++b) {
      const Instance& I = c->inst[(size_t)b];
      if (I.n == 0) continue;
      const double ihs = 2.0 / I.skin;
      ihs_max = std::max(ihs_max, ihs);
      ihs_min = std::min(ihs_min, ihs);
      for (int64_t i = 0; i < I.n && !I.vel.empty(); ++i) {
        const double* v = &I.vel[3 * (size_t)i];
        rate0 = std::max(rate0, sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]) * c->cfg.dt * ihs);
      }
    }
  }
  const double gmag = sqrt((c->cfg.gravity[0] * c->cfg.gravity[0] +
                            c->cfg.gravity[1] * c->cfg.gravity[1]) +
                           c->cfg.gravity[2] * c->cfg.gravity[2]);
  if (!walls_fit(c, c->dynamic ? 1 : c->cfg.rebuild_interval))
    return set_err(DEM_EINVAL,
                   "a translating wall moves more than half the skin between two contact "
                   "searches; lower rebuild_interval or dt, or raise neighbor_threshold");
  c->dyn_acc = 0.0;
  c->dyn_rate = rate0;
  c->dyn_grav = gmag * c->cfg.dt * c->cfg.dt * ihs_max;
  c->dyn_wrate = wall_rate(c);
  c->dyn_wacc = 0.0;
  int max_nb = c->cfg.max_neighbors;
  if (max_nb == 0) max_nb = (int)std::min(512.0, ceil(bound_nb));
  c->max_nb = max_nb;
  c->n = (int)N;
  c->n_keys = total_keys;
  const int64_t npad = ((N + 63) / 64) * 64;
  c->cap = npad * max_nb;

  StepParams& sp = c->sp;
  sp.dt = c->cfg.dt;
  sp.hdt = 0.5 * c->cfg.dt;
  for (int k = 0; k < 3; ++k) sp.g[k] = c->cfg.gravity[k];
  sp.n = (int)N;
  sp.max_nb = max_nb;
  sp.rolling = c->cfg.rolling_model;
  sp.model = c->cfg.contact_model;
  sp.n_keys = (uint32_t)total_keys;
  sp.drift_scale = ihs_min == ihs_max ? c->cfg.dt * ihs_max : 0.0;

  // allocations
  const size_t NN = (size_t)std::max<int64_t>(N, 1);
  int rc = DEM_OK;
  for (int b = 0; b < 2 && rc == DEM_OK; ++b) {
    rc = rc ? rc : dalloc_t(c, &c->pos[b], NN);
    rc = rc ? rc : dalloc_t(c, &c->vel[b], NN);
    rc = rc ? rc : dalloc_t(c, &c->omg[b], NN);
    rc = rc ? rc : dalloc_t(c, &c->gid[b], NN);
    rc = rc ? rc : dalloc_t(c, &c->info[b], NN);
    rc = rc ? rc : dalloc_t(c, &c->F[b], NN);
    rc = rc ? rc : dalloc_t(c, &c->T[b], NN);
    rc = rc ? rc : dalloc_t(c, &c->wid[b], NN * kWallSlots);
    rc = rc ? rc : dalloc_t(c, &c->whist[b], NN * kWallSlots * 3);
    rc = rc ? rc : dalloc_t(c, &c->nbr[b], (size_t)std::max<int64_t>(c->cap, 1));
    rc = rc ? rc : dalloc_t(c, &c->hist[b], (size_t)std::max<int64_t>(c->cap, 1) * 3);
    rc = rc ? rc : dalloc_t(c, &c->rowlen[b], NN);
    rc = rc ? rc : dalloc_t(c, &c->rowcut[b], NN);
  }
  rc = rc ? rc : dalloc_t(c, &c->xref, NN);
  rc = rc ? rc : dalloc_t(c, &c->keys, NN);
  rc = rc ? rc : dalloc_t(c, &c->rank, NN);
  rc = rc ? rc : dalloc_t(c, &c->count, (size_t)total_keys + 1);
  rc = rc ? rc : dalloc_t(c, &c->start, (size_t)total_keys + 2);
  rc = rc ? rc : dalloc_t(c, &c->tile_sums, (size_t)((total_keys + 1 + 1023) / 1024 + 1));
  rc = rc ? rc : dalloc_t(c, &c->perm0, NN);
  rc = rc ? rc : dalloc_t(c, &c->perm, NN);
  rc = rc ? rc : dalloc_t(c, &c->inv, NN);
  rc = rc ? rc : dalloc_t(c, &c->d_pp, (size_t)B * kMaxTypes * kMaxTypes);
  rc = rc ? rc : dalloc_t(c, &c->d_pw, (size_t)B * kMaxTypes * kMaxTypes);
  rc = rc ? rc : dalloc_t(c, &c->d_walls, (size_t)std::max(n_walls, 1));
  rc = rc ? rc : dalloc_t(c, &c->d_inst, (size_t)B);
  rc = rc ? rc : dalloc_t(c, &c->d_flags, 1);
  rc = rc ? rc : dalloc_t(c, &c->d_clock, 1);
  rc = rc ? rc : dalloc_t(c, &c->d_stats, 4);
  rc = rc ? rc : dalloc_t(c, &c->d_ckey, std::max<size_t>(ckey_total, 1));
  rc = rc ? rc : dalloc_t(c, &c->d_key_cell, std::max<size_t>(ckey_total, 1));
  rc = rc ? rc : dalloc_t(c, &c->d_cse, std::max<size_t>(ckey_total, 1));
  rc = rc ? rc : dalloc_t(c, &c->d_drift, (size_t)kDriftSpread * (kDynChunk + 1));
  rc = rc ? rc : dalloc_t(c, &c->d_bacc, 3);
  rc = rc ? rc : dalloc_t(c, &c->d_brec, 3 * (size_t)kDriftSpread);
  if (c->record_pf)
    rc = rc ? rc : dalloc_t(c, &c->pair_force, (size_t)std::max<int64_t>(c->cap, 1) * 3);
  if (!htri.empty()) {
    rc = rc ? rc : dalloc_t(c, &c->d_tri, htri.size());
    rc = rc ? rc : dalloc_t(c, &c->d_mcell, hcell.size());
    rc = rc ? rc : dalloc_t(c, &c->d_mcell_tri, std::max<size_t>(hcell_tri.size(), 1));
    for (int b = 0; b < 2; ++b) {
      rc = rc ? rc : dalloc_t(c, &c->mtri[b], NN * kMeshSlots);
      rc = rc ? rc : dalloc_t(c, &c->mhist[b], NN * kMeshSlots * 3);
    }
    rc = rc ? rc : dalloc_t(c, &c->Fm, NN);
    rc = rc ? rc : dalloc_t(c, &c->Tm, NN);
    c->has_mesh = rc == DEM_OK;
  }
  if (rc == DEM_OK) {
    hipError_t he = hipHostMalloc((void**)&c->h_drift,
                                  sizeof(unsigned long long) * kDriftSpread * (kDynChunk + 1),
                                  hipHostMallocDefault);
    if (he != hipSuccess) {
      c->h_drift = nullptr;
      rc = set_err(DEM_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(he));
    }
  }
  if (rc) {
    free_particles(c);
    return rc;
  }

  // cell-key tables, instance table, walls and material-pair tables
  std::vector<uint32_t> hckey, hkeycell;
  std::vector<InstDev> hinst;
  grid_tables(c, &hckey, &hkeycell, &hinst);
  std::vector<WallDev> hwalls;
  std::vector<PairCoef> pp((size_t)B * kMaxTypes * kMaxTypes), pw(pp.size());
  memset(pp.data(), 0, pp.size() * sizeof(PairCoef));
  memset(pw.data(), 0, pw.size() * sizeof(PairCoef));
  for (int b = 0; b < B; ++b) {
    Instance& I = c->inst[(size_t)b];
    const InstDev& D = hinst[(size_t)b];
    for (WallDev w : I.walls) {
      w.skin = I.skin;
      for (int k = 0; k < 3; ++k) w.axo[k] = w.ax[k] - w.p[k];
      hwalls.push_back(w);
    }
    for (int ta = 0; ta < kMaxTypes; ++ta)
      for (int tb = 0; tb < kMaxTypes; ++tb) {
        if (!I.mat_set[ta] || !I.mat_set[tb]) continue;
        const dem_material &A = I.mat[ta], &M = I.mat[tb];
        const double Ye = eff_youngs(A, M), Ge = eff_shear(A, M);
        // unlike particle types: mean restitution, friction and rolling friction
        const double e = ta == tb ? A.restitution : 0.5 * (A.restitution + M.restitution);
        const double mu = ta == tb ? A.friction : 0.5 * (A.friction + M.friction);
        const double mur =
            ta == tb ? A.rolling_friction : 0.5 * (A.rolling_friction + M.rolling_friction);
        const size_t idx = (size_t)D.coef_base + (size_t)ta * kMaxTypes + (size_t)tb;
        pp[idx] = make_coef(c->cfg, Ye, Ge, e, mu, mur);
        // particle type ta against wall material tb: the wall's e, mu, mu_r
        pw[idx] = make_coef(c->cfg, Ye, Ge, M.restitution, M.friction, M.rolling_friction);
      }
  }

  // packed particle state (1/m and 1/I are stored: the law needs 1/m_i + 1/m_j)
  std::vector<double4> hpos(NN), hvel(NN), homg(NN);
  bool all_type0 = true;
  for (const Instance& I : c->inst)
    for (int32_t t : I.type) all_type0 = all_type0 && t == 0;
  c->pair_mode = all_type0 ? (B == 1 ? 1 : 2) : 0;
  std::vector<int> hgid(NN), hinfo(NN);
  int64_t q = 0;
  for (int b = 0; b < B; ++b) {
    Instance& I = c->inst[(size_t)b];
    I.p_begin = q;
    const bool hv = !I.vel.empty(), hw = !I.omg.empty(), ht = !I.type.empty();
    for (int64_t i = 0; i < I.n; ++i, ++q) {
      const int t = ht ? I.type[(size_t)i] : 0;
      const double R = I.rad[(size_t)i];
      const double m = I.mat[t].density * (4.0 / 3.0) * kPi * R * R * R;
      const double Iner = 0.4 * m * R * R;
      const double* x = &I.pos[3 * (size_t)i];
      hpos[(size_t)q] = make_double4(x[0], x[1], x[2], R);
      hvel[(size_t)q] = hv ? make_double4(I.vel[3 * i], I.vel[3 * i + 1], I.vel[3 * i + 2], 1.0 / m)
                           : make_double4(0.0, 0.0, 0.0, 1.0 / m);
      homg[(size_t)q] = hw ? make_double4(I.omg[3 * i], I.omg[3 * i + 1], I.omg[3 * i + 2], 1.0 / Iner)
                           : make_double4(0.0, 0.0, 0.0, 1.0 / Iner);
      hgid[(size_t)q] = (int)q;
      hinfo[(size_t)q] = t | (b << kInstShift);
    }
  }
  hipStream_t s = c->stream;
  if ((rc = wait_user(c))) return rc;
  if (!hckey.empty()) {
    HIPCHK(hipMemcpyAsync(c->d_ckey, hckey.data(), hckey.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_key_cell, hkeycell.data(), hkeycell.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipMemcpyAsync(c->d_inst, hinst.data(), hinst.size() * sizeof(InstDev),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->d_pp, pp.data(), pp.size() * sizeof(PairCoef), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->d_pw, pw.data(), pw.size() * sizeof(PairCoef), hipMemcpyHostToDevice, s));
  if (!hwalls.empty())
    HIPCHK(hipMemcpyAsync(c->d_walls, hwalls.data(), hwalls.size() * sizeof(WallDev),
                          hipMemcpyHostToDevice, s));
  if (c->has_mesh) {
    HIPCHK(hipMemcpyAsync(c->d_tri, htri.data(), htri.size() * sizeof(TriDev),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_mcell, hcell.data(), hcell.size() * sizeof(int),
                          hipMemcpyHostToDevice, s));
    if (!hcell_tri.empty())
      HIPCHK(hipMemcpyAsync(c->d_mcell_tri, hcell_tri.data(), hcell_tri.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
    HIPCHK(launch_fill_i32(c->mtri[0], -1, (int64_t)NN * kMeshSlots, s));
    HIPCHK(launch_fill_i32((int*)c->mhist[0], 0, (int64_t)NN * kMeshSlots * 6, s));
  }
  c->cur = 0;
  c->pcur = 0;
  if (N > 0) {
    HIPCHK(hipMemcpyAsync(c->pos[0], hpos.data(), N * sizeof(double4), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->vel[0], hvel.data(), N * sizeof(double4), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->omg[0], homg.data(), N * sizeof(double4), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->gid[0], hgid.data(), N * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->info[0], hinfo.data(), N * sizeof(int), hipMemcpyHostToDevice, s));
  }
  // zero-filled: forces of both parities, empty old list and wall slots
  c->sp.bacc = c->d_bacc;
  c->sp.brec = c->d_brec;
  HIPCHK(launch_fill_i32((int*)c->d_bacc, 0, 6, s));
  HIPCHK(launch_fill_i32((int*)c->d_brec, 0, 6 * kDriftSpread, s));
  HIPCHK(launch_fill_i32((int*)c->F[0], 0, (int64_t)NN * 8, s));
  HIPCHK(launch_fill_i32((int*)c->T[0], 0, (int64_t)NN * 8, s));
  HIPCHK(launch_fill_i32((int*)c->F[1], 0, (int64_t)NN * 8, s));
  HIPCHK(launch_fill_i32((int*)c->T[1], 0, (int64_t)NN * 8, s));
  HIPCHK(launch_fill_i32(c->rowlen[0], 0, (int64_t)NN, s));
  HIPCHK(launch_fill_i32(c->wid[0], -1, (int64_t)NN * kWallSlots, s));
  HIPCHK(launch_fill_i32(c->d_flags, 0, 1, s));
  HIPCHK(launch_fill_i32((int*)c->d_clock, 0, 2, s));
  HIPCHK(launch_fill_i32((int*)c->xref, 0, (int64_t)NN * 8, s));
  c->step = 0;
  c->host_base = 0;
  c->n_rebuilds = 0;
  if ((rc = enqueue_rebuild(c, 0, 0, 0, next_eval_rel(c)))) return rc;
  int flags = 0;
  if ((rc = read_flags(c, &flags))) return rc;
  c->ready = true;
  return flags_to_error(c, flags);
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

const char* dem_last_error(dem_ctx*) { return g_err.c_str(); }

void* dem_stream(dem_ctx* c) { return c ? (void*)c->stream : nullptr; }

int dem_create(const dem_config* cfg, dem_ctx** out) {
  if (!cfg || !out) return set_err(DEM_EINVAL, "null argument");
  *out = nullptr;
  if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return set_err(DEM_EINVAL, "dt must be > 0");
  for (int k = 0; k < 3; ++k)
    if (!(cfg->domain_hi[k] > cfg->domain_lo[k]))
      return set_err(DEM_EINVAL, "empty domain along axis %d", k);
  if (cfg->rebuild_interval < 0)
    return set_err(DEM_EINVAL, "rebuild_interval must be >= 1 (constant) or 0 (dynamic)");
  if (!(cfg->neighbor_threshold >= 1.0))
    return set_err(DEM_EINVAL, "neighbor_threshold must be >= 1");
  if (!(cfg->cell_factor >= 1.0)) return set_err(DEM_EINVAL, "cell_factor must be >= 1");
  if (cfg->integrator < 0 || cfg->integrator > 1)
    return set_err(DEM_EINVAL, "integrator must be 0 (Verlet) or 1 (Euler)");
  if (cfg->rolling_model < 0 || cfg->rolling_model > 2)
    return set_err(DEM_EINVAL, "rolling_model must be 0 (none), 1 (constant) or 2 (viscous)");
  if (cfg->contact_model < 0 || cfg->contact_model > 1)
    return set_err(DEM_EINVAL, "contact_model must be 0 (nonlinear) or 1 (linear)");
  if (cfg->contact_model == 1 &&
      !(cfg->characteristic_velocity > 0.0 && std::isfinite(cfg->characteristic_velocity)))
    return set_err(DEM_EINVAL, "the linear model needs characteristic_velocity > 0");
  if (cfg->precision < 0 || cfg->precision > 1)
    return set_err(DEM_EINVAL, "precision must be 0 (FP64) or 1 (FP32 law)");
  if (cfg->force_block != 0 && cfg->force_block != 64 && cfg->force_block != 128 &&
      cfg->force_block != 256)
    return set_err(DEM_EINVAL, "force_block must be 0, 64, 128 or 256");
  if (cfg->n_instances < 1 || cfg->n_instances > kMaxInstances)
    return set_err(DEM_EINVAL, "n_instances must be in [1, %d]", kMaxInstances);
  if (cfg->max_neighbors < 0 || cfg->max_neighbors > 4096)
    return set_err(DEM_EINVAL, "max_neighbors out of range");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_err(DEM_ENODEV, "no HIP device: %s", hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return set_err(DEM_ENODEV, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_err(DEM_ENODEV, "device %d is %s, this library is built for gfx950", dev,
                   prop.gcnArchName);
  dem_ctx* c = new dem_ctx();
  c->cfg = *cfg;
  c->force_block = cfg->force_block ? cfg->force_block : kBlock;
  c->device = dev;
  c->inst.resize((size_t)cfg->n_instances);
  e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_user, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete c;
    return set_err(DEM_EHIP, "stream/event creation: %s", hipGetErrorString(e));
  }
  *out = c;
  return DEM_OK;
}

void dem_destroy(dem_ctx* c) {
  if (!c) return;
  free_particles(c);
  for (hipEvent_t ev : c->tev) (void)hipEventDestroy(ev);
  if (c->ev_user) (void)hipEventDestroy(c->ev_user);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int dem_set_material(dem_ctx* c, int32_t instance, int32_t type, const dem_material* m) {
  if (!c || !m) return set_err(DEM_EINVAL, "null argument");
  if (int rc = check_instance(c, instance)) return rc;
  if (type < 0 || type >= kMaxTypes) return set_err(DEM_EINVAL, "type %d out of [0, 16)", type);
  if (!(m->density > 0.0) || !(m->youngs > 0.0) || !(m->poisson > -1.0 && m->poisson < 0.5) ||
      !(m->restitution > 0.0 && m->restitution <= 1.0) || !(m->friction >= 0.0) ||
      !(m->rolling_friction >= 0.0))
    return set_err(DEM_EINVAL, "invalid material values for type %d", type);
  Instance& I = c->inst[(size_t)instance];
  if (I.staged) return set_err(DEM_ESTATE, "materials are set before dem_set_particles");
  I.mat[type] = *m;
  I.mat_set[type] = true;
  return DEM_OK;
}

int dem_add_planar_wall(dem_ctx* c, int32_t instance, const double point[3],
                        const double normal[3], const double* extent, int32_t material,
                        const double axis_point[3], const double omega[3], double t_on,
                        double t_off, int32_t* wall_id) {
  if (!c || !point || !normal) return set_err(DEM_EINVAL, "null argument");
  if (int rc = check_instance(c, instance)) return rc;
  Instance& I = c->inst[(size_t)instance];
  if ((int)I.walls.size() >= kMaxWalls) return set_err(DEM_EINVAL, "at most 32 walls");
  if (material < 0 || material >= kMaxTypes || !I.mat_set[material])
    return set_err(DEM_EINVAL, "wall material %d not set", material);
  if (I.staged) return set_err(DEM_ESTATE, "walls are added before dem_set_particles");
  WallDev W;
  memset(&W, 0, sizeof(W));
  W.kind = 0;
  if (!unit3(normal, W.nrm)) return set_err(DEM_EINVAL, "zero or non-finite wall normal");
  if (extent) {
    double d = (extent[0] * W.nrm[0] + extent[1] * W.nrm[1]) + extent[2] * W.nrm[2];
    double u[3] = {extent[0] - d * W.nrm[0], extent[1] - d * W.nrm[1], extent[2] - d * W.nrm[2]};
    if (!unit3(u, W.u)) return set_err(DEM_EINVAL, "extent axis parallel to the normal");
    W.vax[0] = W.nrm[1] * W.u[2] - W.nrm[2] * W.u[1];
    W.vax[1] = W.nrm[2] * W.u[0] - W.nrm[0] * W.u[2];
    W.vax[2] = W.nrm[0] * W.u[1] - W.nrm[1] * W.u[0];
    W.hu = extent[3];
    W.hv = extent[4];
    if (!(W.hu > 0.0 && W.hv > 0.0)) return set_err(DEM_EINVAL, "extent half-widths must be > 0");
    W.bounded = 1;
  }
  for (int k = 0; k < 3; ++k) {
    W.p[k] = point[k];
    W.omega[k] = omega ? omega[k] : 0.0;
    W.ax[k] = axis_point ? axis_point[k] : point[k];
  }
  W.material = material;
  W.t_on = t_on;
  W.t_off = t_off;
  if (wall_id) *wall_id = (int32_t)I.walls.size();
  I.walls.push_back(W);
  return DEM_OK;
}

int dem_add_cylinder_wall(dem_ctx* c, int32_t instance, const double axis_point[3],
                          const double axis_dir[3], double radius, double s_min, double s_max,
                          int32_t inside, int32_t material, double omega, double t_on,
                          double t_off, int32_t* wall_id) {
  if (!c || !axis_point || !axis_dir) return set_err(DEM_EINVAL, "null argument");
  if (int rc = check_instance(c, instance)) return rc;
  Instance& I = c->inst[(size_t)instance];
  if ((int)I.walls.size() >= kMaxWalls) return set_err(DEM_EINVAL, "at most 32 walls");
  if (material < 0 || material >= kMaxTypes || !I.mat_set[material])
    return set_err(DEM_EINVAL, "wall material %d not set", material);
  if (!(radius > 0.0) || !(s_max >= s_min))
    return set_err(DEM_EINVAL, "cylinder needs radius > 0 and s_max >= s_min");
  if (I.staged) return set_err(DEM_ESTATE, "walls are added before dem_set_particles");
  WallDev W;
  memset(&W, 0, sizeof(W));
  W.kind = 1;
  if (!unit3(axis_dir, W.nrm)) return set_err(DEM_EINVAL, "zero or non-finite axis");
  for (int k = 0; k < 3; ++k) {
    W.p[k] = axis_point[k];
    W.ax[k] = axis_point[k];
    W.omega[k] = omega * W.nrm[k];
  }
  W.radius = radius;
  W.smin = s_min;
  W.smax = s_max;
  W.inside = inside ? 1 : 0;
  W.material = material;
  W.t_on = t_on;
  W.t_off = t_off;
  if (wall_id) *wall_id = (int32_t)I.walls.size();
  I.walls.push_back(W);
  return DEM_OK;
}

int dem_add_cone_wall(dem_ctx* c, int32_t instance, const double axis_point[3],
                      const double axis_dir[3], double radius0, double slope, double s_min,
                      double s_max, int32_t inside, int32_t material, double omega, double t_on,
                      double t_off, int32_t* wall_id) {
  if (!c || !axis_point || !axis_dir) return set_err(DEM_EINVAL, "null argument");
  if (int rc = check_instance(c, instance)) return rc;
  Instance& I = c->inst[(size_t)instance];
  if ((int)I.walls.size() >= kMaxWalls) return set_err(DEM_EINVAL, "at most 32 walls");
  if (material < 0 || material >= kMaxTypes || !I.mat_set[material])
    return set_err(DEM_EINVAL, "wall material %d not set", material);
  if (!(s_max >= s_min) || !std::isfinite(slope) || !std::isfinite(radius0))
    return set_err(DEM_EINVAL, "cone needs finite radius0 and slope and s_max >= s_min");
  if (!(radius0 + slope * s_min > 0.0) || !(radius0 + slope * s_max > 0.0))
    return set_err(DEM_EINVAL, "cone radius must stay > 0 over [s_min, s_max]");
  if (I.staged) return set_err(DEM_ESTATE, "walls are added before dem_set_particles");
  WallDev W;
  memset(&W, 0, sizeof(W));
  W.kind = 2;
  if (!unit3(axis_dir, W.nrm)) return set_err(DEM_EINVAL, "zero or non-finite axis");
  for (int k = 0; k < 3; ++k) {
    W.p[k] = axis_point[k];
    W.ax[k] = axis_point[k];
    W.omega[k] = omega * W.nrm[k];
  }
  W.radius = radius0;
  W.slope = slope;
  W.q = sqrt(1.0 + slope * slope);
  W.smin = s_min;
  W.smax = s_max;
  W.inside = inside ? 1 : 0;
  W.material = material;
  W.t_on = t_on;
  W.t_off = t_off;
  if (wall_id) *wall_id = (int32_t)I.walls.size();
  I.walls.push_back(W);
  return DEM_OK;
}

int dem_add_mesh_wall(dem_ctx* c, int32_t instance, int64_t n_vertices, const double* vertices,
                      int64_t n_triangles, const int32_t* triangles, int32_t material,
                      const double axis_point[3], const double omega[3], double t_on,
                      double t_off, int32_t* wall_id) {
  if (!c || !vertices || !triangles) return set_err(DEM_EINVAL, "null argument");
  if (int rc = check_instance(c, instance)) return rc;
  Instance& I = c->inst[(size_t)instance];
  if ((int)I.walls.size() >= kMaxWalls) return set_err(DEM_EINVAL, "at most 32 walls");
  if (material < 0 || material >= kMaxTypes || !I.mat_set[material])
    return set_err(DEM_EINVAL, "wall material %d not set", material);
  if (I.staged) return set_err(DEM_ESTATE, "walls are added before dem_set_particles");
  if (n_vertices < 3 || n_vertices > ((int64_t)1 << 30))
    return set_err(DEM_EINVAL, "n_vertices must be in [3, 2^30]");
  if (n_triangles < 1 || (int64_t)I.tris.size() + n_triangles > kMaxMeshTriangles)
    return set_err(DEM_EINVAL, "1 to %d triangles per instance", kMaxMeshTriangles);
  for (int64_t k = 0; k < 3 * n_vertices; ++k)
    if (!std::isfinite(vertices[k])) return set_err(DEM_EINVAL, "non-finite vertex");
  const int wl = (int)I.walls.size();
  std::vector<HostTri> add((size_t)n_triangles);
  for (int64_t f = 0; f < n_triangles; ++f) {
    HostTri& h = add[(size_t)f];
    h.wall = wl;
    for (int cc = 0; cc < 3; ++cc) {
      const int32_t v = triangles[3 * f + cc];
      if (v < 0 || v >= n_vertices)
        return set_err(DEM_EINVAL, "triangle %lld: corner index out of range", (long long)f);
      h.v[cc] = v;
      for (int k = 0; k < 3; ++k) h.p[cc][k] = vertices[3 * (int64_t)v + k];
    }
    const double e01[3] = {h.p[1][0] - h.p[0][0], h.p[1][1] - h.p[0][1], h.p[1][2] - h.p[0][2]};
    const double e02[3] = {h.p[2][0] - h.p[0][0], h.p[2][1] - h.p[0][1], h.p[2][2] - h.p[0][2]};
    const double N[3] = {e01[1] * e02[2] - e01[2] * e02[1], e01[2] * e02[0] - e01[0] * e02[2],
                         e01[0] * e02[1] - e01[1] * e02[0]};
    const double len = sqrt((N[0] * N[0] + N[1] * N[1]) + N[2] * N[2]);
    if (!(len > 0.0) || !std::isfinite(len))
      return set_err(DEM_EINVAL, "triangle %lld is degenerate", (long long)f);
  }
  WallDev W;
  memset(&W, 0, sizeof(W));
  W.kind = 3;
  for (int k = 0; k < 3; ++k) {
    W.p[k] = vertices[k];
    W.ax[k] = axis_point ? axis_point[k] : vertices[k];
    W.omega[k] = omega ? omega[k] : 0.0;
  }
  W.material = material;
  W.t_on = t_on;
  W.t_off = t_off;
  I.tris.insert(I.tris.end(), add.begin(), add.end());
  if (wall_id) *wall_id = wl;
  I.walls.push_back(W);
  return DEM_OK;
}

int dem_get_mesh_contacts(dem_ctx* c, int32_t instance, int64_t cap, int64_t* triples,
                          double* delta_t, int64_t* n_out) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (cap < 0) return set_err(DEM_EINVAL, "cap must be >= 0");
  if (!c->has_mesh) {
    if (n_out) *n_out = 0;
    return DEM_OK;
  }
  if (int rc = wait_user(c)) return rc;
  HostSnapshot h;
  if (int rc = snapshot(c, h, false, false, false)) return rc;
  const size_t n = (size_t)c->n;
  std::vector<int> tr(n * kMeshSlots);
  std::vector<double> th(n * kMeshSlots * 3);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(tr.data(), c->mtri[c->pcur], tr.size() * sizeof(int),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(th.data(), c->mhist[c->pcur], th.size() * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
  }
  if (int rc = finish(c)) return rc;
  struct Rec {
    int64_t i, tri;
    double d[3];
  };
  std::vector<Rec> out;
  const Instance& In = c->inst[(size_t)instance];
  for (size_t p = 0; p < n; ++p) {
    if ((h.info[p] >> kInstShift) != instance) continue;
    for (int sl = 0; sl < kMeshSlots; ++sl) {
      const int t = tr[(size_t)sl * n + p];
      if (t < 0) break;
      Rec r;
      r.i = h.gid[p] - In.p_begin;
      r.tri = t;
      for (int k = 0; k < 3; ++k) r.d[k] = th[(size_t)(3 * sl + k) * n + p];
      out.push_back(r);
    }
  }
  std::sort(out.begin(), out.end(),
            [](const Rec& a, const Rec& b) { return a.i != b.i ? a.i < b.i : a.tri < b.tri; });
  if (n_out) *n_out = (int64_t)out.size();
  if ((int64_t)out.size() > cap)
    return set_err(DEM_EINVAL, "cap %lld < %zu mesh contacts", (long long)cap, out.size());
  for (size_t m = 0; m < out.size(); ++m) {
    if (triples) {
      triples[3 * m] = out[m].i;
      triples[3 * m + 1] = c->tri_wall[(size_t)out[m].tri];
      triples[3 * m + 2] = c->tri_local[(size_t)out[m].tri];
    }
    if (delta_t)
      for (int k = 0; k < 3; ++k) delta_t[3 * m + k] = out[m].d[k];
  }
  return DEM_OK;
}

int dem_set_wall_motion(dem_ctx* c, int32_t instance, int32_t wall_id,
                        const double velocity[3]) {
  if (!c || !velocity) return set_err(DEM_EINVAL, "null argument");
  if (int rc = check_instance(c, instance)) return rc;
  Instance& I = c->inst[(size_t)instance];
  if (wall_id < 0 || wall_id >= (int32_t)I.walls.size())
    return set_err(DEM_EINVAL, "instance %d has no wall %d", instance, wall_id);
  if (I.staged) return set_err(DEM_ESTATE, "wall motion is set before dem_set_particles");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(velocity[k])) return set_err(DEM_EINVAL, "non-finite wall velocity");
  for (int k = 0; k < 3; ++k) I.walls[(size_t)wall_id].vel[k] = velocity[k];
  return DEM_OK;
}

int dem_set_particles(dem_ctx* c, int32_t instance, int64_t n, const double* pos,
                      const double* vel, const double* omega, const double* radius,
                      const int32_t* type) {
  if (!c) return set_err(DEM_EINVAL, "null context");
  if (int rc = check_instance(c, instance)) return rc;
  if (n < 0 || n > kMaxParticles) return set_err(DEM_EINVAL, "n out of range (at most 2^29)");
  if (n > 0 && (!pos || !radius)) return set_err(DEM_EINVAL, "pos and radius are required");
  Instance& I = c->inst[(size_t)instance];
  for (int64_t i = 0; i < n; ++i) {
    if (!(radius[i] > 0.0) || !std::isfinite(radius[i]))
      return set_err(DEM_EINVAL, "radius[%lld] must be > 0", (long long)i);
    int t = type ? type[i] : 0;
    if (t < 0 || t >= kMaxTypes || !I.mat_set[t])
      return set_err(DEM_EINVAL, "particle %lld has type %d without material", (long long)i, t);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(pos[3 * i + k]) || (vel && !std::isfinite(vel[3 * i + k])) ||
          (omega && !std::isfinite(omega[3 * i + k])))
        return set_err(DEM_EINVAL, "non-finite state of particle %lld", (long long)i);
  }
  // setting particles again restarts the batch from the staged inputs
  free_particles(c);
  c->failed = false;
  c->fail_code = 0;
  I.n = n;
  I.pos.assign(pos, pos + 3 * n);
  I.rad.assign(radius, radius + n);
  I.vel.assign(vel ? vel : pos, vel ? vel + 3 * n : pos);
  I.omg.assign(omega ? omega : pos, omega ? omega + 3 * n : pos);
  I.type.assign(type ? type : (const int32_t*)nullptr, type ? type + n : (const int32_t*)nullptr);
  I.staged = true;
  if (c->inst.size() == 1) return commit(c);
  return DEM_OK;
}

int dem_set_instance_domain(dem_ctx* c, int32_t instance, const double lo[3],
                            const double hi[3]) {
  if (!c || !lo || !hi) return set_err(DEM_EINVAL, "null argument");
  if (int rc = check_instance(c, instance)) return rc;
  Instance& I = c->inst[(size_t)instance];
  if (I.staged) return set_err(DEM_ESTATE, "the domain is set before dem_set_particles");
  for (int k = 0; k < 3; ++k)
    if (!(hi[k] > lo[k]) || !std::isfinite(lo[k]) || !std::isfinite(hi[k]))
      return set_err(DEM_EINVAL, "empty domain along axis %d", k);
  for (int k = 0; k < 3; ++k) {
    I.lo[k] = lo[k];
    I.hi[k] = hi[k];
  }
  I.own_domain = true;
  return DEM_OK;
}

int dem_commit(dem_ctx* c) {
  if (!c) return set_err(DEM_EINVAL, "null context");
  if (c->ready) return DEM_OK;
  return require_ready(c);
}

int dem_set_particles_device(dem_ctx* c, int32_t instance, int64_t n, const double* pos,
                             const double* vel, const double* omega, const double* radius,
                             const int32_t* type) {
  if (!c) return set_err(DEM_EINVAL, "null context");
  if (n < 0 || n > kMaxParticles) return set_err(DEM_EINVAL, "n out of range (at most 2^29)");
  // validation needs the values on the host; stage them once
  std::vector<double> hp(3 * (size_t)n), hv, hw, hr((size_t)n);
  std::vector<int32_t> ht;
  if (int rc = wait_user(c)) return rc;
  if (n > 0) {
    if (!pos || !radius) return set_err(DEM_EINVAL, "pos and radius are required");
    HIPCHK(hipMemcpyAsync(hp.data(), pos, hp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(hr.data(), radius, hr.size() * 8, hipMemcpyDeviceToHost, c->stream));
    if (vel) {
      hv.resize(3 * (size_t)n);
      HIPCHK(hipMemcpyAsync(hv.data(), vel, hv.size() * 8, hipMemcpyDeviceToHost, c->stream));
    }
    if (omega) {
      hw.resize(3 * (size_t)n);
      HIPCHK(hipMemcpyAsync(hw.data(), omega, hw.size() * 8, hipMemcpyDeviceToHost, c->stream));
    }
    if (type) {
      ht.resize((size_t)n);
      HIPCHK(hipMemcpyAsync(ht.data(), type, ht.size() * 4, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return dem_set_particles(c, instance, n, hp.data(), vel ? hv.data() : nullptr,
                           omega ? hw.data() : nullptr, hr.data(), type ? ht.data() : nullptr);
}

int dem_step(dem_ctx* c, int64_t n_steps) {
  if (int rc = require_ready(c)) return rc;
  if (n_steps < 0) return set_err(DEM_EINVAL, "n_steps must be >= 0");
  if (c->failed)
    return set_err(DEM_ESTATE, "a previous error (%d) is sticky; call dem_set_particles",
                   c->fail_code);
  if (n_steps == 0 || c->n == 0) {
    c->step += n_steps;
    return DEM_OK;
  }
  int rc = wait_user(c);
  if (rc) return rc;
  if (c->dynamic) {
    if ((rc = step_dynamic(c, n_steps))) return rc;
    c->step += n_steps;
    int flags = 0;
    if ((rc = read_flags(c, &flags))) return rc;
    if ((rc = collect_timing(c))) return rc;
    return flags_to_error(c, flags);
  }
  const int64_t K = c->cfg.rebuild_interval;
  const int64_t s0 = c->step, s_end = s0 + n_steps;
  const bool graphs = !c->timing;
  if (graphs && n_steps >= K && (rc = prepare_chunk_graphs(c))) return rc;
  if (c->cfg.integrator == 0) {
    HIPCHK(launch_kick_drift(c->sp, c->d_inst, pbufs(c, c->cur), c->info[c->pcur],
                             c->F[c->pcur], c->T[c->pcur], nullptr, c->d_clock,
                             s0 + 1 - c->host_base, c->stream));
    int64_t s = s0 + 1;
    while (s <= s_end) {
      if (graphs && s % K == 0 && s + K - 1 <= s_end - 1) {
        if ((rc = launch_chunk(c, s))) return rc;
        s += K;
        continue;
      }
      if (s % K == 0 && (rc = eager_rebuild(c, s - c->host_base))) return rc;
      if ((rc = eager_force(c, s < s_end ? 0 : 1, s - c->host_base))) return rc;
      s += 1;
    }
  } else {
    int64_t s = s0 + 1;
    while (s <= s_end) {
      if (graphs && (s - 1) % K == 0 && s + K - 1 <= s_end) {
        if ((rc = launch_chunk(c, s - 1))) return rc;
        s += K;
        continue;
      }
      if ((rc = eager_force(c, 2, (s - 1) - c->host_base))) return rc;
      if (s % K == 0 && (rc = eager_rebuild(c, s - c->host_base))) return rc;
      s += 1;
    }
  }
  c->step = s_end;
  int flags = 0;
  if ((rc = read_flags(c, &flags))) return rc;
  if ((rc = collect_timing(c))) return rc;
  return flags_to_error(c, flags);
}

int dem_get_state(dem_ctx* c, int32_t instance, double* pos, double* vel, double* omega,
                  uint8_t* active, double* time_out) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (int rc = wait_user(c)) return rc;
  HostSnapshot h;
  if (int rc = snapshot(c, h, pos != nullptr, vel != nullptr, omega != nullptr)) return rc;
  const int64_t base = c->inst[(size_t)instance].p_begin;
  for (int p = 0; p < c->n; ++p) {
    if ((h.info[p] >> kInstShift) != instance) continue;
    const int64_t g = h.gid[p] - base;
    if (pos) {
      pos[3 * g] = h.pos[p].x;
      pos[3 * g + 1] = h.pos[p].y;
      pos[3 * g + 2] = h.pos[p].z;
    }
    if (vel) {
      vel[3 * g] = h.vel[p].x;
      vel[3 * g + 1] = h.vel[p].y;
      vel[3 * g + 2] = h.vel[p].z;
    }
    if (omega) {
      omega[3 * g] = h.omg[p].x;
      omega[3 * g + 1] = h.omg[p].y;
      omega[3 * g + 2] = h.omg[p].z;
    }
    if (active) active[g] = (h.info[p] & kInactive) ? 0 : 1;
  }
  if (time_out) *time_out = (double)c->step * c->cfg.dt;
  return DEM_OK;
}

int dem_get_state_device(dem_ctx* c, int32_t instance, double* pos, double* vel, double* omega,
                         uint8_t* active) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  const size_t n = (size_t)c->inst[(size_t)instance].n;
  std::vector<double> p(pos ? 3 * n : 0), v(vel ? 3 * n : 0), w(omega ? 3 * n : 0);
  std::vector<uint8_t> a(active ? n : 0);
  int rc = dem_get_state(c, instance, pos ? p.data() : nullptr, vel ? v.data() : nullptr,
                         omega ? w.data() : nullptr, active ? a.data() : nullptr, nullptr);
  if (rc) return rc;
  if (pos) HIPCHK(hipMemcpyAsync(pos, p.data(), p.size() * 8, hipMemcpyHostToDevice, c->stream));
  if (vel) HIPCHK(hipMemcpyAsync(vel, v.data(), v.size() * 8, hipMemcpyHostToDevice, c->stream));
  if (omega) HIPCHK(hipMemcpyAsync(omega, w.data(), w.size() * 8, hipMemcpyHostToDevice, c->stream));
  if (active) HIPCHK(hipMemcpyAsync(active, a.data(), a.size(), hipMemcpyHostToDevice, c->stream));
  return finish(c);
}

int dem_get_forces(dem_ctx* c, int32_t instance, double* force, double* torque) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (int rc = wait_user(c)) return rc;
  HostSnapshot h;
  if (int rc = snapshot(c, h, false, false, false)) return rc;
  const size_t n = (size_t)c->n;
  std::vector<double4> F(n), T(n);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(F.data(), c->F[c->pcur], n * sizeof(double4), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(T.data(), c->T[c->pcur], n * sizeof(double4), hipMemcpyDeviceToHost,
                          c->stream));
  }
  if (int rc = finish(c)) return rc;
  const int64_t base = c->inst[(size_t)instance].p_begin;
  for (size_t p = 0; p < n; ++p) {
    if ((h.info[p] >> kInstShift) != instance) continue;
    const int64_t g = h.gid[p] - base;
    if (force) {
      force[3 * g] = F[p].x;
      force[3 * g + 1] = F[p].y;
      force[3 * g + 2] = F[p].z;
    }
    if (torque) {
      torque[3 * g] = T[p].x;
      torque[3 * g + 1] = T[p].y;
      torque[3 * g + 2] = T[p].z;
    }
  }
  return DEM_OK;
}

int dem_get_contacts(dem_ctx* c, int32_t instance, int64_t cap, int64_t* pairs, double* delta_t,
                     uint8_t* touching, int64_t* n_out) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (cap < 0) return set_err(DEM_EINVAL, "cap must be >= 0");
  if (int rc = wait_user(c)) return rc;
  HostSnapshot h;
  if (int rc = snapshot(c, h, true, false, false)) return rc;
  const size_t n = (size_t)c->n;
  std::vector<int> rl(n), nb((size_t)c->cap);
  std::vector<double> hs((size_t)c->cap * 3);
  const int L = c->pcur;
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(rl.data(), c->rowlen[L], n * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(nb.data(), c->nbr[L], (size_t)c->cap * sizeof(int),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(hs.data(), c->hist[L], (size_t)c->cap * 3 * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
  }
  if (int rc = finish(c)) return rc;
  struct Rec {
    int64_t i, j;
    double d[3];
    uint8_t t;
  };
  std::vector<Rec> out;
  const int64_t base = c->inst[(size_t)instance].p_begin;
  for (size_t p = 0; p < n; ++p) {
    if ((h.info[p] >> kInstShift) != instance) continue;
    for (int k = 0; k < rl[p]; ++k) {
      const int64_t e = nbr_entry((int)p, k, c->max_nb);
      const int jr = nb[(size_t)e];
      const int q = jr & 0x7fffffff;  // bit 31: touching at the last evaluation
      if (h.gid[p] >= h.gid[q]) continue;
      Rec r;
      r.i = h.gid[p] - base;
      r.j = h.gid[q] - base;
      const bool has_hist = (jr & (int)0x80000000u) != 0;
      r.d[0] = has_hist ? hs[(size_t)e] : 0.0;
      r.d[1] = has_hist ? hs[(size_t)c->cap + (size_t)e] : 0.0;
      r.d[2] = has_hist ? hs[2 * (size_t)c->cap + (size_t)e] : 0.0;
      const double dx = h.pos[q].x - h.pos[p].x, dy = h.pos[q].y - h.pos[p].y,
                   dz = h.pos[q].z - h.pos[p].z;
      const double rsum = h.pos[p].w + h.pos[q].w;
      r.t = ((dx * dx + dy * dy) + dz * dz) < rsum * rsum ? 1 : 0;
      out.push_back(r);
    }
  }
  std::sort(out.begin(), out.end(),
            [](const Rec& a, const Rec& b) { return a.i != b.i ? a.i < b.i : a.j < b.j; });
  if (n_out) *n_out = (int64_t)out.size();
  if ((int64_t)out.size() > cap) return set_err(DEM_EINVAL, "cap %lld < %zu contacts", (long long)cap, out.size());
  for (size_t m = 0; m < out.size(); ++m) {
    if (pairs) {
      pairs[2 * m] = out[m].i;
      pairs[2 * m + 1] = out[m].j;
    }
    if (delta_t)
      for (int k = 0; k < 3; ++k) delta_t[3 * m + k] = out[m].d[k];
    if (touching) touching[m] = out[m].t;
  }
  return DEM_OK;
}

int dem_restore(dem_ctx* c, int32_t instance, int64_t n_pairs, const int64_t* pairs,
                const double* delta_t, int64_t n_wall, const int64_t* wall_pairs,
                const double* wall_delta_t, const double* force, const double* torque,
                int64_t step) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (c->failed) return set_err(DEM_ESTATE, "a previous error is sticky");
  if (n_pairs < 0 || n_wall < 0) return set_err(DEM_EINVAL, "negative count");
  if ((n_pairs > 0 && (!pairs || !delta_t)) || (n_wall > 0 && (!wall_pairs || !wall_delta_t)))
    return set_err(DEM_EINVAL, "null array");
  if (int rc = wait_user(c)) return rc;
  const bool moving = c->n > 0 && wall_rate(c) > 0.0;
  if (step >= 0 && moving) {
    c->step = step;
    c->host_base = step;
    HIPCHK(hipMemcpyAsync(c->d_clock, &c->host_base, sizeof(int64_t), hipMemcpyHostToDevice,
                          c->stream));
    // translating walls: search again with the walls where they are at the
    // restored time (the lists were built with them elsewhere)
    {
      if (int rc = enqueue_rebuild(c, 0, 1, 0, next_eval_rel(c))) return rc;
      c->dyn_acc = 0.0;
      c->dyn_wacc = 0.0;
      int flags = 0;
      if (int rc = read_flags(c, &flags)) return rc;
      if (int rc = flags_to_error(c, flags)) return rc;
    }
  }
  HostSnapshot h;
  if (int rc = snapshot(c, h, true, false, false)) return rc;
  const size_t n = (size_t)c->n;
  const int L = c->pcur;
  const Instance& In = c->inst[(size_t)instance];
  const int64_t base = In.p_begin;
  std::vector<int> where((size_t)In.n, -1);  // instance gid -> sorted index
  for (size_t p = 0; p < n; ++p)
    if ((h.info[p] >> kInstShift) == instance) where[(size_t)(h.gid[p] - base)] = (int)p;
  std::vector<int> rl(n), nb((size_t)c->cap);
  std::vector<double> hs((size_t)c->cap * 3);
  std::vector<int> w(n * kWallSlots);
  std::vector<double> wh(n * kWallSlots * 3);
  std::vector<double4> F(n), T(n);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(rl.data(), c->rowlen[L], n * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(nb.data(), c->nbr[L], (size_t)c->cap * sizeof(int),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(hs.data(), c->hist[L], (size_t)c->cap * 3 * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(w.data(), c->wid[L], w.size() * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(wh.data(), c->whist[L], wh.size() * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(F.data(), c->F[L], n * sizeof(double4), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(T.data(), c->T[L], n * sizeof(double4), hipMemcpyDeviceToHost,
                          c->stream));
  }
  if (int rc = finish(c)) return rc;
  auto sorted = [&](int64_t g) -> int {
    return g >= 0 && g < In.n ? where[(size_t)g] : -1;
  };
  // entries of this instance start without history, as after a search
  for (size_t p = 0; p < n; ++p) {
    if ((h.info[p] >> kInstShift) != instance) continue;
    for (int a = 0; a < 3 * kWallSlots; ++a) wh[(size_t)a * n + p] = 0.0;
    for (int k = 0; k < rl[p]; ++k) {
      const size_t e = (size_t)nbr_entry((int)p, k, c->max_nb);
      nb[e] &= 0x7fffffff;
      hs[e] = hs[(size_t)c->cap + e] = hs[2 * (size_t)c->cap + e] = 0.0;
    }
  }
  // a pair that does not touch at the current positions keeps no history:
  // the first force evaluation, here, would restart it at zero (and the row
  // cuts of the force kernel may not read its entry until it can touch)
  auto set_entry = [&](int p, int q, double sgn, const double* d) -> bool {
    for (int k = 0; k < rl[(size_t)p]; ++k) {
      const size_t e = (size_t)nbr_entry(p, k, c->max_nb);
      if ((nb[e] & 0x7fffffff) != q) continue;
      const double4 xp = h.pos[(size_t)p], xq = h.pos[(size_t)q];
      const double dx = xq.x - xp.x, dy = xq.y - xp.y, dz = xq.z - xp.z;
      const double rsum = xp.w + xq.w;
      if (!(((dx * dx + dy * dy) + dz * dz) < rsum * rsum)) return true;
      nb[e] = q | (int)0x80000000u;
      for (int a = 0; a < 3; ++a) hs[(size_t)a * (size_t)c->cap + e] = sgn * d[a];
      return true;
    }
    return false;
  };
  for (int64_t m = 0; m < n_pairs; ++m) {
    const int p = sorted(pairs[2 * m]), q = sorted(pairs[2 * m + 1]);
    if (p < 0 || q < 0 || p == q)
      return set_err(DEM_EINVAL, "pair %lld: particle out of range", (long long)m);
    // history of i -> j, and the exact negative from j's side
    if (!set_entry(p, q, 1.0, delta_t + 3 * m) || !set_entry(q, p, -1.0, delta_t + 3 * m))
      return set_err(DEM_EINVAL, "pair (%lld, %lld) is not in the contact list",
                     (long long)pairs[2 * m], (long long)pairs[2 * m + 1]);
  }
  for (int64_t m = 0; m < n_wall; ++m) {
    const int p = sorted(wall_pairs[2 * m]);
    const int64_t wall = wall_pairs[2 * m + 1];
    if (p < 0 || wall < 0 || wall >= (int64_t)In.walls.size())
      return set_err(DEM_EINVAL, "wall contact %lld out of range", (long long)m);
    bool found = false;
    for (int sl = 0; sl < kWallSlots && !found; ++sl) {
      if (w[(size_t)sl * n + (size_t)p] != In.w_begin + (int)wall) continue;
      for (int a = 0; a < 3; ++a) wh[(size_t)(3 * sl + a) * n + (size_t)p] = wall_delta_t[3 * m + a];
      found = true;
    }
    if (!found)
      return set_err(DEM_EINVAL, "particle %lld is not a candidate of wall %lld",
                     (long long)wall_pairs[2 * m], (long long)wall);
  }
  for (int64_t g = 0; g < In.n && (force || torque); ++g) {
    const size_t p = (size_t)where[(size_t)g];
    if (force) F[p] = make_double4(force[3 * g], force[3 * g + 1], force[3 * g + 2], 0.0);
    if (torque) T[p] = make_double4(torque[3 * g], torque[3 * g + 1], torque[3 * g + 2], 0.0);
  }
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(c->nbr[L], nb.data(), (size_t)c->cap * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->hist[L], hs.data(), (size_t)c->cap * 3 * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->whist[L], wh.data(), wh.size() * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->F[L], F.data(), n * sizeof(double4), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(c->T[L], T.data(), n * sizeof(double4), hipMemcpyHostToDevice,
                          c->stream));
  }
  if (step >= 0 && !moving) {
    c->step = step;
    c->host_base = step;
    HIPCHK(hipMemcpyAsync(c->d_clock, &c->host_base, sizeof(int64_t), hipMemcpyHostToDevice,
                          c->stream));
  }
  return finish(c);
}

int dem_restore_mesh_contacts(dem_ctx* c, int32_t instance, int64_t n_tri,
                              const int64_t* triples, const double* delta_t) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (c->failed) return set_err(DEM_ESTATE, "a previous error is sticky");
  if (n_tri < 0) return set_err(DEM_EINVAL, "negative count");
  if (n_tri > 0 && (!triples || !delta_t)) return set_err(DEM_EINVAL, "null array");
  if (!c->has_mesh) {
    if (n_tri > 0) return set_err(DEM_EINVAL, "no mesh walls");
    return DEM_OK;
  }
  if (int rc = wait_user(c)) return rc;
  HostSnapshot h;
  if (int rc = snapshot(c, h, true, false, false)) return rc;
  const size_t n = (size_t)c->n;
  const int L = c->pcur;
  const Instance& In = c->inst[(size_t)instance];
  std::vector<int> where((size_t)In.n, -1);
  for (size_t p = 0; p < n; ++p)
    if ((h.info[p] >> kInstShift) == instance) where[(size_t)(h.gid[p] - In.p_begin)] = (int)p;
  std::vector<int> tr(n * kMeshSlots);
  std::vector<double> th(n * kMeshSlots * 3);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(tr.data(), c->mtri[L], tr.size() * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(th.data(), c->mhist[L], th.size() * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
  }
  if (int rc = finish(c)) return rc;
  for (size_t p = 0; p < n; ++p) {
    if ((h.info[p] >> kInstShift) != instance) continue;
    for (int a = 0; a < 3 * kMeshSlots; ++a) th[(size_t)a * n + p] = 0.0;
  }
  for (int64_t m = 0; m < n_tri; ++m) {
    const int64_t g = triples[3 * m], wl = triples[3 * m + 1], tl = triples[3 * m + 2];
    const int p = g >= 0 && g < In.n ? where[(size_t)g] : -1;
    if (p < 0 || wl < 0 || wl >= (int64_t)In.walls.size() || In.walls[(size_t)wl].kind != 3 ||
        tl < 0 || tl >= In.walls[(size_t)wl].tri_count)
      return set_err(DEM_EINVAL, "mesh contact %lld out of range", (long long)m);
    const int gt = In.walls[(size_t)wl].tri_begin + (int)tl;
    bool found = false;
    for (int sl = 0; sl < kMeshSlots && !found; ++sl) {
      if (tr[(size_t)sl * n + (size_t)p] != gt) continue;
      for (int a = 0; a < 3; ++a) th[(size_t)(3 * sl + a) * n + (size_t)p] = delta_t[3 * m + a];
      found = true;
    }
    if (!found)
      return set_err(DEM_EINVAL, "particle %lld is not a candidate of triangle %lld of wall %lld",
                     (long long)g, (long long)tl, (long long)wl);
  }
  if (n > 0)
    HIPCHK(hipMemcpyAsync(c->mhist[L], th.data(), th.size() * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
  return finish(c);
}

}  // extern "C"

namespace {

// Candidate pairs of an instance into caller device buffers; scratch is
// device memory of at least pairs_scratch_ints(c->n) ints.
int contacts_device(dem_ctx* c, int32_t instance, int64_t cap, int64_t* pairs,
                    double* delta_t, uint8_t* touching, int64_t* n_out, int* scratch) {
  const int L = c->pcur;
  const int64_t nb = (c->n + kBlock - 1) / kBlock;
  HIPCHK(launch_pairs_count(c->sp, instance, c->info[L], c->gid[L], nlist(c, L), scratch,
                            c->stream));
  int total = 0;
  HIPCHK(hipMemcpyAsync(&total, scratch + 2 * nb, sizeof(int), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (n_out) *n_out = total;
  if (total > cap)
    return set_err(DEM_EINVAL, "cap %lld < %d contacts", (long long)cap, total);
  HIPCHK(launch_pairs_fill(c->sp, instance, (int)c->inst[(size_t)instance].p_begin,
                           c->pos[c->cur], c->info[L], c->gid[L], nlist(c, L), scratch, pairs,
                           delta_t, touching, c->stream));
  return finish(c);
}

int contacts_device_check(dem_ctx* c, int32_t instance, int64_t cap) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (cap < 0) return set_err(DEM_EINVAL, "cap must be >= 0");
  if (c->cap >= ((int64_t)1 << 31))
    return set_err(DEM_EINVAL, "%lld list entries: too many for 32-bit pair offsets",
                   (long long)c->cap);
  return wait_user(c);
}

}  // namespace

extern "C" {

int dem_get_contacts_device(dem_ctx* c, int32_t instance, int64_t cap, int64_t* pairs,
                            double* delta_t, uint8_t* touching, int64_t* n_out) {
  if (int rc = contacts_device_check(c, instance, cap)) return rc;
  int* scratch = nullptr;
  const size_t bytes = (size_t)pairs_scratch_ints(c->n) * sizeof(int);
  HIPCHK(hipMalloc((void**)&scratch, bytes));
  const int rc = contacts_device(c, instance, cap, pairs, delta_t, touching, n_out, scratch);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(scratch);
  return rc;
}

// ------------------------------------------------------ allocation-free variant
//
// dem_get_contacts_device_noalloc keeps its workspace in `scratch`, a
// file-scope device array: one copy per GPU, held until the process ends,
// shared by every call on that GPU (calls that overlap on one GPU race).
// On the host the array's name stands for a host-side shadow, not a device
// address, so host code never hands it to a kernel or a copy: it uses the
// device address hipGetSymbolAddress returns, looked up once per device with
// that device current.  Every word the call reads is written by the same
// call first, so nothing needs clearing between calls.

}  // extern "C"

namespace {

constexpr int kNoAllocMaxParticles = 1 << 24;
constexpr int64_t kNoAllocBlocks = kNoAllocMaxParticles / kBlock;
// block counts, their scan (one more word), the scan's tile sums
constexpr int64_t kNoAllocScratchInts =
    kNoAllocBlocks + (kNoAllocBlocks + 2) + ((kNoAllocBlocks + 1 + 1023) / 1024 + 1);
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) int scratch[kNoAllocScratchInts];

std::mutex g_scratch_mu;
int* g_scratch_dev[kNoAllocMaxDevices] = {};

// device address of `scratch` on device dev (current)
int noalloc_scratch(int dev, int** out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return set_err(DEM_ENODEV, "device %d beyond the %d the workspace table holds", dev,
                   kNoAllocMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_err(DEM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                     hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<int*>(p);
  }
  *out = g_scratch_dev[dev];
  return DEM_OK;
}

}  // namespace

extern "C" {

int dem_get_contacts_device_noalloc(dem_ctx* c, int32_t instance, int64_t cap, int64_t* pairs,
                                    double* delta_t, uint8_t* touching, int64_t* n_out) {
  if (int rc = contacts_device_check(c, instance, cap)) return rc;
  if (pairs_scratch_ints(c->n) > kNoAllocScratchInts)
    return set_err(DEM_EINVAL, "%d particles: the allocation-free workspace holds %d", c->n,
                   kNoAllocMaxParticles);
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != c->device)
    return set_err(DEM_EINVAL, "the context lives on device %d but device %d is current",
                   c->device, dev);
  int* ws = nullptr;
  if (int rc = noalloc_scratch(dev, &ws)) return rc;
  return contacts_device(c, instance, cap, pairs, delta_t, touching, n_out, ws);
}

int dem_record_contact_forces(dem_ctx* c, int32_t enable) {
  if (!c) return set_err(DEM_EINVAL, "null context");
  if (int rc = wait_user(c)) return rc;
  const bool on = enable != 0;
  if (on == c->record_pf) return DEM_OK;
  destroy_graphs(c);  // the captured force launches hold the record's address
  HIPCHK(hipStreamSynchronize(c->stream));
  c->record_pf = on;
  if (!c->ready) return DEM_OK;
  if (!on) {
    dfree(c, c->pair_force);
    c->pair_force = nullptr;
    return DEM_OK;
  }
  const size_t m = (size_t)std::max<int64_t>(c->cap, 1) * 3;
  if (int rc = dalloc_t(c, &c->pair_force, m)) {
    c->record_pf = false;
    return rc;
  }
  HIPCHK(launch_fill_i32((int*)c->pair_force, 0, (int64_t)m * 2, c->stream));
  return finish(c);
}

int dem_get_contact_forces(dem_ctx* c, int32_t instance, int64_t cap, int64_t* pairs,
                           double* force, int64_t* n_out) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (cap < 0) return set_err(DEM_EINVAL, "cap must be >= 0");
  if (!c->pair_force)
    return set_err(DEM_ESTATE, "call dem_record_contact_forces(ctx, 1) before dem_step");
  if (c->cfg.integrator == 1 && c->cfg.rebuild_interval > 0 &&
      c->step % c->cfg.rebuild_interval == 0 && c->step > 0)
    return set_err(DEM_ESTATE,
                   "the last step ended with a contact search (explicit Euler): the record "
                   "belongs to the previous contact list");
  if (int rc = wait_user(c)) return rc;
  HostSnapshot h;
  if (int rc = snapshot(c, h, false, false, false)) return rc;
  const size_t n = (size_t)c->n;
  std::vector<int> rl(n), nb((size_t)c->cap);
  std::vector<double> pf((size_t)c->cap * 3);
  const int L = c->pcur;
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(rl.data(), c->rowlen[L], n * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(nb.data(), c->nbr[L], (size_t)c->cap * sizeof(int),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(pf.data(), c->pair_force, (size_t)c->cap * 3 * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
  }
  if (int rc = finish(c)) return rc;
  struct Rec {
    int64_t i, j;
    double f[3];
  };
  std::vector<Rec> out;
  const int64_t base = c->inst[(size_t)instance].p_begin;
  for (size_t p = 0; p < n; ++p) {
    if ((h.info[p] >> kInstShift) != instance) continue;
    for (int k = 0; k < rl[p]; ++k) {
      const int64_t e = nbr_entry((int)p, k, c->max_nb);
      const int jr = nb[(size_t)e];
      const int q = jr & 0x7fffffff;
      if (h.gid[p] >= h.gid[q]) continue;
      // bit 31: the pair touched at the last evaluation, which wrote its force
      const bool t = (jr & (int)0x80000000u) != 0;
      Rec r;
      r.i = h.gid[p] - base;
      r.j = h.gid[q] - base;
      for (int a = 0; a < 3; ++a) r.f[a] = t ? pf[(size_t)a * (size_t)c->cap + (size_t)e] : 0.0;
      out.push_back(r);
    }
  }
  std::sort(out.begin(), out.end(),
            [](const Rec& a, const Rec& b) { return a.i != b.i ? a.i < b.i : a.j < b.j; });
  if (n_out) *n_out = (int64_t)out.size();
  if ((int64_t)out.size() > cap)
    return set_err(DEM_EINVAL, "cap %lld < %zu pairs", (long long)cap, out.size());
  for (size_t m = 0; m < out.size(); ++m) {
    if (pairs) {
      pairs[2 * m] = out[m].i;
      pairs[2 * m + 1] = out[m].j;
    }
    if (force)
      for (int a = 0; a < 3; ++a) force[3 * m + a] = out[m].f[a];
  }
  return DEM_OK;
}

int dem_get_wall_contacts(dem_ctx* c, int32_t instance, int64_t cap, int64_t* pairs,
                          double* delta_t, int64_t* n_out) {
  if (int rc = require_ready(c)) return rc;
  if (int rc = check_instance(c, instance)) return rc;
  if (cap < 0) return set_err(DEM_EINVAL, "cap must be >= 0");
  if (int rc = wait_user(c)) return rc;
  HostSnapshot h;
  if (int rc = snapshot(c, h, false, false, false)) return rc;
  const size_t n = (size_t)c->n;
  std::vector<int> w(n * kWallSlots);
  std::vector<double> wh(n * kWallSlots * 3);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(w.data(), c->wid[c->pcur], w.size() * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(wh.data(), c->whist[c->pcur], wh.size() * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
  }
  if (int rc = finish(c)) return rc;
  struct Rec {
    int64_t i, w;
    double d[3];
  };
  std::vector<Rec> out;
  const Instance& In = c->inst[(size_t)instance];
  for (size_t p = 0; p < n; ++p) {
    if ((h.info[p] >> kInstShift) != instance) continue;
    for (int s = 0; s < kWallSlots; ++s) {
      const int wi = w[(size_t)s * n + p];
      if (wi < 0) break;
      Rec r;
      r.i = h.gid[p] - In.p_begin;
      r.w = wi - In.w_begin;
      for (int k = 0; k < 3; ++k) r.d[k] = wh[(size_t)(3 * s + k) * n + p];
      out.push_back(r);
    }
  }
  std::sort(out.begin(), out.end(),
            [](const Rec& a, const Rec& b) { return a.i != b.i ? a.i < b.i : a.w < b.w; });
  if (n_out) *n_out = (int64_t)out.size();
  if ((int64_t)out.size() > cap) return set_err(DEM_EINVAL, "cap %lld < %zu wall contacts", (long long)cap, out.size());
  for (size_t m = 0; m < out.size(); ++m) {
    if (pairs) {
      pairs[2 * m] = out[m].i;
      pairs[2 * m + 1] = out[m].w;
    }
    if (delta_t)
      for (int k = 0; k < 3; ++k) delta_t[3 * m + k] = out[m].d[k];
  }
  return DEM_OK;
}

int dem_resort(dem_ctx* c) {
  if (int rc = require_ready(c)) return rc;
  if (c->failed) return set_err(DEM_ESTATE, "a previous error is sticky");
  if (int rc = wait_user(c)) return rc;
  if (c->n == 0) return DEM_OK;
  if (int rc = enqueue_rebuild(c, 0, 1, c->step - c->host_base, next_eval_rel(c))) return rc;
  c->dyn_acc = 0.0;
  c->dyn_wacc = 0.0;
  int flags = 0;
  if (int rc = read_flags(c, &flags)) return rc;
  return flags_to_error(c, flags);
}

int dem_get_stats(dem_ctx* c, dem_stats* out) {
  if (int rc = require_ready(c)) return rc;
  if (!out) return set_err(DEM_EINVAL, "null argument");
  if (int rc = wait_user(c)) return rc;
  unsigned long long v[4] = {0, 0, 0, 0};
  if (c->n > 0) {
    HIPCHK(launch_fill_i32((int*)c->d_stats, 0, 8, c->stream));
    HIPCHK(launch_stats(c->sp, c->pos[c->cur], c->info[c->pcur], nlist(c, c->pcur),
                        wslots(c, c->pcur), c->d_stats, c->stream));
    HIPCHK(hipMemcpyAsync(v, c->d_stats, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  }
  if (int rc = finish(c)) return rc;
  memset(out, 0, sizeof(*out));
  out->n_particles = c->n;
  out->n_active = (int64_t)v[0];
  out->n_list_entries = (int64_t)v[1];
  out->n_touching = (int64_t)v[2];
  out->n_wall_candidates = (int64_t)v[3];
  out->step = c->step;
  out->n_rebuilds = c->n_rebuilds;
  out->max_neighbors = c->max_nb;
  out->precision = c->cfg.precision;
  const Instance& I0 = c->inst[0];
  out->r_s = I0.rs;
  out->cell_size = I0.h;
  out->skin = I0.skin;
  out->d_max = I0.dmax;
  out->n_cells = c->n_keys;
  out->device_bytes = (int64_t)c->dev_bytes;
  return DEM_OK;
}

// Per-kernel timing for benchmarks: when enabled, dem_step launches eagerly
// (no graphs) with HIP events around every force launch and every contact
// search; dem_get_timing returns the accumulated milliseconds and counts.
// Autotuner: every trial is a stretch of ordinary steps of the simulation
// (or, for the cell size, forced re-sorts), so tuning advances the run with
// unchanged physics; only summation orders differ between settings.
int dem_autotune(dem_ctx* c, int32_t trial_steps, dem_tuning* out) {
  if (int rc = require_ready(c)) return rc;
  if (!out) return set_err(DEM_EINVAL, "null argument");
  if (trial_steps < 10 || trial_steps > 100000)
    return set_err(DEM_EINVAL, "trial_steps must be in [10, 100000]");
  if (c->failed) return set_err(DEM_ESTATE, "a previous error is sticky");
  memset(out, 0, sizeof(*out));
  for (int k = 0; k < 8; ++k) out->schedules[k] = -1;
  if (c->n == 0) {
    out->force_block = c->force_block;
    out->rebuild_interval = c->cfg.rebuild_interval;
    out->cell_factor = c->cell_factor;
    return DEM_OK;
  }
  const bool timing0 = c->timing;
  int64_t steps = 0;
  int rc = DEM_OK;
  auto forced_search = [&]() -> int {
    int r = enqueue_rebuild(c, 0, 1, c->step - c->host_base, next_eval_rel(c));
    if (r) return r;
    int flags = 0;
    if ((r = read_flags(c, &flags))) return r;
    c->dyn_acc = 0.0;
    c->dyn_wacc = 0.0;
    return flags_to_error(c, flags);
  };
  auto run = [&](int64_t n) -> int {
    steps += n;
    return dem_step(c, n);
  };
  // 1. threads per force workgroup: force-kernel time from HIP events
  const int blocks[3] = {64, 128, 256};
  double best = HUGE_VAL;
  int best_block = c->force_block;
  for (int k = 0; k < 3; ++k) {
    c->force_block = blocks[k];
    destroy_graphs(c);
    c->timing = true;
    c->t_force_ms = c->t_search_ms = 0;
    c->n_force = c->n_search = 0;
    if ((rc = run(trial_steps))) break;
    out->block_ms[k] = c->t_force_ms / (double)std::max<int64_t>(c->n_force, 1);
    if (out->block_ms[k] < best) {
      best = out->block_ms[k];
      best_block = blocks[k];
    }
  }
  c->timing = false;
  c->force_block = best_block;
  destroy_graphs(c);
  if (rc) return rc;
  // 2. cell edge: time of a forced contact search for h / d_max from r_s / d_max up
  double f0 = HUGE_VAL;
  for (const Instance& I : c->inst)
    if (I.n > 0) f0 = std::min(f0, I.rs / I.dmax);
  const double fmul[4] = {1.0, 1.15, 1.3, 1.5};
  best = HUGE_VAL;
  double best_cf = c->cell_factor;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (int k = 0; k < 4 && rc == DEM_OK; ++k) {
    const double cf = f0 * fmul[k];
    out->cell_factors[k] = cf;
    if ((rc = regrid(c, cf))) break;
    if ((rc = forced_search())) break;  // first search on new cells: untimed
    float total = 0.f;
    for (int r = 0; r < 3 && rc == DEM_OK; ++r) {
      hipError_t he = hipEventRecord(e0, c->stream);
      if (he == hipSuccess &&
          (rc = enqueue_rebuild(c, 0, 1, c->step - c->host_base, next_eval_rel(c))) == DEM_OK) {
        he = hipEventRecord(e1, c->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        total += ms;
      }
      if (he != hipSuccess) rc = set_err(DEM_EHIP, "timing events: %s", hipGetErrorString(he));
    }
    out->search_ms[k] = total / 3.0;
    if (rc == DEM_OK && out->search_ms[k] < best) {
      best = out->search_ms[k];
      best_cf = cf;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = regrid(c, best_cf))) return rc;
  // 3. search schedule: whole steps per wall-clock time.  The dynamic trial
  // runs first and measures the largest per-step drift; constant intervals
  // are tried only while K drifts stay below a quarter of half the skin.
  bool can_dynamic = true;
  for (const Instance& I : c->inst)
    if (I.n > 0 && !(I.skin > 0.0)) can_dynamic = false;
  const int Ks[5] = {5, 10, 20, 40, 80};
  int n_sched = 0;
  // without a skin every displacement trips the guard: the schedule stays
  if (can_dynamic) {
    out->schedules[n_sched++] = 0;
    for (int k = 0; k < 5; ++k) out->schedules[n_sched++] = Ks[k];
  }
  const int K0 = c->cfg.rebuild_interval;
  best = HUGE_VAL;
  int best_K = K0;
  double rate = 0.0;  // largest per-step drift in half skins, from the dynamic trial
  for (int k = 0; k < n_sched && rc == DEM_OK; ++k) {
    const int K = out->schedules[k];
    if (K > 0 && (rate * K * 4.0 >= 1.0 || !walls_fit(c, K))) {
      out->schedule_ms[k] = -1.0;  // unsafe for the guard or a moving wall: not tried
      continue;
    }
    c->cfg.rebuild_interval = K;
    c->dynamic = K == 0;
    destroy_graphs(c);
    if ((rc = forced_search())) break;
    const int64_t warm = K > 0 ? 2 * (int64_t)K : 2 * (int64_t)kDynChunk;
    if ((rc = run(warm))) break;  // captures the graphs of this schedule
    const auto t0 = std::chrono::steady_clock::now();
    if ((rc = run(trial_steps))) break;
    const auto t1 = std::chrono::steady_clock::now();
    out->schedule_ms[k] = std::chrono::duration<double, std::milli>(t1 - t0).count() / trial_steps;
    if (K == 0) rate = c->dyn_rate;
    if (out->schedule_ms[k] < best) {
      best = out->schedule_ms[k];
      best_K = K;
    }
  }
  if (rc) return rc;
  if (n_sched == 0) best = HUGE_VAL;
  c->cfg.rebuild_interval = best_K;
  c->dynamic = best_K == 0;
  destroy_graphs(c);
  if ((rc = forced_search())) return rc;
  c->timing = timing0;
  c->t_force_ms = c->t_search_ms = 0;
  c->n_force = c->n_search = 0;
  out->force_block = c->force_block;
  out->rebuild_interval = best_K;
  out->cell_factor = c->cell_factor;
  out->ms_per_step = best;
  out->steps = steps;
  return DEM_OK;
}

int dem_set_timing(dem_ctx* c, int32_t enable) {
  if (!c) return set_err(DEM_EINVAL, "null context");
  c->timing = enable != 0;
  c->t_force_ms = c->t_search_ms = 0;
  c->n_force = c->n_search = 0;
  return DEM_OK;
}

int dem_get_timing(dem_ctx* c, double* out4) {
  if (!c || !out4) return set_err(DEM_EINVAL, "null argument");
  out4[0] = c->t_force_ms;
  out4[1] = (double)c->n_force;
  out4[2] = c->t_search_ms;
  out4[3] = (double)c->n_search;
  return DEM_OK;
}

}  // extern "C"
