// Device-side data structures and kernel launch interface of the MI355X DEM
// library.  Shared by the HIP kernels (dem_kernels.hip) and the host runtime
// behind the C ABI (dem_api.hip).  Nothing here is visible to library users.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace demgpu {

constexpr int kMaxTypes = 16;
constexpr int kMaxWalls = 32;
constexpr int kWallSlots = 4;   // particle-wall contacts kept per particle
constexpr int kMeshSlots = 8;   // particle-triangle candidates kept per particle
constexpr int kBlock = 256;     // threads per workgroup (4 wave64)
constexpr int kWave = 64;
constexpr int kTypeMask = 0xffff;
constexpr int kInactive = 1 << 16;  // flag bit in the per-particle info word
constexpr int kInstShift = 20;      // info bits 20..30: instance of the particle
constexpr int kDriftSpread = 32;  // words per drift record
constexpr int kMaxInstances = 2048;
constexpr int kMaxMeshTriangles = 1 << 24;  // per instance
// Particles per context: while the contact search builds a row, the top three
// bits of each entry carry the pair's gap class, so sorted indices stay below
// 2^29.
constexpr int kClassShift = 29;
constexpr int64_t kMaxParticles = (int64_t)1 << kClassShift;

// Sticky error bits raised by kernels (read once per dem_step call).
enum : int {
  kFlagGuard = 1,         // a particle moved more than skin/2 between searches
  kFlagNonFinite = 2,     // NaN/Inf in the state
  kFlagNbrOverflow = 4,   // a particle had more candidate neighbours than max_nb
  kFlagWallOverflow = 8,  // more wall candidates than kWallSlots
  kFlagMeshOverflow = 16, // more triangle candidates than kMeshSlots
};

// Per material pair constants of the Hertz-Mindlin law (effective-parameter
// table of Sec. 2.1), with Y_e, G_e the effective moduli and
// beta = ln e / sqrt(ln^2 e + pi^2):  kn = 4/3 Y_e, kt = 8 G_e,
// en = -2 sqrt(5/6) beta sqrt(2 Y_e), et = -2 sqrt(5/6) beta sqrt(8 G_e),
// so that k_n = kn q, k_t = kt q, eta_n = en sqrt(m_e q), eta_t = et sqrt(m_e q)
// with q = sqrt(R_e delta_n); mu and mur are the friction coefficients.
// Linear model: kn = kt = (16/15) Y_e (15 V^2 / (16 Y_e))^(1/5) and en = et =
// 2 / sqrt(1 + (pi / ln e)^2), so that k = kn (R_e^2 m_e)^(1/5) and eta = en
// sqrt(m_e k) (Eqs. linearkn, linearetan).
struct PairCoef {
  double kn, kt, en, et, mu, mur, pad0, pad1;
};

// Wall.  kind 0: plane (point p, unit normal nrm into the domain, optional
// rectangular extent along u / vax).  kind 2: cone, as the cylinder with the
// surface at radius + slope s.  kind 1: cylinder (axis point p, unit axis
// nrm, radius, axial range [smin, smax], particles inside or outside).
// kind 3: triangle mesh (its triangles in the triangle table, found through
// a uniform grid over the mesh at time 0; p is its first corner).  Translation with velocity vel: at time t the point and the
// rotation axis sit at p + vel t and ax + vel t.  Surface velocity at a
// contact point x_c: vel + omega x (x_c - ax(t)).  Active for t_on <= t < t_off.
struct WallDev {
  int kind, bounded, inside, material;
  double p[3], nrm[3], u[3], vax[3];
  double hu, hv, radius, smin, smax;
  double omega[3], ax[3];
  double t_on, t_off;
  double skin;  // the owning instance's skin (contact-search margin)
  double slope, q;  // cone: radius + slope s at axial coordinate s; q = sqrt(1 + slope^2)
  double vel[3];
  double axo[3];  // ax - p: the rotation axis moves with the wall
  // mesh: triangles [tri_begin, tri_begin + tri_count); grid cell (cx, cy,
  // cz) = floor((x - vel t - mlo) / mh) lists its triangles at
  // cell_tri[cell[cell_base + c] .. cell[cell_base + c + 1]), c = cx + mnc0
  // (cy + mnc1 cz)
  int tri_begin, tri_count, cell_base, pad;
  int mnc[3], pad2;
  double mlo[3], mh;
};

// One triangle of a mesh wall: corners at time 0 (the particles' side is the
// side of (p1 - p0) x (p2 - p0)), edge vectors e_c = p_{c+1} - p_c, unit
// normal, the mesh's own corner indices (names of its edges and vertices)
// and the owning wall.
struct TriDev {
  double p[3][3];
  double e[3][3];
  double n[3];
  int v[3];
  int wall;
};

// Particle-triangle candidates: slot s of particle i at s * n + i (global
// triangle index or -1), tangential overlaps in 3 * kMeshSlots planes.
struct MeshSlots {
  int* tri;
  double* hist;
};

// Triangle table and mesh grids (all null when no instance has a mesh).
struct MeshTables {
  const TriDev* tri;
  const int* cell;
  const int* cell_tri;
};

// Uniform cell grid of one instance: cell (cx,cy,cz) = floor((x - lo)/h).
// Cells are ordered along a Morton (Z-order) curve (the bits of the three
// coordinates interleaved; axes with fewer bits drop out of the interleave at
// the top), and a cell's key is its rank in that order among the grid's
// cells: key = ckey[(cz * nc[1] + cy) * nc[0] + cx], 0 .. n_keys - 1, so the
// key space has no unused keys (a power-of-two Morton range would).
struct GridDev {
  double lo[3], hi[3], h;
  int nc[3];
  const uint32_t* ckey;
  int64_t n_keys;  // nc[0] * nc[1] * nc[2]
};

// One independent simulation of a batch.  Its cells use the global keys
// [key_base, key_base + grid.n_keys); its walls are walls[wall_begin,
// wall_end); its material-pair constants start at coef_base in the tables.
struct InstDev {
  GridDev grid;
  uint32_t key_base;
  int wall_begin, wall_end;
  int coef_base;
  double rs2;     // squared search radius
  double guard2;  // (skin/2)^2
  double skin;    // r_s - d_max
  double ihs;     // 2 / skin (drift in units of half the skin)
};

struct StepParams {
  double dt, hdt;
  double g[3];
  int n;           // number of particles of all instances (active + inactive)
  int max_nb;      // neighbour slots per particle
  int rolling;     // 0 none, 1 constant torque, 2 viscous torque
  int model;       // 0 nonlinear (Hertz-Mindlin), 1 linear spring-dashpot
  uint32_t n_keys; // total cell keys; key n_keys collects inactive particles
  double drift_scale;  // dt * 2 / skin when every instance has the same skin,
                       // else 0 (then taken per particle from its instance)
  // Displacement bound since the last contact search, in units of half the
  // skin of each particle's instance, for the row cuts (see NbrList): the
  // force evaluation at absolute step s (positions x^s) uses
  // acc(s) = bacc[(s - 1) % 3] + sqrt(max of brec[s % 3]), where brec[s % 3]
  // (kDriftSpread words, non-negative doubles as bits) holds the largest
  // squared drift |v| dt (half skins) of the update that produced x^s.  The
  // evaluation writes bacc[s % 3] = acc(s), raises brec[(s + 1) % 3] with
  // its own update and clears brec[(s + 2) % 3]; a search at step s sets
  // bacc[(s - 1) % 3] and brec[s % 3] to zero.  No particle has moved more
  // than acc(s) half skins from where the last search saw it.
  double* bacc;             // 3 words
  unsigned long long* brec; // 3 * kDriftSpread words
};

// Particle arrays in sorted (spatial) order.  pos = (x, y, z, R),
// vel = (v, 1/m), omg = (omega, 1/I).
struct ParticleBufs {
  double4* pos;
  double4* vel;
  double4* omg;
};

// Neighbour list, one row per particle in wave-slab column-major layout:
// entry (i, k) lives at ((i / 64) * max_nb + k) * 64 + i % 64.  Bit 31 of a
// neighbour index is set while the pair touches; the stored history of an
// entry without bit 31 is undefined and stands for zero.
//
// A search orders each row by the gap g = d - (R_i + R_j) it found: the
// touching pairs first, then the pairs with g < s/8, g < s/4, g < s/2 and the
// rest (s the skin); rowcut packs the ends of the middle three groups (10
// bits each, 1023 = the whole row).  Two particles that each moved at most
// acc s/2 since the search come at most acc s closer, so while acc < f the
// entries with g >= f s cannot touch and the force evaluation reads the row
// only up to the matching end (f = 1/8, 1/4, 1/2).
struct NbrList {
  int* nbr;      // sorted index of the neighbour
  double* hist;  // 3 planes of tangential overlap (x, y, z), stride cap
  int* rowlen;
  int64_t cap;   // entries per plane
  int* rowcut;   // per particle: the three row cuts
};

// Gap classes of the row cuts: fractions of the skin.
constexpr double kCutFrac[3] = {0.125, 0.25, 0.5};
constexpr int kCutBits = 10;
constexpr int kCutMask = (1 << kCutBits) - 1;  // a stored cut of 1023 means "the whole row"

// Particle-wall slots: slot s of particle i at s * n + i.
struct WallSlots {
  int* wid;      // wall id or -1
  double* hist;  // 3 * kWallSlots planes of n
};

__host__ __device__ inline int64_t nbr_entry(int i, int k, int max_nb) {
  return ((int64_t)(i >> 6) * max_nb + k) * 64 + (i & 63);
}

// ---------------------------------------------------------------- launches
// Every launcher enqueues on `s` and returns the hipError_t of the launch.

hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s);
hipError_t launch_keys(const InstDev* inst, const StepParams& sp, const double4* pos,
                       const double4* vel, int* info, const double4* xref, int check_guard,
                       uint32_t* keys, int* rank, int* count, int* flags, hipStream_t s);
// exclusive scan of count[0..m) into start[0..m], start[m] = total; with cse
// also cse[key_cell[k]] = (start[k], start[k + 1]) for the keys k < n_cells
hipError_t launch_scan(const int* count, int* start, int64_t m, int* tile_sums, hipStream_t s,
                       const uint32_t* key_cell = nullptr, int2* cse = nullptr,
                       int64_t n_cells = 0);
hipError_t launch_scatter(int n, const uint32_t* keys, const int* rank, const int* start,
                          int* perm0, hipStream_t s);
hipError_t launch_cell_rank(int n, int64_t n_keys, const int* perm0, const uint32_t* keys,
                            const int* start, const int* gid, int* perm, hipStream_t s);
// perm: new -> old index; inv receives old -> new
// The particle-wall and particle-triangle searches take the walls where they
// are at time (*clock + step_rel) dt.
// It also restarts the displacement bound (StepParams) for the force
// evaluation at step *clock + bound_step_rel.
hipError_t launch_reorder(const StepParams& sp, const InstDev* inst, const int* perm, int* inv,
                          ParticleBufs src,
                          ParticleBufs dst, const int* gid_src, int* gid_dst,
                          const int* info_src, int* info_dst, double4* xref,
                          WallSlots ws_src, WallSlots ws_dst, const WallDev* walls,
                          MeshTables mt, MeshSlots ms_src, MeshSlots ms_dst,
                          const double4* F_src, const double4* T_src, double4* F_dst,
                          double4* T_dst, const int64_t* clock, int64_t step_rel,
                          int64_t bound_step_rel, int* flags, hipStream_t s);
// cse: (start, end) of every cell in sorted order, indexed by the cell's
// position (key_base + (cz * nc[1] + cy) * nc[0] + cx)
hipError_t launch_search(const InstDev* inst, int n_inst, const StepParams& sp,
                         const double4* pos, const int* info, const int2* cse, const int* perm,
                         const int* inv, NbrList old_l, NbrList new_l, int* flags,
                         hipStream_t s);

// force + integration kernels.  mode: 0 = velocity Verlet fused (second half
// kick of this step, first half kick and drift of the next), 1 = velocity
// Verlet last step of a call (second half kick, forces stored), 2 = explicit
// Euler (forces at the current state, then the update; forces stored).
// xsel (may be null): particles i with xsel[i] >= 0 add the force and torque
// Fx[i] / Tx[i] to their contact sums (the mesh contacts of the same state;
// xsel is the first mesh candidate slot).  pf (may be null): the force of
// every touching pair on the row's particle is also written to entry (i, k)
// of three planes of l.cap doubles (a per-contact record for tests).
// pair_mode: 1 when the batch is one instance whose particles all have type
// 0 (every particle pair takes the pair table's first entry), 2 when every
// particle has type 0 (the first entry of the particle's own row), else 0.
hipError_t launch_force(int mode, int precision, const StepParams& sp, const InstDev* inst,
                        const PairCoef* pp,
                        const PairCoef* pw, const WallDev* walls, ParticleBufs in,
                        ParticleBufs out, const int* info, NbrList l, WallSlots ws,
                        double4* F, double4* T, const int64_t* clock, int64_t step_rel,
                        const int* flags, unsigned long long* drift, const int* xsel,
                        const double4* Fx, const double4* Tx, double* pf, int block,
                        int pair_mode, hipStream_t s);
// Contacts of the particles with triangle candidates at time (*clock +
// step_rel) dt (tangential overlaps updated): their force and torque into
// Fm / Tm (written for those particles only).
hipError_t launch_mesh(int precision, const StepParams& sp, const PairCoef* pw,
                       const WallDev* walls, MeshTables mt, ParticleBufs in, const int* info,
                       MeshSlots ms, double4* Fm, double4* Tm, const int64_t* clock,
                       int64_t step_rel, const int* flags, hipStream_t s);
// first half kick + drift from stored forces (start of a velocity-Verlet call).
// When drift is not null, both launchers raise the kDriftSpread words at
// drift (as the bits of non-negative doubles) so that their maximum is the
// largest squared drift |v| dt of the step, in units of half the particle's
// skin (each wavefront raises one word: spreading the atomics over several
// words keeps them from queueing on one address).
// The kick and drift produce the positions of step *clock + step_rel, whose
// displacement-bound record (StepParams) they raise.
hipError_t launch_kick_drift(const StepParams& sp, const InstDev* inst, ParticleBufs st,
                             const int* info, const double4* F, const double4* T,
                             unsigned long long* drift, const int64_t* clock, int64_t step_rel,
                             hipStream_t s);
hipError_t launch_tick(int64_t* clock, int64_t k, hipStream_t s);
// statistics: out[0] active, [1] list entries, [2] touching entries, [3] wall slots
hipError_t launch_stats(const StepParams& sp, const double4* pos, const int* info,
                        NbrList l, WallSlots ws, unsigned long long* out, hipStream_t s);

// Candidate pairs of instance inst on the device (see dem_get_contacts_device).
// scratch holds pairs_scratch_ints(sp.n) ints: block counts, their exclusive
// scan (scratch[nb + nb] is the total afterwards) and the scan's tile sums.
int64_t pairs_scratch_ints(int n);
hipError_t launch_pairs_count(const StepParams& sp, int inst, const int* info, const int* gid,
                              NbrList l, int* scratch, hipStream_t s);
hipError_t launch_pairs_fill(const StepParams& sp, int inst, int gid_base, const double4* pos,
                             const int* info, const int* gid, NbrList l, const int* scratch,
                             int64_t* pairs, double* delta_t, uint8_t* touching, hipStream_t s);

}  // namespace demgpu
