// HIP kernels (gfx950, wave64) of the soft-sphere DEM hot path.
//
// Method: Golshan et al., "Lethe-DEM" (arXiv 2106.09576).
//   contact search   Sec. 3.2: particles sorted into cells, broad search over
//                    a cell and its neighbour cells, fine search keeping pairs
//                    closer than the threshold; rerun every K steps (Sec. 3.1)
//   contact law      Sec. 2.1: Eqs. (deltan), (vecn), (delta_t), (vrt),
//                    (normal_force), (tangential_force), (nonlinearkn)-
//                    (nonlinearetat), effective-parameter table, (torque_t),
//                    constant rolling model, (coulomb_overlap)-(coulomb_overlap3)
//   walls            Sec. 2.1 last paragraph: same law against a wall
//   integration      Sec. 2.2: Eqs. (integ_EE), (halfstep), (newvv)
//
// Design (MI355X): one thread per particle everywhere.  The force kernel is a
// gather over each particle's full neighbour row, so every particle sums its
// own forces in a fixed order (deterministic, no atomics).  Both directions of
// a pair keep their own copy of the tangential overlap; the contact law is
// written so that evaluating it from j's side gives exactly -F and -delta_t
// (IEEE negation symmetry; this file is compiled without FP contraction), so
// the two copies never drift apart.  Rows are stored column-major inside each
// wavefront's slab, so every load of a neighbour index or history component is
// one coalesced 64-lane access.  The force kernel also integrates its own
// particle (ping-pong state buffers), so a time step is one launch.
#include "dem_device.hpp"

namespace demgpu {

// ------------------------------------------------------------------ helpers

// Blocks of a 1-D launch are spread over the 8 XCDs round-robin; remap so each
// XCD works on a contiguous range of particles (neighbours then share its L2).
__device__ inline int xcd_block() {
  const unsigned nb = gridDim.x;
  const unsigned b = blockIdx.x;
  if ((nb & 7u) != 0u) return (int)b;
  return (int)((b & 7u) * (nb >> 3) + (b >> 3));
}

static inline unsigned grid_for(int64_t n, int block = kBlock) {
  int64_t b = (n + block - 1) / block;
  if (b < 1) b = 1;
  b = (b + 7) & ~int64_t(7);
  return (unsigned)b;
}

__device__ inline bool finite3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

__device__ inline int cell_coord(double x, double lo, double h, int nc) {
  int c = (int)floor((x - lo) / h);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ inline uint32_t cell_key(const GridDev& g, int cx, int cy, int cz) {
  return g.ckey[(cz * g.nc[1] + cy) * g.nc[0] + cx];  // fewer than 2^30 cells
}

// Slot of the displacement-bound ring (StepParams) for absolute step s + d
// (s >= 0; 2^32 = 1 mod 3, so s mod 3 follows from its two 32-bit halves).
__device__ __forceinline__ int bound_slot(int64_t s, int d) {
  const uint64_t u = (uint64_t)s;
  const uint32_t r = ((uint32_t)(u >> 32) % 3u + (uint32_t)u % 3u) % 3u;
  return (int)((r + 3u + (uint32_t)d) % 3u);
}

// ------------------------------------------------------------------ fill

__global__ void k_fill_i32(int* p, int v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + kBlock - 1) / kBlock;
  unsigned nb = (unsigned)(b > 65536 ? 65536 : b);
  hipLaunchKernelGGL(k_fill_i32, dim3(nb), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

// ------------------------------------------------------------- sort: keys

// Cell key of every particle; deactivates particles outside the domain box,
// checks the displacement guard and non-finite states, counts per cell (the
// returned atomic slot is the particle's provisional rank in its cell).
__global__ void k_keys(const InstDev* __restrict__ inst, StepParams sp,
                       const double4* __restrict__ pos,
                       const double4* __restrict__ vel, int* __restrict__ info,
                       const double4* __restrict__ xref, int check_guard,
                       uint32_t* __restrict__ keys, int* __restrict__ rank,
                       int* __restrict__ count, int* __restrict__ flags) {
  int i = xcd_block() * kBlock + threadIdx.x;
  // every lane stays to the end: the ranks are handed out per run of equal
  // keys in the wavefront (below)
  const bool valid = i < sp.n;
  int inf = valid ? info[i] : kInactive;
  uint32_t key = valid ? sp.n_keys : 0xffffffffu;
  if (valid && !(inf & kInactive)) {
    const InstDev& I = inst[inf >> kInstShift];
    const GridDev& g = I.grid;
    double4 p = pos[i];
    double4 v = vel[i];
    if (!finite3(p.x, p.y, p.z) || !finite3(v.x, v.y, v.z)) atomicOr(flags, kFlagNonFinite);
    if (check_guard) {
      double4 r = xref[i];
      double dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z;
      double d2 = (dx * dx + dy * dy) + dz * dz;
      if (d2 > I.guard2) atomicOr(flags, kFlagGuard);
    }
    bool inside = p.x >= g.lo[0] && p.x < g.hi[0] && p.y >= g.lo[1] && p.y < g.hi[1] &&
                  p.z >= g.lo[2] && p.z < g.hi[2];
    if (!inside) {
      info[i] = inf | kInactive;
    } else {
      int cx = cell_coord(p.x, g.lo[0], g.h, g.nc[0]);
      int cy = cell_coord(p.y, g.lo[1], g.h, g.nc[1]);
      int cz = cell_coord(p.z, g.lo[2], g.h, g.nc[2]);
      key = I.key_base + cell_key(g, cx, cy, cz);
    }
  }
  // Particles come in the previous search's spatial order, so lanes with the
  // same cell mostly sit side by side: the first lane of each run of equal
  // keys reserves the whole run with one atomic and hands consecutive ranks
  // to the run (the order within a cell is fixed later by k_cell_rank).
  const int lane = threadIdx.x & 63;
  const uint32_t prev = __shfl_up(key, 1, 64);
  const bool first = lane == 0 || prev != key;
  const unsigned long long starts = __builtin_amdgcn_ballot_w64(first);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int lead = 63 - __builtin_clzll(starts & upto);
  const unsigned long long after = lane == 63 ? 0ull : (starts & ~upto);
  const int next = after ? __builtin_ctzll(after) : 64;
  int base = 0;
  if (first && valid) base = atomicAdd(&count[key], next - lane);
  base = __shfl(base, lead, 64);
  if (valid) {
    keys[i] = key;
    rank[i] = base + (lane - lead);
  }
}

hipError_t launch_keys(const InstDev* inst, const StepParams& sp, const double4* pos,
                       const double4* vel, int* info, const double4* xref, int check_guard,
                       uint32_t* keys, int* rank, int* count, int* flags, hipStream_t s) {
  if (sp.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_keys, dim3(grid_for(sp.n)), dim3(kBlock), 0, s, inst, sp, pos, vel, info,
                     xref, check_guard, keys, rank, count, flags);
  return hipGetLastError();
}

// ------------------------------------------------------------- sort: scan
// Three-phase exclusive scan: tile sums, one-block scan of the tile sums,
// tile-local scan plus offset.  Tiles of 1024 elements (256 threads x 4).

constexpr int kScanTile = 1024;

__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
  // 256 threads, 4 waves: wave-level inclusive scan via shuffles, then waves.
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  int wsum = 0;
  for (int k = 0; k < w; ++k) wsum += sh[k];
  int tot = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  *total = tot;
  return x - v + wsum;
}

__global__ void k_scan_tiles(const int* __restrict__ in, int64_t m, int* __restrict__ tsum) {
  __shared__ int sh[4];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
  int s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < m) s += in[base + k];
  int tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// One workgroup: thread t takes the contiguous chunk [t c, (t + 1) c) of the
// nt tile sums (c = ceil(nt / kBlock)), adds it up (independent loads, not
// one dependent round per kBlock sums), the chunk totals are scanned across
// the workgroup, and each thread writes its chunk's exclusive prefixes.
__global__ void k_scan_sums(int* __restrict__ tsum, int64_t nt) {
  __shared__ int sh[4];
  const int64_t c = (nt + kBlock - 1) / kBlock;
  const int64_t a = (int64_t)threadIdx.x * c;
  const int64_t b = a + c < nt ? a + c : nt;
  int s = 0;
#pragma unroll 8
  for (int64_t i = a; i < b; ++i) s += tsum[i];
  int tot;
  int ex = block_exclusive_scan(s, sh, &tot);
  for (int64_t i = a; i < b; ++i) {
    const int v = tsum[i];
    tsum[i] = ex;
    ex += v;
  }
}

// With cse: also the (start, end) pair of each of the first n_cells keys,
// stored at that key's cell (key_cell), for lookups by cell position.
__global__ void k_scan_apply(const int* __restrict__ in, int64_t m, const int* __restrict__ tsum,
                             int* __restrict__ out, const uint32_t* __restrict__ key_cell,
                             int2* __restrict__ cse, int64_t n_cells) {
  __shared__ int sh[4];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
  int v[4];
  int s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < m) ? in[base + k] : 0;
    s += v[k];
  }
  int tot;
  int ex = block_exclusive_scan(s, sh, &tot) + tsum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < m) out[base + k] = ex;
    if (cse && base + k < n_cells) cse[key_cell[base + k]] = make_int2(ex, ex + v[k]);
    ex += v[k];
  }
  // the element after the last one holds the total
  if (base <= m - 1 && m - 1 < base + 4) out[m] = ex;
}

hipError_t launch_scan(const int* count, int* start, int64_t m, int* tile_sums, hipStream_t s,
                       const uint32_t* key_cell, int2* cse, int64_t n_cells) {
  if (m <= 0) return hipSuccess;
  int64_t nt = (m + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kBlock), 0, s, count, m, tile_sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, tile_sums, nt);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(kBlock), 0, s, count, m, tile_sums,
                     start, key_cell, cse, n_cells);
  return hipGetLastError();
}

// ---------------------------------------------------------- sort: scatter

__global__ void k_scatter(int n, const uint32_t* __restrict__ keys, const int* __restrict__ rank,
                          const int* __restrict__ start, int* __restrict__ perm0) {
  int i = xcd_block() * kBlock + threadIdx.x;
  if (i >= n) return;
  perm0[start[keys[i]] + rank[i]] = i;
}

hipError_t launch_scatter(int n, const uint32_t* keys, const int* rank, const int* start,
                          int* perm0, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(kBlock), 0, s, n, keys, rank, start,
                     perm0);
  return hipGetLastError();
}

// Within a cell, order particles by gid so the sorted order (and with it every
// summation order) is independent of atomic arrival order.  Inactive particles
// (last key) keep their arrival order: they take part in no computation.
__global__ void k_cell_rank(int n, uint32_t n_keys, const int* __restrict__ perm0,
                            const uint32_t* __restrict__ keys, const int* __restrict__ start,
                            const int* __restrict__ gid, int* __restrict__ perm) {
  int p = xcd_block() * kBlock + threadIdx.x;
  if (p >= n) return;
  int o = perm0[p];
  uint32_t k = keys[o];
  if (k == n_keys) {
    perm[p] = o;
    return;
  }
  int s = start[k], e = start[k + 1];
  int g = gid[o];
  int r = 0;
  for (int q = s; q < e; ++q) r += gid[perm0[q]] < g ? 1 : 0;
  perm[s + r] = o;
}

hipError_t launch_cell_rank(int n, int64_t n_keys, const int* perm0, const uint32_t* keys,
                            const int* start, const int* gid, int* perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cell_rank, dim3(grid_for(n)), dim3(kBlock), 0, s, n, (uint32_t)n_keys,
                     perm0, keys, start, gid, perm);
  return hipGetLastError();
}

// ------------------------------------------------------------------ walls

// Candidate / touching predicates of particle centre x (radius R) against a
// wall at time t, evaluated without square roots; when touching also the unit
// normal from the particle to the wall, the overlap and the lever arm of the
// contact point about the wall's rotation axis (x_c - ax(t)).
struct WallGeo {
  bool candidate, touching;
  double n[3], dn, arm[3];
};

__device__ inline double dot3(const double* a, const double* b) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

__device__ inline void wall_geo(const WallDev& W, const double x[3], double R, double skin,
                                bool need_contact, double t, WallGeo& g) {
  g.candidate = false;
  g.touching = false;
  const double P[3] = {W.p[0] + W.vel[0] * t, W.p[1] + W.vel[1] * t, W.p[2] + W.vel[2] * t};
  double rel[3] = {x[0] - P[0], x[1] - P[1], x[2] - P[2]};
  if (W.kind == 0) {
    double dist = dot3(rel, W.nrm);
    if (W.bounded) {
      double a = dot3(rel, W.u), b = dot3(rel, W.vax);
      if (!(fabs(a) <= W.hu && fabs(b) <= W.hv)) return;
    }
    g.candidate = (dist < R + skin) && (dist > -R);
    g.touching = dist < R;
    if (g.touching && need_contact) {
      for (int k = 0; k < 3; ++k) {
        g.n[k] = -W.nrm[k];
        g.arm[k] = (rel[k] - dist * W.nrm[k]) - W.axo[k];
      }
      g.dn = R - dist;
    }
    return;
  }
  double sax = dot3(rel, W.nrm);
  if (!(sax >= W.smin && sax <= W.smax)) return;
  double r[3] = {rel[0] - sax * W.nrm[0], rel[1] - sax * W.nrm[1], rel[2] - sax * W.nrm[2]};
  double rho2 = dot3(r, r);
  if (!(rho2 > 0.0)) return;
  if (W.kind == 2) {
    // cone: distance (r(s) - rho) / q inside, (rho - r(s)) / q outside, tested
    // as rho^2 against squared bounds; outward normal (e_rho - slope nrm) / q
    const double q = W.q;
    const double rs = W.radius + W.slope * sax;
    if (W.inside) {
      double lo = rs - (R + skin) * q;
      double hi = rs + R * q;
      bool above = (lo <= 0.0) || (rho2 > lo * lo);
      g.candidate = above && (hi > 0.0) && (rho2 < hi * hi);
      double lt = rs - R * q;
      g.touching = (lt <= 0.0) || (rho2 > lt * lt);
    } else {
      double hi = rs + (R + skin) * q;
      double lo = rs - R * q;
      bool above = (lo <= 0.0) || (rho2 > lo * lo);
      g.candidate = above && (hi > 0.0) && (rho2 < hi * hi);
      double lt = rs + R * q;
      g.touching = (lt > 0.0) && (rho2 < lt * lt);
    }
    if (g.touching && need_contact) {
      double rho = sqrt(rho2);
      double er[3] = {r[0] / rho, r[1] / rho, r[2] / rho};
      double dist = W.inside ? (rs - rho) / q : (rho - rs) / q;
      g.dn = R - dist;
      for (int k = 0; k < 3; ++k) {
        const double m = (er[k] - W.slope * W.nrm[k]) / q;
        g.n[k] = W.inside ? m : -m;
        g.arm[k] = (rel[k] + dist * g.n[k]) - W.axo[k];
      }
    }
    return;
  }
  const double Rc = W.radius;
  if (W.inside) {
    double lo = Rc - (R + skin);
    double hi = Rc + R;
    bool above = (lo <= 0.0) || (rho2 > lo * lo);
    g.candidate = above && (rho2 < hi * hi);
    double lt = Rc - R;
    g.touching = (lt <= 0.0) || (rho2 > lt * lt);
  } else {
    double hi = Rc + R + skin;
    double lo = Rc - R;
    bool above = (lo <= 0.0) || (rho2 > lo * lo);
    g.candidate = above && (rho2 < hi * hi);
    double lt = Rc + R;
    g.touching = rho2 < lt * lt;
  }
  if (g.touching && need_contact) {
    double rho = sqrt(rho2);
    double er[3] = {r[0] / rho, r[1] / rho, r[2] / rho};
    double dist = W.inside ? (Rc - rho) : (rho - Rc);
    g.dn = R - dist;
    for (int k = 0; k < 3; ++k) {
      g.n[k] = W.inside ? er[k] : -er[k];
      g.arm[k] = (sax * W.nrm[k] + Rc * er[k]) - W.axo[k];
    }
  }
}

// ------------------------------------------------------------ mesh walls

// Closest point of the closed triangle T, moved by vel t, to the point x: the
// projection onto the triangle's plane when it lies strictly inside all
// three edges (a face), else the closest of the three edges' own closest
// points (the projection onto the edge line clamped to the edge), on an edge
// when strictly inside it and on a corner otherwise.  s is the signed
// distance from the plane along the unit normal, d2 the squared distance.
struct TriGeo {
  int feature;  // 0 face, 1 edge (corners a, b = a + 1 mod 3), 2 vertex (corner a)
  int a, b;
  double s, d2;
  double q[3];
};

__device__ inline void cross3(const double* a, const double* b, double* r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ inline void tri_closest(const TriDev& T, const double vel[3], double t,
                                   const double x[3], TriGeo& g) {
  double P[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < 3; ++k) P[c][k] = T.p[c][k] + vel[k] * t;
  const double rel[3] = {x[0] - P[0][0], x[1] - P[0][1], x[2] - P[0][2]};
  g.s = dot3(rel, T.n);
  bool inside = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double r[3] = {x[0] - P[c][0], x[1] - P[c][1], x[2] - P[c][2]};
    double cr[3];
    cross3(T.e[c], r, cr);
    if (!(dot3(cr, T.n) > 0.0)) inside = false;
  }
  if (inside) {
    g.feature = 0;
    g.a = g.b = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) g.q[k] = x[k] - g.s * T.n[k];
    g.d2 = g.s * g.s;
    return;
  }
  g.d2 = INFINITY;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double* E = T.e[c];
    const double r[3] = {x[0] - P[c][0], x[1] - P[c][1], x[2] - P[c][2]};
    const double u = dot3(r, E) / dot3(E, E);
    const double uc = u <= 0.0 ? 0.0 : (u >= 1.0 ? 1.0 : u);
    const double q[3] = {P[c][0] + uc * E[0], P[c][1] + uc * E[1], P[c][2] + uc * E[2]};
    const double dq[3] = {x[0] - q[0], x[1] - q[1], x[2] - q[2]};
    const double d2 = dot3(dq, dq);
    if (d2 < g.d2) {
      g.d2 = d2;
      g.q[0] = q[0];
      g.q[1] = q[1];
      g.q[2] = q[2];
      const int c1 = c == 2 ? 0 : c + 1;
      if (u <= 0.0) {
        g.feature = 2;
        g.a = g.b = c;
      } else if (u >= 1.0) {
        g.feature = 2;
        g.a = g.b = c1;
      } else {
        g.feature = 1;
        g.a = c;
        g.b = c1;
      }
    }
  }
}

// ----------------------------------------------------------------- reorder

// Gather every particle array into sorted order, record the reference
// position of the displacement guard, and redo the particle-wall search at
// the new position carrying the tangential overlap of walls already listed.
__global__ void k_reorder(StepParams sp, const InstDev* __restrict__ inst,
                          const int* __restrict__ perm, int* __restrict__ inv, ParticleBufs src,
                          ParticleBufs dst, const int* __restrict__ gid_src,
                          int* __restrict__ gid_dst, const int* __restrict__ info_src,
                          int* __restrict__ info_dst, double4* __restrict__ xref,
                          WallSlots ws_src, WallSlots ws_dst, const WallDev* __restrict__ walls,
                          MeshTables mt, MeshSlots ms_src, MeshSlots ms_dst,
                          const double4* __restrict__ F_src, const double4* __restrict__ T_src,
                          double4* __restrict__ F_dst, double4* __restrict__ T_dst,
                          const int64_t* __restrict__ clock, int64_t step_rel,
                          int64_t bound_step_rel, int* __restrict__ flags) {
  int p = xcd_block() * kBlock + threadIdx.x;
  const int n = sp.n;
  if (blockIdx.x == 0 && threadIdx.x < kDriftSpread) {
    // the positions of the next force evaluation are where this search sees them
    const int r = bound_slot(*clock + bound_step_rel, 0);
    sp.brec[r * kDriftSpread + threadIdx.x] = 0ull;
    if (threadIdx.x == 0) sp.bacc[bound_slot(*clock + bound_step_rel, -1)] = 0.0;
  }
  if (p >= n) return;
  const double t = (double)(*clock + step_rel) * sp.dt;  // walls where they are now
  int o = perm[p];
  inv[o] = p;
  double4 ps = src.pos[o];
  dst.pos[p] = ps;
  dst.vel[p] = src.vel[o];
  dst.omg[p] = src.omg[o];
  gid_dst[p] = gid_src[o];
  int inf = info_src[o];
  info_dst[p] = inf;
  xref[p] = ps;
  if (F_src) {
    F_dst[p] = F_src[o];
    T_dst[p] = T_src[o];
  }
  int c = 0;
  if (!(inf & kInactive)) {
    const InstDev& I = inst[inf >> kInstShift];
    double x[3] = {ps.x, ps.y, ps.z};
    for (int w = I.wall_begin; w < I.wall_end; ++w) {
      if (walls[w].kind == 3) continue;
      WallGeo g;
      wall_geo(walls[w], x, ps.w, I.skin, false, t, g);
      if (!g.candidate) continue;
      if (c == kWallSlots) {
        atomicOr(flags, kFlagWallOverflow);
        break;
      }
      double h0 = 0.0, h1 = 0.0, h2 = 0.0;
      for (int s = 0; s < kWallSlots; ++s) {
        int ow = ws_src.wid[(int64_t)s * n + o];
        if (ow < 0) break;
        if (ow == w) {
          h0 = ws_src.hist[(int64_t)(3 * s + 0) * n + o];
          h1 = ws_src.hist[(int64_t)(3 * s + 1) * n + o];
          h2 = ws_src.hist[(int64_t)(3 * s + 2) * n + o];
          break;
        }
      }
      ws_dst.wid[(int64_t)c * n + p] = w;
      ws_dst.hist[(int64_t)(3 * c + 0) * n + p] = h0;
      ws_dst.hist[(int64_t)(3 * c + 1) * n + p] = h1;
      ws_dst.hist[(int64_t)(3 * c + 2) * n + p] = h2;
      ++c;
    }
  }
  for (; c < kWallSlots; ++c) ws_dst.wid[(int64_t)c * n + p] = -1;
  if (!mt.tri) return;
  // particle-triangle candidates: the triangles listed in the centre's cell
  // of each mesh grid that lie less than R + skin away from it, with the
  // centre less than R behind their plane; overlaps carried by triangle
  int cm = 0;
  if (!(inf & kInactive)) {
    const InstDev& I = inst[inf >> kInstShift];
    const double x[3] = {ps.x, ps.y, ps.z};
    const double R = ps.w;
    const double m = R + I.skin;
    for (int w = I.wall_begin; w < I.wall_end && cm <= kMeshSlots; ++w) {
      const WallDev& W = walls[w];
      if (W.kind != 3) continue;
      int c3[3];
      bool in = true;
      for (int k = 0; k < 3; ++k) {
        const double u = (x[k] - W.vel[k] * t - W.mlo[k]) / W.mh;
        if (!(u >= 0.0 && u < (double)W.mnc[k])) in = false;
        c3[k] = in ? (int)u : 0;
      }
      if (!in) continue;
      const int cb = W.cell_base + c3[0] + W.mnc[0] * (c3[1] + W.mnc[1] * c3[2]);
      const int q1 = mt.cell[cb + 1];
      for (int q = mt.cell[cb]; q < q1; ++q) {
        const int tr = mt.cell_tri[q];
        TriGeo g;
        tri_closest(mt.tri[tr], W.vel, t, x, g);
        if (!(g.s > -R && g.d2 < m * m)) continue;
        if (cm == kMeshSlots) {
          atomicOr(flags, kFlagMeshOverflow);
          ++cm;
          break;
        }
        double h0 = 0.0, h1 = 0.0, h2 = 0.0;
        for (int s = 0; s < kMeshSlots; ++s) {
          const int ot = ms_src.tri[(int64_t)s * n + o];
          if (ot < 0) break;
          if (ot == tr) {
            h0 = ms_src.hist[(int64_t)(3 * s + 0) * n + o];
            h1 = ms_src.hist[(int64_t)(3 * s + 1) * n + o];
            h2 = ms_src.hist[(int64_t)(3 * s + 2) * n + o];
            break;
          }
        }
        ms_dst.tri[(int64_t)cm * n + p] = tr;
        ms_dst.hist[(int64_t)(3 * cm + 0) * n + p] = h0;
        ms_dst.hist[(int64_t)(3 * cm + 1) * n + p] = h1;
        ms_dst.hist[(int64_t)(3 * cm + 2) * n + p] = h2;
        ++cm;
      }
    }
  }
  for (int c2 = cm < kMeshSlots ? cm : kMeshSlots; c2 < kMeshSlots; ++c2)
    ms_dst.tri[(int64_t)c2 * n + p] = -1;
}

hipError_t launch_reorder(const StepParams& sp, const InstDev* inst, const int* perm, int* inv,
                          ParticleBufs src, ParticleBufs dst, const int* gid_src, int* gid_dst,
                          const int* info_src, int* info_dst, double4* xref,
                          WallSlots ws_src, WallSlots ws_dst, const WallDev* walls,
                          MeshTables mt, MeshSlots ms_src, MeshSlots ms_dst,
                          const double4* F_src, const double4* T_src, double4* F_dst,
                          double4* T_dst, const int64_t* clock, int64_t step_rel,
                          int64_t bound_step_rel, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_reorder, dim3(grid_for(sp.n)), dim3(kBlock), 0, s, sp, inst, perm, inv,
                     src, dst,
                     gid_src, gid_dst, info_src, info_dst, xref, ws_src, ws_dst, walls, mt,
                     ms_src, ms_dst, F_src, T_src, F_dst, T_dst, clock, step_rel,
                     bound_step_rel, flags);
  return hipGetLastError();
}

// ------------------------------------------------------------------ search

// Broad + fine search for particle p (sorted order): scan its own and the 26
// surrounding cells and keep q != p with |x_q - x_p|^2 < r_s^2 (evaluated in
// a fixed order without fused operations).  Pairs that touch now go to the
// front of the row (during the next steps the
// history accesses of a wavefront then stay in few cache lines), the others
// behind them in the order of their gap class (the row cuts of NbrList).
// Then the tangential overlaps are carried over (below).
// Positions of the search block's own sorted particles, staged in LDS: the
// cells around a block's particles hold many of the block's particles (a
// window with a halo of further sorted neighbours measured slower, its LDS
// footprint lowering occupancy).
struct SearchTile {
  double4 p[kBlock];
  int lo, hi;  // staged particles [lo, hi)
  __device__ __forceinline__ void stage(const double4* __restrict__ pos, int first, int n) {
    const int a = first;
    const int b = first + kBlock < n ? first + kBlock : n;
    for (int t = threadIdx.x; t < b - a; t += kBlock) p[t] = pos[a + t];
    if (threadIdx.x == 0) {
      lo = a;
      hi = b > a ? b : a;
    }
  }
  __device__ __forceinline__ double4 get(const double4* __restrict__ pos, int q) const {
    return (q >= lo && q < hi) ? p[q - lo] : pos[q];
  }
};

// Gap class of a candidate pair at distance^2 d2 (radius sum rsum, skin sk):
// 0 touching, 1..3 gap d - rsum below kCutFrac[0..2] skins, 4 farther
// (compared as squares, so no square root; the force evaluation keeps a
// relative margin far above the rounding of these comparisons).
__device__ __forceinline__ int gap_class(double d2, double rsum, double sk) {
  const double a = rsum + kCutFrac[0] * sk, b = rsum + kCutFrac[1] * sk,
               c = rsum + kCutFrac[2] * sk;
  return d2 < rsum * rsum ? 0 : (d2 < a * a ? 1 : (d2 < b * b ? 2 : (d2 < c * c ? 3 : 4)));
}

// Five counters, one per gap class, kept in registers (an array indexed by a
// class would be placed in memory).
struct Five {
  int v0 = 0, v1 = 0, v2 = 0, v3 = 0, v4 = 0;
  __device__ __forceinline__ int get(int i) const {
    return i == 0 ? v0 : (i == 1 ? v1 : (i == 2 ? v2 : (i == 3 ? v3 : v4)));
  }
  __device__ __forceinline__ void bump(int i) {
    v0 += i == 0 ? 1 : 0;
    v1 += i == 1 ? 1 : 0;
    v2 += i == 2 ? 1 : 0;
    v3 += i == 3 ? 1 : 0;
    v4 += i == 4 ? 1 : 0;
  }
  __device__ __forceinline__ void set(int i, int x) {
    v0 = i == 0 ? x : v0;
    v1 = i == 1 ? x : v1;
    v2 = i == 2 ? x : v2;
    v3 = i == 3 ? x : v3;
    v4 = i == 4 ? x : v4;
  }
};

constexpr unsigned kRowIndexMask = (1u << kClassShift) - 1u;

// A row under construction in the contact search: its first kRowLds entries
// in the workgroup's LDS (column threadIdx.x, so the lanes of a wavefront
// always hit distinct banks), the rest in place in the neighbour list.
constexpr int kRowLds = 11;
constexpr int kCarryBatch = 4;
struct BuildRow {
  int* lds;  // &buf[0][threadIdx.x], stride kBlock
  int* nbr;
  int p, max_nb;
  __device__ __forceinline__ unsigned load(int t) const {
    return t < kRowLds ? (unsigned)lds[t * kBlock] : (unsigned)nbr[nbr_entry(p, t, max_nb)];
  }
  __device__ __forceinline__ void store(int t, unsigned v) const {
    if (t < kRowLds)
      lds[t * kBlock] = (int)v;
    else
      nbr[nbr_entry(p, t, max_nb)] = (int)v;
  }
};

// One class of the in-place row sort (below): fill the free slots of class C
// in order; an entry found in one of them that belongs to class k != C goes
// to the next free slot of class k, whose occupant moves on in turn, until
// an entry of class C comes back for the slot.
template <int C>
__device__ __forceinline__ void place_class(const BuildRow& row, Five& nx, const Five& en) {
  for (int t = nx.get(C); t < en.get(C); ++t) {
    unsigned v = row.load(t);
    int k = (int)(v >> kClassShift);
    while (k != C) {
      const int u = nx.get(k);
      nx.bump(k);
      const unsigned f = row.load(u);
      row.store(u, v & kRowIndexMask);
      v = f;
      k = (int)(v >> kClassShift);
    }
    row.store(t, v & kRowIndexMask);
  }
  nx.set(C, en.get(C));
}

// kOne: the batch has a single instance, whose table entry then sits in
// scalar registers.  Eight wavefronts per SIMD (at most 64 VGPRs; both
// instantiations fit without spills): the scan is bound by the latency of
// its candidate loads.
template <bool kOne>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8)))
k_search(const InstDev* __restrict__ inst, StepParams sp,
                         const double4* __restrict__ pos,
                         const int* __restrict__ info, const int2* __restrict__ cse,
                         const int* __restrict__ perm, const int* __restrict__ inv,
                         NbrList old_l, NbrList new_l, int* __restrict__ flags) {
  const int b0 = xcd_block() * kBlock;
  int p = b0 + threadIdx.x;
  __shared__ SearchTile tile;
  __shared__ int rowbuf[kRowLds][kBlock];
  tile.stage(pos, b0, sp.n);
  __syncthreads();
  if (p >= sp.n) return;
  const int max_nb = sp.max_nb;
  const int inf = info[p];
  if (inf & kInactive) {
    new_l.rowlen[p] = 0;
    new_l.rowcut[p] = 0;
    return;
  }
  const BuildRow row{&rowbuf[0][threadIdx.x], new_l.nbr, p, max_nb};
  const InstDev& I = inst[kOne ? 0 : inf >> kInstShift];
  const GridDev& g = I.grid;
  const double rs2 = I.rs2;
  const double sk = I.skin;
  const uint32_t kbase = I.key_base;
  const double4 pp = pos[p];
  const int cx = cell_coord(pp.x, g.lo[0], g.h, g.nc[0]);
  const int cy = cell_coord(pp.y, g.lo[1], g.h, g.nc[1]);
  const int cz = cell_coord(pp.z, g.lo[2], g.h, g.nc[2]);
  // one pass: every candidate is stored in the order found, its gap class in
  // the entry's top bits
  int len = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = cz + dz;
    if (z < 0 || z >= g.nc[2]) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = cy + dy;
      if (y < 0 || y >= g.nc[1]) continue;
      // the cells of row (y, z), each with its (start, end) in sorted order
      // (fewer than 2^30 cells: the index fits an int)
      const int2* crow = cse + kbase + (z * g.nc[1] + y) * g.nc[0];
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = cx + dx;
        if (x < 0 || x >= g.nc[0]) continue;
        const int2 se = crow[x];
        const int s = se.x, e = se.y;
        for (int q = s; q < e; ++q) {
          if (q == p) continue;
          const double4 pq = tile.get(pos, q);
          const double ddx = pq.x - pp.x, ddy = pq.y - pp.y, ddz = pq.z - pp.z;
          const double d2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
          if (!(d2 < rs2)) continue;
          const int c = gap_class(d2, pp.w + pq.w, sk);
          if (len < max_nb) row.store(len, (unsigned)q | ((unsigned)c << kClassShift));
          ++len;
        }
      }
    }
  }
  int front = 0;
  int cut = (kCutMask << (2 * kCutBits)) | (kCutMask << kCutBits) | kCutMask;
  if (len > max_nb) {
    // the row is incomplete and the step fails; leave valid indices behind
    atomicOr(flags, kFlagNbrOverflow);
    len = max_nb;
    for (int k = 0; k < len; ++k) row.store(k, row.load(k) & kRowIndexMask);
  } else {
    // sort the row by class in place (each entry moves once), clearing the
    // class bits
    Five at;
    for (int t = 0; t < len; ++t) at.bump((int)(row.load(t) >> kClassShift));
    Five nx, en;
    nx.v0 = 0;
    en.v0 = nx.v1 = at.v0;
    en.v1 = nx.v2 = en.v0 + at.v1;
    en.v2 = nx.v3 = en.v1 + at.v2;
    en.v3 = nx.v4 = en.v2 + at.v3;
    en.v4 = len;
    place_class<0>(row, nx, en);
    place_class<1>(row, nx, en);
    place_class<2>(row, nx, en);
    place_class<3>(row, nx, en);
    for (int t = nx.v4; t < len; ++t) row.store(t, row.load(t) & kRowIndexMask);
    front = at.v0;
    const int c1 = en.v1 < kCutMask ? en.v1 : kCutMask;
    const int c2 = en.v2 < kCutMask ? en.v2 : kCutMask;
    const int c3 = en.v3 < kCutMask ? en.v3 : kCutMask;
    cut = c1 | (c2 << kCutBits) | (c3 << (2 * kCutBits));
  }
  new_l.rowlen[p] = len;
  new_l.rowcut[p] = cut;
  // history carry-over for pairs that touched at the last force evaluation
  // and touch now (a pair that does not touch now has its overlap restarted
  // at zero by the first evaluation, at these positions, anyway): every entry
  // of p's old row with bit 31 names its partner by old index; inv maps it to
  // the new index, which is looked up among the touching entries of the new
  // row.  Entries without bit 31 have zero history, which is never stored.
  // The old entries, their inverse-permutation lookups and the histories of
  // the matched pairs are fetched kCarryBatch entries at a time, so that
  // their loads are in flight together.
  const int op = perm[p];
  const int olen = old_l.rowlen[op];
  for (int k0 = 0; k0 < olen; k0 += kCarryBatch) {
    int oj[kCarryBatch], qn[kCarryBatch];
#pragma unroll
    for (int j = 0; j < kCarryBatch; ++j)
      oj[j] = k0 + j < olen ? old_l.nbr[nbr_entry(op, k0 + j, max_nb)] : 0;
#pragma unroll
    for (int j = 0; j < kCarryBatch; ++j)
      qn[j] = (oj[j] & (int)0x80000000u) ? inv[oj[j] & 0x7fffffff] : -1;
    int mj[kCarryBatch];
#pragma unroll
    for (int j = 0; j < kCarryBatch; ++j) {
      mj[j] = -1;
      if (qn[j] < 0) continue;
      const unsigned q = (unsigned)qn[j];
      for (int m = 0; m < front; ++m) {
        if (row.load(m) == q) {
          row.store(m, q | 0x80000000u);
          mj[j] = m;
          break;
        }
      }
    }
    double h0[kCarryBatch], h1[kCarryBatch], h2[kCarryBatch];
#pragma unroll
    for (int j = 0; j < kCarryBatch; ++j) {
      if (mj[j] < 0) continue;
      const int64_t oe = nbr_entry(op, k0 + j, max_nb);
      h0[j] = old_l.hist[oe];
      h1[j] = old_l.hist[old_l.cap + oe];
      h2[j] = old_l.hist[2 * old_l.cap + oe];
    }
#pragma unroll
    for (int j = 0; j < kCarryBatch; ++j) {
      if (mj[j] < 0) continue;
      const int64_t ne = nbr_entry(p, mj[j], max_nb);
      new_l.hist[ne] = h0[j];
      new_l.hist[new_l.cap + ne] = h1[j];
      new_l.hist[2 * new_l.cap + ne] = h2[j];
    }
  }
  // the part of the row held in LDS goes out entry by entry for the whole
  // wavefront at once (whole cache lines; the part beyond is in place)
  for (int k = 0; k < kRowLds; ++k)
    if (k < len) new_l.nbr[nbr_entry(p, k, max_nb)] = rowbuf[k][threadIdx.x];
}

hipError_t launch_search(const InstDev* inst, int n_inst, const StepParams& sp,
                         const double4* pos, const int* info, const int2* cse, const int* perm,
                         const int* inv, NbrList old_l, NbrList new_l, int* flags,
                         hipStream_t s) {
  if (sp.n <= 0) return hipSuccess;
  if (n_inst == 1)
    hipLaunchKernelGGL(k_search<true>, dim3(grid_for(sp.n)), dim3(kBlock), 0, s, inst, sp, pos,
                       info, cse, perm, inv, old_l, new_l, flags);
  else
    hipLaunchKernelGGL(k_search<false>, dim3(grid_for(sp.n)), dim3(kBlock), 0, s, inst, sp, pos,
                       info, cse, perm, inv, old_l, new_l, flags);
  return hipGetLastError();
}

// ------------------------------------------------------------- contact law

// Square roots and reciprocals.  Double: the hardware estimates refined by two
// Newton-Raphson steps each (rsqrt: y <- y (3 - x y^2) / 2; reciprocal:
// y <- y (2 - x y)), a few ulp from the correctly rounded value, far cheaper
// than the correctly rounded library sequences.  Float: the single hardware
// instructions (about 1 ulp).  Every function of a symmetric argument returns
// the same value whichever side of the pair evaluates it.
template <typename R>
struct Fast;

template <>
struct Fast<double> {
  static __device__ __forceinline__ double rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
  }
  static __device__ __forceinline__ double rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
  }
  static __device__ __forceinline__ double sqrt(double x) {
    return x > 0.0 ? x * rsqrt(x) : 0.0;
  }
  // fifth root: a single-precision estimate 2^(log2(x) / 5) refined by two
  // steps of Newton's iteration for y^5 = x, y <- (4 y + x / y^4) / 5 (the
  // error squares at each step: about 1e-7, 1e-14, then FP64 rounding)
  static __device__ __forceinline__ double root5(double x) {
    if (!(x > 0.0)) return 0.0;
    double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)x) * 0.2f);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double y2 = y * y;
      y = 0.8 * y + (0.2 * x) * rcp(y2 * y2);
    }
    return y;
  }
};

template <>
struct Fast<float> {
  static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float root5(float x) { return ::powf(x, 0.2f); }
};

// The spring-dashpot law (Sec. 2.1) in arithmetic type R for one contact,
// given the overlap dn >= 0, the unit normal n from body i to body j, the
// contact relative velocity vij, wrel = omega_i - omega_j, the rolling speed
// vr = |V_omega| (table of rolling models; used by the viscous model), the effective mass
// and radius and the lever arm Ri.  The tangential overlap dtl stays in FP64
// and is updated in place (Eq. delta_t before the force, Coulomb truncation
// of Eqs. coulomb_overlap..3 after it).  Output: force and torque on body i.
// model 0, Hertz-Mindlin: k_n = (4/3) Y_e q, k_t = 8 G_e q, eta = -2 sqrt(5/6)
// beta sqrt(S m_e), q = sqrt(R_e dn); the per-pair constants are c.kn = 4/3
// Y_e, c.kt = 8 G_e, c.en = -2 sqrt(5/6) beta sqrt(2 Y_e), c.et = -2 sqrt(5/6)
// beta sqrt(8 G_e).  model 1, linear (Eqs. linearkn, linearetan, the same
// constants tangentially): k = c.kn (R_e^2 m_e)^(1/5) with c.kn = (16/15) Y_e
// (15 V^2 / (16 Y_e))^(1/5), eta = c.en sqrt(m_e k) with c.en = 2 / sqrt(1 +
// (pi / ln e)^2).
template <typename R>
__device__ __forceinline__ void hm_law(const PairCoef& c, int rolling, int model, double dt,
                                       R dn, const R n[3], const R vij[3], const R wrel[3],
                                       R vr, R me, R Re, R Ri, double dtl[3],
                                       double Fi[3], double Mi[3]) {
  using M = Fast<R>;
  const R vn = (vij[0] * n[0] + vij[1] * n[1]) + vij[2] * n[2];
  const R vrn[3] = {vn * n[0], vn * n[1], vn * n[2]};
  const R vrt[3] = {vij[0] - vrn[0], vij[1] - vrn[1], vij[2] - vrn[2]};
  dtl[0] = dtl[0] + (double)vrt[0] * dt;
  dtl[1] = dtl[1] + (double)vrt[1] * dt;
  dtl[2] = dtl[2] + (double)vrt[2] * dt;
  R kn, kt, etan, etat;
  if (model == 0) {
    const R q = M::sqrt(Re * dn);
    kn = (R)c.kn * q;
    kt = (R)c.kt * q;
    const R sq = M::sqrt(me * q);
    etan = (R)c.en * sq;
    etat = (R)c.et * sq;
  } else {
    kn = (R)c.kn * M::root5((Re * Re) * me);
    kt = kn;
    etan = (R)c.en * M::sqrt(me * kn);
    etat = etan;
  }
  const R knd = kn * dn;
  R Fn[3], Ft[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Fn[k] = -(knd * n[k]) - etan * vrn[k];
    Ft[k] = -(kt * (R)dtl[k]) - etat * vrt[k];
  }
  const R fn2 = (Fn[0] * Fn[0] + Fn[1] * Fn[1]) + Fn[2] * Fn[2];
  const R ft2 = (Ft[0] * Ft[0] + Ft[1] * Ft[1]) + Ft[2] * Ft[2];
  const R fn = M::sqrt(fn2);
  const R mufn = (R)c.mu * fn;
  if (ft2 >= mufn * mufn && ft2 > (R)0) {
    const R ratio = mufn * M::rsqrt(ft2);
    const R mikt = -M::rcp(kt);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R fhat = ratio * Ft[k];
      dtl[k] = (double)((fhat + etat * vrt[k]) * mikt);
      Ft[k] = fhat;
    }
  }
  R Mr[3] = {(R)0, (R)0, (R)0};
  if (rolling != 0) {
    const R wn2 = (wrel[0] * wrel[0] + wrel[1] * wrel[1]) + wrel[2] * wrel[2];
    if (wn2 > (R)0) {
      R mag = (R)c.mur * Re * fn;  // constant torque; viscous: times |V_omega|
      if (rolling == 2) mag = mag * vr;
      const R sc = -mag * M::rsqrt(wn2);
      Mr[0] = sc * wrel[0];
      Mr[1] = sc * wrel[1];
      Mr[2] = sc * wrel[2];
    }
  }
  const R nx[3] = {n[1] * Ft[2] - n[2] * Ft[1], n[2] * Ft[0] - n[0] * Ft[2],
                   n[0] * Ft[1] - n[1] * Ft[0]};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Fi[k] = (double)(Fn[k] + Ft[k]);
    Mi[k] = (double)(Ri * nx[k] + Mr[k]);
  }
}

// Particle i against a touching neighbour j, evaluated from i's side
// (pos = (x, R), vel = (v, 1/m), omg = (omega, 1/I)).  Written so that the
// evaluation from j's side gives exactly -F and -delta_t: every symmetric
// quantity is formed from commutative operations of the two particles' data.
template <typename R>
__device__ __forceinline__ void pp_contact(const PairCoef& c, int rolling, int model, double dt,
                                           double4 xi, double4 vi, double4 wi, double4 xj,
                                           double4 vj, double4 wj, double dtl[3], double Fi[3],
                                           double Mi[3]);

template <>
__device__ __forceinline__ void pp_contact<double>(const PairCoef& c, int rolling, int model,
                                                   double dt,
                                                   double4 xi, double4 vi, double4 wi,
                                                   double4 xj, double4 vj, double4 wj,
                                                   double dtl[3], double Fi[3], double Mi[3]) {
  using M = Fast<double>;
  const double dx[3] = {xj.x - xi.x, xj.y - xi.y, xj.z - xi.z};
  const double d2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
  const double Ri = xi.w, Rj = xj.w;
  const double rsum = Ri + Rj;
  const double inv_d = M::rsqrt(d2);
  double dn = rsum - d2 * inv_d;
  if (dn < 0.0) dn = 0.0;
  const double n[3] = {dx[0] * inv_d, dx[1] * inv_d, dx[2] * inv_d};
  const double rw[3] = {Ri * wi.x + Rj * wj.x, Ri * wi.y + Rj * wj.y, Ri * wi.z + Rj * wj.z};
  // rolling velocity V_omega = (R_i w_i + R_j w_j) x n, part of the contact velocity
  const double vroll[3] = {rw[1] * n[2] - rw[2] * n[1], rw[2] * n[0] - rw[0] * n[2],
                           rw[0] * n[1] - rw[1] * n[0]};
  const double vij[3] = {(vi.x - vj.x) + vroll[0], (vi.y - vj.y) + vroll[1],
                         (vi.z - vj.z) + vroll[2]};
  const double wrel[3] = {wi.x - wj.x, wi.y - wj.y, wi.z - wj.z};
  const double me = M::rcp(vi.w + vj.w);
  const double Re = (Ri * Rj) * M::rcp(rsum);
  const double vr = rolling == 2 ? M::sqrt(dot3(vroll, vroll)) : 0.0;
  hm_law<double>(c, rolling, model, dt, dn, n, vij, wrel, vr, me, Re, Ri, dtl, Fi, Mi);
}

// FP32 contact law.  The overlap is formed without cancellation:
// dn = (rsum^2 - d^2) / (rsum + d) with the numerator from FP64 positions.
template <>
__device__ __forceinline__ void pp_contact<float>(const PairCoef& c, int rolling, int model,
                                                  double dt,
                                                  double4 xi, double4 vi, double4 wi,
                                                  double4 xj, double4 vj, double4 wj,
                                                  double dtl[3], double Fi[3], double Mi[3]) {
  using M = Fast<float>;
  const double dx[3] = {xj.x - xi.x, xj.y - xi.y, xj.z - xi.z};
  const double d2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
  const double rsum = xi.w + xj.w;
  const float d2f = (float)d2;
  const float inv_d = M::rsqrt(d2f);
  const float num = (float)(rsum * rsum - d2);
  float dn = num * M::rcp((float)rsum + d2f * inv_d);
  if (dn < 0.0f) dn = 0.0f;
  const float n[3] = {(float)dx[0] * inv_d, (float)dx[1] * inv_d, (float)dx[2] * inv_d};
  const float Ri = (float)xi.w, Rj = (float)xj.w;
  const float rw[3] = {Ri * (float)wi.x + Rj * (float)wj.x, Ri * (float)wi.y + Rj * (float)wj.y,
                       Ri * (float)wi.z + Rj * (float)wj.z};
  const float vroll[3] = {rw[1] * n[2] - rw[2] * n[1], rw[2] * n[0] - rw[0] * n[2],
                          rw[0] * n[1] - rw[1] * n[0]};
  const float vij[3] = {(float)(vi.x - vj.x) + vroll[0], (float)(vi.y - vj.y) + vroll[1],
                        (float)(vi.z - vj.z) + vroll[2]};
  const float wrel[3] = {(float)(wi.x - wj.x), (float)(wi.y - wj.y), (float)(wi.z - wj.z)};
  const float me = M::rcp((float)(vi.w + vj.w));
  const float Re = (Ri * Rj) * M::rcp(Ri + Rj);
  const float vr =
      rolling == 2 ? M::sqrt((vroll[0] * vroll[0] + vroll[1] * vroll[1]) + vroll[2] * vroll[2])
                   : 0.0f;
  hm_law<float>(c, rolling, model, dt, dn, n, vij, wrel, vr, me, Re, Ri, dtl, Fi, Mi);
}

// The law against wall W, a body of infinite mass and radius whose contact
// point moves with the wall's surface velocity: unit normal gn from the
// particle to the wall, overlap gdn, lever arm of the contact point about the
// wall's rotation axis.
template <typename R>
__device__ __forceinline__ void wall_law(const PairCoef& c, int rolling, int model, double dt,
                                         const WallDev& W, const double gn[3], double gdn,
                                         const double arm[3], double4 xi, double4 vi,
                                         double4 wi, double dtl[3], double Fi[3],
                                         double Mi[3]) {
  const double dn = gdn < 0.0 ? 0.0 : gdn;
  const double vw[3] = {W.vel[0] + (W.omega[1] * arm[2] - W.omega[2] * arm[1]),
                        W.vel[1] + (W.omega[2] * arm[0] - W.omega[0] * arm[2]),
                        W.vel[2] + (W.omega[0] * arm[1] - W.omega[1] * arm[0])};
  const double Ri = xi.w;
  const double rw[3] = {Ri * wi.x, Ri * wi.y, Ri * wi.z};
  const double vd[3] = {(vi.x - vw[0]) + (rw[1] * gn[2] - rw[2] * gn[1]),
                        (vi.y - vw[1]) + (rw[2] * gn[0] - rw[0] * gn[2]),
                        (vi.z - vw[2]) + (rw[0] * gn[1] - rw[1] * gn[0])};
  const double wd[3] = {wi.x - W.omega[0], wi.y - W.omega[1], wi.z - W.omega[2]};
  const R n[3] = {(R)gn[0], (R)gn[1], (R)gn[2]};
  const R vij[3] = {(R)vd[0], (R)vd[1], (R)vd[2]};
  const R wrel[3] = {(R)wd[0], (R)wd[1], (R)wd[2]};
  // rolling speed against a wall: |R_i (omega_i - Omega_wall) x n|
  R vr = (R)0;
  if (rolling == 2) {
    const R rr[3] = {(R)Ri * wrel[0], (R)Ri * wrel[1], (R)Ri * wrel[2]};
    const R vroll[3] = {rr[1] * n[2] - rr[2] * n[1], rr[2] * n[0] - rr[0] * n[2],
                        rr[0] * n[1] - rr[1] * n[0]};
    vr = Fast<R>::sqrt((vroll[0] * vroll[0] + vroll[1] * vroll[1]) + vroll[2] * vroll[2]);
  }
  const R me = Fast<R>::rcp((R)vi.w);
  hm_law<R>(c, rolling, model, dt, (R)dn, n, vij, wrel, vr, me, (R)Ri, (R)Ri, dtl, Fi, Mi);
}

// Particle against wall W at time t.
template <typename R>
__device__ __forceinline__ void pw_contact(const PairCoef& c, int rolling, int model, double dt,
                                           const WallDev& W, double skin, double t, double4 xi,
                                           double4 vi, double4 wi, double dtl[3],
                                           double Fi[3], double Mi[3]) {
  const double x[3] = {xi.x, xi.y, xi.z};
  WallGeo g;
  wall_geo(W, x, xi.w, skin, true, t, g);
  if (!g.touching) {
    dtl[0] = dtl[1] = dtl[2] = 0.0;
    Fi[0] = Fi[1] = Fi[2] = 0.0;
    Mi[0] = Mi[1] = Mi[2] = 0.0;
    return;
  }
  wall_law<R>(c, rolling, model, dt, W, g.n, g.dn, g.arm, xi, vi, wi, dtl, Fi, Mi);
}

// ------------------------------------------------------------------- force
//
// One thread per particle walks its row in order (every load of a row entry
// is one coalesced access for the wavefront); the neighbour's velocities and
// the pair history are loaded only when the pair touches.  Bit 31 of a row
// entry marks "touching at the last evaluation" (history may be non-zero);
// histories of other entries are zero and are neither read nor written.

constexpr int kTouchedBit = (int)0x80000000u;
constexpr int kIndexMask = 0x7fffffff;

// Accesses to data that only the particle's own thread touches in a force
// launch (its row, row length, pair and wall histories, its new state) are
// non-temporal: they are not reused from the caches within the launch, and
// leaving L2 to the neighbour gathers, which are, made the launch 3-4 %
// faster.
template <typename T>
__device__ __forceinline__ T ld_own(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_own(T v, T* p) {
  __builtin_nontemporal_store(v, p);
}
typedef double own_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_own(const double4& v, double4* p) {
  const own_d4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<own_d4*>(p));
}

// The states of the BS consecutive sorted particles of a force block, staged
// in LDS: in spatial (Morton) order most neighbours of a block's particles lie
// inside the block, and they are then read from LDS instead of through the
// cache hierarchy.
template <int BS>
struct Tile {
  double4 p[BS], v[BS], w[BS];
  int in[BS];
  int lo, hi;  // staged particles [lo, hi)

  __device__ __forceinline__ void stage(const ParticleBufs& src, const int* __restrict__ info,
                                        int first, int n) {
    const int a = first;
    const int b = first + BS < n ? first + BS : n;
    for (int t = threadIdx.x; t < b - a; t += BS) {
      p[t] = src.pos[a + t];
      v[t] = src.vel[a + t];
      w[t] = src.omg[a + t];
      in[t] = info[a + t];
    }
    if (threadIdx.x == 0) {
      lo = a;
      hi = b > a ? b : a;
    }
  }
  __device__ __forceinline__ bool has(int j) const { return j >= lo && j < hi; }
  __device__ __forceinline__ double4 pos(const ParticleBufs& g, int j) const {
    return has(j) ? p[j - lo] : g.pos[j];
  }
  __device__ __forceinline__ double4 vel(const ParticleBufs& g, int j) const {
    return has(j) ? v[j - lo] : g.vel[j];
  }
  __device__ __forceinline__ double4 omg(const ParticleBufs& g, int j) const {
    return has(j) ? w[j - lo] : g.omg[j];
  }
  __device__ __forceinline__ int info(const int* __restrict__ g, int j) const {
    return has(j) ? in[j - lo] : g[j];
  }
};

// Square of a step's drift |v| dt in units of half the skin: scale = dt * 2 /
// skin.  Maxima of squares are taken on the device, the root on the host.
__device__ __forceinline__ double drift2(const double4& v, double scale) {
  const double s2 = scale * scale;
  return ((v.x * v.x + v.y * v.y) + v.z * v.z) * s2;
}

// dt * 2 / skin of the particle's instance (uniform when all skins agree)
__device__ __forceinline__ double drift_scale(const StepParams& sp,
                                              const InstDev* __restrict__ inst, int inf) {
  return sp.drift_scale > 0.0 ? sp.drift_scale : sp.dt * inst[inf >> kInstShift].ihs;
}

// Forces on particle i and its integration; returns the squared drift of
// this step in units of half the instance's skin (for the dynamic search
// trigger) when asked for it.
template <typename R, int MODE, int MODEL, bool REC, int PAIRS, typename TileT>
__device__ __forceinline__ double force_particle(
    const int i, const StepParams& sp, const InstDev* __restrict__ inst,
    const PairCoef* __restrict__ ppc, const PairCoef* __restrict__ pwc,
    const WallDev* __restrict__ walls, ParticleBufs in, ParticleBufs out,
    const int* __restrict__ info, NbrList l, WallSlots ws, double4* __restrict__ Fo,
    double4* __restrict__ To, const int64_t* __restrict__ clock, int64_t step_rel,
    const int* __restrict__ flags, const bool want_drift, const int* __restrict__ xsel,
    const double4* __restrict__ Fx, const double4* __restrict__ Tx, const TileT& tile,
    const int len, const int jr0, double* __restrict__ pf) {
  const int n = sp.n;
  double4 xi = tile.pos(in, i);
  // the particle's own velocity and spin stay in the LDS tile during the row
  // walk and are read where they are used (registers for the neighbour's)
  const int own = i - tile.lo;
  const int inf = tile.info(info, i);
  // frozen after an error, and for inactive particles: carry the state over
  if ((inf & kInactive) || *flags != 0) {
    out.pos[i] = xi;
    out.vel[i] = tile.v[own];
    out.omg[i] = tile.w[own];
    if (MODE != 0) {
      Fo[i] = make_double4(0.0, 0.0, 0.0, 0.0);
      To[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    }
    return 0.0;
  }
  // material-pair row of (instance, type i): instance b's table starts at
  // b * kMaxTypes^2, so it follows from the info word without a lookup
  const int ti = inf & kTypeMask;
  const int row = ((inf >> kInstShift) * kMaxTypes + ti) * kMaxTypes;
  const PairCoef* __restrict__ ppi = ppc + row;
  const PairCoef* __restrict__ pwi = pwc + row;
  // PAIRS 1: a single instance whose particles all have type 0, so every
  // pair takes the table's first entry, read once for the wavefront;
  // PAIRS 2: every particle has type 0, so the pair's entry is the first of
  // the particle's own row (its load does not wait for the neighbour's
  // type), read once for the wavefront when all its lanes share the row
  PairCoef pc0;
  if (PAIRS == 1) pc0 = ppc[0];
  bool uni = false;  // PAIRS 2: the wavefront's lanes share one row
  if (PAIRS == 2) {
    const int rowu = __builtin_amdgcn_readfirstlane(row);
    uni = __builtin_amdgcn_ballot_w64(row != rowu) == 0ull;
    if (uni) pc0 = ppc[rowu];
  }
  const double dt = sp.dt;
  double F[3] = {0.0, 0.0, 0.0};
  double T[3] = {0.0, 0.0, 0.0};
  const int max_nb = sp.max_nb;
  const int64_t cap = l.cap;
  // the index of entry k + 1 is loaded while entry k is worked on (the
  // row walk is a chain of dependent loads; one index ahead costs one VGPR);
  // the row length and entry 0 come from the caller
  int jr_next = jr0;
  for (int k = 0; k < len; ++k) {
    const int64_t e = nbr_entry(i, k, max_nb);
    const int jr = jr_next;
    if (k + 1 < len) jr_next = ld_own(l.nbr + e + 64);  // entry (i, k + 1)
    const int j = jr & kIndexMask;
    // a pair touching at the last evaluation most likely still touches: its
    // history is loaded together with the neighbour's position
    double dtl[3] = {0.0, 0.0, 0.0};
    if (jr & kTouchedBit) {
      dtl[0] = ld_own(l.hist + e);
      dtl[1] = ld_own(l.hist + cap + e);
      dtl[2] = ld_own(l.hist + 2 * cap + e);
    }
    const double4 xj = tile.pos(in, j);
    const double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const double rsum = xi.w + xj.w;
    if (d2 < rsum * rsum) {
      const double4 vj = tile.vel(in, j);
      const double4 wj = tile.omg(in, j);
      int oi = own;
      asm volatile("" : "+v"(oi));  // keeps the LDS reads inside the loop
      const double4 vi = tile.v[oi];
      const double4 wi = tile.w[oi];
      double Fi[3], Mi[3];
      if (PAIRS == 1) {
        pp_contact<R>(pc0, sp.rolling, MODEL, dt, xi, vi, wi, xj, vj, wj, dtl, Fi, Mi);
      } else if (PAIRS == 2) {
        if (uni)
          pp_contact<R>(pc0, sp.rolling, MODEL, dt, xi, vi, wi, xj, vj, wj, dtl, Fi, Mi);
        else
          pp_contact<R>(ppi[0], sp.rolling, MODEL, dt, xi, vi, wi, xj, vj, wj, dtl, Fi, Mi);
      } else {
        const int tj = tile.info(info, j) & kTypeMask;
        pp_contact<R>(ppi[tj], sp.rolling, MODEL, dt, xi, vi, wi, xj, vj, wj, dtl, Fi, Mi);
      }
      st_own(dtl[0], l.hist + e);
      st_own(dtl[1], l.hist + cap + e);
      st_own(dtl[2], l.hist + 2 * cap + e);
      if (!(jr & kTouchedBit)) st_own(j | kTouchedBit, l.nbr + e);
      if (REC) {
        pf[e] = Fi[0];
        pf[cap + e] = Fi[1];
        pf[2 * cap + e] = Fi[2];
      }
      F[0] += Fi[0];
      F[1] += Fi[1];
      F[2] += Fi[2];
      T[0] += Mi[0];
      T[1] += Mi[1];
      T[2] += Mi[2];
    } else if (jr & kTouchedBit) {
      st_own(0.0, l.hist + e);
      st_own(0.0, l.hist + cap + e);
      st_own(0.0, l.hist + 2 * cap + e);
      st_own(j, l.nbr + e);
    }
  }
  double4 vi = tile.v[own];
  double4 wi = tile.w[own];
  // walls: time of this force evaluation
  const double t = (double)(*clock + step_rel) * dt;
  for (int s = 0; s < kWallSlots; ++s) {
    const int w = ws.wid[(int64_t)s * n + i];
    if (w < 0) break;
    const WallDev& W = walls[w];
    double dtl[3] = {ws.hist[(int64_t)(3 * s) * n + i], ws.hist[(int64_t)(3 * s + 1) * n + i],
                     ws.hist[(int64_t)(3 * s + 2) * n + i]};
    double Fi[3], Mi[3];
    if (t >= W.t_on && t < W.t_off) {
      pw_contact<R>(pwi[W.material], sp.rolling, MODEL, dt, W, W.skin, t, xi, vi, wi, dtl, Fi,
                    Mi);
    } else {
      dtl[0] = dtl[1] = dtl[2] = 0.0;
      Fi[0] = Fi[1] = Fi[2] = 0.0;
      Mi[0] = Mi[1] = Mi[2] = 0.0;
    }
    st_own(dtl[0], ws.hist + (int64_t)(3 * s) * n + i);
    st_own(dtl[1], ws.hist + (int64_t)(3 * s + 1) * n + i);
    st_own(dtl[2], ws.hist + (int64_t)(3 * s + 2) * n + i);
    F[0] += Fi[0];
    F[1] += Fi[1];
    F[2] += Fi[2];
    T[0] += Mi[0];
    T[1] += Mi[1];
    T[2] += Mi[2];
  }
  if (xsel && xsel[i] >= 0) {
    const double4 fx = Fx[i], tx = Tx[i];
    F[0] += fx.x;
    F[1] += fx.y;
    F[2] += fx.z;
    T[0] += tx.x;
    T[1] += tx.y;
    T[2] += tx.z;
  }
  // integration of particle i (vel.w = 1/m, omg.w = 1/I)
  const double im = vi.w, iI = wi.w;
  const double a[3] = {F[0] * im + sp.g[0], F[1] * im + sp.g[1], F[2] * im + sp.g[2]};
  const double al[3] = {T[0] * iI, T[1] * iI, T[2] * iI};
  double drift = 0.0;
  if (MODE == 2) {
    // explicit Euler, Eq. (integ_EE): x with the old velocity
    if (want_drift) drift = drift2(vi, drift_scale(sp, inst, inf));
    xi.x = xi.x + vi.x * dt;
    xi.y = xi.y + vi.y * dt;
    xi.z = xi.z + vi.z * dt;
    vi.x = vi.x + a[0] * dt;
    vi.y = vi.y + a[1] * dt;
    vi.z = vi.z + a[2] * dt;
    wi.x = wi.x + al[0] * dt;
    wi.y = wi.y + al[1] * dt;
    wi.z = wi.z + al[2] * dt;
  } else {
    const double h = sp.hdt;
    // second half kick of this step, Eq. (newvv)
    vi.x = vi.x + a[0] * h;
    vi.y = vi.y + a[1] * h;
    vi.z = vi.z + a[2] * h;
    wi.x = wi.x + al[0] * h;
    wi.y = wi.y + al[1] * h;
    wi.z = wi.z + al[2] * h;
    if (MODE == 0) {
      // first half kick and drift of the next step, Eq. (halfstep)
      vi.x = vi.x + a[0] * h;
      vi.y = vi.y + a[1] * h;
      vi.z = vi.z + a[2] * h;
      wi.x = wi.x + al[0] * h;
      wi.y = wi.y + al[1] * h;
      wi.z = wi.z + al[2] * h;
      xi.x = xi.x + vi.x * dt;
      xi.y = xi.y + vi.y * dt;
      xi.z = xi.z + vi.z * dt;
      if (want_drift) drift = drift2(vi, drift_scale(sp, inst, inf));
    }
  }
  st_own(xi, out.pos + i);
  st_own(vi, out.vel + i);
  st_own(wi, out.omg + i);
  if (MODE != 0) {
    Fo[i] = make_double4(F[0], F[1], F[2], 0.0);
    To[i] = make_double4(T[0], T[1], T[2], 0.0);
  }
  return drift;
}

// Largest value of a wavefront (shuffles), then one atomic per wavefront on
// one of kDriftSpread words: non-negative doubles order like their bit
// patterns.  Every lane of the wavefront calls it; waves_per_block is the
// block size in wavefronts.
__device__ __forceinline__ void wave_max_store(unsigned long long* dst, double v,
                                               int waves_per_block = kBlock / 64) {
  const int w = (blockIdx.x * waves_per_block + (threadIdx.x >> 6)) & (kDriftSpread - 1);
  if ((threadIdx.x & 63) == 0 && v > 0.0)
    atomicMax(dst + w, (unsigned long long)__double_as_longlong(v));
}
// returns the wavefront's maximum
__device__ __forceinline__ double wave_max_to(unsigned long long* dst, double v,
                                              int waves_per_block = kBlock / 64) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  wave_max_store(dst, v, waves_per_block);
  return v;
}

// Occupancy floor: four wavefronts per SIMD (128 VGPRs, no spills), except
// for the linear law with explicit Euler, which would spill there and keeps
// three.
// REC: also write every touching pair's force to pf (the per-contact record;
// a separate instantiation, so the record costs the plain kernel nothing).
// PAIRS: how a pair finds its material-pair constants (see force_particle).
template <typename R, int MODE, int MODEL, int BS, bool REC, int PAIRS>
__global__ void __launch_bounds__(BS)
    __attribute__((amdgpu_waves_per_eu(MODE == 2 && MODEL == 1 ? 3 : 4)))
k_force(StepParams sp, const InstDev* __restrict__ inst, const PairCoef* __restrict__ ppc,
        const PairCoef* __restrict__ pwc, const WallDev* __restrict__ walls, ParticleBufs in,
        ParticleBufs out, const int* __restrict__ info, NbrList l, WallSlots ws,
        double4* __restrict__ Fo, double4* __restrict__ To, const int64_t* __restrict__ clock,
        int64_t step_rel, const int* __restrict__ flags, unsigned long long* __restrict__ drift,
        const int* __restrict__ xsel, const double4* __restrict__ Fx,
        const double4* __restrict__ Tx, double* __restrict__ pf) {
  const int b0 = xcd_block() * BS;
  const int i = b0 + threadIdx.x;
  const int64_t step = *clock + step_rel;  // these positions are x^step
  // the row length, its cuts and the first row entry do not depend on the
  // tile: their loads are issued before it is staged (entry 0 exists for
  // every row)
  int len = 0, cut = 0, jr0 = 0;
  if (i < sp.n) {
    len = ld_own(l.rowlen + i);
    cut = ld_own(l.rowcut + i);
    jr0 = ld_own(l.nbr + nbr_entry(i, 0, sp.max_nb));
  }
  // displacement bound of x^step since the last search (half skins): the
  // previous evaluation's bound plus the largest drift of the update since;
  // then the row cut it allows (uniform across the wavefront; a relative
  // margin of 1e-6 covers every rounding of the bound and of the gaps)
  int u_cut;
  {
    // the record's words, read with one address for the whole wavefront
    // (non-negative doubles order like their bit patterns)
    const unsigned long long* rw = sp.brec + bound_slot(step, 0) * kDriftSpread;
    unsigned long long mb = 0ull;
#pragma unroll
    for (int w = 0; w < kDriftSpread; ++w) mb = rw[w] > mb ? rw[w] : mb;
    const double m2 = __longlong_as_double((long long)mb);
    const double acc = sp.bacc[bound_slot(step, -1)] + sqrt(m2);
    if (blockIdx.x == 0 && threadIdx.x < kDriftSpread) {
      sp.brec[bound_slot(step, 2) * kDriftSpread + threadIdx.x] = 0ull;
      if (threadIdx.x == 0) sp.bacc[bound_slot(step, 0)] = acc;
    }
    const double accm = acc * (1.0 + 1e-6);
    u_cut = accm < kCutFrac[0] ? 0 : (accm < kCutFrac[1] ? 1 : (accm < kCutFrac[2] ? 2 : 3));
    u_cut = __builtin_amdgcn_readfirstlane(u_cut);
  }
  if (u_cut < 3) {
    const int c = (cut >> (kCutBits * u_cut)) & kCutMask;
    if (c != kCutMask && c < len) len = c;
  }
  __shared__ Tile<BS> tile;
  tile.stage(in, info, b0, sp.n);
  __syncthreads();
  double d = 0.0;
  if (i < sp.n)
    d = force_particle<R, MODE, MODEL, REC, PAIRS>(i, sp, inst, ppc, pwc, walls, in, out, info,
                                                  l, ws, Fo, To, clock, step_rel, flags,
                                                  MODE != 1, xsel, Fx, Tx, tile, len, jr0, pf);
  if (MODE != 1) {
    // this launch's own update produced x^(step + 1)
    const double dm = wave_max_to(sp.brec + bound_slot(step, 1) * kDriftSpread, d, BS / 64);
    if (drift) wave_max_store(drift, dm, BS / 64);
  }
}

hipError_t launch_force(int mode, int precision, const StepParams& sp, const InstDev* inst,
                        const PairCoef* pp,
                        const PairCoef* pw, const WallDev* walls, ParticleBufs in,
                        ParticleBufs out, const int* info, NbrList l, WallSlots ws,
                        double4* F, double4* T, const int64_t* clock, int64_t step_rel,
                        const int* flags, unsigned long long* drift, const int* xsel,
                        const double4* Fx, const double4* Tx, double* pf, int block,
                        int pair_mode, hipStream_t s) {
  if (sp.n <= 0) return hipSuccess;
  if (block != 64 && block != 128 && block != 256) return hipErrorInvalidValue;
  dim3 gr(grid_for(sp.n, block)), bl(block);
#define DEM_LAUNCH_REC(RT, M, L, REC, PAIRS)                                                    \
  do {                                                                                          \
    if (block == 64)                                                                            \
      hipLaunchKernelGGL((k_force<RT, M, L, 64, REC, PAIRS>), gr, bl, 0, s, sp, inst, pp, pw,   \
                         walls, in, out, info, l, ws, F, T, clock, step_rel, flags, drift,      \
                         xsel, Fx, Tx, pf);                                                     \
    else if (block == 128)                                                                      \
      hipLaunchKernelGGL((k_force<RT, M, L, 128, REC, PAIRS>), gr, bl, 0, s, sp, inst, pp, pw,  \
                         walls, in, out, info, l, ws, F, T, clock, step_rel, flags, drift,      \
                         xsel, Fx, Tx, pf);                                                     \
    else                                                                                        \
      hipLaunchKernelGGL((k_force<RT, M, L, 256, REC, PAIRS>), gr, bl, 0, s, sp, inst, pp, pw,  \
                         walls, in, out, info, l, ws, F, T, clock, step_rel, flags, drift,      \
                         xsel, Fx, Tx, pf);                                                     \
  } while (0)
#define DEM_LAUNCH(RT, M, L)                                     \
  do {                                                           \
    if (pf) DEM_LAUNCH_REC(RT, M, L, true, 0);                   \
    else if (pair_mode == 1) DEM_LAUNCH_REC(RT, M, L, false, 1); \
    else if (pair_mode == 2) DEM_LAUNCH_REC(RT, M, L, false, 2); \
    else DEM_LAUNCH_REC(RT, M, L, false, 0);                     \
  } while (0)
#define DEM_LAUNCH_MODE(RT, L)                \
  do {                                        \
    if (mode == 0) DEM_LAUNCH(RT, 0, L);      \
    else if (mode == 1) DEM_LAUNCH(RT, 1, L); \
    else DEM_LAUNCH(RT, 2, L);                \
  } while (0)
  if (precision == 0) {
    if (sp.model == 0) DEM_LAUNCH_MODE(double, 0);
    else DEM_LAUNCH_MODE(double, 1);
  } else {
    if (sp.model == 0) DEM_LAUNCH_MODE(float, 0);
    else DEM_LAUNCH_MODE(float, 1);
  }
#undef DEM_LAUNCH_MODE
#undef DEM_LAUNCH
#undef DEM_LAUNCH_REC
  return hipGetLastError();
}

// ------------------------------------------------------------ mesh contacts
//
// One thread per particle over its triangle candidates (at most kMeshSlots).
// Every candidate reports its closest point and feature.  A face touches
// when the centre is less than R above its plane.  The distance restricted
// to one triangle is convex, so a point on an edge or at a vertex is a local
// minimum of the distance over the surface exactly when every triangle
// around it has it as its closest point: an edge or vertex counts when every
// candidate triangle of the same mesh that contains it reports it, once, in
// the slot of the first candidate reporting it, and touches when closer
// than R.  Slots without a contact restart their tangential overlap at zero.

// three wavefronts per SIMD fit without spills (168 VGPRs)
template <typename R>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
k_mesh(StepParams sp, const PairCoef* __restrict__ pwc, const WallDev* __restrict__ walls,
       MeshTables mt, ParticleBufs in, const int* __restrict__ info, MeshSlots ms,
       double4* __restrict__ Fm, double4* __restrict__ Tm, const int64_t* __restrict__ clock,
       int64_t step_rel, const int* __restrict__ flags) {
  const int i = xcd_block() * kBlock + threadIdx.x;
  const int n = sp.n;
  if (i >= n) return;
  double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
  const int inf = info[i];
  // only particles with candidates: the force kernel reads Fm / Tm for them
  if (ms.tri[i] < 0) return;
  if (!(inf & kInactive) && *flags == 0) {
    const double4 xi = in.pos[i], vi = in.vel[i], wi = in.omg[i];
    const double x[3] = {xi.x, xi.y, xi.z};
    const double rad = xi.w;
    const double t = (double)(*clock + step_rel) * sp.dt;
    const int row = ((inf >> kInstShift) * kMaxTypes + (inf & kTypeMask)) * kMaxTypes;
    // features reported by the candidates
    int tri[kMeshSlots], wl[kMeshSlots], kind[kMeshSlots], fa[kMeshSlots], fb[kMeshSlots];
    int tv[kMeshSlots][3];
    unsigned near = 0u;  // bit k: slot k's closest point is closer than R (faces: above the plane)
#pragma unroll
    for (int k = 0; k < kMeshSlots; ++k) {
      const int tr = ms.tri[(int64_t)k * n + i];
      tri[k] = tr;
      wl[k] = -1;
      kind[k] = fa[k] = fb[k] = -1;
      tv[k][0] = tv[k][1] = tv[k][2] = -1;
      if (tr < 0) continue;
      const TriDev& Tt = mt.tri[tr];
      TriGeo g;
      tri_closest(Tt, walls[Tt.wall].vel, t, x, g);
      wl[k] = Tt.wall;
      tv[k][0] = Tt.v[0];
      tv[k][1] = Tt.v[1];
      tv[k][2] = Tt.v[2];
      kind[k] = g.feature;
      const bool close = g.feature == 0 ? g.s < rad : (g.d2 < rad * rad && g.d2 > 0.0);
      if (close) near |= 1u << k;
      if (g.feature == 0) {
        fa[k] = tr;
      } else if (g.feature == 1) {
        const int va = Tt.v[g.a], vb = Tt.v[g.b];
        fa[k] = va < vb ? va : vb;
        fb[k] = va < vb ? vb : va;
      } else {
        fa[k] = Tt.v[g.a];
      }
    }
    // which slots carry a contact (the arrays above end here)
    unsigned used = 0u, contact = 0u;
#pragma unroll
    for (int k = 0; k < kMeshSlots; ++k) {
      if (tri[k] < 0) continue;
      used |= 1u << k;
      const WallDev& W = walls[wl[k]];
      bool c = false;
      if (t >= W.t_on && t < W.t_off) {
        if (kind[k] == 0) {
          c = (near >> k) & 1u;
        } else {
          bool dropped = false, owner = true;
#pragma unroll
          for (int j = 0; j < kMeshSlots; ++j) {
            if (tri[j] < 0 || wl[j] != wl[k]) continue;
            const bool same = kind[j] == kind[k] && fa[j] == fa[k] && fb[j] == fb[k];
            const bool has_a = tv[j][0] == fa[k] || tv[j][1] == fa[k] || tv[j][2] == fa[k];
            const bool has_b = tv[j][0] == fb[k] || tv[j][1] == fb[k] || tv[j][2] == fb[k];
            if (has_a && (kind[k] == 2 || has_b) && !same) dropped = true;
            if (j < k && same) owner = false;
          }
          c = !dropped && owner && ((near >> k) & 1u);
        }
      }
      if (c) contact |= 1u << k;
    }
    // the law for each contact, geometry evaluated again
#pragma unroll 1
    for (int k = 0; k < kMeshSlots; ++k) {
      if (!((used >> k) & 1u)) continue;
      const int64_t h = (int64_t)(3 * k) * n + i;
      if (!((contact >> k) & 1u)) {
        ms.hist[h] = 0.0;
        ms.hist[h + n] = 0.0;
        ms.hist[h + 2 * (int64_t)n] = 0.0;
        continue;
      }
      const TriDev& Tt = mt.tri[ms.tri[(int64_t)k * n + i]];
      const WallDev& W = walls[Tt.wall];
      TriGeo g;
      tri_closest(Tt, W.vel, t, x, g);
      double gn[3], gdn;
      if (g.feature == 0) {
        gn[0] = -Tt.n[0];
        gn[1] = -Tt.n[1];
        gn[2] = -Tt.n[2];
        gdn = rad - g.s;
      } else {
        const double dist = sqrt(g.d2);
        gn[0] = (g.q[0] - x[0]) / dist;
        gn[1] = (g.q[1] - x[1]) / dist;
        gn[2] = (g.q[2] - x[2]) / dist;
        gdn = rad - dist;
      }
      const double arm[3] = {g.q[0] - (W.ax[0] + W.vel[0] * t), g.q[1] - (W.ax[1] + W.vel[1] * t),
                             g.q[2] - (W.ax[2] + W.vel[2] * t)};
      double dtl[3] = {ms.hist[h], ms.hist[h + n], ms.hist[h + 2 * (int64_t)n]};
      double Fi[3], Mi[3];
      wall_law<R>(pwc[row + W.material], sp.rolling, sp.model, sp.dt, W, gn, gdn, arm, xi, vi, wi,
                  dtl, Fi, Mi);
      ms.hist[h] = dtl[0];
      ms.hist[h + n] = dtl[1];
      ms.hist[h + 2 * (int64_t)n] = dtl[2];
      F[0] += Fi[0];
      F[1] += Fi[1];
      F[2] += Fi[2];
      T[0] += Mi[0];
      T[1] += Mi[1];
      T[2] += Mi[2];
    }
  }
  Fm[i] = make_double4(F[0], F[1], F[2], 0.0);
  Tm[i] = make_double4(T[0], T[1], T[2], 0.0);
}

hipError_t launch_mesh(int precision, const StepParams& sp, const PairCoef* pw,
                       const WallDev* walls, MeshTables mt, ParticleBufs in, const int* info,
                       MeshSlots ms, double4* Fm, double4* Tm, const int64_t* clock,
                       int64_t step_rel, const int* flags, hipStream_t s) {
  if (sp.n <= 0) return hipSuccess;
  if (precision == 0)
    hipLaunchKernelGGL(k_mesh<double>, dim3(grid_for(sp.n)), dim3(kBlock), 0, s, sp, pw, walls,
                       mt, in, info, ms, Fm, Tm, clock, step_rel, flags);
  else
    hipLaunchKernelGGL(k_mesh<float>, dim3(grid_for(sp.n)), dim3(kBlock), 0, s, sp, pw, walls,
                       mt, in, info, ms, Fm, Tm, clock, step_rel, flags);
  return hipGetLastError();
}

// ------------------------------------------------------ kick-drift, clock

// first half kick and drift of particle i from the stored forces; returns the
// squared drift in units of half the skin when asked for it
__device__ __forceinline__ double kick_drift_one(int i, const StepParams& sp, const InstDev* __restrict__ inst,
                                 ParticleBufs st, const int* __restrict__ info,
                                 const double4* __restrict__ F,
                                 const double4* __restrict__ T, const bool want_drift) {
  double4 x = st.pos[i], v = st.vel[i], w = st.omg[i];
  double4 f = F[i], tq = T[i];
  const double h = sp.hdt, dt = sp.dt;
  // vel.w = 1/m, omg.w = 1/I
  double a0 = f.x * v.w + sp.g[0], a1 = f.y * v.w + sp.g[1], a2 = f.z * v.w + sp.g[2];
  v.x = v.x + a0 * h;
  v.y = v.y + a1 * h;
  v.z = v.z + a2 * h;
  w.x = w.x + (tq.x * w.w) * h;
  w.y = w.y + (tq.y * w.w) * h;
  w.z = w.z + (tq.z * w.w) * h;
  x.x = x.x + v.x * dt;
  x.y = x.y + v.y * dt;
  x.z = x.z + v.z * dt;
  st.pos[i] = x;
  st.vel[i] = v;
  st.omg[i] = w;
  if (!want_drift) return 0.0;
  return drift2(v, drift_scale(sp, inst, info[i]));
}

__global__ void k_kick_drift(StepParams sp, const InstDev* __restrict__ inst, ParticleBufs st,
                             const int* __restrict__ info, const double4* __restrict__ F,
                             const double4* __restrict__ T,
                             unsigned long long* __restrict__ drift,
                             const int64_t* __restrict__ clock, int64_t step_rel) {
  int i = xcd_block() * kBlock + threadIdx.x;
  double d = 0.0;
  if (i < sp.n && !(info[i] & kInactive)) d = kick_drift_one(i, sp, inst, st, info, F, T, true);
  // the displacement bound's record of the update that produced x^step
  const int64_t step = *clock + step_rel;
  const double dm = wave_max_to(sp.brec + bound_slot(step, 0) * kDriftSpread, d);
  if (drift) wave_max_store(drift, dm);
}

hipError_t launch_kick_drift(const StepParams& sp, const InstDev* inst, ParticleBufs st,
                             const int* info, const double4* F, const double4* T,
                             unsigned long long* drift, const int64_t* clock, int64_t step_rel,
                             hipStream_t s) {
  if (sp.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(sp.n)), dim3(kBlock), 0, s, sp, inst, st, info,
                     F, T, drift, clock, step_rel);
  return hipGetLastError();
}



__global__ void k_tick(int64_t* clock, int64_t k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] += k;
}

hipError_t launch_tick(int64_t* clock, int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, clock, k);
  return hipGetLastError();
}

// -------------------------------------------------------------------- stats

__global__ void k_stats(StepParams sp, const double4* __restrict__ pos,
                        const int* __restrict__ info, NbrList l, WallSlots ws,
                        unsigned long long* out) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  unsigned long long a = 0, e = 0, tch = 0, wc = 0;
  if (i < sp.n && !(info[i] & kInactive)) {
    a = 1;
    double4 xi = pos[i];
    int len = l.rowlen[i];
    e = (unsigned long long)len;
    for (int k = 0; k < len; ++k) {
      int j = l.nbr[nbr_entry(i, k, sp.max_nb)] & 0x7fffffff;
      double4 xj = pos[j];
      double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
      double d2 = (dx * dx + dy * dy) + dz * dz;
      double rs = xi.w + xj.w;
      if (d2 < rs * rs) ++tch;
    }
    for (int s = 0; s < kWallSlots; ++s)
      if (ws.wid[(int64_t)s * sp.n + i] >= 0) ++wc;
  }
  // wave reduction, then one atomic per wave
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    e += __shfl_down(e, o, 64);
    tch += __shfl_down(tch, o, 64);
    wc += __shfl_down(wc, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&out[0], a);
    atomicAdd(&out[1], e);
    atomicAdd(&out[2], tch);
    atomicAdd(&out[3], wc);
  }
}

hipError_t launch_stats(const StepParams& sp, const double4* pos, const int* info, NbrList l,
                        WallSlots ws, unsigned long long* out, hipStream_t s) {
  if (sp.n <= 0) return hipSuccess;
  unsigned nb = (unsigned)((sp.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_stats, dim3(nb), dim3(kBlock), 0, s, sp, pos, info, l, ws, out);
  return hipGetLastError();
}

// ------------------------------------------------ contact list on the device
//
// The candidate pairs of one instance, each once as (gid_i, gid_j) with
// gid_i < gid_j, written to caller buffers in the sorted order of the first
// particle and then its row order: a per-block count, a scan of the block
// counts, and a fill in which each block recounts its threads' pairs and
// places them after its block's offset.  Only the block counts and their
// scan need memory beyond the outputs.

__device__ __forceinline__ int pairs_of_row(const StepParams& sp, int inst, int p,
                                            const int* __restrict__ info,
                                            const int* __restrict__ gid, const NbrList& l) {
  if (p >= sp.n) return 0;
  const int inf = info[p];
  if ((inf & kInactive) || (inf >> kInstShift) != inst) return 0;
  const int g = gid[p];
  const int len = l.rowlen[p];
  int c = 0;
  for (int k = 0; k < len; ++k) {
    const int q = l.nbr[nbr_entry(p, k, sp.max_nb)] & kIndexMask;
    c += gid[q] > g ? 1 : 0;
  }
  return c;
}

__global__ void k_pairs_count(StepParams sp, int inst, const int* __restrict__ info,
                              const int* __restrict__ gid, NbrList l, int* __restrict__ bcount) {
  __shared__ int sh[4];
  const int p = blockIdx.x * kBlock + threadIdx.x;
  const int c = pairs_of_row(sp, inst, p, info, gid, l);
  int tot;
  block_exclusive_scan(c, sh, &tot);
  if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}

__global__ void k_pairs_fill(StepParams sp, int inst, int gid_base,
                             const double4* __restrict__ pos, const int* __restrict__ info,
                             const int* __restrict__ gid, NbrList l,
                             const int* __restrict__ bstart, int64_t* __restrict__ pairs,
                             double* __restrict__ delta_t, uint8_t* __restrict__ touching) {
  __shared__ int sh[4];
  const int p = blockIdx.x * kBlock + threadIdx.x;
  const int c = pairs_of_row(sp, inst, p, info, gid, l);
  int tot;
  int64_t o = (int64_t)bstart[blockIdx.x] + block_exclusive_scan(c, sh, &tot);
  if (c == 0) return;
  const int g = gid[p];
  const double4 xp = pos[p];
  const int len = l.rowlen[p];
  for (int k = 0; k < len; ++k) {
    const int64_t e = nbr_entry(p, k, sp.max_nb);
    const int jr = l.nbr[e];
    const int q = jr & kIndexMask;
    const int gq = gid[q];
    if (!(gq > g)) continue;
    if (pairs) {
      pairs[2 * o] = g - gid_base;
      pairs[2 * o + 1] = gq - gid_base;
    }
    if (delta_t) {
      // bit 31: the pair touched at the last evaluation and holds a history
      const bool h = (jr & kTouchedBit) != 0;
      delta_t[3 * o] = h ? l.hist[e] : 0.0;
      delta_t[3 * o + 1] = h ? l.hist[l.cap + e] : 0.0;
      delta_t[3 * o + 2] = h ? l.hist[2 * l.cap + e] : 0.0;
    }
    if (touching) {
      const double4 xq = pos[q];
      const double dx = xq.x - xp.x, dy = xq.y - xp.y, dz = xq.z - xp.z;
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      const double rs = xp.w + xq.w;
      touching[o] = d2 < rs * rs ? 1 : 0;
    }
    ++o;
  }
}

int64_t pairs_scratch_ints(int n) {
  const int64_t nb = (n + kBlock - 1) / kBlock;
  return nb + (nb + 2) + ((nb + 1 + kScanTile - 1) / kScanTile + 1);
}

hipError_t launch_pairs_count(const StepParams& sp, int inst, const int* info, const int* gid,
                              NbrList l, int* scratch, hipStream_t s) {
  const int64_t nb = (sp.n + kBlock - 1) / kBlock;
  int* bcount = scratch;
  int* bstart = scratch + nb;
  int* tiles = bstart + nb + 2;
  if (nb > 0)
    hipLaunchKernelGGL(k_pairs_count, dim3((unsigned)nb), dim3(kBlock), 0, s, sp, inst, info,
                       gid, l, bcount);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nb == 0) return launch_fill_i32(bstart, 0, 1, s);
  return launch_scan(bcount, bstart, nb, tiles, s);
}

hipError_t launch_pairs_fill(const StepParams& sp, int inst, int gid_base, const double4* pos,
                             const int* info, const int* gid, NbrList l, const int* scratch,
                             int64_t* pairs, double* delta_t, uint8_t* touching,
                             hipStream_t s) {
  const int64_t nb = (sp.n + kBlock - 1) / kBlock;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pairs_fill, dim3((unsigned)nb), dim3(kBlock), 0, s, sp, inst, gid_base,
                     pos, info, gid, l, scratch + nb, pairs, delta_t, touching);
  return hipGetLastError();
}

}  // namespace demgpu
