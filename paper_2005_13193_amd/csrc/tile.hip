// Column-tiled gathers and scatter for particles ordered by cell.
//
// After pt_sort_particles the particles of a column of kTileX x kTileY cells
// are contiguous and ordered by layer z.  Work items are runs of layers of
// one column (gather) or half-column (scatter); a launch holds one workgroup
// per compute unit, and the workgroups draw items from per-XCD counters until
// every item is taken.  Each workgroup marches up in z through its item with
// a ring of padded coefficient planes of the column's tile in LDS, so that
// every coefficient is read from HBM about once per column (plus the halo
// rows/columns shared with neighbouring columns, which hit in L2, and the
// planes at item ends).
//
// tile_gather: both Heun stages (forward) or the step adjoint's gather half
// (backward) per particle.  Four loader waves fill the ring with direct
// global-to-LDS loads several planes ahead; eight compute waves evaluate the
// particles of the current slab of layers, four lanes per point.  Points
// whose stencil is not in the ring (the predictor left the column or moved
// more than one layer) are deferred to gather_deferred, which redoes them from
// global memory.
//
// tile_scatter: the adjoint of the 64-term sums into the coefficient
// gradient, summed in 64-bit fixed point in an LDS ring and added to HBM one
// plane at a time; launches by colour keep concurrent workgroups on disjoint
// coefficients, and stencils that do not fit go to scatter_deferred.
#include "pt_common.h"
#include "pt_inertial.h"

namespace pt {

constexpr int kSlab = 2;          // layers per iteration
constexpr int kGatherSeg = 128;   // most layers per gather work item
constexpr int kScatterSeg = 256;  // most layers per scatter work item
// The particle table indexes half-layers: the rows 0..15 and 16..31 of a
// column layer (key >> 9 with 32 x 32 columns).
constexpr int kHalfShift = 9;     // log2(kTileX * kTileY / 2)
constexpr int kMaxSlots = 64;     // slots for the largest |ub| (see zero_int)
constexpr int kTableBad = kMaxSlots + 1;  // defer header: particle table found invalid
constexpr int kDeferHeader = 512; // bytes before the deferred list
static_assert(kTileX * kTileY == (2 << kHalfShift), "half-layer shift");

struct TileArgs {
  GridDev g;
  const void* coeff;
  const int32_t* lstart;  // [ncol * nz + 1]: first particle of each (column, layer)
  int ncx, ncy, ncol, nseg, seg_len;
  int color;              // scatter: colour of this launch
  const int4* items;      // work items (column, half, z0, z1)
  const int* item_range;  // [begin, end) of this launch's items in `items`
  int* item_ctr;          // 8 zeroed counters of this launch (one per XCD range)
  int64_t np;
  double dt;
  const double* x;        // [3][np] positions (sorted)
  double* x_out;          // fwd: new positions
  const double* lam;      // bwd: dL/dx_out  [3][np]
  double* xbn;            // bwd: dL/dx_n    [3][np]
  float* u0;              // bwd: stage-1 velocity  [3][np]
  float* ub0;             // bwd: adjoint of stage-1 velocity [3][np]
  float* ub1;             // bwd: adjoint of stage-2 velocity, dt/2 lam [3][np]
  const double* disp;     // inertial: displacement increments [3][np] or null
  float* vel_out;         // inertial: new particle velocities [3][np] or null
  InertialCoef ik;        // inertial: step coefficients
  float* out;             // interpolation modes: [3][np] or [12][np]
  float* saved;           // fwd save: [21][np] rows u0 (0-2), du_c/dx_d at x_n
                          // (3 + 3c + d) and at x* (12 + 3c + d)
  float* gcoeff;          // scatter target (padded FP32)
  uint32_t* defer;        // scatter: deferred stencils (2 p + stage)
  int* defer_count;
  int* err;
};

__device__ __forceinline__ float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
  return v;
}

__device__ __forceinline__ float pick4(const float w[4], int i) {
  return i == 0 ? w[0] : i == 1 ? w[1] : i == 2 ? w[2] : w[3];
}

// ---------------------------------------------------- point evaluation ---
struct Pt {
  int a, b, c;     // cell
  float t[3];      // local coordinates
  bool in_ring;    // stencil resident in LDS
};

// X0, Y0: padded index of LDS column/row 0; cells a with a - X0 in
// [0, kTileX + 2M) have their 4x4 stencil columns inside the tile.
template <int M>
__device__ __forceinline__ Pt locate_pt(const GridDev& g, const double p[3], int X0, int Y0,
                                        int zlo, int zhi, int* err) {
  Pt q;
  bool bad = false;
  double t0, t1, t2;
  q.a = cell_1d(p[0], g.cs[0], g.nx, &t0, &bad);
  q.b = cell_1d(p[1], g.cs[1], g.ny, &t1, &bad);
  q.c = cell_1d(p[2], g.cs[2], g.nz, &t2, &bad);
  if (bad) *err = 1;
  q.t[0] = (float)t0;
  q.t[1] = (float)t1;
  q.t[2] = (float)t2;
  const int lx = q.a - X0, ly = q.b - Y0;
  q.in_ring = lx >= 0 && lx < kTileX + 2 * M && ly >= 0 && ly < kTileY + 2 * M && q.c >= zlo &&
              q.c <= zhi;
  return q;
}

// Value of lane D of this lane's quad (one DPP move).
template <int D>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, D * 0x55, 0xF, 0xF, true);
}
template <int D>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(quad_bcast<D>(__float_as_int(v)));
}

// v[i] for a lane-dependent i (i >= 2: v[2]) as two selects.  The values are
// pinned in registers first (an empty asm statement): otherwise the compiler
// may turn the choice into an indexed access, which moves the whole array to
// scratch memory.
template <typename T>
__device__ __forceinline__ T pick3(const T v[3], int i) {
  T a = v[0], b = v[1], c = v[2];
  asm("" : "+v"(a), "+v"(b), "+v"(c));
  return i == 0 ? a : i == 1 ? b : c;
}

// The grid axis a lane of a quad locates (lane d < 3: axis d; lane 3 repeats
// axis 2).  Formed once per kernel: a lane-dependent choice between the
// grid's fields inside a loop compiles to a memory load and a full wait.
struct LaneAxis {
  double cs;  // grid units per length
  int n;      // points
};

__device__ __forceinline__ LaneAxis lane_axis(const GridDev& g, int lane) {
  LaneAxis ax;
  ax.cs = lane == 0 ? g.cs[0] : lane == 1 ? g.cs[1] : g.cs[2];
  ax.n = lane == 0 ? g.nx : lane == 1 ? g.ny : g.nz;
  return ax;
}

// locate_pt<0> run by the four lanes of a particle's quad together: each
// lane locates its axis ax in FP64 (xd: that axis of the point) and the quad
// shares the cells and local coordinates, instead of every lane locating all
// three axes.  All four lanes of the quad must take part.
__device__ __forceinline__ Pt locate_quad(const LaneAxis& ax, double xd, int X0, int Y0,
                                          int zlo, int zhi, int* err) {
  bool bad = false;
  double t;
  const int cell = cell_1d(xd, ax.cs, ax.n, &t, &bad);
  if (bad) *err = 1;
  const float tf = (float)t;
  Pt q;
  q.a = quad_bcast<0>(cell);
  q.b = quad_bcast<1>(cell);
  q.c = quad_bcast<2>(cell);
  q.t[0] = quad_bcast<0>(tf);
  q.t[1] = quad_bcast<1>(tf);
  q.t[2] = quad_bcast<2>(tf);
  const int lx = q.a - X0, ly = q.b - Y0;
  q.in_ring =
      lx >= 0 && lx < kTileX + 2 && ly >= 0 && ly < kTileY + 2 && q.c >= zlo && q.c <= zhi;
  return q;
}

// Value (GRAD: and gradient) of the three components at a point, read from
// global memory (points whose stencil is not resident in LDS).
template <typename CT, bool GRAD>
__device__ __forceinline__ void eval_global(const CT* __restrict__ coeff, const GridDev& g,
                                            const Pt& q, float out[12]) {
  float wx[4], wy[4], wz[4], dx[4], dy[4], dz[4];
  bspline_w(q.t[0], wx);
  bspline_w(q.t[1], wy);
  bspline_w(q.t[2], wz);
  if (GRAD) {
    bspline_dw(q.t[0], dx);
    bspline_dw(q.t[1], dy);
    bspline_dw(q.t[2], dz);
  }
  const int64_t off = ((int64_t)q.c * g.py + q.b) * g.px + q.a;
  for (int comp = 0; comp < 3; ++comp) {
    const CT* base = coeff + comp * g.comp + off;
    float v = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
    for (int k = 0; k < 4; ++k) {
      float ty = 0.f, tdy = 0.f, tdx = 0.f;
      for (int j = 0; j < 4; ++j) {
        const CT* row = base + k * g.plane + j * g.px;
        const float r0 = load_coeff(row), r1 = load_coeff(row + 1);
        const float r2 = load_coeff(row + 2), r3 = load_coeff(row + 3);
        const float sx = wx[0] * r0 + wx[1] * r1 + wx[2] * r2 + wx[3] * r3;
        ty += wy[j] * sx;
        if (GRAD) {
          tdy += dy[j] * sx;
          tdx += wy[j] * (dx[0] * r0 + dx[1] * r1 + dx[2] * r2 + dx[3] * r3);
        }
      }
      v += wz[k] * ty;
      if (GRAD) {
        gx += wz[k] * tdx;
        gy += wz[k] * tdy;
        gz += dz[k] * ty;
      }
    }
    out[comp] = v;
    if (GRAD) {
      out[3 + 3 * comp + 0] = gx * g.inv_h[0];
      out[3 + 3 * comp + 1] = gy * g.inv_h[1];
      out[3 + 3 * comp + 2] = gz * g.inv_h[2];
    }
  }
}

// ------------------------------------------------------- gather kernels ---
// The gather ring holds kGRing dense planes [3][kTileY+5][kTileX+5] of 32-bit
// words (FP32 values; BF16 values widened on arrival).  Four loader waves fill
// it with direct global-to-LDS loads; eight compute waves only read it.  The
// load queue of a wave retires in order, so keeping the plane loads in waves
// of their own means the compute waves never wait on them, and the loaders
// wait for exactly their own loads before the barrier that publishes them.
// A one-cell margin around the column, so that predictor points that moved
// one cell out of it still find their stencil in the ring: 9 slots, planes
// zs-1 .. zs+5 in use and zs+6, zs+7 in flight during slab zs.
constexpr int kGRing = 9;
constexpr int kGTW = kTileX + 5, kGTH = kTileY + 5;
constexpr int kGComp = kGTW * kGTH;            // 1369 words per component
constexpr int kGSlot = 3 * kGComp + 29;        // slot pitch (words), 40 mod 64
static_assert(kGSlot % 64 == 40, "planes of one stencil in distinct LDS banks");
constexpr int kCompute = 512;                  // compute threads (8 waves)
// Loader waves: a wave has at most 63 memory operations in flight, so the
// plane loads in flight per compute unit grow with the loader count; 4 (one
// per SIMD) measured best (2 and 3 slower or equal; 5 and more leave the
// compute waves too few registers).
constexpr int kLoaders = 4;
constexpr int kGTB = kCompute + 64 * kLoaders;
constexpr int kGChunks = (kGComp + 63) / 64;   // 64-word chunks per component (20)
constexpr int kGChunksPerLoader = (kGChunks + kLoaders - 1) / kLoaders;
constexpr int kGGroups = kCompute / 4;

// Modes of the tiled gather: the fused Heun step, its adjoint's gathers, the
// two stages of a Heun step in a field that changes over the step (stage 1
// with the field at t_n, stage 2 with the field at t_n + dt), and the
// inertial / diffusive particle step (both stages, velocities carried).
enum {
  TILE_RK2_FWD = 0,
  TILE_RK2_BWD_GRAD = 1,
  TILE_TV_STAGE1 = 2,
  TILE_TV_STAGE2 = 3,
  TILE_INERTIAL = 4,
  TILE_INTERP3 = 5,   // (u, v, w) at the particles
  TILE_INTERP12 = 6,  // (u, v, w) and the nine velocity gradients
  TILE_RK2_FWD_SAVE = 7,  // the Heun step from values and gradients at both
                          // stage points, keeping u0 and the gradients
  TILE_RK2_FWD_GRAD12 = 8  // the Heun step, writing also (u, v, w) and the
                           // nine gradients at x_n
};

__device__ __forceinline__ int gslot(int P) { return (P + kGRing) % kGRing; }

// Value (GRAD: and gradient) at a resident point; every lane of the quad
// returns the full result.  Lane k of the quad takes plane k of the 4x4x4
// stencil and reads its 12 x-runs of 4 words (3 components x 4 rows) as word
// pairs; with the slot pitch of 40 banks mod 64, the 16 words of the 4 planes
// of one point fall into distinct banks, and each LDS instruction moves twice
// the data of a single-word read.
template <typename CT, bool GRAD>
__device__ __forceinline__ void eval_ring(const uint32_t* ring, const GridDev& g, const Pt& q,
                                          int X0, int Y0, int lane, float out[12]) {
  float wx[4], wy[4], wz[4], dwx[4], dwy[4], dwz[4];
  bspline_w(q.t[0], wx);
  bspline_w(q.t[1], wy);
  bspline_w(q.t[2], wz);
  if (GRAD) {
    bspline_dw(q.t[0], dwx);
    bspline_dw(q.t[1], dwy);
    bspline_dw(q.t[2], dwz);
  }
  const float wzk = pick4(wz, lane);
  const float dwzk = GRAD ? pick4(dwz, lane) : 0.0f;
  const uint32_t* base = ring + gslot(q.c + lane) * kGSlot + (q.b - Y0) * kGTW + (q.a - X0);
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    float A = 0.f, Bx = 0.f, By = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t* r = base + comp * kGComp + j * kGTW;
      const float v0 = __uint_as_float(r[0]), v1 = __uint_as_float(r[1]);
      const float v2 = __uint_as_float(r[2]), v3 = __uint_as_float(r[3]);
      const float sx = wx[0] * v0 + wx[1] * v1 + wx[2] * v2 + wx[3] * v3;
      A += wy[j] * sx;
      if (GRAD) {
        const float sdx = dwx[0] * v0 + dwx[1] * v1 + dwx[2] * v2 + dwx[3] * v3;
        Bx += wy[j] * sdx;
        By += dwy[j] * sx;
      }
    }
    out[comp] = quad_sum(wzk * A);
    if (GRAD) {
      out[3 + 3 * comp + 0] = quad_sum(wzk * Bx) * g.inv_h[0];
      out[3 + 3 * comp + 1] = quad_sum(wzk * By) * g.inv_h[1];
      out[3 + 3 * comp + 2] = quad_sum(dwzk * A) * g.inv_h[2];
    }
  }
}

// Per-particle data of one pass.
struct PData {
  double x[3];
  double lam[3];  // backward: dL/dx_out; inertial: displacement increment
  float un[3];    // stage 2: velocity of stage 1; inertial: particle velocity
  int p;
  bool ok;
};

template <int MODE>
__device__ __forceinline__ void load_pdata(const TileArgs& a, int64_t p, bool ok, PData* d) {
  const int64_t np = a.np;
  const int64_t i = ok ? p : 0;  // always a valid address: the load is always issued
  d->ok = ok;
  d->p = (int)p;
#pragma unroll
  for (int c = 0; c < 3; ++c) d->x[c] = a.x[c * np + i];
  if (MODE == TILE_RK2_BWD_GRAD) {
#pragma unroll
    for (int c = 0; c < 3; ++c) d->lam[c] = a.lam[c * np + i];
  }
  if (MODE == TILE_TV_STAGE2) {
#pragma unroll
    for (int c = 0; c < 3; ++c) d->un[c] = a.u0[c * np + i];
  }
  if (MODE == TILE_INERTIAL) {
    // a null velocity (tracer) or increment reads as zero (uniform branches)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d->un[c] = a.u0 ? a.u0[c * np + i] : 0.0f;
      d->lam[c] = a.disp ? a.disp[c * np + i] : 0.0;
    }
  }
}

// Outputs of one particle, held in registers until the wave's next flush.
// Stores are issued only right after the wave has waited for all its
// memory operations: a store still in flight makes every later wait for a
// load a wait for everything, including the loads just issued for the next
// pass, so stores must not sit between the loads and their use.
struct Pend {
  int64_t off;  // c * np + p for lane c < 3 of the quad (fwd save: p for
                // every lane), or -1
  double d;     // x_out (forward modes) or dL/dx_n (backward)
  float f0, f1, f2; // stage 1: u_n; backward: u0, ub0, ub1; fwd save: row c
                    // of the gradient at x_n (lane 3: u0)
  float g0, g1, g2; // fwd save: row c of the gradient at x*
  int defer;    // quad lane 0: particle to redo from global memory, or -1
};

// Deferred particles of one flush get list slots from one counter draw per
// wave; the returned base is used at the next flush, after the wave's next
// full wait, so the draw never stalls the wave.
struct DeferBatch {
  uint64_t mask;  // lanes with a particle to defer
  int leader;     // lane that drew the slots
  int base;       // first slot (valid in the leader lane)
  int part;       // this lane's particle
};

template <int MODE>
__device__ __forceinline__ void flush_pend(const TileArgs& a, Pend* o, DeferBatch* db, int* lerr) {
  const int64_t np = a.np;
  const int lane64 = threadIdx.x & 63;
  if (db->mask) {
    const int base = __shfl(db->base, db->leader, 64);
    const int rank = __popcll(db->mask & ((1ull << lane64) - 1ull));
    if (db->part >= 0 && (int64_t)(base + rank) < np) ((int32_t*)a.defer)[base + rank] = db->part;
  }
  if (o->off >= 0) {
    if (MODE == TILE_INTERP3) {
      a.out[(int64_t)(lane64 & 3) * np + o->off] = o->f0;
    } else if (MODE == TILE_INTERP12 || MODE == TILE_RK2_FWD_GRAD12) {
      const int q = lane64 & 3;
      const int64_t r = 3 * q;
      a.out[r * np + o->off] = o->f0;
      a.out[(r + 1) * np + o->off] = o->f1;
      a.out[(r + 2) * np + o->off] = o->f2;
      if (MODE == TILE_RK2_FWD_GRAD12 && q < 3) a.x_out[q * np + o->off] = o->d;
    } else if (MODE == TILE_RK2_FWD_SAVE) {
      const int q = lane64 & 3;
      const int64_t p = o->off;
      float* ra = a.saved + (int64_t)(q < 3 ? 3 + 3 * q : 0) * np + p;
      ra[0] = o->f0;
      ra[np] = o->f1;
      ra[2 * np] = o->f2;
      if (q < 3) {
        a.x_out[q * np + p] = o->d;
        float* rb = a.saved + (int64_t)(12 + 3 * q) * np + p;
        rb[0] = o->g0;
        rb[np] = o->g1;
        rb[2 * np] = o->g2;
      }
    } else if (MODE == TILE_RK2_BWD_GRAD) {
      a.xbn[o->off] = o->d;
      a.u0[o->off] = o->f0;
      a.ub0[o->off] = o->f1;
      a.ub1[o->off] = o->f2;
    } else {
      if (MODE == TILE_TV_STAGE1) a.u0[o->off] = o->f0;
      if (MODE == TILE_INERTIAL && a.vel_out) a.vel_out[o->off] = o->f0;
      a.x_out[o->off] = o->d;
    }
  }
  if (*lerr) {
    *a.err = 1;
    *lerr = 0;
  }
  const uint64_t m = __ballot(o->defer >= 0);
  db->mask = m;
  db->part = o->defer;
  if (m) {
    db->leader = __ffsll((unsigned long long)m) - 1;
    if (lane64 == db->leader) db->base = atomicAdd(a.defer_count, __popcll(m));
  }
  o->off = -1;
  o->defer = -1;
}

// Both Heun stages (forward), the whole step adjoint (backward) or one stage
// of the time-varying step of one particle from the ring, into o.  A particle
// whose predictor point is not resident is deferred to the cleanup kernel,
// which redoes it from global memory.
template <typename CT, int MODE>
__device__ __forceinline__ void ring_particle(const TileArgs& a, const uint32_t* ring,
                                              const PData& d, int X0, int Y0, int zz, int lane,
                                              const LaneAxis& ax, float* umax, Pend* o,
                                              int* lerr) {
  const GridDev& g = a.g;
  const int64_t np = a.np, p = d.p;
  const double* xn = d.x;
  // this lane's axis of x_n (lane 3: axis 2), for the quad-shared locates
  const double xnl = pick3(xn, lane);
  // resident cells: layers zz-1 .. zz+kSlab (planes zz-1 .. zz+5)
  const Pt qn = locate_quad(ax, xnl, X0, Y0, zz - 1, zz + kSlab, lerr);
  if (!qn.in_ring) {  // cannot happen for a correctly sorted particle; kept safe
    if (lane == 0) o->defer = d.p;
    return;
  }
  // lane c < 3 keeps component c (selects, not indexing: register arrays
  // indexed by a lane-dependent value would live in scratch memory)
  if (MODE == TILE_TV_STAGE1) {
    // u^n at x; the positions are written back in the sorted order
    float u0[12];
    eval_ring<CT, false>(ring, g, qn, X0, Y0, lane, u0);
    if (lane < 3) {
      o->off = lane * np + p;
      o->f0 = lane == 0 ? u0[0] : lane == 1 ? u0[1] : u0[2];
      o->d = lane == 0 ? xn[0] : lane == 1 ? xn[1] : xn[2];
    }
  } else if (MODE == TILE_TV_STAGE2) {
    // x* = x + dt u^n (from stage 1), u^{n+1}(x*) from the ring
    const float unl = pick3(d.un, lane);
    const Pt qs = locate_quad(ax, xnl + a.dt * (double)unl, X0, Y0, zz - 1, zz + kSlab, lerr);
    if (!qs.in_ring) {
      if (lane == 0) o->defer = d.p;
      return;
    }
    float u1[12];
    eval_ring<CT, false>(ring, g, qs, X0, Y0, lane, u1);
    if (lane < 3) {
      const double h = 0.5 * a.dt;
      const double x0 = lane == 0 ? xn[0] : lane == 1 ? xn[1] : xn[2];
      const float ua = lane == 0 ? d.un[0] : lane == 1 ? d.un[1] : d.un[2];
      const float ub = lane == 0 ? u1[0] : lane == 1 ? u1[1] : u1[2];
      o->off = lane * np + p;
      o->d = x0 + h * ((double)ua + (double)ub);
    }
  } else if (MODE == TILE_INTERP3 || MODE == TILE_INTERP12) {
    // lane c < 3 writes row c (INTERP3); lane c writes rows 3c .. 3c+2
    // (INTERP12)
    float o12[12];
    eval_ring<CT, MODE == TILE_INTERP12>(ring, g, qn, X0, Y0, lane, o12);
    if (MODE == TILE_INTERP3) {
      if (lane < 3) {
        o->off = p;
        o->f0 = lane == 0 ? o12[0] : lane == 1 ? o12[1] : o12[2];
      }
    } else {
      o->off = p;
      o->f0 = lane == 0 ? o12[0] : lane == 1 ? o12[3] : lane == 2 ? o12[6] : o12[9];
      o->f1 = lane == 0 ? o12[1] : lane == 1 ? o12[4] : lane == 2 ? o12[7] : o12[10];
      o->f2 = lane == 0 ? o12[2] : lane == 1 ? o12[5] : lane == 2 ? o12[8] : o12[11];
    }
  } else if (MODE == TILE_INERTIAL) {
    float u0[12], u1[12];
    eval_ring<CT, false>(ring, g, qn, X0, Y0, lane, u0);
    // this lane's axis (lane 3: axis 2) of the predictor point
    const double xsl = inertial_predict(a.ik, xnl, (double)pick3(d.un, lane),
                                        (double)pick3(u0, lane), pick3(d.lam, lane));
    const Pt qs = locate_quad(ax, xsl, X0, Y0, zz - 1, zz + kSlab, lerr);
    if (!qs.in_ring) {
      if (lane == 0) o->defer = d.p;
      return;
    }
    eval_ring<CT, false>(ring, g, qs, X0, Y0, lane, u1);
    if (lane < 3) {
      const double xl = xsl;
      const double ua = lane == 0 ? u0[0] : lane == 1 ? u0[1] : u0[2];
      const double ub = lane == 0 ? u1[0] : lane == 1 ? u1[1] : u1[2];
      const double vl = lane == 0 ? d.un[0] : lane == 1 ? d.un[1] : d.un[2];
      o->off = lane * np + p;
      o->d = inertial_correct(a.ik, xl, ua, ub);
      o->f0 = (float)inertial_velocity(a.ik, vl, ua, ub);
    }
  } else if (MODE == TILE_RK2_FWD) {
    float u0[12], u1[12];
    eval_ring<CT, false>(ring, g, qn, X0, Y0, lane, u0);
    const float u0l = pick3(u0, lane);
    const Pt qs = locate_quad(ax, xnl + a.dt * (double)u0l, X0, Y0, zz - 1, zz + kSlab, lerr);
    if (!qs.in_ring) {
      if (lane == 0) o->defer = d.p;
      return;
    }
    eval_ring<CT, false>(ring, g, qs, X0, Y0, lane, u1);
    if (lane < 3) {
      const double h = 0.5 * a.dt;
      const double x0 = xnl;
      const float ua = lane == 0 ? u0[0] : lane == 1 ? u0[1] : u0[2];
      const float ub = lane == 0 ? u1[0] : lane == 1 ? u1[1] : u1[2];
      o->off = lane * np + p;
      o->d = x0 + h * ((double)ua + (double)ub);
    }
  } else if (MODE == TILE_RK2_FWD_GRAD12) {
    // values and gradients at x_n (written out, rows as TILE_INTERP12),
    // values at x*
    float on[12], os[12];
    eval_ring<CT, true>(ring, g, qn, X0, Y0, lane, on);
    const float onl = pick3(on, lane);
    const Pt qs = locate_quad(ax, xnl + a.dt * (double)onl, X0, Y0, zz - 1, zz + kSlab, lerr);
    if (!qs.in_ring) {
      if (lane == 0) o->defer = d.p;
      return;
    }
    eval_ring<CT, false>(ring, g, qs, X0, Y0, lane, os);
    const float ua = lane == 0 ? on[0] : lane == 1 ? on[1] : on[2];
    const float ub = lane == 0 ? os[0] : lane == 1 ? os[1] : os[2];
    o->off = p;
    o->d = xnl + 0.5 * a.dt * ((double)ua + (double)ub);
    o->f0 = lane == 0 ? on[0] : lane == 1 ? on[3] : lane == 2 ? on[6] : on[9];
    o->f1 = lane == 0 ? on[1] : lane == 1 ? on[4] : lane == 2 ? on[7] : on[10];
    o->f2 = lane == 0 ? on[2] : lane == 1 ? on[5] : lane == 2 ? on[8] : on[11];
  } else if (MODE == TILE_RK2_FWD_SAVE) {
    float on[12], os[12];
    eval_ring<CT, true>(ring, g, qn, X0, Y0, lane, on);
    const float onl = pick3(on, lane);
    const Pt qs = locate_quad(ax, xnl + a.dt * (double)onl, X0, Y0, zz - 1, zz + kSlab, lerr);
    if (!qs.in_ring) {
      if (lane == 0) o->defer = d.p;
      return;
    }
    eval_ring<CT, true>(ring, g, qs, X0, Y0, lane, os);
    // lane c < 3: x_out[c] and row c of both gradients; lane 3: u0
    const float ua = lane == 0 ? on[0] : lane == 1 ? on[1] : on[2];
    const float ub = lane == 0 ? os[0] : lane == 1 ? os[1] : os[2];
    o->off = p;
    o->d = xnl + 0.5 * a.dt * ((double)ua + (double)ub);
    o->f0 = lane == 0 ? on[3] : lane == 1 ? on[6] : lane == 2 ? on[9] : on[0];
    o->f1 = lane == 0 ? on[4] : lane == 1 ? on[7] : lane == 2 ? on[10] : on[1];
    o->f2 = lane == 0 ? on[5] : lane == 1 ? on[8] : lane == 2 ? on[11] : on[2];
    o->g0 = lane == 0 ? os[3] : lane == 1 ? os[6] : os[9];
    o->g1 = lane == 0 ? os[4] : lane == 1 ? os[7] : os[10];
    o->g2 = lane == 0 ? os[5] : lane == 1 ? os[8] : os[11];
  } else {
    float on[12], os[12];
    eval_ring<CT, true>(ring, g, qn, X0, Y0, lane, on);
    const float onl = pick3(on, lane);
    const Pt qs = locate_quad(ax, xnl + a.dt * (double)onl, X0, Y0, zz - 1, zz + kSlab, lerr);
    if (!qs.in_ring) {
      if (lane == 0) o->defer = d.p;
      return;
    }
    eval_ring<CT, true>(ring, g, qs, X0, Y0, lane, os);
    const double* lam = d.lam;
    float ub1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) ub1[c] = (float)(0.5 * a.dt * lam[c]);
    double xbs[3], xb[3];
    float ub0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xbs[c] = (double)(ub1[0] * os[3 + c] + ub1[1] * os[6 + c] + ub1[2] * os[9 + c]);
      ub0[c] = (float)(0.5 * a.dt * lam[c] + a.dt * xbs[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xb[c] = lam[c] + xbs[c] +
              (double)(ub0[0] * on[3 + c] + ub0[1] * on[6 + c] + ub0[2] * on[9 + c]);
      *umax = fmaxf(*umax, fmaxf(fabsf(ub0[c]), fabsf(ub1[c])));
    }
    if (lane < 3) {
      o->off = lane * np + p;
      o->d = lane == 0 ? xb[0] : lane == 1 ? xb[1] : xb[2];
      o->f0 = lane == 0 ? on[0] : lane == 1 ? on[1] : on[2];
      o->f1 = lane == 0 ? ub0[0] : lane == 1 ? ub0[1] : ub0[2];
      o->f2 = lane == 0 ? ub1[0] : lane == 1 ? ub1[1] : ub1[2];
    }
  }
}

// Work items of a launch.  The items are cut into 8 contiguous ranges, one
// per XCD (blocks are dealt to the XCDs round-robin, block b to XCD b % 8):
// neighbouring columns of similar layers run on one XCD and share its L2.
// The blocks of an XCD take the items of its range from a counter, then help
// the other ranges; a block ends when every range is used up (at most 8 more
// counter draws), so the launch needs only as many blocks as fit on the chip
// and no block is left idle behind a heavy item.
// Starts with a barrier: the previous item's LDS contents are no longer read.
__device__ __forceinline__ bool next_item(const TileArgs& a, int* range_k, int* col, int* half,
                                          int* z0, int* z1) {
  __shared__ int s_next[2];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int begin = a.item_range[0], n = a.item_range[1] - begin;
    const int per = (n + 7) / 8;
    const int x0 = blockIdx.x & 7;
    int k = *range_k, item = -1;
    for (; k < 8; ++k) {
      const int x = (x0 + k) & 7;
      const int lo = x * per, hi = min(n, lo + per);
      if (lo >= hi) continue;
      const int t = atomicAdd(a.item_ctr + x, 1);
      if (lo + t < hi) {
        item = begin + lo + t;
        break;
      }
    }
    s_next[0] = item;
    s_next[1] = k;
  }
  __syncthreads();
  const int item = s_next[0];
  *range_k = s_next[1];
  if (item < 0) return false;
  const int4 it = a.items[item];
  *col = it.x;
  *half = it.y;
  *z0 = it.z;
  *z1 = it.w;
  return true;
}

// Loader side: per lane the in-plane offsets of its chunks (same for every
// plane and component), then one direct-to-LDS load per chunk.
// BF16 values are copied as 2-byte values into the low halves of 32-bit ring
// words (half the HBM bytes of FP32), then widened in place to FP32 words by
// the loader lane that copied them, once they have arrived: the compute waves
// always read FP32 words and pay no conversion per read.
template <typename CT>
struct RingLoader {
  static constexpr int kCopies = 3 * kGChunksPerLoader;  // direct-to-LDS copies per plane
  int rel[kGChunksPerLoader];
  bool act[kGChunksPerLoader];
  int chunk0, lane;

  __device__ __forceinline__ void init(const GridDev& g, int X0, int Y0, int loader, int l) {
    chunk0 = loader;
    lane = l;
#pragma unroll
    for (int m = 0; m < kGChunksPerLoader; ++m) {
      const int c = loader + kLoaders * m;
      const int r = 64 * c + lane;
      act[m] = c < kGChunks && r < kGComp;
      const int rr = min(r, kGComp - 1);
      const int y = rr / kGTW, x = rr - y * kGTW;
      // ring words outside the padded grid (the margin of the first and last
      // columns) are never read by a cell of the grid: any valid address
      const int X = min(max(X0 + x, 0), g.px - 1), Y = min(max(Y0 + y, 0), g.py - 1);
      rel[m] = Y * g.px + X;
    }
  }

  __device__ __forceinline__ void load(const CT* coeff, const GridDev& g, uint32_t* ring,
                                       int P) const {
    const int Pc = min(max(P, 0), g.nz + 2);
    uint32_t* slot = ring + gslot(P) * kGSlot;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      const CT* base = coeff + comp * g.comp + (int64_t)Pc * g.plane;
#pragma unroll
      for (int m = 0; m < kGChunksPerLoader; ++m) {
        const int c = chunk0 + kLoaders * m;
        if (c < kGChunks && act[m]) {
          const auto* src = (const __attribute__((address_space(1))) void*)(base + rel[m]);
          auto* dst = (__attribute__((address_space(3))) void*)(slot + comp * kGComp + 64 * c);
          if constexpr (sizeof(CT) == 4) __builtin_amdgcn_global_load_lds(src, dst, 4, 0, 0);
          else __builtin_amdgcn_global_load_lds(src, dst, 2, 0, 0);
        }
      }
    }
  }

  // BF16: plane P's words of this lane, copied and arrived, to FP32 words.
  __device__ __forceinline__ void widen(uint32_t* ring, int P) const {
    if constexpr (sizeof(CT) == 2) {
      uint32_t* slot = ring + gslot(P) * kGSlot;
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
#pragma unroll
        for (int m = 0; m < kGChunksPerLoader; ++m) {
          const int c = chunk0 + kLoaders * m;
          if (c < kGChunks && act[m]) {
            uint32_t* w = slot + comp * kGComp + 64 * c + lane;
            *w = *w << 16;
          }
        }
      }
    }
  }
};

// s_waitcnt vmcnt(0) with the other counters left alone
#define PT_WAIT_VMCNT0() __builtin_amdgcn_s_waitcnt(0x0F70)
// s_waitcnt vmcnt(N) with the other counters left alone (N < 64).
#define PT_WAIT_VMCNT(N) \
  __builtin_amdgcn_s_waitcnt(((N) & 0xF) | (((N) >> 4) << 14) | 0x0F70)

// Workgroup barrier that waits only for this wave's LDS operations.  A
// __syncthreads() would also wait for every global access of the wave (its
// fence covers the direct-to-LDS copies, tracked by the vector memory
// counter), which would drain the loaders' prefetches at every step; here the
// loaders wait for exactly the copies the next step reads.  The memory
// clobber keeps the compiler from moving accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <typename CT, int MODE>
__global__ __launch_bounds__(kGTB) void tile_gather(TileArgs a) {
  extern __shared__ uint32_t gsm[];
  uint32_t* ring = gsm;
  int* lst = (int*)(gsm + kGRing * kGSlot);  // layer starts of the segment
  const GridDev& g = a.g;
  const int wave = threadIdx.x >> 6;
  const bool loader = wave >= kCompute / 64;
  float umax = 0.0f;  // largest |ub| of this thread's particles (adjoint)
  Pend pend;
  pend.off = -1;
  pend.defer = -1;
  DeferBatch db;
  db.mask = 0;
  int lerr = 0;  // a non-finite position was met
  int col, half_unused, z0, z1, range_k = 0;
  while (next_item(a, &range_k, &col, &half_unused, &z0, &z1)) {
  const int cy = col / a.ncx, cx = col - cy * a.ncx;
  const int X0 = cx * kTileX - 1, Y0 = cy * kTileY - 1;  // ring origin: one-cell margin
  const int nl = z1 - z0;
  const int32_t* ls = a.lstart + 2 * ((int64_t)col * g.nz + z0);
  const CT* coeff = (const CT*)a.coeff;

  RingLoader<CT> rl;
  if (loader) {
    rl.init(g, X0, Y0, wave - kCompute / 64, threadIdx.x & 63);
    for (int P = z0 - 1; P <= z0 + 5; ++P) rl.load(coeff, g, ring, P);
    PT_WAIT_VMCNT0();  // planes z0-1 .. z0+5 are in
    for (int P = z0 - 1; P <= z0 + 5; ++P) rl.widen(ring, P);
  } else {
    for (int i = threadIdx.x; i <= nl; i += kCompute) lst[i] = ls[2 * i];
  }
  lds_barrier();

  const int lane = threadIdx.x & 3, grp = threadIdx.x >> 2;
  const LaneAxis ax = lane_axis(g, lane);
  PData pd[2];
  auto prefetch = [&](int set, int s) {
    const int zs = z0 + s * kSlab;
    int64_t pb = 0, pe = 0;
    if (zs < z1) {
      pb = lst[zs - z0];
      pe = lst[min(zs + kSlab, z1) - z0];
    }
    load_pdata<MODE>(a, pb + grp, pb + grp < pe, &pd[set]);
  };
  if (!loader) {
    prefetch(0, 0);
    prefetch(1, 1);
  }
  for (int s0 = 0; z0 + s0 * kSlab < z1; s0 += 2) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int s = s0 + half;
      const int zs = z0 + s * kSlab;
      if (zs < z1) {
        if (loader) {
          // the planes the next slab adds go into the slots of zs-3, zs-2
          // (free since the previous step) while this slab is evaluated
          rl.load(coeff, g, ring, zs + 6);
          rl.load(coeff, g, ring, zs + 7);
          PT_WAIT_VMCNT0();
          rl.widen(ring, zs + 6);
          rl.widen(ring, zs + 7);
        } else {
          const int64_t pb = lst[zs - z0];
          const int64_t pe = lst[min(zs + kSlab, z1) - z0];
          // passes of kGGroups particles.  Each pass starts with a full wait
          // (the data of this pass was loaded during the previous one), then
          // stores the previous pass's outputs, then loads the next pass into
          // the register set not in use (a copy between sets would also make
          // the wave wait for loads in flight).
          const int npass = (int)((pe - pb + kGGroups - 1) / kGGroups);
          PData sb;
          for (int k = 0; k < npass; k += 2) {  // npass uniform
            PT_WAIT_VMCNT0();
            flush_pend<MODE>(a, &pend, &db, &lerr);
            if (k + 1 < npass) {
              const int64_t pn = pb + (int64_t)(k + 1) * kGGroups + grp;
              load_pdata<MODE>(a, pn, pn < pe, &sb);
            }
            if (pd[half].ok)
              ring_particle<CT, MODE>(a, ring, pd[half], X0, Y0, zs, lane, ax, &umax, &pend, &lerr);
            if (k + 1 >= npass) break;
            PT_WAIT_VMCNT0();
            flush_pend<MODE>(a, &pend, &db, &lerr);
            if (k + 2 < npass) {
              const int64_t pn = pb + (int64_t)(k + 2) * kGGroups + grp;
              load_pdata<MODE>(a, pn, pn < pe, &pd[half]);
            }
            if (sb.ok)
              ring_particle<CT, MODE>(a, ring, sb, X0, Y0, zs, lane, ax, &umax, &pend, &lerr);
          }
          prefetch(half, s + 2);
        }
        lds_barrier();
      }
    }
  }
  if (loader) PT_WAIT_VMCNT0();  // no copy into the ring outlives the item
  }  // items
  if (!loader) {
    // the last outputs, then the list slots of the last deferred batch
    PT_WAIT_VMCNT0();
    flush_pend<MODE>(a, &pend, &db, &lerr);
    PT_WAIT_VMCNT0();
    flush_pend<MODE>(a, &pend, &db, &lerr);
  }
  if (MODE == TILE_RK2_BWD_GRAD) {
    // block maximum of |ub| for the fixed-point scale of the scatter
    float* smax = (float*)(lst + a.seg_len + 4);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) umax = fmaxf(umax, __shfl_xor(umax, o, 64));
    if ((threadIdx.x & 63) == 0) smax[wave] = umax;
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = 0.0f;
      for (int w = 0; w < kGTB / 64; ++w) m = fmaxf(m, smax[w]);
      atomicMax(a.defer_count + 1 + (blockIdx.x & (kMaxSlots - 1)), __float_as_int(m));
    }
  }
}

// Particles deferred by tile_gather, redone from global memory.
template <typename CT, int MODE>
__global__ __launch_bounds__(256) void gather_deferred(TileArgs a) {
  const int64_t n = min((int64_t)*a.defer_count, a.np);
  const GridDev& g = a.g;
  const CT* coeff = (const CT*)a.coeff;
  const int64_t np = a.np;
  const int32_t* list = (const int32_t*)a.defer;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const int64_t p = list[i];
    if (p < 0 || p >= np) continue;
    double xn[3] = {a.x[p], a.x[np + p], a.x[2 * np + p]};
    const Pt qn = locate_pt<0>(g, xn, 0, 0, 0, -1, a.err);
    if (MODE == TILE_INTERP3 || MODE == TILE_INTERP12) {
      constexpr int kOut = MODE == TILE_INTERP12 ? 12 : 3;
      float o12[12];
      eval_global<CT, MODE == TILE_INTERP12>(coeff, g, qn, o12);
      for (int r = 0; r < kOut; ++r) a.out[r * np + p] = o12[r];
    } else if (MODE == TILE_TV_STAGE1) {
      float u0[12];
      eval_global<CT, false>(coeff, g, qn, u0);
      for (int c = 0; c < 3; ++c) {
        a.u0[c * np + p] = u0[c];
        a.x_out[c * np + p] = xn[c];
      }
    } else if (MODE == TILE_TV_STAGE2) {
      double xs[3];
      float ua[3];
      for (int c = 0; c < 3; ++c) {
        ua[c] = a.u0[c * np + p];
        xs[c] = xn[c] + a.dt * (double)ua[c];
      }
      const Pt qs = locate_pt<0>(g, xs, 0, 0, 0, -1, a.err);
      float u1[12];
      eval_global<CT, false>(coeff, g, qs, u1);
      for (int c = 0; c < 3; ++c)
        a.x_out[c * np + p] = xn[c] + 0.5 * a.dt * ((double)ua[c] + (double)u1[c]);
    } else if (MODE == TILE_INERTIAL) {
      float u0[12], u1[12];
      eval_global<CT, false>(coeff, g, qn, u0);
      double xs[3], vn[3];
      for (int c = 0; c < 3; ++c) {
        vn[c] = a.u0 ? (double)a.u0[c * np + p] : 0.0;
        xs[c] = inertial_predict(a.ik, xn[c], vn[c], (double)u0[c],
                                 a.disp ? a.disp[c * np + p] : 0.0);
      }
      const Pt qs = locate_pt<0>(g, xs, 0, 0, 0, -1, a.err);
      eval_global<CT, false>(coeff, g, qs, u1);
      for (int c = 0; c < 3; ++c) {
        a.x_out[c * np + p] = inertial_correct(a.ik, xs[c], (double)u0[c], (double)u1[c]);
        if (a.vel_out)
          a.vel_out[c * np + p] =
              (float)inertial_velocity(a.ik, vn[c], (double)u0[c], (double)u1[c]);
      }
    } else if (MODE == TILE_RK2_FWD_GRAD12) {
      float on[12], os[12];
      eval_global<CT, true>(coeff, g, qn, on);
      double xs[3];
      for (int c = 0; c < 3; ++c) xs[c] = xn[c] + a.dt * (double)on[c];
      const Pt qs = locate_pt<0>(g, xs, 0, 0, 0, -1, a.err);
      eval_global<CT, false>(coeff, g, qs, os);
      for (int c = 0; c < 3; ++c)
        a.x_out[c * np + p] = xn[c] + 0.5 * a.dt * ((double)on[c] + (double)os[c]);
      for (int r = 0; r < 12; ++r) a.out[r * np + p] = on[r];
    } else if (MODE == TILE_RK2_FWD_SAVE) {
      float on[12], os[12];
      eval_global<CT, true>(coeff, g, qn, on);
      double xs[3];
      for (int c = 0; c < 3; ++c) xs[c] = xn[c] + a.dt * (double)on[c];
      const Pt qs = locate_pt<0>(g, xs, 0, 0, 0, -1, a.err);
      eval_global<CT, true>(coeff, g, qs, os);
      for (int c = 0; c < 3; ++c)
        a.x_out[c * np + p] = xn[c] + 0.5 * a.dt * ((double)on[c] + (double)os[c]);
      for (int r = 0; r < 12; ++r) a.saved[r * np + p] = on[r];
      for (int r = 3; r < 12; ++r) a.saved[(r + 9) * np + p] = os[r];
    } else if (MODE == TILE_RK2_FWD) {
      float u0[12], u1[12];
      eval_global<CT, false>(coeff, g, qn, u0);
      double xs[3];
      for (int c = 0; c < 3; ++c) xs[c] = xn[c] + a.dt * (double)u0[c];
      const Pt qs = locate_pt<0>(g, xs, 0, 0, 0, -1, a.err);
      eval_global<CT, false>(coeff, g, qs, u1);
      for (int c = 0; c < 3; ++c)
        a.x_out[c * np + p] = xn[c] + 0.5 * a.dt * ((double)u0[c] + (double)u1[c]);
    } else {
      float on[12], os[12];
      eval_global<CT, true>(coeff, g, qn, on);
      double xs[3], lam[3];
      for (int c = 0; c < 3; ++c) {
        xs[c] = xn[c] + a.dt * (double)on[c];
        lam[c] = a.lam[c * np + p];
      }
      const Pt qs = locate_pt<0>(g, xs, 0, 0, 0, -1, a.err);
      eval_global<CT, true>(coeff, g, qs, os);
      float ub1[3];
      for (int c = 0; c < 3; ++c) ub1[c] = (float)(0.5 * a.dt * lam[c]);
      double xbs[3];
      float ub0[3];
      for (int c = 0; c < 3; ++c) {
        xbs[c] = (double)(ub1[0] * os[3 + c] + ub1[1] * os[6 + c] + ub1[2] * os[9 + c]);
        ub0[c] = (float)(0.5 * a.dt * lam[c] + a.dt * xbs[c]);
      }
      float m = 0.0f;
      for (int c = 0; c < 3; ++c) {
        a.xbn[c * np + p] = lam[c] + xbs[c] +
                            (double)(ub0[0] * on[3 + c] + ub0[1] * on[6 + c] + ub0[2] * on[9 + c]);
        a.u0[c * np + p] = on[c];
        a.ub0[c * np + p] = ub0[c];
        a.ub1[c * np + p] = ub1[c];
        m = fmaxf(m, fmaxf(fabsf(ub0[c]), fabsf(ub1[c])));
      }
      atomicMax(a.defer_count + 1 + (int)(p & (kMaxSlots - 1)), __float_as_int(m));
    }
  }
}

// ------------------------------------------------------- scatter kernel ---
// Adjoint of the 64-term sums of both Heun stages:
//   g_coeff += W(x^n)^T ub0 + W(x*)^T ub1  over the particles.
// Each workgroup takes a 32 x 16 half of a column over a segment of layers and
// sums the contributions in an LDS ring of planes of its tile (one-cell
// margin, so predictor points that moved one cell out still land in it).  A
// plane is added to g_coeff once nothing more can reach it.  Launches run one
// colour (parities of cx, the half-row and the segment) at a time, so no two
// concurrent workgroups touch the same coefficient and the order of the
// additions to each coefficient is fixed.  Stencils that do not fit the tile
// (periodic wrap, or a move of more than one cell) go to a list that
// scatter_deferred adds with atomics after all colours.
//
// The LDS sums are fixed point: LDS atomic adds of FP32 values run at a small
// fraction of the rate of integer ones on this hardware (measured about 0.33
// against 7.6 lane operations per clock per CU for 64-bit integers).  Every
// contribution w * ub is formed in FP32 with ub pre-scaled by 2^k (k chosen
// per launch from the largest |ub|, so that |w ub 2^k| < 2^31), rounded to
// the nearest 32-bit integer and added as a 64-bit integer; the plane flush
// converts back.  The rounding of each contribution is at most 2^-(k+1)
// absolute (about 2^-31 of the largest |ub|) and unbiased.  (Two components
// in the two halves of one 64-bit word would halve the LDS and a third of the
// atomics, but each half then needs a range bound per work item, and bounds
// from particle counts per layer leave too coarse a resolution in dense
// clusters.)
constexpr int kSTW = kTileX + 5;           // 37: tile width with margin
constexpr int kSTH = kTileY / 2 + 5;       // 21
constexpr int kSComp = kSTW * kSTH;        // 777
constexpr int kSPlane = 3 * kSComp;        // 2331
constexpr int kSSlot = kSPlane + 1;        // slot pitch (64-bit words)
// A slab touches planes zs-1 .. zs+5 and then frees zs-1 and zs, which the
// next slab's planes zs+6 and zs+7 take over: 7 slots.
constexpr int kSRing = 7;
// Loader waves read the particles of the chunk after next, locate both
// stages of each particle (FP64 positions, one lane per particle) and leave a
// ready-to-scatter record per particle in LDS; the compute waves only form
// the weights and add the contributions.  The compute waves then issue no
// global loads in their passes (only, at a slab's end, those of the next
// flush's gradient values): a load into registers that a later pass reuses
// makes the compiler wait for every memory operation in flight before
// issuing it, a full memory round trip per pass.
constexpr int kSCompute = 512;             // compute threads (8 waves)
constexpr int kSLoaders = 2;               // loader waves
constexpr int kSTB = kSCompute + 64 * kSLoaders;
constexpr int kSLanes = 8;                 // lanes per particle
constexpr int kSPer = (kSPlane + kSCompute - 1) / kSCompute;  // plane words per thread (5)
constexpr int kSChunk = 64 * kSLoaders;    // particles per chunk, one per loader lane
// Record of a particle in a chunk buffer (32-bit words [kSRec][kSChunk]):
//   0: stage-1 stencil, ring row-column offset | first plane's slot << 12,
//      or kSNoRing when the stencil is not in the ring (deferred)
//   1-3: stage-1 local coordinates (FP32)
//   4-7: the same for the stage-2 (predictor) point
//   8-10: stage-1 velocity adjoint ub0 times the fixed-point scale
//   11-13: stage-2 velocity adjoint ub1 times the scale
//   14: particle index
constexpr int kSRec = 15;
constexpr uint32_t kSNoRing = 0xFFFFFFFFu;

__device__ __forceinline__ int sslot(int P) { return (P + 2 * kSRing) % kSRing; }

// Tile point of element e of a plane: component, row, column.
__device__ __forceinline__ void selem(int e, int* c, int* y, int* x) {
  *c = e / kSComp;
  const int r = e - *c * kSComp;
  *y = r / kSTW;
  *x = r - *y * kSTW;
}

// Adds the 64-point stencil of one stage of a particle to the ring.  word:
// record word 0 or 4 (not kSNoRing); t: local coordinates; us: scaled
// velocity adjoint.  lane = (i, kh) of the particle's 16 / NK lanes:
// x-offset i, planes k = NK kh .. NK kh + NK - 1.
template <int NK>
__device__ __forceinline__ void scatter_ring(long long* ring, uint32_t word, const float t[3],
                                             int lane, const float us[3]) {
  float wx[4], wy[4], wz[4];
  bspline_w(t[0], wx);
  bspline_w(t[1], wy);
  bspline_w(t[2], wz);
  const int i = lane & 3, kh = lane >> 2;
  const float wxi = pick4(wx, i);
  const int off = (int)(word & 0xFFFu) + i, slot0 = (int)(word >> 12);
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    const int k = NK * kh + kk;
    const float wzk = pick4(wz, k);
    int slot = slot0 + k;
    slot -= slot >= kSRing ? kSRing : 0;
    long long* pl = ring + slot * kSSlot + off;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float w = wxi * wy[j] * wzk;
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const int v = __float2int_rn(w * us[comp]);
        atomicAdd((unsigned long long*)(pl + comp * kSComp + j * kSTW),
                  (unsigned long long)(long long)v);
      }
    }
  }
}

// Stage 1 of a particle, and stage 2 with it when both points share a cell
// (pair): one atomic per point then adds w1 s0 + w2 s1, rounded once.  About
// half of the particles at usual Courant numbers, so it saves a good part of
// the LDS atomics.  word: record word 0 (not
// kSNoRing); t1, t2: local coordinates of the two points; s0, s1: scaled
// stage adjoints.
template <int NK>
__device__ __forceinline__ void scatter_ring2(long long* ring, uint32_t word, const float t1[3],
                                              const float t2[3], bool pair, int lane,
                                              const float s0[3], const float s1[3]) {
  float wx[4], wy[4], wz[4], vx[4], vy[4], vz[4];
  bspline_w(t1[0], wx);
  bspline_w(t1[1], wy);
  bspline_w(t1[2], wz);
  bspline_w(t2[0], vx);
  bspline_w(t2[1], vy);
  bspline_w(t2[2], vz);
  const int i = lane & 3, kh = lane >> 2;
  const float wxi = pick4(wx, i), vxi = pick4(vx, i);
  float u1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u1[c] = pair ? s1[c] : 0.0f;
  const int off = (int)(word & 0xFFFu) + i, slot0 = (int)(word >> 12);
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    const int k = NK * kh + kk;
    const float wzk = pick4(wz, k), vzk = pick4(vz, k);
    const float a1 = wxi * wzk, a2 = vxi * vzk;
    int slot = slot0 + k;
    slot -= slot >= kSRing ? kSRing : 0;
    long long* pl = ring + slot * kSSlot + off;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float w1 = a1 * wy[j], w2 = a2 * vy[j];
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const int v = __float2int_rn(fmaf(w2, u1[comp], w1 * s0[comp]));
        atomicAdd((unsigned long long*)(pl + comp * kSComp + j * kSTW),
                  (unsigned long long)(long long)v);
      }
    }
  }
}

// A particle's inputs as loaded: x (lo, hi words of each component), u0,
// ub0, ub1.
struct SRaw {
  uint32_t w[15];
};

__device__ __forceinline__ void load_sraw(const TileArgs& a, int64_t p, SRaw* r) {
  const int64_t np = a.np;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint2 xw = *(const uint2*)(a.x + c * np + p);
    r->w[2 * c] = xw.x;
    r->w[2 * c + 1] = xw.y;
    r->w[6 + c] = __float_as_uint(a.u0[c * np + p]);
    r->w[9 + c] = __float_as_uint(a.ub0[c * np + p]);
    r->w[12 + c] = __float_as_uint(a.ub1[c * np + p]);
  }
}

// Record word 0 or 4 of a located point: cells with tile-local index in
// [0, kTileX + 2) x [0, kTileY/2 + 2) and layers zs-1 .. zs+kSlab have their
// stencils inside the tile and the ring.
__device__ __forceinline__ uint32_t ring_word(const Pt& q, int X0, int Y0, int zs) {
  const int lx = q.a - X0, ly = q.b - Y0;
  const bool in = lx >= 0 && lx < kTileX + 2 && ly >= 0 && ly < kTileY / 2 + 2 &&
                  q.c >= zs - 1 && q.c <= zs + kSlab;
  return in ? (uint32_t)(ly * kSTW + lx) | ((uint32_t)sslot(q.c) << 12) : kSNoRing;
}

// Builds the record of particle p of slab zs in slot l of chunk buffer pb.
__device__ __forceinline__ void store_srec(const TileArgs& a, const SRaw& r, int64_t p, int X0,
                                           int Y0, int zs, float scale, uint32_t* pb, int l,
                                           int* lerr) {
  double x[3], xs[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    x[c] = __longlong_as_double((long long)((uint64_t)r.w[2 * c] |
                                            ((uint64_t)r.w[2 * c + 1] << 32)));
    xs[c] = x[c] + a.dt * (double)__uint_as_float(r.w[6 + c]);
  }
  const Pt qn = locate_pt<0>(a.g, x, 0, 0, 0, -1, lerr);
  const Pt qs = locate_pt<0>(a.g, xs, 0, 0, 0, -1, lerr);
  uint32_t w[kSRec];
  w[0] = ring_word(qn, X0, Y0, zs);
  w[4] = ring_word(qs, X0, Y0, zs);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    w[1 + c] = __float_as_uint(qn.t[c]);
    w[5 + c] = __float_as_uint(qs.t[c]);
    w[8 + c] = __float_as_uint(__uint_as_float(r.w[9 + c]) * scale);
    w[11 + c] = __float_as_uint(__uint_as_float(r.w[12 + c]) * scale);
  }
  w[14] = (uint32_t)p;
#pragma unroll
  for (int k = 0; k < kSRec; ++k) pb[k * kSChunk + l] = w[k];
}

// Deferred stencils (2 p + stage) collect in a small LDS list that the
// workgroup copies to the global list at slab ends (see dump_deferred), so
// that the compute waves issue no global memory operation they would have to
// wait for.  Past the LDS capacity an entry goes straight to the global list.
constexpr int kSDefCap = 512;

__device__ __forceinline__ void defer_stencil(const TileArgs& a, int* sdef_n, uint32_t* sdef,
                                              int64_t p, int stage) {
  const uint32_t e = (uint32_t)(2 * p + stage);
  const int k = atomicAdd(sdef_n, 1);
  if (k < kSDefCap) {
    sdef[k] = e;
  } else {
    const int i = atomicAdd(a.defer_count, 1);
    if ((int64_t)i < 2 * a.np) a.defer[i] = e;
    PT_WAIT_VMCNT0();  // leave no store in flight on this rare path
  }
}

// Copies the LDS list to the global list when it is at least half full (or
// always, with force) and empties it.  Called by the whole workgroup after a
// barrier; ends with one.
__device__ __forceinline__ void dump_deferred(const TileArgs& a, int* sdef_n, uint32_t* sdef,
                                              int* s_base, bool force) {
  const int n = min(*sdef_n, kSDefCap);
  if (n == 0 || (!force && n < kSDefCap / 2)) return;  // uniform
  if (threadIdx.x == 0) *s_base = atomicAdd(a.defer_count, n);
  lds_barrier();
  const int64_t base = *s_base;
  for (int i = threadIdx.x; i < n; i += kSCompute)
    if (i < n && threadIdx.x < kSCompute && base + i < 2 * a.np) a.defer[base + i] = sdef[i];
  lds_barrier();
  if (threadIdx.x == 0) *sdef_n = 0;
  lds_barrier();
}

// Both stages of staged particle q of chunk buffer pb, on the particle's
// 16 / NK lanes (lane: this thread's index among them).
template <int NK>
__device__ __forceinline__ void scatter_particle(const TileArgs& a, long long* ring,
                                                 const uint32_t* pb, int q, int lane, int* sdef_n,
                                                 uint32_t* sdef) {
  float tn[3], ts[3], s0[3], s1[3];
  const uint32_t wn = pb[q], ws = pb[4 * kSChunk + q];
  const uint32_t pq = pb[14 * kSChunk + q];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s0[c] = __uint_as_float(pb[(8 + c) * kSChunk + q]);
    s1[c] = __uint_as_float(pb[(11 + c) * kSChunk + q]);
    tn[c] = __uint_as_float(pb[(1 + c) * kSChunk + q]);
    ts[c] = __uint_as_float(pb[(5 + c) * kSChunk + q]);
  }
  const bool pair = wn == ws && wn != kSNoRing;
  if (wn != kSNoRing) scatter_ring2<NK>(ring, wn, tn, ts, pair, lane, s0, s1);
  else if (lane == 0) defer_stencil(a, sdef_n, sdef, pq, 0);
  if (!pair) {
    if (ws != kSNoRing) scatter_ring<NK>(ring, ws, ts, lane, s1);
    else if (lane == 0) defer_stencil(a, sdef_n, sdef, pq, 1);
  }
}

__device__ __forceinline__ float scatter_scale(const TileArgs& a) {
  float m = 0.0f;
  for (int i = 1; i <= kMaxSlots; ++i) m = fmaxf(m, __int_as_float(a.defer_count[i]));
  if (!(m > 0.0f) || !(m < 3.0e38f)) return 1.0f;
  int e;
  frexpf(m, &e);  // m < 2^e
  // 2^126 at most: the scale and its inverse stay finite and normal
  return ldexpf(1.0f, min(30 - e, 126));
}

// Offsets in g_coeff, less the plane term, of the plane words this thread
// flushes for the current tile (-1: outside the padded grid).  They depend on
// the tile only, so they are formed once per work item.
__device__ __forceinline__ void flush_offsets(const GridDev& g, int X0, int Y0,
                                              int64_t off[kSPer]) {
#pragma unroll
  for (int q = 0; q < kSPer; ++q) {
    const int e = threadIdx.x + q * kSCompute;
    int c, y, x;
    selem(e, &c, &y, &x);
    const int X = X0 + x, Y = Y0 + y;
    off[q] = (e < kSPlane && X >= 0 && X < g.px && Y >= 0 && Y < g.py)
                 ? c * g.comp + (int64_t)Y * g.px + X
                 : -1;
  }
}

// 64-bit fixed-point sum to FP32: the high and low halves converted in FP32
// and combined with one fused multiply-add (at most one FP32 rounding more
// than a direct conversion, far below the accumulated FP32 rounding of the
// gradient).
__device__ __forceinline__ float fixed_to_float(long long acc, float inv_scale) {
  const float hi = (float)(int)(acc >> 32);
  const float lo = (float)(uint32_t)acc;
  return fmaf(hi, 4294967296.0f, lo) * inv_scale;
}

// The plane flush at a slab's end is a read-modify-write of the gradient
// without atomics: the colours keep every other workgroup of the launch off
// these points, and this workgroup writes them only in that flush, so values
// loaded at the slab before's end are still current, and the stores cost
// far less than atomics.  Lanes and planes outside the padded grid load a
// valid word they then ignore, so that every slab end issues the same loads.
struct SPre {
  float v[2][kSPer];
};

__device__ __forceinline__ void prefetch_splanes(const TileArgs& a, const int64_t off[kSPer],
                                                 int P0, SPre* pre) {
  const GridDev& g = a.g;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int P = min(max(P0 + h, 0), g.nz + 2);
    const float* gp = a.gcoeff + (int64_t)P * g.plane;
#pragma unroll
    for (int q = 0; q < kSPer; ++q) pre->v[h][q] = gp[off[q] >= 0 ? off[q] : 0];
  }
}

// Reads planes P0, P0 + 1 of the ring and clears them for reuse (all of the
// thread's LDS reads issued before any conversion), then writes prefetched
// value + plane sum back to the gradient.  Planes outside the padded grid
// are skipped.
__device__ __forceinline__ void flush_splanes_rmw(const TileArgs& a, long long* ring,
                                                  const int64_t off[kSPer], int P0,
                                                  float inv_scale, const SPre& pre) {
  const GridDev& g = a.g;
  long long acc[2][kSPer];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const long long* sl = ring + sslot(P0 + h) * kSSlot;
#pragma unroll
    for (int q = 0; q < kSPer; ++q)
      acc[h][q] = sl[min((int)threadIdx.x + q * kSCompute, kSPlane - 1)];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    long long* sl = ring + sslot(P0 + h) * kSSlot;
#pragma unroll
    for (int q = 0; q < kSPer; ++q) {
      const int e = threadIdx.x + q * kSCompute;
      if (e < kSPlane) sl[e] = 0;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int P = P0 + h;
    if (P < 0 || P >= g.nz + 3) continue;
    float* gp = a.gcoeff + (int64_t)P * g.plane;
#pragma unroll
    for (int q = 0; q < kSPer; ++q)
      if (acc[h][q] != 0 && off[q] >= 0)
        gp[off[q]] = pre.v[h][q] + fixed_to_float(acc[h][q], inv_scale);
  }
}

// Adds finished planes P0 .. P0 + NP - 1 of the ring to the gradient with one
// FP32 atomic add per point (the planes past a work item's last slab) and
// clears them for reuse.  All of the thread's LDS reads are issued before
// any conversion or global atomic.  Planes outside the padded grid are
// skipped.
template <int NP>
__device__ __forceinline__ void flush_splanes(const TileArgs& a, long long* ring,
                                              const int64_t off[kSPer], int P0, float inv_scale) {
  const GridDev& g = a.g;
  long long acc[NP][kSPer];
#pragma unroll
  for (int h = 0; h < NP; ++h) {
    const long long* sl = ring + sslot(P0 + h) * kSSlot;
#pragma unroll
    for (int q = 0; q < kSPer; ++q) {
      const int e = min((int)threadIdx.x + q * kSCompute, kSPlane - 1);  // a word of the plane
      acc[h][q] = sl[e];
    }
  }
#pragma unroll
  for (int h = 0; h < NP; ++h) {
    long long* sl = ring + sslot(P0 + h) * kSSlot;
#pragma unroll
    for (int q = 0; q < kSPer; ++q) {
      const int e = threadIdx.x + q * kSCompute;
      if (e < kSPlane) sl[e] = 0;
    }
  }
#pragma unroll
  for (int h = 0; h < NP; ++h) {
    const int P = P0 + h;
    if (P < 0 || P >= g.nz + 3) continue;
    float* gp = a.gcoeff + (int64_t)P * g.plane;
#pragma unroll
    for (int q = 0; q < kSPer; ++q)
      if (acc[h][q] != 0 && off[q] >= 0) atomicAdd(gp + off[q], fixed_to_float(acc[h][q], inv_scale));
  }
}

__global__ __launch_bounds__(kSTB) void tile_scatter(TileArgs a) {
  extern __shared__ long long ssm[];
  long long* ring = ssm;
  uint32_t* pbuf = (uint32_t*)(ssm + kSRing * kSSlot);  // [2][kSRec][kSChunk]
  int* lst = (int*)(pbuf + 2 * kSRec * kSChunk);       // [2 (nl + 1)] half-layer starts
  int* sdef_n = lst + 2 * (kScatterSeg + 2);  // LDS deferred list: length, base, entries
  int* s_base = sdef_n + 1;
  uint32_t* sdef = (uint32_t*)(sdef_n + 4);
  const GridDev& g = a.g;
  const float scale = scatter_scale(a), inv_scale = 1.0f / scale;
  // the wave index in a scalar register: loader / compute branches are uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool loader = wave >= kSCompute / 64;
  int lerr = 0;  // a non-finite position was met
  if (threadIdx.x == 0) *sdef_n = 0;  // published by the barrier in next_item
  int col, half, z0, z1, range_k = 0;
  while (next_item(a, &range_k, &col, &half, &z0, &z1)) {
  const int cy = col / a.ncx, cx = col - cy * a.ncx;
  const int X0 = cx * kTileX - 1, Y0 = cy * kTileY + half * (kTileY / 2) - 1;
  int64_t foff[kSPer];
  SPre pre;  // the gradient values of the next flush
  if (!loader) {
    flush_offsets(g, X0, Y0, foff);
    prefetch_splanes(a, foff, z0 - 1, &pre);
  }
  const int lane = threadIdx.x & (kSLanes - 1), grp = threadIdx.x / kSLanes;
  const int nl = z1 - z0;
  // starts of this half and of the next half-layer, for layers z0 .. z1
  const int32_t* hs = a.lstart + 2 * ((int64_t)col * g.nz + z0) + half;
  for (int i = threadIdx.x; i < nl; i += kSTB) {
    lst[2 * i] = hs[2 * i];
    lst[2 * i + 1] = hs[2 * i + 1];
  }
  for (int e = threadIdx.x; e < kSRing * kSSlot; e += kSTB) ring[e] = 0;
  __syncthreads();

  // The particles of slab zs (layers zs, zs+1 of this half): one virtual list
  // of n0 + n1, taken in chunks of kSChunk.  Chunks run in slab order, each
  // slab taking at least one.
  auto slab_count = [&](int zs, int64_t* r0, int64_t* n0, int64_t* r1) {
    *r0 = *n0 = *r1 = 0;
    if (zs >= z1) return (int64_t)0;
    const int i0 = zs - z0;
    *r0 = lst[2 * i0];
    *n0 = lst[2 * i0 + 1] - *r0;
    int64_t n1 = 0;
    if (zs + 1 < z1) {
      *r1 = lst[2 * i0 + 2];
      n1 = lst[2 * i0 + 3] - *r1;
    }
    return *n0 + n1;
  };
  auto nchunks = [](int64_t n) { return n > 0 ? (int)((n + kSChunk - 1) / kSChunk) : 1; };
  auto advance = [&](int* zs, int* j) {
    int64_t r0, n0, r1;
    if (*j + 1 >= nchunks(slab_count(*zs, &r0, &n0, &r1))) {
      *zs += kSlab;
      *j = 0;
    } else {
      ++*j;
    }
  };

  // Loader side: raw inputs of this lane's particle of chunk (lzs, lj), in
  // flight while the compute waves work on the chunk before it.
  const int ll = threadIdx.x - kSCompute;  // loader lane 0 .. kSChunk-1
  SRaw raw;
  int64_t raw_p = -1;
  int lzs = z0, lj = 0;
  // particle of this lane in chunk j of a slab (r0, n0, r1: slab_count), or -1
  auto particle = [&](int j, int64_t n, int64_t r0, int64_t n0, int64_t r1) {
    const int64_t v = (int64_t)j * kSChunk + ll;
    return v < n ? (v < n0 ? r0 + v : r1 + (v - n0)) : (int64_t)-1;
  };
  auto issue = [&]() {
    int64_t r0, n0, r1;
    const int64_t n = slab_count(lzs, &r0, &n0, &r1);
    raw_p = particle(lj, n, r0, n0, r1);
    if (raw_p >= 0) load_sraw(a, raw_p, &raw);
  };
  auto finish = [&](int buf) {
    if (raw_p >= 0)
      store_srec(a, raw, raw_p, X0, Y0, lzs, scale, pbuf + buf * kSRec * kSChunk, ll, &lerr);
  };
  if (loader) {
    issue();
    finish(0);  // chunk 0
    advance(&lzs, &lj);
    issue();    // chunk 1
  }
  lds_barrier();
  int zs = z0, j = 0, b = 0;
  while (zs < z1) {  // uniform
    int64_t r0, n0, r1;
    const int64_t n = slab_count(zs, &r0, &n0, &r1);
    const bool slab_end = j + 1 >= nchunks(n);
    if (loader) {
      // The slab bounds of the chunk after next are read first, while the
      // LDS queue is short (right after the barrier, before the compute
      // waves' atomics); then the chunk after this one is finished into
      // buffer b ^ 1 (last read before the previous barrier) and the loads
      // of the one after that are issued.
      int nzs = lzs, nj = lj;
      advance(&nzs, &nj);
      int64_t nr0, nn0, nr1;
      const int64_t nn = slab_count(nzs, &nr0, &nn0, &nr1);
      const int64_t np2 = particle(nj, nn, nr0, nn0, nr1);
      finish(b ^ 1);
      lzs = nzs;
      lj = nj;
      raw_p = np2;
      if (raw_p >= 0) load_sraw(a, raw_p, &raw);
    } else {
      const uint32_t* pb = pbuf + b * kSRec * kSChunk;
      const int cnt = (int)min((int64_t)kSChunk, n - (int64_t)j * kSChunk);
      // Chunks of at most 32 particles (most slabs outside dense clusters)
      // take 16 lanes per particle, so that all compute waves share the
      // work; larger ones 8.  The wave's particles are spaced apart in the
      // chunk, so that in dense cells they do not all add to the same LDS
      // words in one instruction.
      if (cnt <= kSCompute / 16) {
        const int nslot = (cnt + 3) / 4, sub = (threadIdx.x & 63) >> 4;
        if (wave < nslot && sub * nslot + wave < cnt)
          scatter_particle<1>(a, ring, pb, sub * nslot + wave, threadIdx.x & 15, sdef_n, sdef);
      } else {
        const int nslot = (cnt + 7) / 8, sub = grp & 7;
        for (int r = wave; r < nslot; r += kSCompute / 64) {
          const int q = sub * nslot + r;
          if (q < cnt) scatter_particle<2>(a, ring, pb, q, lane, sdef_n, sdef);
        }
      }
    }
    if (slab_end) {
      lds_barrier();
      // planes zs-1 and zs are complete: later particles sit in layers
      // >= zs+2 and their predictor points in layers >= zs+1.  The next
      // slab flushes planes zs+1 and zs+2.
      if (!loader) {
        flush_splanes_rmw(a, ring, foff, zs - 1, inv_scale, pre);
        prefetch_splanes(a, foff, zs + 1, &pre);
      }
      dump_deferred(a, sdef_n, sdef, s_base, false);
    }
    lds_barrier();  // the next chunk is in LDS
    if (slab_end) {
      zs += kSlab;
      j = 0;
    } else {
      ++j;
    }
    b ^= 1;
  }
  // planes above the last flushed one: the last slab accepted cells up to
  // last_zs + kSlab, whose stencils reach plane last_zs + kSlab + 3 (z1 + 3
  // for an even item length, z1 + 4 for an odd one)
  const int last_zs = z0 + ((nl - 1) / kSlab) * kSlab;
  static_assert(kSlab + 3 == 5, "end-of-item flush covers five planes");
  if (!loader) {
    flush_splanes<3>(a, ring, foff, last_zs + 1, inv_scale);
    flush_splanes<2>(a, ring, foff, last_zs + 4, inv_scale);
  }
  lds_barrier();
  }  // items
  __syncthreads();
  dump_deferred(a, sdef_n, sdef, s_base, true);
  if (lerr) *a.err = 1;
}

// Stencils that did not fit their column's tile, added with atomics once all
// colours are done.
__global__ __launch_bounds__(256) void scatter_deferred(TileArgs a) {
  const int64_t n = min((int64_t)*a.defer_count, 2 * a.np);
  const GridDev& g = a.g;
  const int64_t np = a.np;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t e = a.defer[i];
    const int64_t p = e >> 1;
    if (p >= np) continue;
    const int stage = e & 1;
    double x[3];
    float gu[3];
    for (int c = 0; c < 3; ++c) {
      const double xn = a.x[c * np + p];
      if (stage == 0) {
        x[c] = xn;
        gu[c] = a.ub0[c * np + p];
      } else {
        x[c] = xn + a.dt * (double)a.u0[c * np + p];
        gu[c] = a.ub1[c * np + p];
      }
    }
    bool bad = false;
    double t0, t1, t2;
    const int ca = cell_1d(x[0], g.cs[0], g.nx, &t0, &bad);
    const int cb = cell_1d(x[1], g.cs[1], g.ny, &t1, &bad);
    const int cc = cell_1d(x[2], g.cs[2], g.nz, &t2, &bad);
    float wx[4], wy[4], wz[4];
    bspline_w((float)t0, wx);
    bspline_w((float)t1, wy);
    bspline_w((float)t2, wz);
    const int64_t off = ((int64_t)cc * g.py + cb) * g.px + ca;
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j)
        for (int ii = 0; ii < 4; ++ii) {
          const float w = wx[ii] * wy[j] * wz[k];
          for (int c = 0; c < 3; ++c)
            unsafeAtomicAdd(a.gcoeff + c * g.comp + off + k * g.plane + j * g.px + ii, w * gu[c]);
        }
  }
}

__global__ void zero_defer_count(int* p) { p[0] = 0; }

// defer header: [0] deferred-list length, [1 .. kMaxSlots] largest |ub|
// (float bits) per group of gather blocks
__global__ void zero_int(int* p) {
  if (threadIdx.x <= kTableBad) p[threadIdx.x] = 0;
}

// A particle table handed over from an earlier call: entries 0 .. nl must
// rise from 0 to np.  Any other table raises the flag.
__global__ __launch_bounds__(256) void check_table(const int32_t* __restrict__ ls, int64_t nl,
                                                   int64_t np, int* bad) {
  const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (h > nl) return;
  const int64_t v = ls[h];
  bool ok = v >= 0 && v <= np;
  if (h == 0) ok = ok && v == 0;
  if (h == nl) ok = ok && v == np;
  else ok = ok && v <= (int64_t)ls[h + 1];
  if (!ok) atomicOr(bad, 1);
}

// The scatter's counterpart: after a failed check every stencil (2 p + stage)
// is deferred.
// Both fallbacks run on a fixed grid (grid-stride loops): they are launched
// on every call and almost always find the flag clear.
constexpr int kFallbackBlocks = 1024;

__global__ __launch_bounds__(256) void scatter_fallback(int* header, uint32_t* __restrict__ list,
                                                        int64_t np) {
  if (header[kTableBad] == 0) return;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 2 * np; i += stride)
    list[i] = (uint32_t)i;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    header[0] = (int)(2 * np < 0x7fffffff ? 2 * np : 0x7fffffff);
}

// After a failed check: empty every layer and put every particle on the
// deferred list, so that all of them are evaluated from global memory.
__global__ __launch_bounds__(256) void table_fallback(int32_t* __restrict__ ls, int64_t nl,
                                                      int64_t np, int* header,
                                                      int32_t* __restrict__ list) {
  if (header[kTableBad] == 0) return;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i <= nl || i < np; i += stride) {
    if (i <= nl) ls[i] = 0;
    if (i < np) list[i] = (int32_t)i;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) header[0] = (int)np;
}

// ------------------------------------------------------- layer table ---
template <typename K>
__global__ __launch_bounds__(256) void layer_table(const K* __restrict__ keys, int64_t np,
                                                   int64_t nlayers, int32_t* __restrict__ ls) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i > np) return;
  const int64_t lprev = i == 0 ? -1 : (int64_t)(keys[i - 1] >> kHalfShift);
  const int64_t lcur = i == np ? nlayers : (int64_t)(keys[i] >> kHalfShift);
  for (int64_t L = lprev + 1; L <= lcur && L <= nlayers; ++L) ls[L] = (int32_t)i;
}

// ------------------------------------------------------- work items ---
// Work items split each column (gather) or half-column (scatter) into runs of
// layers holding at most pmax particles (but at least lmin layers, the last
// run excepted) and at most lmax layers, so that dense clusters are spread
// over many workgroups.  Scatter items carry a colour: parities of cx, of the
// half-row 2 cy + h and of the run index; runs of one colour never share a
// coefficient because every run between two of them is at least lmin = 6
// layers long and a run touches planes z0-1 .. z1+4 only (z1+4: an odd-length
// run's last slab accepts cells up to z1+1).
// Gather units are (z-block of lmax layers, column), ordered z-block first
// and, inside a z-block, by groups of 8 x 4 neighbouring columns: the
// workgroups that run at the same time on one XCD take neighbouring columns
// over the same layers, so the halo rows and columns they share are read
// from HBM once and then hit in that XCD's L2.  Ragged groups leave empty
// units, which emit no item.
constexpr int kGroupW = 8, kGroupH = 4;

struct ItemCfg {
  int pmax, lmin, lmax, scatter;
  int ncy, ngx, ngy;  // gather: columns in y, column groups in x and y
};

__device__ __forceinline__ bool gather_unit(const ItemCfg& cfg, int ncx, int u, int* col,
                                            int* zb) {
  const int per_zb = cfg.ngx * cfg.ngy * kGroupW * kGroupH;
  *zb = u / per_zb;
  const int r = u - *zb * per_zb;
  const int grp = r / (kGroupW * kGroupH), l = r % (kGroupW * kGroupH);
  const int cx = (grp % cfg.ngx) * kGroupW + l % kGroupW;
  const int cy = (grp / cfg.ngx) * kGroupH + l / kGroupW;
  *col = cy * ncx + cx;
  return cx < ncx && cy < cfg.ncy;
}

__device__ __forceinline__ int unit_layer_count(const int32_t* hs, int nz, int u, int z,
                                                bool scatter) {
  if (!scatter) {
    const int64_t b = 2 * ((int64_t)u * nz + z);
    return hs[b + 2] - hs[b];
  }
  const int64_t b = 2 * ((int64_t)(u >> 1) * nz + z) + (u & 1);
  return hs[b + 1] - hs[b];
}

// One wave per unit: the lanes load the unit's layer counts 64 at a time
// (coalesced), and the greedy cut then runs over them in layer order, every
// lane holding the same state (the counts taken with readlane), so that the
// cuts are those of a sequential pass over the layers.
template <bool WRITE>
__global__ __launch_bounds__(256) void build_items(const int32_t* __restrict__ hs, int nunits,
                                                   int nz, int ncx, ItemCfg cfg,
                                                   int* __restrict__ offsets,
                                                   int4* __restrict__ items, int64_t capacity) {
  const int lane = threadIdx.x & 63;
  const int u = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (u >= nunits) return;  // the whole wave
  const bool sc = cfg.scatter != 0;
  if (!sc) {
    // gather: the layers of one z-block of one column
    int col = 0, zb = 0;
    const bool real = gather_unit(cfg, ncx, u, &col, &zb);
    const int zs = zb * cfg.lmax, ze = min(nz, zs + cfg.lmax);
    int n = 0, z0 = zs, acc = 0;
    const int o = WRITE ? offsets[u] : 0;
    if (real) {
      for (int zc = zs; zc < ze; zc += 64) {
        const int cl = zc + lane < ze ? unit_layer_count(hs, nz, col, zc + lane, false) : 0;
        const int m = min(64, ze - zc);
        for (int jj = 0; jj < m; ++jj) {
          const int z = zc + jj;
          const int c = __builtin_amdgcn_readlane(cl, jj);
          if (z > z0 && z - z0 >= cfg.lmin && acc + c > cfg.pmax) {
            if (WRITE && lane == 0 && o + n < capacity) items[o + n] = make_int4(col, 0, z0, z);
            ++n;
            z0 = z;
            acc = 0;
          }
          acc += c;
        }
      }
      if (WRITE && lane == 0 && o + n < capacity) items[o + n] = make_int4(col, 0, z0, ze);
      ++n;
    }
    if (!WRITE && lane == 0) offsets[u] = n;
    return;
  }
  const int col = u >> 1, half = u & 1;
  const int cx = col % ncx, hy = 2 * (col / ncx) + half;
  const int base = (cx & 1) | ((hy & 1) << 1);
  int n_even = 0, n_odd = 0, k = 0, z0 = 0, acc = 0;
  const int o_even = WRITE ? offsets[base * nunits + u] : 0;
  const int o_odd = WRITE ? offsets[(base | 4) * nunits + u] : 0;
  auto emit = [&](int za, int zb) {
    const bool odd = k & 1;
    const int at = odd ? o_odd + n_odd : o_even + n_even;
    if (WRITE && lane == 0 && at < capacity) items[at] = make_int4(col, half, za, zb);
    if (odd) ++n_odd;
    else ++n_even;
    ++k;
  };
  for (int zc = 0; zc < nz; zc += 64) {
    const int cl = zc + lane < nz ? unit_layer_count(hs, nz, u, zc + lane, true) : 0;
    const int m = min(64, nz - zc);
    for (int jj = 0; jj < m; ++jj) {
      const int z = zc + jj;
      const int c = __builtin_amdgcn_readlane(cl, jj);
      const int len = z - z0;
      if (len > 0 && (len >= cfg.lmax || (len >= cfg.lmin && acc + c > cfg.pmax))) {
        emit(z0, z);
        z0 = z;
        acc = 0;
      }
      acc += c;
    }
  }
  emit(z0, nz);
  if (!WRITE && lane < 8)
    offsets[lane * nunits + u] = lane == base ? n_even : lane == (base | 4) ? n_odd : 0;
}

// Exclusive scan of n counts in one workgroup; range[c] = first item of
// colour c (c = 0 .. ncolors), the counts being colour-major.
__global__ __launch_bounds__(1024) void scan_items(int* data, int n, int nunits, int ncolors,
                                                   int* range) {
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (n + 1023) / 1024;
  const int b = tid * per;
  int tot = 0;
  for (int i = 0; i < per; ++i)
    if (b + i < n) tot += data[b + i];
  int incl = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wave; ++w) woff += wsum[w];
  int run = woff + incl - tot;
  for (int i = 0; i < per; ++i) {
    if (b + i < n) {
      const int v = data[b + i];
      data[b + i] = run;
      if ((b + i) % nunits == 0) range[(b + i) / nunits] = run;
      run += v;
    }
  }
  if (tid == 1023) range[ncolors] = woff + incl;
}

// ------------------------------------------------------------ host side ---
// number of half-layers (entries of the particle table minus one)
int64_t tile_nlayers(const pt_grid* g) {
  const int64_t ncx = (g->nx + kTileX - 1) / kTileX, ncy = (g->ny + kTileY - 1) / kTileY;
  return 2 * ncx * ncy * g->nz;
}

size_t tile_defer_bytes(int64_t np) { return 8 * (size_t)np + kDeferHeader; }

pt_status build_layer_table(const pt_grid* g, int64_t np, const void* keys, int key_bytes,
                            int32_t* ls, hipStream_t s) {
  const int64_t nl = tile_nlayers(g);
  if (key_bytes == 4)
    hipLaunchKernelGGL(layer_table<uint32_t>, dim3(grid_1d(np + 1, 256)), dim3(256), 0, s,
                       (const uint32_t*)keys, np, nl, ls);
  else
    hipLaunchKernelGGL(layer_table<uint64_t>, dim3(grid_1d(np + 1, 256)), dim3(256), 0, s,
                       (const uint64_t*)keys, np, nl, ls);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

static TileArgs tile_args(const pt_grid* g, const void* coeff, const int32_t* ls, int64_t np,
                          double dt, int seg) {
  TileArgs a{};
  a.g = make_grid_dev(g);
  a.coeff = coeff;
  a.lstart = ls;
  a.ncx = (g->nx + kTileX - 1) / kTileX;
  a.ncy = (g->ny + kTileY - 1) / kTileY;
  a.ncol = a.ncx * a.ncy;
  a.seg_len = g->nz <= seg ? g->nz : seg;
  a.nseg = (g->nz + a.seg_len - 1) / a.seg_len;
  a.np = np;
  a.dt = dt;
  a.err = device_error_flag();
  return a;
}

// Items workspace: colour ranges (bytes 0..63), item counters (64..319),
// per-unit counts / offsets, items.
constexpr size_t kItemsHeader = 512;

constexpr int kItemPmax = 8192;

static int64_t item_bound(int64_t nunits, int nz, int64_t np, int lmax) {
  return nunits * ((nz + lmax - 1) / lmax + 1) + 2 * ((np + kItemPmax - 1) / kItemPmax) + 8;
}

// Most layers per work item.  The longest runs are the cheapest per layer
// (each item flushes or loads a few planes beyond its own), but a launch
// needs about two items per compute unit (eight colours for the scatter):
// small grids get shorter runs.
static int item_lmax(const pt_grid* g, bool scatter) {
  const int64_t ncol = (int64_t)((g->nx + kTileX - 1) / kTileX) * ((g->ny + kTileY - 1) / kTileY);
  const int64_t want = scatter ? 8 * 2 * 256 : 2 * 256;  // items per launch, all colours
  const int64_t units = scatter ? 2 * ncol : ncol;
  const int64_t l = (int64_t)g->nz * units / want;
  const int lo = scatter ? 8 : 16, hi = scatter ? kScatterSeg : kGatherSeg;
  return (int)(l < lo ? lo : (l > hi ? hi : l));
}

// Units of the item builder: half-columns (scatter) or (z-block, column)
// slots of the grouped column order (gather).
static int64_t item_units(const pt_grid* g, bool scatter, ItemCfg* cfg) {
  const int ncx = (g->nx + kTileX - 1) / kTileX, ncy = (g->ny + kTileY - 1) / kTileY;
  if (cfg) {
    cfg->ncy = ncy;
    cfg->ngx = (ncx + kGroupW - 1) / kGroupW;
    cfg->ngy = (ncy + kGroupH - 1) / kGroupH;
  }
  if (scatter) return 2 * (int64_t)ncx * ncy;
  const int lmax = item_lmax(g, false);
  const int64_t nzb = (g->nz + lmax - 1) / lmax;
  return nzb * ((ncx + kGroupW - 1) / kGroupW) * ((ncy + kGroupH - 1) / kGroupH) * kGroupW *
         kGroupH;
}

// Workspace of build_tile_items: counts/offsets, colour ranges and items.
size_t tile_items_bytes(const pt_grid* g, int64_t np, bool scatter) {
  const int64_t nunits = item_units(g, scatter, nullptr);
  // a gather unit spans one z-block: at most 1 + (splits by particle count)
  const int64_t bound = scatter ? item_bound(nunits, g->nz, np, item_lmax(g, true))
                                : nunits + 2 * ((np + kItemPmax - 1) / kItemPmax) + 8;
  return kItemsHeader + 4 * (size_t)(8 * nunits) + 16 * (size_t)bound;
}

struct ItemSet {
  const int4* items;
  const int* range;  // [ncolors + 1]
  int* ctr;          // [ncolors][8] zeroed item counters
  int64_t bound;
};

// Scatter items of each launch (colour) and XCD range, the segments that
// next_item deals from, reordered by decreasing estimated cost, particles +
// 32 x layers (a layer's flush and barriers cost about what 32 particles
// cost): the workgroups of an XCD take the long items first and the short
// ones fill in at the end, which shortens the wait for the last workgroup of
// a launch.  The items of one launch are disjoint, so their order changes no
// result.  Segments longer than kOrderMax keep the order they were built in.
constexpr int kOrderMax = 3072;
constexpr int kOrderBins = 32;
__global__ __launch_bounds__(256) void order_items(int4* __restrict__ items,
                                                   const int* __restrict__ range,
                                                   const int32_t* __restrict__ ls, int nz,
                                                   int cost_max) {
  __shared__ int4 s_it[kOrderMax];
  __shared__ unsigned char s_bin[kOrderMax];
  __shared__ int s_cnt[kOrderBins];
  const int c = blockIdx.x >> 3, x = blockIdx.x & 7;
  const int begin = range[c], n = range[c + 1] - begin;
  const int per = (n + 7) / 8;
  const int lo = x * per, hi = min(n, lo + per), len = hi - lo;
  if (len <= 1 || len > kOrderMax) return;  // uniform over the block
  if (threadIdx.x < kOrderBins) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  int4* seg = items + begin + lo;
  for (int i = threadIdx.x; i < len; i += 256) {
    const int4 it = seg[i];  // (column, half, z0, z1)
    s_it[i] = it;
    // particles of the half-column over layers z0 .. z1-1: entry 2 z + half
    // of the column's table starts half `half` of layer z
    const int32_t* L = ls + 2 * (int64_t)it.x * nz + it.y;
    int64_t p = 0;
    for (int z = it.z; z < it.w; ++z) p += L[2 * z + 1] - L[2 * z];
    const int64_t cost = p + 32 * (int64_t)(it.w - it.z);
    const int b = (int)min<int64_t>(kOrderBins - 1, cost * kOrderBins / cost_max);
    s_bin[i] = (unsigned char)(kOrderBins - 1 - b);  // the costliest first
    atomicAdd(&s_cnt[kOrderBins - 1 - b], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int o = 0;
    for (int b = 0; b < kOrderBins; ++b) {
      const int t = s_cnt[b];
      s_cnt[b] = o;
      o += t;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < len; i += 256) seg[atomicAdd(&s_cnt[s_bin[i]], 1)] = s_it[i];
}

__global__ void zero_ctr(int* p) {
  if (threadIdx.x < 64) p[threadIdx.x] = 0;
}

static pt_status build_tile_items(const pt_grid* g, int64_t np, const int32_t* hs, bool scatter,
                                  void* ws, ItemSet* out, hipStream_t s) {
  const int ncx = (g->nx + kTileX - 1) / kTileX;
  const int lmax = item_lmax(g, scatter);
  ItemCfg cfg{kItemPmax, scatter ? 6 : 2, lmax, scatter ? 1 : 0, 0, 0, 0};
  const int64_t nunits64 = item_units(g, scatter, &cfg);
  const int ncolors = scatter ? 8 : 1;
  if (nunits64 * ncolors > (int64_t)1 << 26) return PT_ERR_UNSUPPORTED;
  const int nunits = (int)nunits64;
  char* p = (char*)ws;
  int* range = (int*)p;
  int* ctr = (int*)(p + 64);  // [8 colours][8 XCD ranges]
  int* offsets = (int*)(p + kItemsHeader);
  int4* items = (int4*)(p + kItemsHeader + 4 * (size_t)(8 * nunits));
  const unsigned blocks = (unsigned)((nunits + 3) / 4);  // a wave per unit
  const int64_t bound = scatter ? item_bound(nunits, g->nz, np, lmax)
                                : nunits + 2 * ((np + kItemPmax - 1) / kItemPmax) + 8;
  hipLaunchKernelGGL(build_items<false>, dim3(blocks), dim3(256), 0, s, hs, nunits, g->nz, ncx,
                     cfg, offsets, items, bound);
  hipLaunchKernelGGL(scan_items, dim3(1), dim3(1024), 0, s, offsets, nunits * ncolors, nunits,
                     ncolors, range);
  hipLaunchKernelGGL(build_items<true>, dim3(blocks), dim3(256), 0, s, hs, nunits, g->nz, ncx,
                     cfg, offsets, items, bound);
  PT_LAUNCH_CHECK();
  if (scatter) {
    // the gather keeps its order: neighbouring columns of one XCD share halo
    // lines in its L2 when they run together
    hipLaunchKernelGGL(order_items, dim3(8 * ncolors), dim3(256), 0, s, items, range, hs, g->nz,
                       kItemPmax + 32 * lmax);
    PT_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(zero_ctr, dim3(1), dim3(64), 0, s, ctr);
  PT_LAUNCH_CHECK();
  out->items = items;
  out->range = range;
  out->ctr = ctr;
  out->bound = bound;
  return PT_OK;
}

// Blocks of a tiled launch: per_cu per compute unit (the gathers hold one
// workgroup per CU, the scatter two), a multiple of 8 (the XCD ranges), at
// most one per item.
static unsigned item_blocks(int64_t bound, int per_cu = 1) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  const int64_t want = ((int64_t)cus * per_cu + 7) / 8 * 8;
  const int64_t cap = (bound + 7) / 8 * 8;
  return (unsigned)(want < cap ? want : cap);
}

template <typename F>
static bool allow_lds(F* fn, size_t bytes) {
  return hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes) == hipSuccess;
}

static const char* gather_name(int mode) {
  switch (mode) {
    case TILE_RK2_FWD: return "tile_rk2_fwd";
    case TILE_RK2_BWD_GRAD: return "tile_rk2_bwd_gather";
    case TILE_TV_STAGE1: return "tile_tv_stage1";
    case TILE_INERTIAL: return "tile_inertial";
    case TILE_INTERP3: return "tile_interp";
    case TILE_INTERP12: return "tile_interp_grad";
    case TILE_RK2_FWD_SAVE: return "tile_rk2_fwd_save";
    case TILE_RK2_FWD_GRAD12: return "tile_rk2_fwd_grad";
    default: return "tile_tv_stage2";
  }
}

// check: the particle table comes from an earlier call; verify it on the
// device first (a table that fails sends every particle down the deferred
// path, which needs no table).
static pt_status launch_gather(const pt_grid* g, TileArgs a, pt_dtype dtype, int mode,
                               void* defer, void* items_ws, bool check, hipStream_t s) {
  a.defer_count = (int*)defer;
  a.defer = (uint32_t*)((char*)defer + kDeferHeader);
  hipLaunchKernelGGL(zero_int, dim3(1), dim3(128), 0, s, a.defer_count);
  PT_LAUNCH_CHECK();
  if (check) {
    const int64_t nl = tile_nlayers(g);
    hipLaunchKernelGGL(check_table, dim3(grid_1d(nl + 1, 256)), dim3(256), 0, s, a.lstart, nl,
                       a.np, a.defer_count + kTableBad);
    hipLaunchKernelGGL(table_fallback, dim3(kFallbackBlocks), dim3(256), 0, s,
                       (int32_t*)a.lstart, nl, a.np, a.defer_count, (int32_t*)a.defer);
    PT_LAUNCH_CHECK();
  }
  ItemSet it;
  pt_status st = build_tile_items(g, a.np, a.lstart, false, items_ws, &it, s);
  if (st != PT_OK) return st;
  a.items = it.items;
  a.item_range = it.range;
  a.item_ctr = it.ctr;
  const unsigned blocks = item_blocks(it.bound);
  const size_t lds = sizeof(uint32_t) * ((size_t)kGRing * kGSlot + a.seg_len + 4 + kGTB / 64);
#define PT_TG(CT, MD)                                                                  \
  do {                                                                                 \
    if (!allow_lds(tile_gather<CT, MD>, lds)) return PT_ERR_HIP;                       \
    {                                                                                  \
      TimedLaunch t(gather_name(MD), s);                                               \
      hipLaunchKernelGGL((tile_gather<CT, MD>), dim3(blocks), dim3(kGTB), lds, s, a);  \
    }                                                                                  \
    hipLaunchKernelGGL((gather_deferred<CT, MD>), dim3(256), dim3(256), 0, s, a);      \
  } while (0)
#define PT_TG_MODES(CT)                                   \
  do {                                                    \
    switch (mode) {                                       \
      case TILE_RK2_FWD: PT_TG(CT, TILE_RK2_FWD); break;  \
      case TILE_RK2_BWD_GRAD: PT_TG(CT, TILE_RK2_BWD_GRAD); break; \
      case TILE_TV_STAGE1: PT_TG(CT, TILE_TV_STAGE1); break; \
      case TILE_INERTIAL: PT_TG(CT, TILE_INERTIAL); break; \
      case TILE_INTERP3: PT_TG(CT, TILE_INTERP3); break; \
      case TILE_INTERP12: PT_TG(CT, TILE_INTERP12); break; \
      case TILE_RK2_FWD_SAVE: PT_TG(CT, TILE_RK2_FWD_SAVE); break; \
      case TILE_RK2_FWD_GRAD12: PT_TG(CT, TILE_RK2_FWD_GRAD12); break; \
      default: PT_TG(CT, TILE_TV_STAGE2); break;          \
    }                                                     \
  } while (0)
  if (dtype == PT_F32) PT_TG_MODES(float);
  else if (dtype == PT_BF16) PT_TG_MODES(uint16_t);
  else return PT_ERR_UNSUPPORTED;  // the ring stages FP32 or BF16 only
#undef PT_TG_MODES
#undef PT_TG
  PT_LAUNCH_CHECK();
  return PT_OK;
}

// defer: tile_defer_bytes(np) bytes; items_ws: tile_items_bytes(g, np, false)
// check: ls was built from positions that may not be in cell order (see
// launch_gather); x_out may then alias x.
pt_status tile_rk2_fwd(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                       int64_t np, double dt, const double* x, double* x_out, void* defer,
                       void* items_ws, bool check, hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, dt, kGatherSeg);
  a.x = x;
  a.x_out = x_out;
  return launch_gather(g, a, dtype, TILE_RK2_FWD, defer, items_ws, check, s);
}

// The same step keeping, per particle, u0 and the velocity gradients at x_n
// and at x* in saved ([21][np] floats, rows as TileArgs::saved) for
// tile_rk2_bwd_saved.  x_out may alias x.
pt_status tile_rk2_fwd_save(const pt_grid* g, const void* coeff, pt_dtype dtype,
                            const int32_t* ls, int64_t np, double dt, const double* x,
                            double* x_out, float* saved, void* defer, void* items_ws, bool check,
                            hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, dt, kGatherSeg);
  a.x = x;
  a.x_out = x_out;
  a.saved = saved;
  return launch_gather(g, a, dtype, TILE_RK2_FWD_SAVE, defer, items_ws, check, s);
}

// The same step writing also (u, v, w) and the nine velocity gradients at x
// to out ([12][np] floats, rows as tile_interp with nout = 12).  x_out may
// alias x.
pt_status tile_rk2_fwd_grad(const pt_grid* g, const void* coeff, pt_dtype dtype,
                            const int32_t* ls, int64_t np, double dt, const double* x,
                            double* x_out, float* out, void* defer, void* items_ws, bool check,
                            hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, dt, kGatherSeg);
  a.x = x;
  a.x_out = x_out;
  a.out = out;
  return launch_gather(g, a, dtype, TILE_RK2_FWD_GRAD12, defer, items_ws, check, s);
}

// Inertial / diffusive step on sorted particles x (table ls, checked on the
// device when `check`): x_out, v_out may alias x, v; v and v_out may be null
// (tracer), disp may be null.
pt_status tile_inertial(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                        int64_t np, const InertialCoef& k, const double* x, const float* v,
                        const double* disp, double* x_out, float* v_out, void* defer,
                        void* items_ws, bool check, hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, 0.0, kGatherSeg);
  a.x = x;
  a.x_out = x_out;
  a.u0 = (float*)v;  // read only in this mode
  a.vel_out = v_out;
  a.disp = disp;
  a.ik = k;
  return launch_gather(g, a, dtype, TILE_INERTIAL, defer, items_ws, check, s);
}

// (u, v, w) (nout = 3) or with the nine gradients (nout = 12) at particles
// in cell order (table ls built from x, checked on the device).
pt_status tile_interp(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                      int64_t np, const double* x, int nout, float* out, void* defer,
                      void* items_ws, hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, 0.0, kGatherSeg);
  a.x = x;
  a.out = out;
  return launch_gather(g, a, dtype, nout == 12 ? TILE_INTERP12 : TILE_INTERP3, defer, items_ws,
                       true, s);
}

// Stage 1 of the time-varying step on sorted particles x (table ls):
// u_n = u^n(x) and x_out = x (the sorted positions handed back).
pt_status tile_tv_stage1(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                         int64_t np, const double* x, double* x_out, float* u_n, void* defer,
                         void* items_ws, hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, 0.0, kGatherSeg);
  a.x = x;
  a.x_out = x_out;
  a.u0 = u_n;
  return launch_gather(g, a, dtype, TILE_TV_STAGE1, defer, items_ws, false, s);
}

// Stage 2: x_out = x + dt/2 (u_n + u^{n+1}(x + dt u_n)); x_out may alias x.
// ls is the table of an earlier stage 1 and is checked on the device.
pt_status tile_tv_stage2(const pt_grid* g, const void* coeff, pt_dtype dtype, int32_t* ls,
                         int64_t np, double dt, const double* x, const float* u_n, double* x_out,
                         void* defer, void* items_ws, hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, dt, kGatherSeg);
  a.x = x;
  a.x_out = x_out;
  a.u0 = (float*)u_n;  // read only in this mode
  return launch_gather(g, a, dtype, TILE_TV_STAGE2, defer, items_ws, true, s);
}

static pt_status launch_scatter(const pt_grid* g, const int32_t* ls, int64_t np, double dt,
                                const double* x, float* u0, float* ub0, float* ub1,
                                float* gcoeff, void* defer, void* items_ws, bool check,
                                hipStream_t s);

// defer: tile_defer_bytes(np) bytes; items_ws: tile_items_bytes(g, np, false)
// followed by tile_items_bytes(g, np, true) bytes.  The gather writes u0,
// ub0 and ub1 for the scatter, which then needs neither lam nor xbn: xbn may
// alias lam (each particle's lam is read before its xbn is written, by the
// same thread, in the gather or in gather_deferred).
pt_status tile_rk2_bwd(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                       int64_t np, double dt, const double* x, const double* lam, double* xbn,
                       float* u0, float* ub0, float* ub1, float* gcoeff, void* defer,
                       void* items_ws, bool check, hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, dt, kGatherSeg);
  a.x = x;
  a.lam = lam;
  a.xbn = xbn;
  a.u0 = u0;
  a.ub0 = ub0;
  a.ub1 = ub1;
  pt_status st = launch_gather(g, a, dtype, TILE_RK2_BWD_GRAD, defer, items_ws, check, s);
  if (st != PT_OK || !gcoeff) return st;
  return launch_scatter(g, ls, np, dt, x, u0, ub0, ub1, gcoeff, defer, items_ws, check, s);
}

// Header of a deferred list cleared: its length, the slots of the largest
// |ub| and the table flag.
pt_status tile_defer_reset(void* defer, hipStream_t s) {
  hipLaunchKernelGGL(zero_int, dim3(1), dim3(128), 0, s, (int*)defer);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

// Slots of the largest |ub| in a deferred-list header (for a gather that
// fills them itself before launch_scatter).
int* tile_umax_slots(void* defer) { return (int*)defer + 1; }

// The scatter alone, after a gather (tiled or not) has written u0, ub0, ub1
// and the largest |ub| into the header of `defer` (cleared before it by
// tile_defer_reset).  check: the table ls comes from positions that may not
// be in cell order, checked here first.
pt_status tile_scatter_only(const pt_grid* g, const int32_t* ls, int64_t np, double dt,
                            const double* x, float* u0, float* ub0, float* ub1, float* gcoeff,
                            void* defer, void* items_ws, bool check, hipStream_t s) {
  if (check) {
    // a table that fails is emptied (no work items), and launch_scatter then
    // sends every stencil to the deferred list
    const int64_t nl = tile_nlayers(g);
    hipLaunchKernelGGL(check_table, dim3(grid_1d(nl + 1, 256)), dim3(256), 0, s, ls, nl, np,
                       (int*)defer + kTableBad);
    hipLaunchKernelGGL(table_fallback, dim3(kFallbackBlocks), dim3(256), 0, s, (int32_t*)ls, nl,
                       np, (int*)defer, (int32_t*)((char*)defer + kDeferHeader));
    PT_LAUNCH_CHECK();
  }
  return launch_scatter(g, ls, np, dt, x, u0, ub0, ub1, gcoeff, defer, items_ws, check, s);
}

// The step adjoint from what tile_rk2_fwd_save kept, one thread per
// particle: with lam = dL/dx_{n+1} and J0, J1 the velocity gradients at x_n
// and x*,
//   ub1 = dt/2 lam,  ub0 = dt/2 lam + dt J1^T ub1,
//   dL/dx_n = lam + J1^T ub1 + J0^T ub0  (written over lam),
// the arithmetic of the adjoint gather; the largest |ub| of each block goes
// to one of the kMaxSlots slots for the scatter's fixed-point scale.
__global__ __launch_bounds__(256) void rk2_bwd_saved(const float* __restrict__ saved, int64_t np,
                                                     double dt, double* __restrict__ lam_xb,
                                                     float* __restrict__ ub0,
                                                     float* __restrict__ ub1, int* umax) {
  __shared__ float smax[4];
  float m = 0.0f;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < np;
       p += (int64_t)gridDim.x * 256) {
    double lam[3];
    float j0[9], j1[9], b0[3], b1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) lam[c] = lam_xb[c * np + p];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      j0[r] = saved[(3 + r) * np + p];
      j1[r] = saved[(12 + r) * np + p];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) b1[c] = (float)(0.5 * dt * lam[c]);
    double xbs[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xbs[c] = (double)(b1[0] * j1[c] + b1[1] * j1[3 + c] + b1[2] * j1[6 + c]);
      b0[c] = (float)(0.5 * dt * lam[c] + dt * xbs[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lam_xb[c * np + p] =
          lam[c] + xbs[c] + (double)(b0[0] * j0[c] + b0[1] * j0[3 + c] + b0[2] * j0[6 + c]);
      ub0[c * np + p] = b0[c];
      ub1[c * np + p] = b1[c];
      m = fmaxf(m, fmaxf(fabsf(b0[c]), fabsf(b1[c])));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(umax + (blockIdx.x & (kMaxSlots - 1)),
              __float_as_int(fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]))));
}

// dL/dx_n (in place of lam) and the coefficient gradient (accumulated into
// gcoeff, if not null) of a Heun step on sorted particles x (table ls,
// checked on the device) whose forward kept saved (tile_rk2_fwd_save).  ub0
// and ub1: [3][np] floats of workspace.
pt_status tile_rk2_bwd_saved(const pt_grid* g, const int32_t* ls, int64_t np, double dt,
                             const double* x, const float* saved, double* lam, float* ub0,
                             float* ub1, float* gcoeff, void* defer, void* items_ws,
                             hipStream_t s) {
  pt_status st = tile_defer_reset(defer, s);
  if (st != PT_OK) return st;
  {
    TimedLaunch t("rk2_bwd_saved", s);
    const unsigned blocks = grid_1d(np, 256) < 8192u ? grid_1d(np, 256) : 8192u;
    hipLaunchKernelGGL(rk2_bwd_saved, dim3(blocks), dim3(256), 0, s, saved, np, dt, lam,
                       ub0, ub1, tile_umax_slots(defer));
    PT_LAUNCH_CHECK();
  }
  if (!gcoeff) return PT_OK;
  // the scatter reads u0 from the saved rows 0..2 ([3][np], read only)
  return tile_scatter_only(g, ls, np, dt, x, const_cast<float*>(saved), ub0, ub1, gcoeff, defer,
                           items_ws, true, s);
}

static pt_status launch_scatter(const pt_grid* g, const int32_t* ls, int64_t np, double dt,
                                const double* x, float* u0, float* ub0, float* ub1,
                                float* gcoeff, void* defer, void* items_ws, bool check,
                                hipStream_t s) {
  pt_status st;
  TileArgs b = tile_args(g, nullptr, ls, np, dt, kScatterSeg);
  b.x = x;
  b.u0 = u0;
  b.ub0 = ub0;
  b.ub1 = ub1;
  b.gcoeff = gcoeff;
  b.defer_count = (int*)defer;
  b.defer = (uint32_t*)((char*)defer + kDeferHeader);
  ItemSet it;
  st = build_tile_items(g, np, ls, true, (char*)items_ws + tile_items_bytes(g, np, false), &it, s);
  if (st != PT_OK) return st;
  b.items = it.items;
  hipLaunchKernelGGL(zero_defer_count, dim3(1), dim3(1), 0, s, b.defer_count);
  PT_LAUNCH_CHECK();
  if (check) {
    // a table the gather found invalid was emptied: every stencil goes to
    // the deferred list
    hipLaunchKernelGGL(scatter_fallback, dim3(kFallbackBlocks), dim3(256), 0, s,
                       b.defer_count, b.defer, np);
    PT_LAUNCH_CHECK();
  }
  const size_t lds = sizeof(long long) * (size_t)kSRing * kSSlot +
                     sizeof(uint32_t) * 2 * kSRec * kSChunk + sizeof(int) * 2 * (kScatterSeg + 2) +
                     sizeof(int) * (4 + (size_t)kSDefCap);
  if (!allow_lds(tile_scatter, lds)) return PT_ERR_HIP;
  const unsigned blocks = item_blocks(it.bound);
  for (int color = 0; color < 8; ++color) {
    b.color = color;
    b.item_range = it.range + color;
    b.item_ctr = it.ctr + 8 * color;
    TimedLaunch t("tile_scatter", s);
    hipLaunchKernelGGL(tile_scatter, dim3(blocks), dim3(kSTB), lds, s, b);
    PT_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(scatter_deferred, dim3(1024), dim3(256), 0, s, b);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
