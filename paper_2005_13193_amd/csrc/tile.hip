// Column-tiled gathers and scatter for particles ordered by cell.
//
// After pt_sort_particles the particles of a column of kTileX x kTileY cells
// are contiguous and ordered by layer z.  One workgroup takes one column over
// a range of layers and marches up in z with a ring of kRing padded
// coefficient planes of the column's (kTileX+3) x (kTileY+3) tile staged in
// LDS, so that every coefficient is read from HBM about once per column
// (plus the three shared halo rows/columns and the planes at segment
// boundaries).  Per slab of kSlab layers the ring holds planes z-1 .. z+5:
// the stencils of the particles of the slab and of points up to one layer
// away (the RK2 predictor moves a particle by at most ~0.6 cell per step).
// Points whose stencil is not in the ring (they left the column or moved
// more than one layer) are evaluated from global memory instead.
//
// Four lanes evaluate one point: lane i holds the x-offset i of the 4x4x4
// stencil, sums the 16 (y, z) rows for each component, and the four partial
// sums are combined with quad DPP moves.
#include "pt_common.h"

namespace pt {

constexpr int kTB = 512;                 // threads per workgroup
constexpr int kGroups = kTB / 4;         // points in flight per pass
constexpr int kTW = kTileX + 3;          // tile width in padded points (35)
constexpr int kTH = kTileY + 3;          // tile height (35)
constexpr int kRing = 8;                 // LDS plane slots (power of two)
constexpr int kSlab = 2;                 // layers per iteration
constexpr int kRowP = 36;                // LDS row pitch (floats)
constexpr int kCompP = kTH * kRowP + 4;  // LDS component pitch
constexpr int kSlotP = 3 * kCompP + 4;   // LDS plane-slot pitch
constexpr int kPlaneElems = 3 * kTW * kTH;
constexpr int kPerThread = (kPlaneElems + kTB - 1) / kTB;  // 8
constexpr int kLayerShift = 10;          // log2(kTileX * kTileY)
static_assert(kTileX * kTileY == (1 << kLayerShift), "layer shift");

struct TileArgs {
  GridDev g;
  const void* coeff;
  const int32_t* lstart;  // [ncol * nz + 1]: first particle of each (column, layer)
  int ncx, ncol, nseg, seg_len;
  int64_t np;
  double dt;
  const double* x;        // [3][np] positions (sorted)
  double* x_out;          // fwd: new positions
  const double* lam;      // bwd: dL/dx_out  [3][np]
  double* xbn;            // bwd: dL/dx_n    [3][np]
  float* u0;              // bwd: stage-1 velocity  [3][np]
  float* ub0;             // bwd: adjoint of stage-1 velocity [3][np]
  float* gcoeff;          // scatter target (padded FP32)
  int* err;
};

// Work item of a block: column and first/last layer.  Blocks are dealt to the
// 8 XCDs round-robin; item numbers are remapped so that each XCD walks a
// contiguous run of neighbouring columns (shared halos stay in its L2).
__device__ __forceinline__ void work_item(const TileArgs& a, int* col, int* z0, int* z1) {
  const int nitems = a.ncol * a.nseg;
  const int b = blockIdx.x;
  const int per = (nitems + 7) / 8;
  int item = (b & 7) * per + (b >> 3);
  if ((b & 7) * per + (b >> 3) >= nitems || (b >> 3) >= per) item = -1;
  if (item < 0) { *col = -1; return; }
  const int seg = item / a.ncol;
  *col = item - seg * a.ncol;
  *z0 = seg * a.seg_len;
  *z1 = min(*z0 + a.seg_len, a.g.nz);
}

__device__ __forceinline__ float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
  return v;
}

// ------------------------------------------------------ plane staging ---
template <typename CT>
struct PlaneLoader {
  const CT* coeff;
  int64_t comp_stride, plane;
  int px, py, X0, Y0;

  __device__ __forceinline__ void load(int P, int npad, float v[kPerThread]) const {
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int e = threadIdx.x + q * kTB;
      const int c = e / (kTW * kTH);
      const int r = e - c * (kTW * kTH);
      const int y = r / kTW, x = r - y * kTW;
      const bool ok = e < kPlaneElems && P >= 0 && P < npad && X0 + x < px && Y0 + y < py;
      v[q] = ok ? load_coeff(coeff + c * comp_stride + (int64_t)P * plane +
                             (int64_t)(Y0 + y) * px + (X0 + x))
                : 0.0f;
    }
  }
};

__device__ __forceinline__ void store_plane(float* lds, int slot, const float v[kPerThread]) {
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int e = threadIdx.x + q * kTB;
    if (e < kPlaneElems) {
      const int c = e / (kTW * kTH);
      const int r = e - c * (kTW * kTH);
      const int y = r / kTW, x = r - y * kTW;
      lds[slot * kSlotP + c * kCompP + y * kRowP + x] = v[q];
    }
  }
}

// ---------------------------------------------------- point evaluation ---
struct Pt {
  int a, b, c;     // cell
  float t[3];      // local coordinates
  bool in_ring;    // stencil resident in LDS
};

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
  q.in_ring = lx >= 0 && lx < kTileX && ly >= 0 && ly < kTileY && q.c >= zlo && q.c <= zhi;
  return q;
}

// Value (GRAD: and gradient) of the three components at a resident point;
// every lane of the quad returns the full result.
template <bool GRAD>
__device__ __forceinline__ void eval_lds(const float* lds, const GridDev& g, const Pt& q, int X0,
                                         int Y0, int lane, float out[12]) {
  float wx[4], wy[4], wz[4], dwx[4], dwy[4], dwz[4];
  bspline_w(q.t[0], wx);
  bspline_w(q.t[1], wy);
  bspline_w(q.t[2], wz);
  if (GRAD) {
    bspline_dw(q.t[0], dwx);
    bspline_dw(q.t[1], dwy);
    bspline_dw(q.t[2], dwz);
  }
  const float wxi = lane == 0 ? wx[0] : lane == 1 ? wx[1] : lane == 2 ? wx[2] : wx[3];
  float dwxi = 0.f;
  if (GRAD) dwxi = lane == 0 ? dwx[0] : lane == 1 ? dwx[1] : lane == 2 ? dwx[2] : dwx[3];
  const int col = (q.a - X0) + lane;
  const int row0 = q.b - Y0;
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    float A = 0.f, B = 0.f, C = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float* pl = lds + ((q.c + k) & (kRing - 1)) * kSlotP + comp * kCompP + col;
      float sy = 0.f, sdy = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float s = pl[(row0 + j) * kRowP];
        sy += wy[j] * s;
        if (GRAD) sdy += dwy[j] * s;
      }
      A += wz[k] * sy;
      if (GRAD) {
        B += wz[k] * sdy;
        C += dwz[k] * sy;
      }
    }
    out[comp] = quad_sum(wxi * A);
    if (GRAD) {
      out[3 + 3 * comp + 0] = quad_sum(dwxi * A) * g.inv_h[0];
      out[3 + 3 * comp + 1] = quad_sum(wxi * B) * g.inv_h[1];
      out[3 + 3 * comp + 2] = quad_sum(wxi * C) * g.inv_h[2];
    }
  }
}

// Same quantity from global memory (points outside the ring; rare, so kept
// out of line).
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

template <typename CT, bool GRAD>
__device__ __forceinline__ void eval_point(const float* lds, const CT* coeff, const GridDev& g,
                                           const Pt& q, int X0, int Y0, int lane, float out[12]) {
  if (q.in_ring) eval_lds<GRAD>(lds, g, q, X0, Y0, lane, out);
  else eval_global<CT, GRAD>(coeff, g, q, out);
}

// ------------------------------------------------------- gather kernels ---
enum { TILE_RK2_FWD = 0, TILE_RK2_BWD_GRAD = 1 };

template <typename CT, int MODE>
__device__ __forceinline__ void process_particle(const TileArgs& a, const float* lds, int64_t p,
                                                 int X0, int Y0, int zz, int lane) {
  const GridDev& g = a.g;
  const CT* coeff = (const CT*)a.coeff;
  const int64_t np = a.np;
  double xn[3] = {a.x[p], a.x[np + p], a.x[2 * np + p]};
  // resident layers of cells: zz-1 .. zz+2 (planes zz-1 .. zz+5)
  const Pt qn = locate_pt(g, xn, X0, Y0, zz - 1, zz + kSlab, a.err);
  if (MODE == TILE_RK2_FWD) {
    float u0[12], u1[12];
    eval_point<CT, false>(lds, coeff, g, qn, X0, Y0, lane, u0);
    double xs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) xs[d] = xn[d] + a.dt * (double)u0[d];
    const Pt qs = locate_pt(g, xs, X0, Y0, zz - 1, zz + kSlab, a.err);
    eval_point<CT, false>(lds, coeff, g, qs, X0, Y0, lane, u1);
    if (lane < 3) {
      const double h = 0.5 * a.dt;
      const double x0 = lane == 0 ? xn[0] : lane == 1 ? xn[1] : xn[2];
      const float ua = lane == 0 ? u0[0] : lane == 1 ? u0[1] : u0[2];
      const float ub = lane == 0 ? u1[0] : lane == 1 ? u1[1] : u1[2];
      a.x_out[lane * np + p] = x0 + h * ((double)ua + (double)ub);
    }
  } else {
    // adjoint of a Heun step: J(x^n) and u0 at x^n, then J(x*) at x*
    float on[12], os[12];
    eval_point<CT, true>(lds, coeff, g, qn, X0, Y0, lane, on);
    double xs[3], lam[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xs[d] = xn[d] + a.dt * (double)on[d];
      lam[d] = a.lam[d * np + p];
    }
    const Pt qs = locate_pt(g, xs, X0, Y0, zz - 1, zz + kSlab, a.err);
    eval_point<CT, true>(lds, coeff, g, qs, X0, Y0, lane, os);
    float ub1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) ub1[d] = (float)(0.5 * a.dt * lam[d]);
    double xbs[3], ub0d[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xbs[d] = (double)(ub1[0] * os[3 + d] + ub1[1] * os[6 + d] + ub1[2] * os[9 + d]);
      ub0d[d] = 0.5 * a.dt * lam[d] + a.dt * xbs[d];
    }
    float ub0[3] = {(float)ub0d[0], (float)ub0d[1], (float)ub0d[2]};
    if (lane < 3) {
      const int d = lane;
      const double xb = lam[d] + xbs[d] +
                        (double)(ub0[0] * on[3 + d] + ub0[1] * on[6 + d] + ub0[2] * on[9 + d]);
      a.xbn[d * np + p] = xb;
      a.u0[d * np + p] = d == 0 ? on[0] : d == 1 ? on[1] : on[2];
      a.ub0[d * np + p] = ub0[d];
    }
  }
}

template <typename CT, int MODE>
__global__ __launch_bounds__(kTB) void tile_gather(TileArgs a) {
  extern __shared__ float lds[];
  int col, z0, z1;
  work_item(a, &col, &z0, &z1);
  if (col < 0) return;
  const GridDev& g = a.g;
  const int cy = col / a.ncx, cx = col - cy * a.ncx;
  const int X0 = cx * kTileX, Y0 = cy * kTileY;
  const int npad = g.nz + 3;
  PlaneLoader<CT> ld{(const CT*)a.coeff, g.comp, g.plane, g.px, g.py, X0, Y0};
  const int lane = threadIdx.x & 3, grp = threadIdx.x >> 2;
  const int32_t* ls = a.lstart + (int64_t)col * g.nz;

  // prologue: planes z0-1 .. z0+5
  {
    float v[kPerThread];
    for (int P = z0 - 1; P <= z0 + 5; ++P) {
      ld.load(P, npad, v);
      store_plane(lds, P & (kRing - 1), v);
    }
  }
  float va[2][kPerThread], vb[2][kPerThread];
  ld.load(z0 + 6, npad, va[0]);
  ld.load(z0 + 7, npad, va[1]);
  ld.load(z0 + 8, npad, vb[0]);
  ld.load(z0 + 9, npad, vb[1]);

  for (int zz = z0; zz < z1; zz += 2 * kSlab) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int zs = zz + half * kSlab;
      if (zs < z1) {
        __syncthreads();
        const int64_t pb = ls[zs];
        const int64_t pe = ls[min(zs + kSlab, z1)];
        for (int64_t p = pb + grp; p < pe; p += kGroups)
          process_particle<CT, MODE>(a, lds, p, X0, Y0, zs, lane);
        __syncthreads();
        float (*v)[kPerThread] = half == 0 ? va : vb;
        store_plane(lds, (zs + 6) & (kRing - 1), v[0]);
        store_plane(lds, (zs + 7) & (kRing - 1), v[1]);
        ld.load(zs + 10, npad, v[0]);
        ld.load(zs + 11, npad, v[1]);
      }
    }
  }
}

// ------------------------------------------------------- scatter kernel ---
// Adjoint of the 64-term sums of both Heun stages, accumulated in an LDS ring
// of the column's planes and flushed to g_coeff once a plane can receive no
// further contribution.  Interior points of a column tile belong to it alone
// and are updated with a plain read-modify-write; the 3-point strips shared
// with neighbouring columns, and stencils outside the ring, use atomics.
__device__ __forceinline__ void scatter_lds(float* lds, const Pt& q, int X0, int Y0, int lane,
                                            const float gu[3]) {
  float wx[4], wy[4], wz[4];
  bspline_w(q.t[0], wx);
  bspline_w(q.t[1], wy);
  bspline_w(q.t[2], wz);
  const float wxi = lane == 0 ? wx[0] : lane == 1 ? wx[1] : lane == 2 ? wx[2] : wx[3];
  const int col = (q.a - X0) + lane;
  const int row0 = q.b - Y0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float* pl = lds + ((q.c + k) & (kRing - 1)) * kSlotP + col;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float w = wxi * wy[j] * wz[k];
#pragma unroll
      for (int comp = 0; comp < 3; ++comp)
        atomicAdd(pl + comp * kCompP + (row0 + j) * kRowP, w * gu[comp]);
    }
  }
}

__device__ __forceinline__ void scatter_global(float* gc, const GridDev& g, const Pt& q, int lane,
                                               const float gu[3]) {
  float wx[4], wy[4], wz[4];
  bspline_w(q.t[0], wx);
  bspline_w(q.t[1], wy);
  bspline_w(q.t[2], wz);
  const float wxi = lane == 0 ? wx[0] : lane == 1 ? wx[1] : lane == 2 ? wx[2] : wx[3];
  const int64_t off = ((int64_t)q.c * g.py + q.b) * g.px + q.a + lane;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) {
      const float w = wxi * wy[j] * wz[k];
      for (int comp = 0; comp < 3; ++comp)
        unsafeAtomicAdd(gc + comp * g.comp + off + k * g.plane + j * g.px, w * gu[comp]);
    }
}

__device__ __forceinline__ void zero_slot(float* lds, int slot) {
  for (int e = threadIdx.x; e < kSlotP; e += kTB) lds[slot * kSlotP + e] = 0.0f;
}

// Add LDS slot into padded plane P of g_coeff.
__device__ __forceinline__ void flush_plane(float* lds, int slot, float* gc, const GridDev& g,
                                            int P, int X0, int Y0) {
  if (P < 0 || P >= g.nz + 3) return;
  for (int e = threadIdx.x; e < kPlaneElems; e += kTB) {
    const int c = e / (kTW * kTH);
    const int r = e - c * (kTW * kTH);
    const int y = r / kTW, x = r - y * kTW;
    const int X = X0 + x, Y = Y0 + y;
    if (X >= g.px || Y >= g.py) continue;
    const float v = lds[slot * kSlotP + c * kCompP + y * kRowP + x];
    if (v == 0.0f) continue;
    float* dst = gc + c * g.comp + (int64_t)P * g.plane + (int64_t)Y * g.px + X;
    // Other columns add into the same points concurrently (the shared 3-point
    // strips, and stencils that left their own column), so every update is
    // an atomic add.
    unsafeAtomicAdd(dst, v);
  }
}

__global__ __launch_bounds__(kTB) void tile_scatter(TileArgs a) {
  extern __shared__ float lds[];
  // one block per whole column (no segments: every plane is flushed once)
  const int b = blockIdx.x;
  const int per = (a.ncol + 7) / 8;
  const int col = (b & 7) * per + (b >> 3);
  if ((b >> 3) >= per || col >= a.ncol) return;
  const GridDev& g = a.g;
  const int cy = col / a.ncx, cx = col - cy * a.ncx;
  const int X0 = cx * kTileX, Y0 = cy * kTileY;
  const int lane = threadIdx.x & 3, grp = threadIdx.x >> 2;
  const int32_t* ls = a.lstart + (int64_t)col * g.nz;
  const int64_t np = a.np;
  for (int s = 0; s < kRing; ++s) zero_slot(lds, s);
  for (int zs = 0; zs < g.nz; zs += kSlab) {
    __syncthreads();
    const int64_t pb = ls[zs];
    const int64_t pe = ls[min(zs + kSlab, g.nz)];
    for (int64_t p = pb + grp; p < pe; p += kGroups) {
      const double xn[3] = {a.x[p], a.x[np + p], a.x[2 * np + p]};
      double xs[3];
      float ub1[3], ub0[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        xs[d] = xn[d] + a.dt * (double)a.u0[d * np + p];
        ub1[d] = (float)(0.5 * a.dt * a.lam[d * np + p]);
        ub0[d] = a.ub0[d * np + p];
      }
      const Pt qn = locate_pt(g, xn, X0, Y0, zs - 1, zs + kSlab, a.err);
      const Pt qs = locate_pt(g, xs, X0, Y0, zs - 1, zs + kSlab, a.err);
      if (qn.in_ring) scatter_lds(lds, qn, X0, Y0, lane, ub0);
      else scatter_global(a.gcoeff, g, qn, lane, ub0);
      if (qs.in_ring) scatter_lds(lds, qs, X0, Y0, lane, ub1);
      else scatter_global(a.gcoeff, g, qs, lane, ub1);
    }
    __syncthreads();
    // planes zs-1 and zs are complete: later layers touch planes >= zs+1
    for (int P = zs - 1; P <= zs; ++P) {
      flush_plane(lds, P & (kRing - 1), a.gcoeff, g, P, X0, Y0);
    }
    __syncthreads();
    zero_slot(lds, (zs - 1) & (kRing - 1));
    zero_slot(lds, zs & (kRing - 1));
  }
  __syncthreads();
  // remaining planes nz-1 .. nz+2 (the last slab flushed up to nz-1 or nz-2)
  const int last_done = ((g.nz - 1) / kSlab) * kSlab;  // zs of the last slab
  for (int P = last_done + 1; P <= g.nz + 2; ++P)
    flush_plane(lds, P & (kRing - 1), a.gcoeff, g, P, X0, Y0);
}

// ------------------------------------------------------- layer table ---
template <typename K>
__global__ __launch_bounds__(256) void layer_table(const K* __restrict__ keys, int64_t np,
                                                   int64_t nlayers, int32_t* __restrict__ ls) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i > np) return;
  const int64_t lprev = i == 0 ? -1 : (int64_t)(keys[i - 1] >> kLayerShift);
  const int64_t lcur = i == np ? nlayers : (int64_t)(keys[i] >> kLayerShift);
  for (int64_t L = lprev + 1; L <= lcur && L <= nlayers; ++L) ls[L] = (int32_t)i;
}

// ------------------------------------------------------------ host side ---
static size_t tile_lds_bytes() { return (size_t)kRing * kSlotP * sizeof(float); }

int64_t tile_nlayers(const pt_grid* g) {
  const int64_t ncx = (g->nx + kTileX - 1) / kTileX, ncy = (g->ny + kTileY - 1) / kTileY;
  return ncx * ncy * g->nz;
}

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
                          double dt) {
  TileArgs a{};
  a.g = make_grid_dev(g);
  a.coeff = coeff;
  a.lstart = ls;
  a.ncx = (g->nx + kTileX - 1) / kTileX;
  a.ncol = a.ncx * ((g->ny + kTileY - 1) / kTileY);
  a.seg_len = g->nz <= 128 ? g->nz : 128;
  a.nseg = (g->nz + a.seg_len - 1) / a.seg_len;
  a.np = np;
  a.dt = dt;
  a.err = device_error_flag();
  return a;
}

template <typename F>
static bool allow_lds(F* fn) {
  return hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)tile_lds_bytes()) == hipSuccess;
}

static pt_status launch_gather(const TileArgs& a, pt_dtype dtype, int mode, hipStream_t s) {
  const int nitems = a.ncol * a.nseg;
  const unsigned blocks = (unsigned)(((nitems + 7) / 8) * 8);
  const size_t lds = tile_lds_bytes();
#define PT_TG(CT, M)                                                               \
  do {                                                                             \
    if (!allow_lds(tile_gather<CT, M>)) return PT_ERR_HIP;                          \
    hipLaunchKernelGGL((tile_gather<CT, M>), dim3(blocks), dim3(kTB), lds, s, a);  \
  } while (0)
  if (dtype == PT_F32) {
    if (mode == TILE_RK2_FWD) PT_TG(float, TILE_RK2_FWD);
    else PT_TG(float, TILE_RK2_BWD_GRAD);
  } else {
    if (mode == TILE_RK2_FWD) PT_TG(uint16_t, TILE_RK2_FWD);
    else PT_TG(uint16_t, TILE_RK2_BWD_GRAD);
  }
#undef PT_TG
  PT_LAUNCH_CHECK();
  return PT_OK;
}

pt_status tile_rk2_fwd(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                       int64_t np, double dt, const double* x, double* x_out, hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, dt);
  a.x = x;
  a.x_out = x_out;
  return launch_gather(a, dtype, TILE_RK2_FWD, s);
}

pt_status tile_rk2_bwd(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                       int64_t np, double dt, const double* x, const double* lam, double* xbn,
                       float* u0, float* ub0, float* gcoeff, hipStream_t s) {
  TileArgs a = tile_args(g, coeff, ls, np, dt);
  a.x = x;
  a.lam = lam;
  a.xbn = xbn;
  a.u0 = u0;
  a.ub0 = ub0;
  a.gcoeff = gcoeff;
  pt_status st = launch_gather(a, dtype, TILE_RK2_BWD_GRAD, s);
  if (st != PT_OK || !gcoeff) return st;
  const unsigned blocks = (unsigned)(((a.ncol + 7) / 8) * 8);
  if (!allow_lds(tile_scatter)) return PT_ERR_HIP;
  hipLaunchKernelGGL(tile_scatter, dim3(blocks), dim3(kTB), tile_lds_bytes(), s, a);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
