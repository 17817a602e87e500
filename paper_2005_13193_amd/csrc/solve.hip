// Operation 1 of Sec. 2.2: periodic cubic-spline coefficients, one periodic
// tridiagonal solve (S[m-1] + 4 S[m] + S[m+1]) / 6 = g[m] per grid line and
// axis.
//
// GPU formulation.  The paper solves each line with the Thomas algorithm.
// Here every line is cut into chunks of kChunk outputs, one chunk per thread,
// and each chunk is solved by the factorised form of the same inverse:
//   A = -(1 / (6 z1)) (1 - z1 q^-1)(1 - z1 q),   z1 = sqrt(3) - 2,
// i.e. a causal recursion c[m] = g[m] + z1 c[m-1], an anti-causal recursion
// d[m] = c[m] + z1 d[m+1], and S = -6 z1 d (q the periodic shift).  Each
// recursion is started kWarm points outside the chunk (periodic indices), so
// a chunk needs no data from other threads; the start-up error is damped by
// |z1|^kWarm = 7.2e-10 before it reaches the chunk, two orders of magnitude
// below FP32 rounding.  Lines are read and written once per axis pass with
// coalesced accesses (lanes across x for the y and z passes; rows staged in
// LDS for the x pass).
#include "pt_common.h"

namespace pt {

constexpr int kChunk = 32;  // outputs per thread
constexpr int kWarm = 16;   // warm-up points of each recursion
constexpr float kZ1 = -0.26794919243112270f;  // sqrt(3) - 2
constexpr float kGain = 1.6076951545867361f;  // -6 z1

enum OutMode { OUT_PLAIN = 0, OUT_PAD_F32 = 1, OUT_PAD_BF16 = 2 };

// Lines along axis A (length na, input stride sa); 64 lanes across x (stride
// 1); third axis B (length nb, input stride sb).  With a padded output the
// lane and B indices run over the padded extents and read the periodic
// source line (X - 1) mod n; the A index writes padded P = m + 1 plus the
// three wrapped copies.
struct StridedArgs {
  const float* in;
  void* out;
  int nx, na, nb;
  int64_t sa, sb;    // input strides
  int lx, lb;        // lane / B extents of the launch (n or n + 3)
  int64_t osa, osb;  // output strides along A and B
};

template <int MODE>
__global__ __launch_bounds__(256) void solve_strided(StridedArgs a) {
  const int X = blockIdx.x * 64 + (threadIdx.x & 63);
  const int chunk = blockIdx.z * 4 + (threadIdx.x >> 6);
  const int B = blockIdx.y;
  const int m0 = chunk * kChunk;
  if (X >= a.lx || m0 >= a.na) return;
  const int x = MODE == OUT_PLAIN ? X : (X - 1 + a.nx) % a.nx;
  const int b = MODE == OUT_PLAIN ? B : (B - 1 + a.nb) % a.nb;
  const float* line = a.in + x + (int64_t)b * a.sb;

  float cbuf[kChunk + kWarm];
  float c = 0.0f;
  int j = ((m0 - kWarm) % a.na + a.na) % a.na;
#pragma unroll
  for (int it = 0; it < kChunk + 2 * kWarm; ++it) {
    c = line[(int64_t)j * a.sa] + kZ1 * c;
    if (it >= kWarm) cbuf[it - kWarm] = c;
    j = (j + 1 == a.na) ? 0 : j + 1;
  }
  float res[kChunk];
  float d = 0.0f;
#pragma unroll
  for (int it = kChunk + kWarm - 1; it >= 0; --it) {
    d = cbuf[it] + kZ1 * d;
    if (it < kChunk) res[it] = kGain * d;
  }
  const int len = min(kChunk, a.na - m0);
  if (MODE == OUT_PLAIN) {
    float* o = (float*)a.out + x + (int64_t)b * a.sb + (int64_t)m0 * a.sa;
#pragma unroll
    for (int it = 0; it < kChunk; ++it)
      if (it < len) o[(int64_t)it * a.sa] = res[it];
  } else {
    const int64_t base = X + (int64_t)B * a.osb;
#pragma unroll
    for (int it = 0; it < kChunk; ++it) {
      if (it < len) {
        const int m = m0 + it;
        float v = res[it];
        int P[2] = {m + 1, m == a.na - 1 ? 0 : (m == 0 ? a.na + 1 : (m == 1 ? a.na + 2 : -1))};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (P[q] < 0) continue;
          int64_t idx = base + (int64_t)P[q] * a.osa;
          if (MODE == OUT_PAD_F32) ((float*)a.out)[idx] = v;
          else ((uint16_t*)a.out)[idx] = f32_to_bf16_rne(v);
        }
      }
    }
  }
}

// x pass: rows (contiguous lines of nx points) staged through LDS.  Element p
// of a row sits at LDS offset p + p/32 so that the 32 chunks of a row start
// in different banks.
constexpr int kRowLds = 8192 + 512;

__global__ __launch_bounds__(256) void solve_rows(const float* __restrict__ in,
                                                  float* __restrict__ out, int nx,
                                                  int64_t nrows, int rows_per_block,
                                                  int cpr) {
  __shared__ float lds[kRowLds];
  const int rs = nx + (nx >> 5) + 1;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int nr = (int)min((int64_t)rows_per_block, nrows - r0);
  const int tid = threadIdx.x;
  const float* src = in + r0 * nx;
  for (int r = 0; r < nr; ++r)
    for (int p = tid; p < nx; p += 256) lds[r * rs + p + (p >> 5)] = src[(int64_t)r * nx + p];
  __syncthreads();

  const int r = tid / cpr, q = tid - r * cpr;
  const int m0 = q * kChunk;
  const bool active = r < nr && m0 < nx;
  float res[kChunk];
  if (active) {
    const float* row = lds + r * rs;
    float cbuf[kChunk + kWarm];
    float c = 0.0f;
    int j = ((m0 - kWarm) % nx + nx) % nx;
#pragma unroll
    for (int it = 0; it < kChunk + 2 * kWarm; ++it) {
      c = row[j + (j >> 5)] + kZ1 * c;
      if (it >= kWarm) cbuf[it - kWarm] = c;
      j = (j + 1 == nx) ? 0 : j + 1;
    }
    float d = 0.0f;
#pragma unroll
    for (int it = kChunk + kWarm - 1; it >= 0; --it) {
      d = cbuf[it] + kZ1 * d;
      if (it < kChunk) res[it] = kGain * d;
    }
  }
  __syncthreads();
  if (active) {
    float* row = lds + r * rs;
    const int len = min(kChunk, nx - m0);
#pragma unroll
    for (int it = 0; it < kChunk; ++it) {
      const int p = m0 + it;
      if (it < len) row[p + (p >> 5)] = res[it];
    }
  }
  __syncthreads();
  float* dst = out + r0 * nx;
  for (int rr = 0; rr < nr; ++rr)
    for (int p = tid; p < nx; p += 256) dst[(int64_t)rr * nx + p] = lds[rr * rs + p + (p >> 5)];
}

// Adjoint of the padding: every grid point collects the padded entries that
// copy it (P = m + 1 along each axis, plus P = 0 for m = n-1, P = n+1 for
// m = 0 and P = n+2 for m = 1).
__global__ __launch_bounds__(256) void fold_pad(const float* __restrict__ gpad,
                                                float* __restrict__ g, int nx, int ny, int nz) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n3 = (int64_t)nx * ny * nz;
  if (i >= n3) return;
  const int x = (int)(i % nx);
  const int y = (int)((i / nx) % ny);
  const int z = (int)(i / ((int64_t)nx * ny));
  const int px = nx + 3, py = ny + 3;
  auto extra = [](int m, int n) { return m == n - 1 ? 0 : (m == 0 ? n + 1 : (m == 1 ? n + 2 : -1)); };
  const int X[2] = {x + 1, extra(x, nx)};
  const int Y[2] = {y + 1, extra(y, ny)};
  const int Z[2] = {z + 1, extra(z, nz)};
  float s = 0.0f;
  for (int c = 0; c < 2; ++c) {
    if (Z[c] < 0) continue;
    for (int b = 0; b < 2; ++b) {
      if (Y[b] < 0) continue;
      for (int a = 0; a < 2; ++a) {
        if (X[a] < 0) continue;
        s += gpad[((int64_t)Z[c] * py + Y[b]) * px + X[a]];
      }
    }
  }
  g[i] = s;
}

// ------------------------------------------------------------ launchers ---

static pt_status pass_rows(const float* in, float* out, int nx, int ny, int nz,
                           hipStream_t s) {
  const int cpr = (nx + kChunk - 1) / kChunk;
  if (cpr > 256) return PT_ERR_UNSUPPORTED;
  const int rpb = 256 / cpr;
  const int64_t nrows = (int64_t)ny * nz;
  const unsigned blocks = (unsigned)((nrows + rpb - 1) / rpb);
  TimedLaunch t("spline_x", s);
  hipLaunchKernelGGL(solve_rows, dim3(blocks), dim3(256), 0, s, in, out, nx, nrows, rpb, cpr);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

// axis 1 = y, axis 2 = z; padded output only for the last pass along y.
static pt_status pass_strided(const float* in, void* out, int nx, int ny, int nz, int axis,
                              int mode, hipStream_t s) {
  StridedArgs a;
  a.in = in;
  a.out = out;
  a.nx = nx;
  if (axis == 1) {
    a.na = ny; a.sa = nx; a.nb = nz; a.sb = (int64_t)nx * ny;
  } else {
    a.na = nz; a.sa = (int64_t)nx * ny; a.nb = ny; a.sb = nx;
  }
  if (mode == OUT_PLAIN) {
    a.lx = nx; a.lb = a.nb; a.osa = a.sa; a.osb = a.sb;
  } else {
    // padded layout [nz+3][ny+3][nx+3], lines along y, B = z
    if (axis != 1) return PT_ERR_UNSUPPORTED;
    a.lx = nx + 3; a.lb = nz + 3; a.osa = nx + 3; a.osb = (int64_t)(nx + 3) * (ny + 3);
  }
  const int nchunks = (a.na + kChunk - 1) / kChunk;
  dim3 grid((a.lx + 63) / 64, a.lb, (nchunks + 3) / 4);
  TimedLaunch t(axis == 2 ? "spline_z" : (mode == OUT_PLAIN ? "spline_y" : "spline_y_pad"), s);
  if (mode == OUT_PLAIN)
    hipLaunchKernelGGL(solve_strided<OUT_PLAIN>, grid, dim3(256), 0, s, a);
  else if (mode == OUT_PAD_F32)
    hipLaunchKernelGGL(solve_strided<OUT_PAD_F32>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(solve_strided<OUT_PAD_BF16>, grid, dim3(256), 0, s, a);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

size_t spline_ws_floats(const pt_grid* g, pt_dtype dtype) {
  const size_t n3 = (size_t)g->nx * g->ny * g->nz;
  return dtype == PT_BF16 ? 2 * n3 : n3;
}

pt_status spline_fwd(const pt_grid* g, const float* field, void* coeff, pt_dtype dtype,
                     float* ws, hipStream_t s) {
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t p3 = (int64_t)(nx + 3) * (ny + 3) * (nz + 3);
  for (int c = 0; c < 3; ++c) {
    const float* f = field + c * n3;
    // x pass into a scratch line set, z pass, then the y pass writes the
    // padded coefficients (the paper's axis order x, z, y).  For FP32 output
    // the component's own output block serves as the first scratch array.
    float* t1 = dtype == PT_F32 ? (float*)coeff + c * p3 : ws;
    float* t2 = dtype == PT_F32 ? ws : ws + n3;
    pt_status st = pass_rows(f, t1, nx, ny, nz, s);
    if (st != PT_OK) return st;
    st = pass_strided(t1, t2, nx, ny, nz, 2, OUT_PLAIN, s);
    if (st != PT_OK) return st;
    void* o = dtype == PT_F32 ? (void*)((float*)coeff + c * p3) : (void*)((uint16_t*)coeff + c * p3);
    st = pass_strided(t2, o, nx, ny, nz, 1, dtype == PT_F32 ? OUT_PAD_F32 : OUT_PAD_BF16, s);
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

pt_status spline_bwd(const pt_grid* g, const float* gcoeff, float* gfield, float* ws,
                     hipStream_t s) {
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t p3 = (int64_t)(nx + 3) * (ny + 3) * (nz + 3);
  for (int c = 0; c < 3; ++c) {
    float* o = gfield + c * n3;
    {
      TimedLaunch t("spline_fold", s);
      hipLaunchKernelGGL(fold_pad, dim3(grid_1d(n3, 256)), dim3(256), 0, s, gcoeff + c * p3, ws,
                       nx, ny, nz);
    }
    PT_LAUNCH_CHECK();
    pt_status st = pass_strided(ws, o, nx, ny, nz, 1, OUT_PLAIN, s);  // y
    if (st != PT_OK) return st;
    st = pass_strided(o, ws, nx, ny, nz, 2, OUT_PLAIN, s);  // z
    if (st != PT_OK) return st;
    st = pass_rows(ws, o, nx, ny, nz, s);  // x
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

}  // namespace pt
