// Operation 1 of Sec. 2.2: periodic cubic-spline coefficients, one periodic
// tridiagonal solve (S[m-1] + 4 S[m] + S[m+1]) / 6 = g[m] per grid line and
// axis, and its adjoint.
//
// GPU formulation.  The paper solves each line with the Thomas algorithm.
// Here the same inverse is applied in factorised form:
//   A = -(1 / (6 z1)) (1 - z1 q^-1)(1 - z1 q),   z1 = sqrt(3) - 2,
// i.e. a causal recursion c[m] = g[m] + z1 c[m-1], an anti-causal recursion
// d[m] = c[m] + z1 d[m+1], and S = -6 z1 d (q the periodic shift).
//
// A line is cut into chunks, one per thread.  Each thread runs both
// recursions over its chunk starting from zero; the true state entering a
// chunk is then an affine function of the local end values of the other
// chunks.  Chunk k maps the state entering it to the state leaving it by
// C -> z1^len_k C + e_k, so the state entering chunk k is
//   C_in(k) = (e_{k-1} + z1^len_{k-1} e_{k-2} + ...) / (1 - z1^n),
// summed once around the periodic line (the denominator closes the loop).
// Each thread then adds z1^(i+1) C_in to its local causal values (and the
// mirrored correction after the anti-causal pass).  The result is the exact
// periodic solve with no overlap between chunks: every input is read from HBM
// once and every output written once.
//
// Axis order.  The axis solves commute, so their order changes only the
// rounding.  The paper's order is x, z, y; here it is z, y, x, so that the
// pass that writes the padded layout (and, in the adjoint, the pass that
// reads it) runs along x and moves whole rows:
//  * solve_lines - lines along y or z: lanes run across x in groups of G
//    consecutive points (coalesced 4G-byte segments); the waves of a
//    workgroup hold consecutive chunks of the same lines and combine their
//    chunk maps through LDS.
//  * solve_rows  - lines along x: one wave per row, staged through LDS so
//    that global loads and stores are contiguous across lanes; lane l then
//    holds a contiguous chunk and the chunk maps are combined by a wave scan.
//    Variants write all padded copies of the row (last forward pass) or sum
//    the padded copies of the row (first adjoint pass).
//  * solve_yx    - the forward y and x passes fused, for rows of 256, 512 or
//    1024 points: a y pass that stores only its chunk carries, then one
//    workgroup per chunk of rows solves along y in registers and along x
//    through LDS and writes the padded rows (one read and one write of the
//    field instead of two of each).
//
// Slab form.  When the grid is split in z (one device's share), the z lines
// of a slab are solved with open ends over the slab plus W field planes on
// each side: the periodic inverse decays like |z1|^d, so the recursions
// started from zero W planes away reach the slab with a relative error of
// order |z1|^W, below FP32 rounding for W >= 14.  The x and y solves are
// whole lines and stay periodic.
#include <math.h>

#include <type_traits>

#include "pt_common.h"

namespace pt {

// z1 = sqrt(3) - 2 and the gain -6 z1 in the arithmetic type T of a pass
// (FP32, or FP64 for FP64 coefficient storage).
template <typename T> __device__ __forceinline__ constexpr T z1c() { return T(-0.26794919243112270); }
template <typename T> __device__ __forceinline__ constexpr T gainc() { return T(1.6076951545867361); }

// z1^k in FP64 (0 once it underflows); the FP32 passes use it rounded to FP32.
static double z1_pow_d(int k) {
  double p = 1.0;
  const double z = sqrt(3.0) - 2.0;
  for (int i = 0; i < k && p != 0.0; ++i) p *= z;
  return p;
}
static float z1_pow(int k) { return (float)z1_pow_d(k); }

// Padded index that also holds grid index m (besides m + 1), or -1.
__device__ __forceinline__ int pad_extra(int m, int n) {
  return m == n - 1 ? 0 : (m == 0 ? n + 1 : (m == 1 ? n + 2 : -1));
}

// ------------------------------------------------------- chunk phases ---
// A thread's chunk lives in v[0..Q) with len <= Q valid points.  The phases
// touch all Q registers with selects instead of branches (FULL: len == Q),
// and points past len stay zero through both recursions.

// Causal recursion from zero; returns the local end state.
template <int Q, bool FULL, typename T>
__device__ __forceinline__ T causal_local(T (&v)[Q], int len) {
  const T z1 = z1c<T>();
  T c = 0, e = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    c = v[i] + z1 * c;
    v[i] = (FULL || i < len) ? c : T(0);
    e = FULL ? c : (i == len - 1 ? c : e);
  }
  return e;
}

// Adds z1^(i+1) cin to point i (the carry entering the chunk).
template <int Q, bool FULL, typename T>
__device__ __forceinline__ void causal_carry(T (&v)[Q], int len, T cin) {
  const T z1 = z1c<T>();
  T p = z1 * cin;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    v[i] += (FULL || i < len) ? p : T(0);
    p *= z1;
  }
}

// Anti-causal recursion from zero (points past len are zero, so it starts at
// len - 1); returns the local state at the chunk start.
template <int Q, typename T>
__device__ __forceinline__ T anticausal_local(T (&v)[Q]) {
  const T z1 = z1c<T>();
  T d = 0;
#pragma unroll
  for (int i = Q - 1; i >= 0; --i) {
    d = v[i] + z1 * d;
    v[i] = d;
  }
  return d;
}

// Adds z1^(len-i) din to point i < len (the carry entering from the right).
template <int Q, bool FULL, typename T>
__device__ __forceinline__ void anticausal_carry(T (&v)[Q], int len, T din) {
  const T z1 = z1c<T>();
  T p = 0;
#pragma unroll
  for (int i = Q - 1; i >= 0; --i) {
    p = (FULL ? i == Q - 1 : i == len - 1) ? z1 * din : p * z1;
    v[i] += p;
  }
}

// ------------------------------------------------------------ x lines ---
enum RowMode { ROW_PLAIN = 0, ROW_PAD_F32 = 1, ROW_PAD_BF16 = 2, ROW_FOLD = 3, ROW_PAD_F64 = 4 };

//  PLAIN: plain rows in and out.
//  PAD_*: plain rows in; the solved row (y, z) is written to every padded
//         row that holds it (y+1 and z+1, plus the wrapped copies), with its
//         x padding.
//  FOLD:  padded rows in: output row (y, z) is the solve of the sum of the
//         padded copies of the row and, along x, of each point's copies.
struct RowArgs {
  const void* in;  // float rows (double for ROW_PAD_F64)
  void* out;
  int nx, ny, nz;
  int q;       // points per lane chunk, ceil(nx / 64)
  int nrows;   // ny * nz
  int pitch;   // LDS words (of the pass's arithmetic type) per wave
  int zpad;    // PAD_*: 1 = rows are grid planes (write z + 1 and its wrapped
               // copy); 0 = rows are already padded planes (write z only)
};

// LDS slot of row element p: one pad word per 16 keeps the chunk view
// (lane l reads l q + i) free of bank conflicts for q = 16.
__device__ __forceinline__ int lds_ix(int p) { return p + (p >> 4); }

template <typename TO, typename T>
__device__ __forceinline__ void put(void* out, int64_t i, T s) {
  if constexpr (sizeof(TO) == 8) ((double*)out)[i] = s;
  else if constexpr (sizeof(TO) == 4) ((float*)out)[i] = s;
  else ((uint16_t*)out)[i] = f32_to_bf16_rne(s);
}

template <int MODE, int Q>
__global__ __launch_bounds__(256) void solve_rows(RowArgs a) {
  // arithmetic (and input) type: FP64 for the FP64 padded output
  using T = typename std::conditional<MODE == ROW_PAD_F64, double, float>::type;
  extern __shared__ __align__(16) unsigned char lds_bytes[];
  T* lds = (T*)lds_bytes;
  const T kZ1 = z1c<T>(), kGain = gainc<T>();
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int r = blockIdx.x * (blockDim.x >> 6) + wid;
  const bool active = r < a.nrows;  // inactive waves still reach the barriers
  const int nx = a.nx, px = nx + 3;
  const int64_t py = a.ny + 3;
  const int y = active ? r % a.ny : 0, z = active ? r / a.ny : 0;
  T* L = lds + wid * a.pitch;

  // 1. contiguous loads (all issued before the first LDS write), then LDS.
  // A row has at most 64 Q + 3 points: Q + 1 loads per lane.
  constexpr int J = Q + 1;
  T w[J];
  if (active) {
    if (MODE == ROW_FOLD) {
      const float* in = (const float*)a.in;
      const int ye = pad_extra(y, a.ny), ze = pad_extra(z, a.nz);
      const float* r00 = in + ((int64_t)(z + 1) * py + (y + 1)) * px;
      const float* r01 = in + ((int64_t)(z + 1) * py + ye) * px;
      const float* r10 = in + ((int64_t)ze * py + (y + 1)) * px;
      const float* r11 = in + ((int64_t)ze * py + ye) * px;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int p = lane + 64 * j;
        w[j] = p < px ? r00[p] : 0.0f;
      }
      if (ye >= 0) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const int p = lane + 64 * j;
          if (p < px) w[j] += r01[p];
        }
      }
      if (ze >= 0) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const int p = lane + 64 * j;
          if (p < px) w[j] += r10[p] + (ye >= 0 ? r11[p] : 0.0f);
        }
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int p = lane + 64 * j;
        if (p < px) L[lds_ix(p)] = w[j];
      }
    } else {
      const T* src = (const T*)a.in + (int64_t)r * nx;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int p = lane + 64 * j;
        w[j] = p < nx ? src[p] : T(0);
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int p = lane + 64 * j;
        if (p < nx) L[lds_ix(p)] = w[j];
      }
    }
  }
  __syncthreads();

  // 2. chunk view: lane l takes points [l q, l q + len)
  const int m0 = lane * a.q;
  const int len = active ? min(max(nx - m0, 0), a.q) : 0;
  const int last = max(len - 1, 0);
  const int off = MODE == ROW_FOLD ? 1 : 0;  // padded position of point x is x + 1
  T v[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int x = min(m0 + min(i, last), nx - 1);  // in the row even when len = 0
    T t = L[lds_ix(x + off)];
    if (MODE == ROW_FOLD) {
      const int xe = pad_extra(x, nx);
      if (xe >= 0) t += L[lds_ix(xe)];
    }
    v[i] = i < len ? t : T(0);
  }
  __syncthreads();

  // 3. the periodic solve of the row
  T a_len = 1;  // z1^len
#pragma unroll
  for (int i = 0; i < Q; ++i) a_len = i < len ? a_len * kZ1 : a_len;
  const T e = causal_local<Q, false>(v, len);
  T sa = a_len, se = e;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T pa = __shfl_up(sa, d), pe = __shfl_up(se, d);
    if (lane >= d) {
      se = sa * pe + se;
      sa = sa * pa;
    }
  }
  {
    // the whole row maps C -> A C + B; periodicity fixes C = B / (1 - A)
    const T A = __shfl(sa, 63), B = __shfl(se, 63);
    const T C0 = B / (T(1) - A);
    const T pa = __shfl_up(sa, 1), pe = __shfl_up(se, 1);
    causal_carry<Q, false>(v, len, lane == 0 ? C0 : pa * C0 + pe);
  }
  const T f = anticausal_local<Q>(v);
  sa = a_len;
  T sf = f;
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    const T pa = __shfl_down(sa, s), pf = __shfl_down(sf, s);
    if (lane + s < 64) {
      sf = sa * pf + sf;
      sa = sa * pa;
    }
  }
  {
    const T A = __shfl(sa, 0), B = __shfl(sf, 0);
    const T D0 = B / (T(1) - A);
    const T pa = __shfl_down(sa, 1), pf = __shfl_down(sf, 1);
    anticausal_carry<Q, false>(v, len, lane == 63 ? D0 : pa * D0 + pf);
  }

  // 4. results back to LDS (padded positions for PAD), then contiguous stores
  const bool pad_out = MODE == ROW_PAD_F32 || MODE == ROW_PAD_BF16 || MODE == ROW_PAD_F64;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (i < len) {
      const int x = m0 + i;
      const T s = kGain * v[i];
      if (pad_out) {
        L[lds_ix(x + 1)] = s;
        const int xe = pad_extra(x, nx);
        if (xe >= 0) L[lds_ix(xe)] = s;
      } else {
        L[lds_ix(x)] = s;
      }
    }
  }
  __syncthreads();
  if (!active) return;
  const int n_out = pad_out ? px : nx;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int p = lane + 64 * j;
    w[j] = p < n_out ? L[lds_ix(p)] : T(0);
  }
  if (pad_out) {
    using TO = typename std::conditional<
        MODE == ROW_PAD_F64, double,
        typename std::conditional<MODE == ROW_PAD_F32, float, uint16_t>::type>::type;
    const int ye = pad_extra(y, a.ny), ze = a.zpad ? pad_extra(z, a.nz) : -1;
    const int Ys[2] = {y + 1, ye}, Zs[2] = {a.zpad ? z + 1 : z, ze};
    for (int zc = 0; zc < 2; ++zc) {
      if (Zs[zc] < 0) continue;
      for (int yc = 0; yc < 2; ++yc) {
        if (Ys[yc] < 0) continue;
        const int64_t row = ((int64_t)Zs[zc] * py + Ys[yc]) * px;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const int p = lane + 64 * j;
          if (p < px) put<TO>(a.out, row + p, w[j]);
        }
      }
    }
  } else {
    T* dst = (T*)a.out + (int64_t)r * nx;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int p = lane + 64 * j;
      if (p < nx) dst[p] = w[j];
    }
  }
}

// ------------------------------------------------------- y / z lines ---
// Lines along axis A (length na), stride sa; lanes across x; third axis B
// (stride sb); plain layout in and out.
struct LineArgs {
  const void* in;  // float, or double for the FP64 passes after the first
  void* out;       // float, or double for the FP64 passes
  int nx, na;
  int64_t sa, sb;
  int G;          // x points per lane group; a wave holds 64 / G chunks
  int K;          // chunks per line
  int L;          // chunk length
  double a_full;   // z1^L (in the pass's arithmetic type, widened)
  double a_last;   // z1^(length of the last, shorter chunk)
  double closure;  // 1 / (1 - z1^na); 1 for open lines
  int open;       // 1: lines with open ends (recursions start from zero at
                  // the ends), 0: periodic lines
  int bx0;        // first x-block of the launch
  float* carry;   // non-null: write only the carries entering each run of
                  // 16 points, [b][na / 16][2][nx] (causal, anti-causal),
                  // for solve_yx (whole chunks of a multiple of 16 points)
  int nbf;        // FOLD input (y lines of the padded adjoint): grid planes
};

// The fold of the adjoint: grid point (x, y, z) sums every padded copy that
// holds it, index m + 1 along each axis plus pad_extra(m) where it exists.
// fold_rows adds to v[i] the x copies (x + 1, and xe) of row i * stride of
// the padded rows at p (the caller picks the y and z copies).
template <int Q>
__device__ __forceinline__ void fold_rows(float* v, const float* p, int64_t stride, int x,
                                          int xe) {
#pragma unroll
  for (int i = 0; i < Q; ++i) v[i] += p[i * stride + x + 1];
  if (xe >= 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] += p[i * stride + xe];
  }
}

// Folded values of Q consecutive grid rows y0 .. y0 + Q - 1 (Q >= 3) at
// column x of grid plane z into v, from the padded gradient in (px, py: the
// padded row length and rows per plane; ny, nz: grid extents): the rows' own
// padded copies, then the wrapped copies of grid rows 0, 1 and ny - 1 (only
// i = 0, 1 and Q - 1 can hold them) and of planes 0, 1 and nz - 1.
template <int Q>
__device__ __forceinline__ void fold_column(float* v, const float* in, int px, int64_t py,
                                            int nx, int ny, int nz, int x, int y0, int z) {
  static_assert(Q >= 3, "rows 0 and 1 and the last must be distinct slots");
  const int xe = pad_extra(x, nx), ze = pad_extra(z, nz);
  const int64_t pl = py * px;
#pragma unroll
  for (int i = 0; i < Q; ++i) v[i] = 0.0f;
  fold_rows<Q>(v, in + (z + 1) * pl + (int64_t)(y0 + 1) * px, px, x, xe);
  if (ze >= 0) fold_rows<Q>(v, in + ze * pl + (int64_t)(y0 + 1) * px, px, x, xe);
  constexpr int kI[3] = {0, 1, Q - 1};
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int ye = pad_extra(y0 + kI[t], ny);
    if (ye < 0) continue;
    float c = 0.0f;
    fold_rows<1>(&c, in + (z + 1) * pl + (int64_t)ye * px, 0, x, xe);
    if (ze >= 0) fold_rows<1>(&c, in + ze * pl + (int64_t)ye * px, 0, x, xe);
    v[kI[t]] += c;
  }
}

template <typename T>
__device__ __forceinline__ T chunk_gain(const LineArgs& a, int k) {
  const int lk = min(max(a.na - k * a.L, 0), a.L);
  return lk == a.L ? (T)a.a_full : (lk == 0 ? T(1) : (T)a.a_last);
}

// FULL: every thread of the launch holds a whole chunk of Q = L points
// (launched only on x-blocks inside nx, with K * L = na).
// CARRY: write only the run carries to a.carry (FULL launches only).
// FOLD: y lines (axis A = y, B = z) of the folded padded gradient (FULL and
// CARRY only): the carries of the adjoint's fused y + x pass.
// TI: input type; T: arithmetic and output type (float, float or float,
// double or double, double).
template <int Q, bool FULL, bool CARRY = false, typename TI = float, typename T = float,
          bool FOLD = false>
__global__ __launch_bounds__(1024) void solve_lines(LineArgs a) {
  static_assert(!FOLD || (FULL && CARRY && std::is_same<T, float>::value),
                "the folded input feeds the carries-only FP32 pass");
  __shared__ T s_e[1024];
  __shared__ T s_f[1024];
  const T kGain = gainc<T>();
  const int lane = threadIdx.x & 63;
  const int xg = lane & (a.G - 1);
  const int k = (threadIdx.x >> 6) * (64 / a.G) + lane / a.G;
  int bx = blockIdx.x, b = blockIdx.y;
  if constexpr (FOLD) {
    // Padded rows start off 128-byte lines, so two neighbouring x-blocks share
    // a line at their border.  Workgroups go to the 8 XCDs round-robin by
    // linear index: renumbered, each XCD takes whole planes (all x-blocks of
    // a plane at once) and fetches a shared line into its L2 once.
    const int nbx = gridDim.x, total = nbx * gridDim.y;
    if (total % 8 == 0) {
      const int id = blockIdx.y * nbx + blockIdx.x;
      const int l = (id % 8) * (total / 8) + id / 8;
      bx = l % nbx;
      b = l / nbx;
    }
  }
  const int x = (bx + a.bx0) * a.G + xg;
  const int m0 = k * a.L;
  const int len = FULL ? Q : (x < a.nx ? min(max(a.na - m0, 0), a.L) : 0);
  const int last = max(len - 1, 0);

  T v[Q];
  if constexpr (FOLD) {
    fold_column<Q>(v, (const float*)a.in, a.nx + 3, a.na + 3, a.nx, a.na, a.nbf, x, m0, b);
  } else {
    // clamped addresses keep every load in bounds; selects zero the rest
    const TI* in = (const TI*)a.in;
    const TI* src = len > 0 ? in + x + (int64_t)b * a.sb + (int64_t)m0 * a.sa : in;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T t = (T)*src;
      v[i] = (FULL || i < len) ? t : T(0);
      src += (FULL || i < last) ? a.sa : 0;
    }
  }

  s_e[k * a.G + xg] = causal_local<Q, FULL>(v, len);
  __syncthreads();
  const T closure = (T)a.closure;
  T s_c;  // the causal carry entering this chunk
  {
    T cin = 0, P = 1;
    const int jn = a.open ? k : a.K;  // chunks before this one (open: no wrap)
    for (int j = 1; j <= jn && P != T(0); ++j) {
      int kk = k - j;
      if (kk < 0) kk += a.K;
      cin += P * s_e[kk * a.G + xg];
      P *= chunk_gain<T>(a, kk);
    }
    causal_carry<Q, FULL>(v, len, cin * closure);
    s_c = cin * closure;
  }
  T cv[Q / 16 > 1 ? Q / 16 - 1 : 1];  // causal values ending runs of 16
  if constexpr (CARRY) {
#pragma unroll
    for (int r = 0; r + 1 < Q / 16; ++r) cv[r] = v[16 * r + 15];
  }
  s_f[k * a.G + xg] = anticausal_local<Q>(v);
  __syncthreads();
  {
    T din = 0, R = 1;
    const int jn = a.open ? a.K - 1 - k : a.K;
    for (int j = 1; j <= jn && R != T(0); ++j) {
      int kk = k + j;
      if (kk >= a.K) kk -= a.K;
      din += R * s_f[kk * a.G + xg];
      R *= chunk_gain<T>(a, kk);
    }
    if constexpr (CARRY) {
      // the state entering each run of 16 points from the left (the causal
      // value before it) and from the right (the anti-causal value after it)
      constexpr int R = Q / 16;
      T cl[R];
      cl[0] = s_c;
#pragma unroll
      for (int r = 1; r < R; ++r) cl[r] = cv[r - 1];
      anticausal_carry<Q, FULL>(v, len, din * closure);
      if (len > 0) {
        T* cr = (T*)a.carry + ((int64_t)b * a.na + m0) / 16 * 2 * a.nx + x;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          cr[2 * r * a.nx] = cl[r];
          cr[(2 * r + 1) * a.nx] = r + 1 < R ? v[16 * (r + 1)] : din * closure;
        }
      }
      return;
    }
    anticausal_carry<Q, FULL>(v, len, din * closure);
  }

  T* o = (T*)a.out + x + (int64_t)b * a.sb + (int64_t)m0 * a.sa;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (FULL || i < len) *o = kGain * v[i];
    o += a.sa;
  }
}

// ------------------------------------------------ fused y + x lines ---
// The y pass and the padded x pass of the forward solve in one read and one
// write of the field.  A carries-only y pass (solve_lines with a.carry) has
// stored the states entering every run of QY rows from either side; a
// workgroup of nx = 64 W threads then takes one run of one plane: thread x
// solves its column of the run along y in registers (the recursions of the
// y pass, started from the stored states), and the rows go through LDS W at
// a time, one wave per row, for the periodic x solve of solve_rows and the
// padded stores.  The arithmetic is that of the two separate passes, with
// the y recursions restarted at every
// run of QY rows from the carries stored there.
struct YXArgs {
  const float* in;     // plain [planes][ny][nx] (z-solved field)
  const float* carry;  // [planes][K][2][nx] from the carries-only y pass
  void* out;           // padded coefficients
  int nx, ny, nz;      // nz: grid planes (for the wrapped z copies with zpad)
  int K;               // chunks per y line (QY rows each)
  int pitch;           // LDS floats per row slot
  int zpad;            // as RowArgs::zpad
};

template <int W, int QY, typename T>
__global__ __launch_bounds__(1024) void solve_yx(YXArgs a) {
  const float kZ1 = z1c<float>(), kGain = gainc<float>();
  extern __shared__ float lds[];
  constexpr int QX = W;  // x points per lane: nx = 64 W
  constexpr int J = QX + 1;
  const int x = threadIdx.x, lane = x & 63, wid = x >> 6;
  const int k = blockIdx.x, z = blockIdx.y;
  const int nx = a.nx, px = nx + 3;
  const int64_t py = a.ny + 3;

  float v[QY];
  {
    const float* src = a.in + ((int64_t)z * a.ny + (int64_t)k * QY) * nx + x;
#pragma unroll
    for (int i = 0; i < QY; ++i) v[i] = src[(int64_t)i * nx];
    const float* cr = a.carry + ((int64_t)z * a.K + k) * 2 * nx + x;
    const float cin = cr[0], din = cr[nx];
    causal_local<QY, true>(v, QY);
    causal_carry<QY, true>(v, QY, cin);
    anticausal_local<QY>(v);
    anticausal_carry<QY, true>(v, QY, din);
  }

  float* L = lds + wid * a.pitch;
  const int m0 = lane * QX;
#pragma unroll
  for (int bt = 0; bt < QY / W; ++bt) {
#pragma unroll
    for (int r = 0; r < W; ++r) lds[r * a.pitch + lds_ix(x)] = kGain * v[bt * W + r];
    __syncthreads();
    const int y = k * QY + bt * W + wid;

    // the periodic x solve of row (y, z), as in solve_rows
    float u[QX];
#pragma unroll
    for (int i = 0; i < QX; ++i) u[i] = L[lds_ix(m0 + i)];
    float a_len = 1.0f;
#pragma unroll
    for (int i = 0; i < QX; ++i) a_len *= kZ1;
    const float e = causal_local<QX, false>(u, QX);
    float sa = a_len, se = e;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float pa = __shfl_up(sa, d), pe = __shfl_up(se, d);
      if (lane >= d) {
        se = sa * pe + se;
        sa = sa * pa;
      }
    }
    {
      const float A = __shfl(sa, 63), B = __shfl(se, 63);
      const float C0 = B / (1.0f - A);
      const float pa = __shfl_up(sa, 1), pe = __shfl_up(se, 1);
      causal_carry<QX, false>(u, QX, lane == 0 ? C0 : pa * C0 + pe);
    }
    const float f = anticausal_local<QX>(u);
    sa = a_len;
    float sf = f;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float pa = __shfl_down(sa, d), pf = __shfl_down(sf, d);
      if (lane + d < 64) {
        sf = sa * pf + sf;
        sa = sa * pa;
      }
    }
    {
      const float A = __shfl(sa, 0), B = __shfl(sf, 0);
      const float D0 = B / (1.0f - A);
      const float pa = __shfl_down(sa, 1), pf = __shfl_down(sf, 1);
      anticausal_carry<QX, false>(u, QX, lane == 63 ? D0 : pa * D0 + pf);
    }
    __syncthreads();  // every lane's reads of the row before the padded writes
#pragma unroll
    for (int i = 0; i < QX; ++i) {
      const int xx = m0 + i;
      const float sv = kGain * u[i];
      L[lds_ix(xx + 1)] = sv;
      const int xe = pad_extra(xx, nx);
      if (xe >= 0) L[lds_ix(xe)] = sv;
    }
    __syncthreads();
    float w[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int p = lane + 64 * j;
      w[j] = p < px ? L[lds_ix(p)] : 0.0f;
    }
    const int ye = pad_extra(y, a.ny), ze = a.zpad ? pad_extra(z, a.nz) : -1;
    const int Ys[2] = {y + 1, ye}, Zs[2] = {a.zpad ? z + 1 : z, ze};
    for (int zc = 0; zc < 2; ++zc) {
      if (Zs[zc] < 0) continue;
      for (int yc = 0; yc < 2; ++yc) {
        if (Ys[yc] < 0) continue;
        const int64_t row = ((int64_t)Zs[zc] * py + Ys[yc]) * px;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const int p = lane + 64 * j;
          if (p < px) put<T>(a.out, row + p, w[j]);
        }
      }
    }
    __syncthreads();  // the slots are refilled by the next batch
  }
}

// ------------------------------------------ fused fold + y + x (adjoint) ---
// The first passes of the adjoint in one read of the padded gradient and one
// write of the plain field: the fold, the y solve and the x solve (the solves
// commute, so y may go first).  A carries-only pass over the folded y lines
// (solve_lines with FOLD) has stored the states entering every run of QY
// rows; a workgroup of nx = 64 W threads takes one run of one plane: thread x
// folds its column of the run and solves it along y in registers from the
// stored states, and the rows go through LDS W at a time, one wave per row,
// for the periodic x solve and contiguous plain stores.
struct FYXArgs {
  const float* in;     // padded gradient [nz+3][ny+3][nx+3]
  const float* carry;  // [nz][K][2][nx] from the folded carries-only y pass
  float* out;          // plain [nz][ny][nx]
  int nx, ny, nz;
  int K;               // runs per y line (QY rows each)
  int pitch;           // LDS floats per row slot
};

template <int W, int QY>
__global__ __launch_bounds__(1024) void solve_fyx(FYXArgs a) {
  const float kZ1 = z1c<float>(), kGain = gainc<float>();
  extern __shared__ float lds[];
  constexpr int QX = W;  // x points per lane: nx = 64 W
  const int x = threadIdx.x, lane = x & 63, wid = x >> 6;
  const int k = blockIdx.x, z = blockIdx.y;
  const int nx = a.nx;

  float v[QY];
  {
    fold_column<QY>(v, a.in, nx + 3, a.ny + 3, nx, a.ny, a.nz, x, k * QY, z);
    const float* cr = a.carry + ((int64_t)z * a.K + k) * 2 * nx + x;
    const float cin = cr[0], din = cr[nx];
    causal_local<QY, true>(v, QY);
    causal_carry<QY, true>(v, QY, cin);
    anticausal_local<QY>(v);
    anticausal_carry<QY, true>(v, QY, din);
  }

  float* L = lds + wid * a.pitch;
  const int m0 = lane * QX;
#pragma unroll
  for (int bt = 0; bt < QY / W; ++bt) {
#pragma unroll
    for (int r = 0; r < W; ++r) lds[r * a.pitch + lds_ix(x)] = kGain * v[bt * W + r];
    __syncthreads();
    const int y = k * QY + bt * W + wid;

    // the periodic x solve of row (y, z), as in solve_rows
    float u[QX];
#pragma unroll
    for (int i = 0; i < QX; ++i) u[i] = L[lds_ix(m0 + i)];
    float a_len = 1.0f;
#pragma unroll
    for (int i = 0; i < QX; ++i) a_len *= kZ1;
    const float e = causal_local<QX, false>(u, QX);
    float sa = a_len, se = e;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float pa = __shfl_up(sa, d), pe = __shfl_up(se, d);
      if (lane >= d) {
        se = sa * pe + se;
        sa = sa * pa;
      }
    }
    {
      const float A = __shfl(sa, 63), B = __shfl(se, 63);
      const float C0 = B / (1.0f - A);
      const float pa = __shfl_up(sa, 1), pe = __shfl_up(se, 1);
      causal_carry<QX, false>(u, QX, lane == 0 ? C0 : pa * C0 + pe);
    }
    const float f = anticausal_local<QX>(u);
    sa = a_len;
    float sf = f;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float pa = __shfl_down(sa, d), pf = __shfl_down(sf, d);
      if (lane + d < 64) {
        sf = sa * pf + sf;
        sa = sa * pa;
      }
    }
    {
      const float A = __shfl(sa, 0), B = __shfl(sf, 0);
      const float D0 = B / (1.0f - A);
      const float pa = __shfl_down(sa, 1), pf = __shfl_down(sf, 1);
      anticausal_carry<QX, false>(u, QX, lane == 63 ? D0 : pa * D0 + pf);
    }
    // each lane writes back only its own chunk: no barrier before the writes
#pragma unroll
    for (int i = 0; i < QX; ++i) L[lds_ix(m0 + i)] = kGain * u[i];
    __syncthreads();
    float* row = a.out + ((int64_t)z * a.ny + y) * nx;
#pragma unroll
    for (int j = 0; j < QX; ++j) row[lane + 64 * j] = L[lds_ix(lane + 64 * j)];
    __syncthreads();  // the slots are refilled by the next batch
  }
}

// ------------------------------------------------------------ launchers ---

template <typename F>
static bool allow_lds(F* fn, size_t bytes) {
  return hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes) == hipSuccess;
}

static pt_status pass_rows(const void* in, void* out, int nx, int ny, int nz, int mode,
                           hipStream_t s, int zpad = 1) {
  RowArgs a;
  a.in = in;
  a.out = out;
  a.nx = nx; a.ny = ny; a.nz = nz;
  a.zpad = zpad;
  a.q = (nx + 63) / 64;
  a.nrows = ny * nz;
  const int px = nx + 3;
  a.pitch = px + (px >> 4) + 1;
  const size_t wb = mode == ROW_PAD_F64 ? 8 : 4;  // bytes per LDS word
  const int waves = 4 * (size_t)a.pitch * wb <= 64 * 1024 ? 4 : 1;
  const size_t lds = (size_t)waves * a.pitch * wb;
  const unsigned blocks = (unsigned)((a.nrows + waves - 1) / waves);
  const char* name = mode == ROW_FOLD ? "spline_x_fold"
                     : mode == ROW_PLAIN ? "spline_x" : "spline_x_pad";
  TimedLaunch t(name, s);
#define PT_ROWS(M, QQ)                                                                  \
  do {                                                                                  \
    if (lds > 65536 && !allow_lds(solve_rows<M, QQ>, lds)) return PT_ERR_HIP;           \
    hipLaunchKernelGGL((solve_rows<M, QQ>), dim3(blocks), dim3(64 * waves), lds, s, a); \
  } while (0)
#define PT_ROWS_Q(M)                    \
  do {                                  \
    if (a.q <= 4) PT_ROWS(M, 4);        \
    else if (a.q <= 8) PT_ROWS(M, 8);   \
    else if (a.q <= 16) PT_ROWS(M, 16); \
    else if (a.q <= 32) PT_ROWS(M, 32); \
    else if (a.q <= 64) PT_ROWS(M, 64); \
    else PT_ROWS(M, 128);               \
  } while (0)
  if (a.q > 128) return PT_ERR_UNSUPPORTED;
  switch (mode) {
    case ROW_PLAIN: PT_ROWS_Q(ROW_PLAIN); break;
    case ROW_PAD_F32: PT_ROWS_Q(ROW_PAD_F32); break;
    case ROW_PAD_BF16: PT_ROWS_Q(ROW_PAD_BF16); break;
    case ROW_PAD_F64: PT_ROWS_Q(ROW_PAD_F64); break;
    default: PT_ROWS_Q(ROW_FOLD); break;
  }
#undef PT_ROWS_Q
#undef PT_ROWS
  PT_LAUNCH_CHECK();
  return PT_OK;
}

// Chunking of a line of length na into at most 16 waves: (Q points per
// chunk at most, G x-points per lane group).  Wide lane groups come first:
// measured at 1024^3, 256-byte row segments (G = 64) beat 128-byte ones by
// 10-20 %, and 64-byte ones are 1.6x slower.  Long lines (the large grids)
// take Q = 64 to keep G = 64.
static bool line_shape(int na, int* Q, int* G, int* waves) {
  static const int kCand[8][2] = {{64, 64}, {32, 64}, {32, 32}, {64, 64}, {64, 32},
                                  {32, 16}, {64, 16}, {64, 8}};
  for (int i = na >= 1024 ? 0 : 1; i < 8; ++i) {
    const int q = kCand[i][0], g = kCand[i][1];
    const int per_wave = 64 / g;
    const int w = (na + per_wave * q - 1) / (per_wave * q);
    if (w <= 16) {
      *Q = q;
      *G = g;
      *waves = w;
      return true;
    }
  }
  return false;
}

// Precisions of a line pass: FP32 in and out, FP32 in and FP64 out (the
// first pass of an FP64 solve), FP64 in and out.
enum { LINES_F32 = 0, LINES_F32_F64 = 1, LINES_F64 = 2 };

// axis 1 = y, axis 2 = z; plain layout in and out.  fold (with carry, axis
// 1): the input is the padded adjoint, read folded.
static pt_status pass_lines(const void* in, void* out, int nx, int ny, int nz, int axis,
                            hipStream_t s, int open = 0, float* carry = nullptr,
                            int prec = LINES_F32, bool fold = false) {
  LineArgs a;
  a.in = in;
  a.out = out;
  a.nx = nx;
  a.open = open;
  a.carry = carry;
  a.nbf = nz;
  if (fold && (!carry || axis != 1 || open)) return PT_ERR_UNSUPPORTED;
  int nb;
  if (axis == 1) {
    a.na = ny; nb = nz;
    a.sa = nx; a.sb = (int64_t)nx * ny;
  } else {
    a.na = nz; nb = ny;
    a.sa = (int64_t)nx * ny; a.sb = nx;
  }
  int Q = 0, G = 0, waves = 0;
  if (!line_shape(a.na, &Q, &G, &waves)) return PT_ERR_UNSUPPORTED;
  a.G = G;
  a.K = waves * (64 / G);
  a.L = (a.na + a.K - 1) / a.K;
  if (prec == LINES_F32) {
    a.a_full = z1_pow(a.L);
    a.a_last = z1_pow(a.na - (a.na / a.L) * a.L);
    a.closure = open ? 1.0f : (float)(1.0 / (1.0 - (double)z1_pow(a.na)));
  } else {
    a.a_full = z1_pow_d(a.L);
    a.a_last = z1_pow_d(a.na - (a.na / a.L) * a.L);
    a.closure = open ? 1.0 : 1.0 / (1.0 - z1_pow_d(a.na));
  }
  // Whole chunks everywhere except possibly a last, partial x-block: the
  // FULL kernel takes the whole x-blocks, the general one the rest.
  const int xblocks = (nx + G - 1) / G;
  const int full_x = (a.L == Q && a.K * a.L == a.na) ? nx / G : 0;
  const dim3 block(64 * waves);
  TimedLaunch t(fold ? "spline_fold_y_carry"
                     : (carry ? "spline_y_carry" : (axis == 2 ? "spline_z" : "spline_y")),
                s);
  if (prec != LINES_F32) {
    if (carry) return PT_ERR_UNSUPPORTED;
#define PT_LINES64(QQ, FF, TI)                                                              \
  hipLaunchKernelGGL((solve_lines<QQ, FF, false, TI, double>), grid2, block, 0, s, a)
#define PT_LINES64_Q(FF, TI)                   \
  do {                                         \
    if (Q == 32) PT_LINES64(32, FF, TI);       \
    else PT_LINES64(64, FF, TI);               \
  } while (0)
    if (full_x > 0) {
      a.bx0 = 0;
      const dim3 grid2(full_x, nb);
      if (prec == LINES_F32_F64) PT_LINES64_Q(true, float);
      else PT_LINES64_Q(true, double);
    }
    if (full_x < xblocks) {
      a.bx0 = full_x;
      const dim3 grid2(xblocks - full_x, nb);
      if (prec == LINES_F32_F64) PT_LINES64_Q(false, float);
      else PT_LINES64_Q(false, double);
    }
#undef PT_LINES64_Q
#undef PT_LINES64
    PT_LAUNCH_CHECK();
    return PT_OK;
  }
  if (carry) {
    if (full_x != xblocks) return PT_ERR_UNSUPPORTED;
    a.bx0 = 0;
    if (fold) {
      if (Q == 32)
        hipLaunchKernelGGL((solve_lines<32, true, true, float, float, true>), dim3(full_x, nb),
                           block, 0, s, a);
      else
        hipLaunchKernelGGL((solve_lines<64, true, true, float, float, true>), dim3(full_x, nb),
                           block, 0, s, a);
      PT_LAUNCH_CHECK();
      return PT_OK;
    }
    if (Q == 32)
      hipLaunchKernelGGL((solve_lines<32, true, true>), dim3(full_x, nb), block, 0, s, a);
    else
      hipLaunchKernelGGL((solve_lines<64, true, true>), dim3(full_x, nb), block, 0, s, a);
    PT_LAUNCH_CHECK();
    return PT_OK;
  }
  if (full_x > 0) {
    a.bx0 = 0;
    if (Q == 32) hipLaunchKernelGGL((solve_lines<32, true>), dim3(full_x, nb), block, 0, s, a);
    else hipLaunchKernelGGL((solve_lines<64, true>), dim3(full_x, nb), block, 0, s, a);
  }
  if (full_x < xblocks) {
    a.bx0 = full_x;
    const dim3 g2(xblocks - full_x, nb);
    if (Q == 32) hipLaunchKernelGGL((solve_lines<32, false>), g2, block, 0, s, a);
    else hipLaunchKernelGGL((solve_lines<64, false>), g2, block, 0, s, a);
  }
  PT_LAUNCH_CHECK();
  return PT_OK;
}

static float* align256f(float* p) {
  return (float*)(((uintptr_t)p + 255) & ~(uintptr_t)255);
}

// The fused y + x pass applies to rows of 256, 512 or 1024 points (one
// thread per point) and y lines that line_shape cuts into whole chunks of 32
// or 64 points; solve_yx takes runs of 16 rows (few enough registers for two
// workgroups per compute unit).  *K, *QY: runs per line and rows per run.
static bool yx_shape(int nx, int ny, int* K, int* QY) {
  if (nx != 256 && nx != 512 && nx != 1024) return false;
  int Q = 0, G = 0, waves = 0;
  if (!line_shape(ny, &Q, &G, &waves)) return false;
  const int k = waves * (64 / G), L = (ny + k - 1) / k;
  if (L != Q || k * L != ny || Q % 16 != 0) return false;
  *K = ny / 16;
  *QY = 16;
  return true;
}

// Carry floats of the fused pass over `planes` planes (0 if it does not apply).
static size_t yx_carry_floats(const pt_grid* g, int planes) {
  int K = 0, QY = 0;
  if (!yx_shape(g->nx, g->ny, &K, &QY)) return 0;
  return 2 * (size_t)K * g->nx * planes;
}


// y then x of `planes` planes of in (plain, z-solved) into the padded out:
// the carries-only y pass into carry, then solve_yx.
static pt_status pass_yx(const float* in, float* carry, void* out, bool bf16, int nx, int ny,
                         int planes, int nz, int zpad, hipStream_t s) {
  int K = 0, QY = 0;
  if (!yx_shape(nx, ny, &K, &QY)) return PT_ERR_UNSUPPORTED;
  pt_status st = pass_lines(in, nullptr, nx, ny, planes, 1, s, 0, carry);
  if (st != PT_OK) return st;
  YXArgs a;
  a.in = in;
  a.carry = carry;
  a.out = out;
  a.nx = nx; a.ny = ny; a.nz = nz;
  a.K = K;
  a.zpad = zpad;
  const int px = nx + 3;
  a.pitch = px + (px >> 4) + 1;
  const int W = nx / 64;
  const size_t lds = (size_t)W * a.pitch * 4;
  const dim3 grid(K, planes);
  TimedLaunch t("spline_yx_pad", s);
#define PT_YX(WW, QQ, TT)                                                             \
  do {                                                                                \
    if (!allow_lds(solve_yx<WW, QQ, TT>, lds)) return PT_ERR_HIP;                     \
    hipLaunchKernelGGL((solve_yx<WW, QQ, TT>), grid, dim3(nx), lds, s, a);            \
  } while (0)
#define PT_YX_W(QQ, TT)                  \
  do {                                   \
    if (W == 4) PT_YX(4, QQ, TT);        \
    else if (W == 8) PT_YX(8, QQ, TT);   \
    else PT_YX(16, QQ, TT);              \
  } while (0)
  if (QY != 16) return PT_ERR_UNSUPPORTED;
  if (bf16) PT_YX_W(16, uint16_t);
  else PT_YX_W(16, float);
#undef PT_YX_W
#undef PT_YX
  PT_LAUNCH_CHECK();
  return PT_OK;
}

// fold + y + x of the padded adjoint gin into the plain out: the folded
// carries-only y pass into carry (n3 / 8 floats), then solve_fyx.
static pt_status pass_fyx(const float* gin, float* carry, float* out, int nx, int ny, int nz,
                          hipStream_t s) {
  int K = 0, QY = 0;
  if (!yx_shape(nx, ny, &K, &QY) || QY != 16) return PT_ERR_UNSUPPORTED;
  pt_status st = pass_lines(gin, nullptr, nx, ny, nz, 1, s, 0, carry, LINES_F32, true);
  if (st != PT_OK) return st;
  FYXArgs a;
  a.in = gin;
  a.carry = carry;
  a.out = out;
  a.nx = nx; a.ny = ny; a.nz = nz;
  a.K = K;
  const int px = nx + 3;
  a.pitch = px + (px >> 4) + 1;
  const int W = nx / 64;
  const size_t lds = (size_t)W * a.pitch * 4;
  const dim3 grid(K, nz);
  TimedLaunch t("spline_fyx", s);
#define PT_FYX(WW)                                                              \
  do {                                                                          \
    if (!allow_lds(solve_fyx<WW, 16>, lds)) return PT_ERR_HIP;                  \
    hipLaunchKernelGGL((solve_fyx<WW, 16>), grid, dim3(nx), lds, s, a);         \
  } while (0)
  if (W == 4) PT_FYX(4);
  else if (W == 8) PT_FYX(8);
  else PT_FYX(16);
#undef PT_FYX
  PT_LAUNCH_CHECK();
  return PT_OK;
}

size_t spline_ws_floats(const pt_grid* g, pt_dtype dtype) {
  const size_t n3 = (size_t)g->nx * g->ny * g->nz;
  if (dtype == PT_F64) return 2 * n3;  // the z- and y-solved component, FP64
  const size_t cf = yx_carry_floats(g, g->nz);
  if (cf) return n3 + 64 + cf;  // z-solved field, then the y carries
  return dtype == PT_BF16 ? 2 * n3 : n3;
}

pt_status spline_fwd(const pt_grid* g, const float* field, void* coeff, pt_dtype dtype,
                     float* ws, hipStream_t s) {
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t p3 = (int64_t)(nx + 3) * (ny + 3) * (nz + 3);
  if (dtype == PT_F64) {
    // FP64 arithmetic throughout: z pass (FP32 field in), y pass in place
    // (a line pass reads all of its lines before it writes any, and
    // workgroups own disjoint lines), x pass into the padded FP64 output
    double* t = (double*)ws;
    for (int c = 0; c < 3; ++c) {
      pt_status st = pass_lines(field + c * n3, t, nx, ny, nz, 2, s, 0, nullptr, LINES_F32_F64);
      if (st != PT_OK) return st;
      st = pass_lines(t, t, nx, ny, nz, 1, s, 0, nullptr, LINES_F64);
      if (st != PT_OK) return st;
      st = pass_rows(t, (double*)coeff + c * p3, nx, ny, nz, ROW_PAD_F64, s);
      if (st != PT_OK) return st;
    }
    return PT_OK;
  }
  const bool fused = yx_carry_floats(g, nz) > 0;
  for (int c = 0; c < 3; ++c) {
    const float* f = field + c * n3;
    void* o = dtype == PT_F32 ? (void*)((float*)coeff + c * p3)
                              : (void*)((uint16_t*)coeff + c * p3);
    if (fused) {
      // z pass into the workspace, then y and x in one pass into the output
      pt_status st = pass_lines(f, ws, nx, ny, nz, 2, s);
      if (st != PT_OK) return st;
      st = pass_yx(ws, align256f(ws + n3), o, dtype == PT_BF16, nx, ny, nz, nz, 1, s);
      if (st != PT_OK) return st;
      continue;
    }
    // z pass into a scratch array, y pass, then the x pass writes the padded
    // coefficients.  For FP32 output the component's own output block (read
    // by the y pass before the x pass overwrites it) is the first scratch,
    // started at a 256-byte boundary inside the block (p3 >= n3 + 279):
    // misaligned rows cost the z and y passes up to 2x.
    float* t1 = dtype == PT_F32 ? align256f((float*)coeff + c * p3) : ws;
    float* t2 = dtype == PT_F32 ? ws : ws + n3;
    pt_status st = pass_lines(f, t1, nx, ny, nz, 2, s);
    if (st != PT_OK) return st;
    st = pass_lines(t1, t2, nx, ny, nz, 1, s);
    if (st != PT_OK) return st;
    st = pass_rows(t2, o, nx, ny, nz, dtype == PT_F32 ? ROW_PAD_F32 : ROW_PAD_BF16, s);
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

size_t spline_slab_ws_floats(const pt_grid* g, int nzl, int W, pt_dtype dtype) {
  const size_t planes = (size_t)(nzl + 3 + 2 * W);
  if (dtype == PT_F64) return 2 * (size_t)g->nx * g->ny * planes;
  const size_t cf = yx_carry_floats(g, (int)planes);
  return (size_t)g->nx * g->ny * planes + (cf ? 64 + cf : 0);
}

// field: planes z0-1-W .. z0+nzl+1+W of the periodic field (nzl + 3 + 2W),
// coeff: [3][nzl+3][ny+3][nx+3], padded plane P = global plane z0-1+P.
pt_status spline_slab_fwd(const pt_grid* g, int nzl, int W, const float* field, void* coeff,
                          pt_dtype dtype, float* ws, hipStream_t s) {
  const int nx = g->nx, ny = g->ny;
  const int nzo = nzl + 3, nzi = nzo + 2 * W;
  const int64_t plane = (int64_t)nx * ny;
  const int64_t pb = (int64_t)(nx + 3) * (ny + 3) * nzo;  // output block per component
  if (dtype == PT_F64) {
    double* t = (double*)ws;
    for (int c = 0; c < 3; ++c) {
      pt_status st = pass_lines(field + c * plane * nzi, t, nx, ny, nzi, 2, s, 1, nullptr,
                                LINES_F32_F64);
      if (st != PT_OK) return st;
      double* mid = t + plane * W;
      st = pass_lines(mid, mid, nx, ny, nzo, 1, s, 0, nullptr, LINES_F64);
      if (st != PT_OK) return st;
      st = pass_rows(mid, (double*)coeff + c * pb, nx, ny, nzo, ROW_PAD_F64, s, 0);
      if (st != PT_OK) return st;
    }
    return PT_OK;
  }
  for (int c = 0; c < 3; ++c) {
    // z with open ends over all nzi planes into the workspace, then y and x
    // of the nzo central planes: fused where solve_yx applies, else y in
    // place (a line pass reads all of its lines before it writes any, and
    // workgroups own disjoint lines) and the x pass; the padded rows get y
    // padding only (the planes are padded z planes already).
    float* t = ws;
    pt_status st = pass_lines(field + c * plane * nzi, t, nx, ny, nzi, 2, s, 1);
    if (st != PT_OK) return st;
    float* mid = t + plane * W;
    void* o = dtype == PT_F32 ? (void*)((float*)coeff + c * pb)
                              : (void*)((uint16_t*)coeff + c * pb);
    if (yx_carry_floats(g, nzi) > 0) {
      st = pass_yx(mid, align256f(t + plane * nzi), o, dtype == PT_BF16, nx, ny, nzo, nzo, 0,
                   s);
      if (st != PT_OK) return st;
      continue;
    }
    st = pass_lines(mid, mid, nx, ny, nzo, 1, s);
    if (st != PT_OK) return st;
    st = pass_rows(mid, o, nx, ny, nzo, dtype == PT_F32 ? ROW_PAD_F32 : ROW_PAD_BF16, s, 0);
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

// Adjoint.  The forward map is pad(A_x^-1 A_y^-1 A_z^-1 g); its transpose is
// A_z^-1 A_y^-1 A_x^-1 fold(S_bar) (A symmetric): the same solves in reverse
// axis order, the first one reading and folding the padded gradient.  Where
// the fused pass applies (rows of 256 to 1024 points), fold, y and x run as
// one pass (the axis solves commute), with the y carries stored in the
// component's output block until the z pass writes it.
pt_status spline_bwd(const pt_grid* g, const float* gcoeff, float* gfield, float* ws,
                     hipStream_t s) {
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t p3 = (int64_t)(nx + 3) * (ny + 3) * (nz + 3);
  const bool fused = yx_carry_floats(g, nz) > 0;
  for (int c = 0; c < 3; ++c) {
    float* o = gfield + c * n3;
    if (fused) {
      pt_status st = pass_fyx(gcoeff + c * p3, o, ws, nx, ny, nz, s);  // fold + y + x
      if (st != PT_OK) return st;
      st = pass_lines(ws, o, nx, ny, nz, 2, s);  // z
      if (st != PT_OK) return st;
      continue;
    }
    pt_status st = pass_rows(gcoeff + c * p3, o, nx, ny, nz, ROW_FOLD, s);  // fold + x
    if (st != PT_OK) return st;
    st = pass_lines(o, ws, nx, ny, nz, 1, s);  // y
    if (st != PT_OK) return st;
    st = pass_lines(ws, o, nx, ny, nz, 2, s);  // z
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

}  // namespace pt
