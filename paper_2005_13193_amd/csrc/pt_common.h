// Internal definitions shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pt_spline.h"

namespace pt {

// Particles are ordered in columns of kTileX x kTileY cells (full height in
// z); see pt_key_layout.
constexpr int kTileX = 32;
constexpr int kTileY = 32;

// Launch-time description of the grid and of the padded coefficient array.
struct GridDev {
  int nx, ny, nz;      // grid points per axis
  int px, py, pz;      // padded extents n + 3
  int64_t plane;       // px * py
  int64_t comp;        // px * py * pz (elements per component)
  double cs[3];        // n / L per axis (grid units per length), host-rounded
  float inv_h[3];      // n / L in FP32 (for physical derivatives)
};

inline GridDev make_grid_dev(const pt_grid* g) {
  GridDev d;
  d.nx = g->nx; d.ny = g->ny; d.nz = g->nz;
  d.px = g->nx + 3; d.py = g->ny + 3; d.pz = g->nz + 3;
  d.plane = (int64_t)d.px * d.py;
  d.comp = d.plane * d.pz;
  d.cs[0] = (double)g->nx / g->lx;
  d.cs[1] = (double)g->ny / g->ly;
  d.cs[2] = (double)g->nz / g->lz;
  for (int i = 0; i < 3; ++i) d.inv_h[i] = (float)d.cs[i];
  return d;
}

// ---------------------------------------------------------------- cells ---
// Shadow position and cell along one axis (Sec. 2.2 / Sec. 3): every step is
// one IEEE double operation, none fused, so the cell index is identical to
// any other implementation of the same sequence.  A non-finite coordinate
// yields cell 0, t = 0 and sets *bad.
__device__ __forceinline__ int cell_1d(double x, double cs, int n, double* t, bool* bad) {
#pragma clang fp contract(off)
  if (!(fabs(x) <= 1.7976931348623157e308)) {  // NaN or +-inf
    *bad = true;
    *t = 0.0;
    return 0;
  }
  const double dn = (double)n;
  double s = x * cs;
  double sw = s;
  // Inside the primary domain floor(s / n) is 0 (a quotient that rounds up to
  // 1 is corrected back by the second test), so the division is only needed
  // outside it; both branches give the same bits.
  if (!(s >= 0.0 && s < dn)) {
    double k = floor(s / dn);
    double kn = k * dn;
    sw = s - kn;
    if (sw < 0.0) sw = sw + dn;
    if (sw >= dn) sw = sw - dn;
  }
  double fa = floor(sw);
  *t = sw - fa;
  int a = (int)fa;
  // sw is in [0, n) by construction; the clamp only guards the memory access.
  a = a < 0 ? 0 : (a > n - 1 ? n - 1 : a);
  return a;
}

// ------------------------------------------------------------- weights ---
// Uniform cubic B-spline pieces on the cell, i = 1..4 <-> coefficient
// offsets -1..+2 (eq. (spline): p = alpha + i - 2), and their t-derivatives,
// in the arithmetic type T of the gather (float, or double for FP64 storage).
template <typename T>
__device__ __forceinline__ void bspline_w(T t, T w[4]) {
  const T s = T(1) - t;
  const T t2 = t * t, t3 = t2 * t;
  const T r6 = T(1) / T(6);
  w[0] = s * s * s * r6;
  w[1] = (T(3) * t3 - T(6) * t2 + T(4)) * r6;
  w[2] = (T(-3) * t3 + T(3) * t2 + T(3) * t + T(1)) * r6;
  w[3] = t3 * r6;
}

template <typename T>
__device__ __forceinline__ void bspline_dw(T t, T w[4]) {
  const T s = T(1) - t;
  w[0] = T(-0.5) * s * s;
  w[1] = t * (T(1.5) * t - T(2));
  w[2] = T(0.5) + t * (T(1) - T(1.5) * t);
  w[3] = T(0.5) * t * t;
}

// Arithmetic type of the gathers for a coefficient storage type: FP32 for
// FP32 and BF16 storage, FP64 for FP64 storage.
template <typename CT> struct AccOf { using T = float; };
template <> struct AccOf<double> { using T = double; };

// ------------------------------------------------------------ bfloat16 ---
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

// Round to nearest, ties to even; NaN stays a (quiet) NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float load_coeff(const float* p) { return *p; }
__device__ __forceinline__ float load_coeff(const uint16_t* p) { return bf16_to_f32(*p); }
__device__ __forceinline__ double load_coeff(const double* p) { return *p; }

// Bytes of one stored coefficient (and of one velocity or interpolated value
// on the FP64 path, which keeps them in FP64 too).
inline size_t dtype_bytes(pt_dtype d) { return d == PT_F64 ? 8 : d == PT_BF16 ? 2 : 4; }
inline size_t value_bytes(pt_dtype d) { return d == PT_F64 ? 8 : 4; }

// ---------------------------------------------------------- host glue ---
// Per-device pointer to the library's non-finite-position flag.
int* device_error_flag();

inline unsigned grid_1d(int64_t n, int block) {
  return (unsigned)((n + block - 1) / block);
}

}  // namespace pt

#define PT_HIP_CHECK(expr)                    \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return PT_ERR_HIP;  \
  } while (0)

#define PT_LAUNCH_CHECK() PT_HIP_CHECK(hipGetLastError())

namespace pt {
// Optional per-kernel timing: while enabled (pt_timing_enable), launches
// wrapped in a TimedLaunch record a pair of HIP events on their stream.
bool timing_on();
void timing_record(const char* name, hipEvent_t start, hipEvent_t stop);

struct TimedLaunch {
  const char* name;
  hipStream_t stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TimedLaunch(const char* n, hipStream_t s) : name(n), stream(s) {
    if (!timing_on()) return;
    if (hipEventCreate(&e0) != hipSuccess) {
      e0 = nullptr;
      return;
    }
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      e0 = e1 = nullptr;
      return;
    }
    (void)hipEventRecord(e0, stream);  // diagnostics: a failed record only loses the sample
  }
  ~TimedLaunch() {
    if (e0 && e1) {
      (void)hipEventRecord(e1, stream);
      timing_record(name, e0, e1);
    }
  }
};
}  // namespace pt
