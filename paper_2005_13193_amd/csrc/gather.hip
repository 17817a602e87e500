// Operations 2 and 3 of Sec. 2.2 (basis functions and the 64-term sum of
// eq. (spline)) at every particle, the Heun RK2 stages built on them, the
// inertial-particle step, and their adjoints.  One thread per particle; the
// 16 x-runs of 4 coefficients per component are read straight from the
// padded array.  Particles that are ordered by cell (pt_sort_particles) make
// neighbouring lanes read neighbouring coefficients, so the reads coalesce
// and hit in L2.
//
// Every kernel is instantiated for the three coefficient storage types; the
// arithmetic type AT is FP32 for FP32 and BF16 storage and FP64 for FP64
// storage, and so is the value type VT of velocities and interpolated values
// handed between kernels or to the caller.
#include "pt_common.h"
#include "pt_inertial.h"

namespace pt {

template <typename AT>
struct Cell {
  int a, b, c;
  AT t[3];
};

template <typename AT>
__device__ __forceinline__ Cell<AT> locate(const GridDev& g, double x, double y, double z,
                                           int* err) {
  Cell<AT> cl;
  bool bad = false;
  double t0, t1, t2;
  cl.a = cell_1d(x, g.cs[0], g.nx, &t0, &bad);
  cl.b = cell_1d(y, g.cs[1], g.ny, &t1, &bad);
  cl.c = cell_1d(z, g.cs[2], g.nz, &t2, &bad);
  if (bad) *err = 1;
  cl.t[0] = (AT)t0;
  cl.t[1] = (AT)t1;
  cl.t[2] = (AT)t2;
  return cl;
}

// Value (and, with GRAD, the three physical derivatives) of each component:
// out[c] = u_c, out[3 + 3c + d] = du_c/dx_d.
template <typename CT, bool GRAD, typename AT = typename AccOf<CT>::T>
__device__ __forceinline__ void spline_eval(const GridDev& g, const CT* __restrict__ coeff,
                                            const Cell<AT>& cl, AT out[12]) {
  AT wx[4], wy[4], wz[4], dx[4], dy[4], dz[4];
  bspline_w(cl.t[0], wx);
  bspline_w(cl.t[1], wy);
  bspline_w(cl.t[2], wz);
  if (GRAD) {
    bspline_dw(cl.t[0], dx);
    bspline_dw(cl.t[1], dy);
    bspline_dw(cl.t[2], dz);
  }
  const int64_t off = ((int64_t)cl.c * g.py + cl.b) * g.px + cl.a;
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    const CT* base = coeff + comp * g.comp + off;
    AT v = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      AT ty = 0, tdy = 0, tdx = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const CT* row = base + k * g.plane + j * g.px;
        const AT r0 = load_coeff(row), r1 = load_coeff(row + 1);
        const AT r2 = load_coeff(row + 2), r3 = load_coeff(row + 3);
        const AT sx = wx[0] * r0 + wx[1] * r1 + wx[2] * r2 + wx[3] * r3;
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
      out[3 + 3 * comp + 0] = gx * (AT)g.cs[0];
      out[3 + 3 * comp + 1] = gy * (AT)g.cs[1];
      out[3 + 3 * comp + 2] = gz * (AT)g.cs[2];
    }
  }
}

// Transposed 64-term sum: g_coeff[comp][stencil] += w_ijk gu[comp] (the
// gradient is FP32 whatever the storage type).
template <typename AT>
__device__ __forceinline__ void spline_scatter(const GridDev& g, float* __restrict__ gc,
                                               const Cell<AT>& cl, const AT gu[3]) {
  AT wx[4], wy[4], wz[4];
  bspline_w(cl.t[0], wx);
  bspline_w(cl.t[1], wy);
  bspline_w(cl.t[2], wz);
  const int64_t off = ((int64_t)cl.c * g.py + cl.b) * g.px + cl.a;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const AT wjk = wz[k] * wy[j];
      float* row = gc + off + k * g.plane + j * g.px;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const AT w = wjk * wx[i];
#pragma unroll
        for (int comp = 0; comp < 3; ++comp)
          unsafeAtomicAdd(row + comp * g.comp + i, (float)(w * gu[comp]));
      }
    }
}

template <typename CT, int NOUT, typename VT = typename AccOf<CT>::T>
__global__ __launch_bounds__(256) void interp_kernel(GridDev g, const CT* __restrict__ coeff,
                                                     int64_t np, const double* __restrict__ pos,
                                                     VT* __restrict__ out, int* err) {
  using AT = typename AccOf<CT>::T;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const Cell<AT> cl = locate<AT>(g, pos[p], pos[np + p], pos[2 * np + p], err);
  AT o[12];
  spline_eval<CT, NOUT == 12>(g, coeff, cl, o);
#pragma unroll
  for (int q = 0; q < NOUT; ++q) out[q * np + p] = (VT)o[q];
}

// Second Heun stage: x* = x + dt u0, u1 = u(x*), x_out = x + dt/2 (u0 + u1).
// x_out may alias x (each thread reads its own particle before writing).
template <typename CT, typename VT = typename AccOf<CT>::T>
__global__ __launch_bounds__(256) void rk2_stage2(GridDev g, const CT* __restrict__ coeff,
                                                  int64_t np, double dt, const double* x,
                                                  const VT* __restrict__ u0, double* x_out,
                                                  int* err) {
  using AT = typename AccOf<CT>::T;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  double xn[3], xs[3];
  VT ua[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xn[d] = x[d * np + p];
    ua[d] = u0[d * np + p];
    xs[d] = xn[d] + dt * (double)ua[d];
  }
  const Cell<AT> cl = locate<AT>(g, xs[0], xs[1], xs[2], err);
  AT ub[12];
  spline_eval<CT, false>(g, coeff, cl, ub);
  const double h = 0.5 * dt;
#pragma unroll
  for (int d = 0; d < 3; ++d) x_out[d * np + p] = xn[d] + h * ((double)ua[d] + (double)ub[d]);
}

// Inertial / diffusive particle step (see pt_inertial.h), both stages in one
// thread: x_out and v_out may alias x and v.
template <typename CT, typename VT = typename AccOf<CT>::T>
__global__ __launch_bounds__(256) void inertial_direct(GridDev g, const CT* __restrict__ coeff,
                                                       int64_t np, InertialCoef k,
                                                       const double* x, const VT* v,
                                                       const double* __restrict__ disp,
                                                       double* x_out, VT* v_out, int* err) {
  using AT = typename AccOf<CT>::T;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  double xn[3], vn[3], xs[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xn[d] = x[d * np + p];
    vn[d] = v ? (double)v[d * np + p] : 0.0;
  }
  const Cell<AT> c0 = locate<AT>(g, xn[0], xn[1], xn[2], err);
  AT u0[12], u1[12];
  spline_eval<CT, false>(g, coeff, c0, u0);
#pragma unroll
  for (int d = 0; d < 3; ++d)
    xs[d] = inertial_predict(k, xn[d], vn[d], (double)u0[d], disp ? disp[d * np + p] : 0.0);
  const Cell<AT> c1 = locate<AT>(g, xs[0], xs[1], xs[2], err);
  spline_eval<CT, false>(g, coeff, c1, u1);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x_out[d * np + p] = inertial_correct(k, xs[d], (double)u0[d], (double)u1[d]);
    if (v_out) v_out[d * np + p] = (VT)inertial_velocity(k, vn[d], (double)u0[d], (double)u1[d]);
  }
}

template <typename CT>
__global__ __launch_bounds__(256) void interp_bwd_kernel(GridDev g, const CT* __restrict__ coeff,
                                                         int64_t np, const double* __restrict__ pos,
                                                         const float* __restrict__ gout,
                                                         double* __restrict__ gpos,
                                                         float* __restrict__ gcoeff, int* err) {
  using AT = typename AccOf<CT>::T;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const Cell<AT> cl = locate<AT>(g, pos[p], pos[np + p], pos[2 * np + p], err);
  const AT gu[3] = {(AT)gout[p], (AT)gout[np + p], (AT)gout[2 * np + p]};
  if (gpos) {
    AT o[12];
    spline_eval<CT, true>(g, coeff, cl, o);
#pragma unroll
    for (int d = 0; d < 3; ++d)
      gpos[d * np + p] += (double)(gu[0] * o[3 + d] + gu[1] * o[6 + d] + gu[2] * o[9 + d]);
  }
  if (gcoeff) spline_scatter(g, gcoeff, cl, gu);
}

// Adjoint of a Heun step, part 1 (at x*): ub1 = dt/2 lam, xbs = J(x*)^T ub1,
// g_coeff += W(x*)^T ub1.  u0 is the stage-1 velocity at x^n.
template <typename CT, typename VT = typename AccOf<CT>::T>
__global__ __launch_bounds__(256) void rk2_bwd_star(GridDev g, const CT* __restrict__ coeff,
                                                    int64_t np, double dt,
                                                    const double* __restrict__ x,
                                                    const VT* __restrict__ u0,
                                                    const double* __restrict__ lam,
                                                    double* __restrict__ xbs,
                                                    float* __restrict__ gcoeff, int* err) {
  using AT = typename AccOf<CT>::T;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  double xs[3];
  AT ub[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xs[d] = x[d * np + p] + dt * (double)u0[d * np + p];
    ub[d] = (AT)(0.5 * dt * lam[d * np + p]);
  }
  const Cell<AT> cl = locate<AT>(g, xs[0], xs[1], xs[2], err);
  AT o[12];
  spline_eval<CT, true>(g, coeff, cl, o);
#pragma unroll
  for (int d = 0; d < 3; ++d)
    xbs[d * np + p] = (double)(ub[0] * o[3 + d] + ub[1] * o[6 + d] + ub[2] * o[9 + d]);
  if (gcoeff) spline_scatter(g, gcoeff, cl, ub);
}

// Part 2 (at x^n): ub0 = dt/2 lam + dt xbs, out = lam + xbs + J(x^n)^T ub0,
// g_coeff += W(x^n)^T ub0.  out may alias lam.
template <typename CT>
__global__ __launch_bounds__(256) void rk2_bwd_n(GridDev g, const CT* __restrict__ coeff,
                                                 int64_t np, double dt,
                                                 const double* __restrict__ x, const double* lam,
                                                 const double* __restrict__ xbs, double* out,
                                                 float* __restrict__ gcoeff, int* err) {
  using AT = typename AccOf<CT>::T;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  double l[3], s[3];
  AT ub[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    l[d] = lam[d * np + p];
    s[d] = xbs[d * np + p];
    ub[d] = (AT)(0.5 * dt * l[d] + dt * s[d]);
  }
  const Cell<AT> cl = locate<AT>(g, x[p], x[np + p], x[2 * np + p], err);
  AT o[12];
  spline_eval<CT, true>(g, coeff, cl, o);
#pragma unroll
  for (int d = 0; d < 3; ++d)
    out[d * np + p] = l[d] + s[d] + (double)(ub[0] * o[3 + d] + ub[1] * o[6 + d] + ub[2] * o[9 + d]);
  if (gcoeff) spline_scatter(g, gcoeff, cl, ub);
}

// The gather half of a Heun step's adjoint, one thread per particle, for the
// column-tiled scatter to finish: xbn = lam + xbs + J(x^n)^T ub0 (may alias
// lam), and the stage-1 velocity and both stage adjoints in FP32 for the
// scatter (ub1 = dt/2 lam, ub0 = dt/2 lam + dt xbs, xbs = J(x*)^T ub1); the
// largest |ub| of each block goes to one of the 64 slots of `umax` (float
// bits, compared as integers: all non-negative).
template <typename CT>
__global__ __launch_bounds__(256) void rk2_bwd_gather_direct(
    GridDev g, const CT* __restrict__ coeff, int64_t np, double dt, const double* __restrict__ x,
    const double* lam, double* xbn, float* __restrict__ u0f, float* __restrict__ ub0f,
    float* __restrict__ ub1f, int* umax, int* err) {
  using AT = typename AccOf<CT>::T;
  __shared__ float s_max[4];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float m = 0.0f;
  if (p < np) {
    double xn[3], l[3], xs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xn[d] = x[d * np + p];
      l[d] = lam[d * np + p];
    }
    const Cell<AT> c0 = locate<AT>(g, xn[0], xn[1], xn[2], err);
    AT on[12], os[12];
    spline_eval<CT, true>(g, coeff, c0, on);
#pragma unroll
    for (int d = 0; d < 3; ++d) xs[d] = xn[d] + dt * (double)on[d];
    const Cell<AT> c1 = locate<AT>(g, xs[0], xs[1], xs[2], err);
    spline_eval<CT, true>(g, coeff, c1, os);
    AT ub1[3], ub0[3];
    double xbs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) ub1[d] = (AT)(0.5 * dt * l[d]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xbs[d] = (double)(ub1[0] * os[3 + d] + ub1[1] * os[6 + d] + ub1[2] * os[9 + d]);
      ub0[d] = (AT)(0.5 * dt * l[d] + dt * xbs[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xbn[d * np + p] =
          l[d] + xbs[d] + (double)(ub0[0] * on[3 + d] + ub0[1] * on[6 + d] + ub0[2] * on[9 + d]);
      u0f[d * np + p] = (float)on[d];
      ub0f[d * np + p] = (float)ub0[d];
      ub1f[d * np + p] = (float)ub1[d];
      m = fmaxf(m, fmaxf(fabsf((float)ub0[d]), fabsf((float)ub1[d])));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
    atomicMax(umax + (blockIdx.x & 63), __float_as_int(m));
  }
}

__global__ __launch_bounds__(256) void scatter_rows_f64(int64_t np, const double* __restrict__ in,
                                                        const int32_t* __restrict__ perm,
                                                        double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const int64_t q = perm[i];
  if ((uint64_t)q >= (uint64_t)np) return;
  out[q] = in[i];
  out[np + q] = in[np + i];
  out[2 * np + q] = in[2 * np + i];
}

// ------------------------------------------------------------ launchers ---
// Calls F.template operator()<CT>() with the storage type of `dtype`.
template <typename F>
static pt_status with_ct(pt_dtype dtype, F&& f) {
  if (dtype == PT_F32) f.template operator()<float>();
  else if (dtype == PT_BF16) f.template operator()<uint16_t>();
  else f.template operator()<double>();
  PT_LAUNCH_CHECK();
  return PT_OK;
}

pt_status interp_fwd(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np,
                     const double* pos, void* out, int nout, hipStream_t s) {
  const GridDev gd = make_grid_dev(g);
  const dim3 grid(grid_1d(np, 256)), block(256);
  int* err = device_error_flag();
  TimedLaunch t("interp", s);
  return with_ct(dtype, [&]<typename CT>() {
    using VT = typename AccOf<CT>::T;
    if (nout == 3)
      hipLaunchKernelGGL((interp_kernel<CT, 3>), grid, block, 0, s, gd, (const CT*)coeff, np, pos,
                         (VT*)out, err);
    else
      hipLaunchKernelGGL((interp_kernel<CT, 12>), grid, block, 0, s, gd, (const CT*)coeff, np,
                         pos, (VT*)out, err);
  });
}

// Second Heun stage alone: x_out = x + dt/2 (u0 + u(x + dt u0)) with the
// given coefficients (x_out may alias x).
pt_status rk2_correct(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np, double dt,
                      const double* x, const void* u0, double* x_out, hipStream_t s) {
  const GridDev gd = make_grid_dev(g);
  TimedLaunch t("rk2_direct_stage2", s);
  return with_ct(dtype, [&]<typename CT>() {
    using VT = typename AccOf<CT>::T;
    hipLaunchKernelGGL(rk2_stage2<CT>, dim3(grid_1d(np, 256)), dim3(256), 0, s, gd,
                       (const CT*)coeff, np, dt, x, (const VT*)u0, x_out, device_error_flag());
  });
}

pt_status rk2_advance(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np, double dt,
                      const double* x, double* x_out, void* u0, hipStream_t s) {
  pt_status st = interp_fwd(g, coeff, dtype, np, x, u0, 3, s);
  if (st != PT_OK) return st;
  return rk2_correct(g, coeff, dtype, np, dt, x, u0, x_out, s);
}

pt_status inertial_advance(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np,
                           const InertialCoef& k, const double* x, const void* v,
                           const double* disp, double* x_out, void* v_out, hipStream_t s) {
  const GridDev gd = make_grid_dev(g);
  TimedLaunch t("inertial_direct", s);
  return with_ct(dtype, [&]<typename CT>() {
    using VT = typename AccOf<CT>::T;
    hipLaunchKernelGGL(inertial_direct<CT>, dim3(grid_1d(np, 256)), dim3(256), 0, s, gd,
                       (const CT*)coeff, np, k, x, (const VT*)v, disp, x_out, (VT*)v_out,
                       device_error_flag());
  });
}

pt_status interp_bwd(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np,
                     const double* pos, const float* gout, double* gpos, float* gcoeff,
                     hipStream_t s) {
  const GridDev gd = make_grid_dev(g);
  return with_ct(dtype, [&]<typename CT>() {
    hipLaunchKernelGGL(interp_bwd_kernel<CT>, dim3(grid_1d(np, 256)), dim3(256), 0, s, gd,
                       (const CT*)coeff, np, pos, gout, gpos, gcoeff, device_error_flag());
  });
}

// Adjoint of one Heun step on particles in the order x is given; lam is
// dL/dx_out in that order; out receives dL/dx (out may alias lam).  u0 holds
// np values of the storage's value type (FP64 for FP64 storage).
pt_status rk2_backward(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np, double dt,
                       const double* x, const double* lam, double* out, float* gcoeff, void* u0,
                       double* xbs, hipStream_t s) {
  pt_status st = interp_fwd(g, coeff, dtype, np, x, u0, 3, s);
  if (st != PT_OK) return st;
  const GridDev gd = make_grid_dev(g);
  const dim3 grid(grid_1d(np, 256)), block(256);
  int* err = device_error_flag();
  TimedLaunch t("rk2_direct_bwd", s);
  return with_ct(dtype, [&]<typename CT>() {
    using VT = typename AccOf<CT>::T;
    hipLaunchKernelGGL(rk2_bwd_star<CT>, grid, block, 0, s, gd, (const CT*)coeff, np, dt, x,
                       (const VT*)u0, lam, xbs, gcoeff, err);
    hipLaunchKernelGGL(rk2_bwd_n<CT>, grid, block, 0, s, gd, (const CT*)coeff, np, dt, x, lam,
                       xbs, out, gcoeff, err);
  });
}

pt_status rk2_bwd_gather(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np,
                        double dt, const double* x, const double* lam, double* xbn, float* u0f,
                        float* ub0f, float* ub1f, int* umax, hipStream_t s) {
  const GridDev gd = make_grid_dev(g);
  TimedLaunch t("rk2_direct_bwd_gather", s);
  return with_ct(dtype, [&]<typename CT>() {
    hipLaunchKernelGGL(rk2_bwd_gather_direct<CT>, dim3(grid_1d(np, 256)), dim3(256), 0, s, gd,
                       (const CT*)coeff, np, dt, x, lam, xbn, u0f, ub0f, ub1f, umax,
                       device_error_flag());
  });
}

pt_status scatter_back(int64_t np, const double* in, const int32_t* perm, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(scatter_rows_f64, dim3(grid_1d(np, 256)), dim3(256), 0, s, np, in, perm, out);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
