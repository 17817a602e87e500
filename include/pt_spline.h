/*
 * pt_spline.h - C ABI of the MI355X (gfx950) periodic cubic-spline particle
 * tracking library.
 *
 * The library implements, on one GPU, the per-step path of the particle
 * tracking method of Buaria & Yeung (Comput. Phys. Commun., "A highly scalable
 * particle tracking algorithm using partitioned global address space (PGAS)
 * programming for extreme-scale turbulence simulations"):
 *   Operation 1 of Sec. 2.2  - cubic-spline coefficients of a periodic field,
 *                              one periodic tridiagonal solve per axis;
 *   Sec. 3                   - particles ordered by the spline cell that
 *                              holds them (the one-device counterpart of the
 *                              paper's position-based particle-to-process
 *                              mapping), as a stable radix sort;
 *   Operations 2 and 3       - basis functions and the 64-term sum of
 *     of Sec. 2.2              eq. (spline), for (u,v,w) and for the nine
 *                              velocity gradients;
 *   eq. (dxdt), Sec. 4.3     - explicit second-order Runge-Kutta advance of
 *                              the particle positions;
 * plus hand-written adjoints of each of these (not in the paper).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller.  No entry
 *    point allocates device memory; scratch space is passed in as a workspace
 *    whose size is given by pt_workspace_bytes().  The library keeps, per
 *    device, one 4-byte error flag in its own static device memory.
 *  - Arrays are dense, C order, x the fastest index:
 *      field   float [3][nz][ny][nx]           grid values of (u, v, w)
 *      coeff   [3][nz+3][ny+3][nx+3]           padded spline coefficients,
 *              float (PT_F32), bfloat16 bits (PT_BF16) or double (PT_F64);
 *              along every axis the
 *              padded index P holds the coefficient of grid line (P-1) mod n,
 *              i.e. the index range 1..N+3 of eq. (spline) shifted to 0-based
 *      pos     double [3][np]                  positions x, y, z, unwrapped
 *  - Every call validates its arguments on the host before launching anything
 *    and returns a pt_status; no exception crosses the ABI.  Work is enqueued
 *    asynchronously on `stream` (0 = the null stream).  HIP launch failures
 *    return PT_ERR_HIP.  A kernel that meets a non-finite position treats it
 *    as the origin, finishes, and raises the device error flag that
 *    pt_last_device_error() reports.
 *  - Gradient outputs named g_* ACCUMULATE (+=) into caller-initialised
 *    buffers, except pt_spline_coeffs_bwd, which overwrites g_field.
 *  - Grid sizes: 4 <= n <= 8192 per axis; np < 2^31.
 */
#ifndef PT_SPLINE_H
#define PT_SPLINE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PT_OK = 0,
  PT_ERR_NULL = -1,        /* a required pointer is NULL */
  PT_ERR_SIZE = -2,        /* grid size, particle count or box length invalid */
  PT_ERR_DTYPE = -3,       /* unknown coefficient dtype */
  PT_ERR_WORKSPACE = -4,   /* workspace NULL or smaller than required */
  PT_ERR_NONFINITE = -5,   /* a kernel met a NaN or infinite position */
  PT_ERR_HIP = -6,         /* a HIP runtime call or launch failed */
  PT_ERR_UNSUPPORTED = -7, /* valid but not supported (e.g. n > 8192) */
  PT_ERR_ARG = -8          /* other invalid argument (bad op code, dt) */
} pt_status;

/* Storage type of the spline coefficients.  PT_F32 and PT_BF16 compute in
 * FP32 (BF16 values widened exactly); PT_F64 is the FP64 form of the same
 * method (the baseline the other two are compared with on the same device):
 * its solves and gathers compute in FP64, and the interpolated values and
 * velocities it reads or writes (out, u_n, vel) are double instead of float.
 * The column-tiled kernels stage FP32 or BF16 coefficients only: with PT_F64
 * the sorted paths (PT_SORT, PT_SORTED) sort as usual and then gather from
 * global memory, one thread per particle. */
typedef enum { PT_F32 = 0, PT_BF16 = 1, PT_F64 = 2 } pt_dtype;

/* Periodic box [0,lx) x [0,ly) x [0,lz) sampled at nx*ny*nz points with
 * uniform spacing lx/nx, ly/ny, lz/nz (Sec. 2.2). */
typedef struct {
  int32_t nx, ny, nz;
  double lx, ly, lz;
} pt_grid;

/* Operation codes for pt_workspace_bytes. */
enum {
  PT_OP_SPLINE = 0,     /* pt_spline_coeffs */
  PT_OP_SORT = 1,       /* pt_sort_particles */
  PT_OP_RK2 = 2,        /* pt_rk2_step (with or without sort) */
  PT_OP_SPLINE_BWD = 3, /* pt_spline_coeffs_bwd */
  PT_OP_RK2_BWD = 4,    /* pt_rk2_step_bwd (with or without sort) */
  PT_OP_SPLINE_SLAB = 5, /* pt_spline_coeffs_slab; np = input planes nzl + 3 + 2 halo */
  PT_OP_SLAB_PARTITION = 6, /* pt_slab_partition */
  PT_OP_INERTIAL = 7,    /* pt_inertial_step (with or without sort) */
  PT_OP_INTERP_SORTED = 8 /* pt_interp_sorted */
};

/* Bytes of workspace the operation needs for this grid, coefficient dtype
 * and particle count (np ignored for PT_OP_SPLINE and PT_OP_SPLINE_BWD; for
 * PT_OP_SPLINE_SLAB it is the slab's input plane count).  The result is a
 * multiple of 256.  Returns PT_ERR_ARG for an unknown op. */
pt_status pt_workspace_bytes(int op, const pt_grid *grid, pt_dtype dtype, int64_t np,
                             size_t *bytes);

/* Layout of the particle sort key (see pt_sort_particles): cells are grouped
 * in columns of tile_x * tile_y cells in the (x, y) plane, running the full
 * height in z; key_bits is the number of significant key bits for this grid.
 * With a = alpha, b = beta, g = gamma (0-based cell indices):
 *   key = (((b/ty * ceil(nx/tx) + a/tx) * nz + g) * ty + b%ty) * tx + a%tx. */
pt_status pt_key_layout(const pt_grid *grid, int32_t *tile_x, int32_t *tile_y,
                        int32_t *key_bits);

/* Operation 1 (Sec. 2.2): spline coefficients of the three components.
 * Along every grid line of every axis the coefficients S solve the periodic
 * tridiagonal system (S[m-1] + 4 S[m] + S[m+1]) / 6 = g[m], m = 0..n-1
 * (indices mod n), so that the tensor-product cubic B-spline with
 * coefficients S interpolates the grid values exactly.  The axis solves
 * commute; they run in the order z, y, x (the paper's order is x, z, y, which
 * differs only in rounding), and the x pass writes the padded layout (rounded
 * to nearest-even for PT_BF16).
 *   field  in   float [3][nz][ny][nx]
 *   coeff  out  [3][nz+3][ny+3][nx+3] of `dtype`; must not overlap field
 *   ws          >= pt_workspace_bytes(PT_OP_SPLINE, ...) bytes */
pt_status pt_spline_coeffs(const pt_grid *grid, const float *field, void *coeff,
                           pt_dtype dtype, void *ws, size_t ws_bytes,
                           hipStream_t stream);

/* Operation 1 for one z-slab of a periodic grid: the share of one device
 * when the grid is split in z, as the paper's domain decomposition splits it
 * across processes (Sec. 3).  The z lines are solved with open ends over the
 * slab plus `halo` field planes on each side: the inverse of the periodic
 * 1-4-1 system decays like |z1|^d (z1 = sqrt(3) - 2, |z1| = 0.268) with the
 * distance d, so the result differs from the periodic solve by a relative
 * amount of order |z1|^halo (halo >= 14 puts it below FP32 rounding).  The x
 * and y lines are whole and solved periodically, as by pt_spline_coeffs.
 *   grid   the whole grid (nx, ny as stored here; nz = all planes)
 *   nzl    planes of the slab, 1 <= nzl <= nz;  halo 1 .. 64
 *   field  in   float [3][nzl + 3 + 2 halo][ny][nx]: the periodic field's
 *               planes z0-1-halo .. z0+nzl+1+halo (indices mod nz), for a
 *               slab starting at plane z0
 *   coeff  out  [3][nzl+3][ny+3][nx+3] of `dtype`, x and y padded as by
 *               pt_spline_coeffs; padded plane P holds plane z0-1+P
 *   ws          >= pt_workspace_bytes(PT_OP_SPLINE_SLAB, grid, dtype,
 *               nzl + 3 + 2 halo) bytes */
pt_status pt_spline_coeffs_slab(const pt_grid *grid, int32_t nzl, int32_t halo,
                                const float *field, void *coeff, pt_dtype dtype, void *ws,
                                size_t ws_bytes, hipStream_t stream);

/* Sec. 2.2 and Sec. 3: map each position to its cell and order particles by
 * cell.  Per axis, in double precision with no fused operations,
 *   s = x * (n / L);  s_w = s - n floor(s / n), then +n if s_w < 0 and -n if
 *   s_w >= n;  alpha = floor(s_w),  t = s_w - alpha in [0, 1)
 * (the shadow position inside the primary domain).  The key is the one given
 * at pt_key_layout; the sort is a stable LSD radix sort, so particles with
 * equal keys keep their input order.
 *   pos         in   double [3][np]
 *   pos_sorted  out  double [3][np], pos_sorted[d][i] = pos[d][perm[i]]
 *                    (may be NULL); must not overlap pos
 *   perm        out  int32 [np], original index of sorted particle i
 *   ids      in/out  int32 [np] particle labels, re-ordered with the positions:
 *                    ids[i] <- ids[perm[i]] (may be NULL)
 *   keys_out    out  uint64 [np] sorted keys (may be NULL)
 *   ws               >= pt_workspace_bytes(PT_OP_SORT, ...) bytes */
pt_status pt_sort_particles(const pt_grid *grid, int64_t np, const double *pos,
                            double *pos_sorted, int32_t *perm, int32_t *ids,
                            uint64_t *keys_out, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* Operations 2 and 3 of Sec. 2.2, eq. (spline): at every particle
 *   g+ = sum_{k,j,i=1..4} b_i(x') c_j(y') d_k(z') S[gamma+k-2][beta+j-2][alpha+i-2]
 * with the cubic B-spline pieces as basis functions, in FP32 (FP64 for
 * PT_F64).
 *   coeff  in   padded coefficients of `dtype`
 *   pos    in   double [3][np] (any order; sorted order is fastest)
 *   out    out  float [3][np] = (u, v, w); double for PT_F64 */
pt_status pt_interp_uvw(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                        int64_t np, const double *pos, void *out, hipStream_t stream);

/* As pt_interp_uvw, plus the nine velocity gradients from the derivatives of
 * the basis functions (Sec. 2.2: the splines are twice differentiable):
 *   out  float [12][np] (double for PT_F64): u, v, w, then du_i/dx_j at
 *        row 3 + 3 i + j. */
pt_status pt_interp_grad(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                         int64_t np, const double *pos, void *out, hipStream_t stream);

/* pt_interp_uvw (nout = 3) or pt_interp_grad (nout = 12) for particles in
 * cell order (as pt_sort_particles leaves them): the column-tiled kernels
 * stage each column's coefficient planes in LDS once and gather from there,
 * the particle-per-thread kernels of pt_interp_uvw / pt_interp_grad read
 * them from global memory.  Particles out of order give the same values more
 * slowly (a particle outside its column's tile is evaluated from global
 * memory, and a cell table that is not a partition of the particles, checked
 * on the device, sends every particle that way).  Fewer than 2^30 particles
 * per call (else PT_ERR_UNSUPPORTED).  PT_F64 gathers from global memory.
 *   pos   in   double [3][np], cell order
 *   nout  3 or 12 (else PT_ERR_ARG)
 *   out   out  float [nout][np] (double for PT_F64), rows as for
 *              pt_interp_grad
 *   ws         >= pt_workspace_bytes(PT_OP_INTERP_SORTED, ...) bytes */
pt_status pt_interp_sorted(const pt_grid *grid, const void *coeff, pt_dtype dtype, int64_t np,
                           const double *pos, int nout, void *out, void *ws, size_t ws_bytes,
                           hipStream_t stream);

/* The sort argument of pt_rk2_step and pt_rk2_step_bwd. */
enum {
  PT_UNSORTED = 0, /* particles in any order, left in it; one thread per particle
                      reads its coefficients from global memory */
  PT_SORT = 1,     /* sort first (as pt_sort_particles); the column-tiled kernels */
  PT_SORTED = 2    /* the particles are already in cell order (as pt_sort_particles
                      leaves them, positions unchanged since) and stay in it; the
                      column-tiled kernels without the sort.  Particles out of order
                      give the same result more slowly: a particle outside its
                      column's tile is evaluated from global memory, and a cell
                      table that is not a partition of the particles (checked on
                      the device) sends every particle that way.
                      PT_SORT and PT_SORTED (and the sorted stages of the
                      time-varying step) take fewer than 2^30 particles per
                      call: more return PT_ERR_UNSUPPORTED. */
};

/* One RK2 step of dx/dt = u(x) (eq. (dxdt)), Heun's form:
 *   u0 = u(x);  x* = x + dt u0;  u1 = u(x*);  x <- x + dt/2 (u0 + u1),
 * velocities from the spline (FP32; FP64 for PT_F64), positions in FP64,
 * stored unwrapped.
 * With sort = PT_SORT the particles are first re-ordered as by
 * pt_sort_particles and pos (and ids, if not NULL) come back in the new
 * order; with PT_UNSORTED or PT_SORTED the order is kept.  Other values of
 * sort return PT_ERR_ARG.
 *   pos  in/out double [3][np];  ids  in/out int32 [np] or NULL
 *   ws          >= pt_workspace_bytes(PT_OP_RK2, ...) bytes */
pt_status pt_rk2_step(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                      int64_t np, double dt, double *pos, int32_t *ids, int sort,
                      void *ws, size_t ws_bytes, hipStream_t stream);

/* The same step out of place, for particles in any order (PT_UNSORTED) or in
 * cell order (PT_SORTED), kept in it: pos_out = the step of pos_in, with the
 * same kernels and the same results bit for bit as pt_rk2_step.  A caller
 * that needs x_n after the step (an adjoint) keeps it without a copy.
 * PT_SORT returns PT_ERR_ARG (it re-orders; use pt_rk2_step).
 *   pos_in   in   double [3][np]
 *   pos_out  out  double [3][np]; may be pos_in, else must not overlap it
 *   ws            >= pt_workspace_bytes(PT_OP_RK2, ...) bytes */
pt_status pt_rk2_step_out(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                          int64_t np, double dt, const double *pos_in, double *pos_out,
                          int sort, void *ws, size_t ws_bytes, hipStream_t stream);

/* The same step in a field that changes over the step, in two calls.  In the
 * paper's production runs (Sec. 4.3, Table 5) the particles are advanced at
 * each sub-step of the flow solver's second-order Runge-Kutta scheme, with
 * the spline coefficients of that sub-step's velocity field: the predictor
 * uses the field at t_n, the corrector the field at t_n + dt.
 *
 * Stage 1, with the coefficients of u(., t_n):
 *   u_n = u^n(x)
 * If sort != 0 the particles are first re-ordered as by pt_sort_particles;
 * pos (and ids, if not NULL) come back in the new order, and ws keeps the
 * table of particles per cell layer for stage 2.
 *   coeff_n  in   padded coefficients of the field at t_n, of `dtype`
 *   pos      in/out double [3][np]  (only re-ordered)
 *   ids      in/out int32 [np] or NULL
 *   u_n      out  float [3][np] (double for PT_F64), in the order pos
 *                 leaves in
 *   ws            >= pt_workspace_bytes(PT_OP_RK2, ...) bytes */
pt_status pt_rk2_stage1(const pt_grid *grid, const void *coeff_n, pt_dtype dtype,
                        int64_t np, double *pos, int32_t *ids, int sort, void *u_n,
                        void *ws, size_t ws_bytes, hipStream_t stream);

/* Stage 2, with the coefficients of u(., t_n + dt):
 *   x* = x + dt u_n;  x <- x + dt/2 (u_n + u^{n+1}(x*))
 * (FP64 positions, FP32 velocities (FP64 for PT_F64)), pos updated in place.  With sorted != 0
 * the particles are taken in the cell order of the stage 1 that sorted them,
 * and ws must be that call's workspace (same grid, np and size).  The table
 * it holds is checked on the device; a table that is not a partition of the
 * np particles (ws reused in between) makes every particle go through the
 * slower path that reads the coefficients from global memory, with the same
 * result.  Positions moved since stage 1 are handled the same way.
 *   coeff_np1  in   padded coefficients of the field at t_n + dt
 *   pos        in/out double [3][np]
 *   u_n        in   float [3][np] (double for PT_F64) from stage 1
 *   ws              >= pt_workspace_bytes(PT_OP_RK2, ...) bytes (unused when
 *                   sorted == 0, may then be NULL) */
pt_status pt_rk2_stage2(const pt_grid *grid, const void *coeff_np1, pt_dtype dtype,
                        int64_t np, double dt, double *pos, const void *u_n, int sorted,
                        void *ws, size_t ws_bytes, hipStream_t stream);

/* Inertial or diffusive particles (Sec. 4.3: inertial particles, and
 * markers of high molecular diffusivity, can move more than one grid spacing
 * per step; the paper gives no equation for them).  One step h = dt of the
 * Stokes-drag particle
 *   dx/dt = v,   dv/dt = (u(x) - v) / tau
 * solved exactly with the fluid velocity seen over the step taken as linear
 * in time from u0 = u(x) to u1 = u(x*), where x* is the end point of the
 * exact solution with the fluid velocity held at u0 (an exponential-integrator
 * form of Heun's predictor-corrector).  With r = dt/tau, E = exp(-r),
 * p1 = (1 - E)/r, p2 = (1 - p1)/r:
 *   x* = x + dt p1 v + dt (1 - p1) u0 + d
 *   x <- x* + dt (1/2 - p2) (u1 - u0)
 *   v <- E v + (p1 - E) u0 + (1 - p1) u1
 * tau = 0 is the fluid tracer (Heun's step of pt_rk2_step, v not used);
 * d is an optional displacement increment per particle, e.g. the random step
 * sqrt(2 kappa dt) xi of a diffusive marker, drawn by the caller.  Steps may
 * move particles any number of cells: a particle whose predicted point leaves
 * its column's tile is evaluated from global memory.
 *   dt > 0, tau >= 0 (finite), else PT_ERR_ARG
 *   pos   in/out double [3][np], unwrapped
 *   vel   in/out float [3][np] (double for PT_F64); may be NULL only if
 *              tau = 0 (then neither read nor written)
 *   disp  in     double [3][np] in the input order, or NULL (no increment)
 *   ids   in/out int32 [np] or NULL
 *   sort  as for pt_rk2_step; with PT_SORT, pos, vel and ids come back in
 *         cell order
 *   ws          >= pt_workspace_bytes(PT_OP_INERTIAL, ...) bytes */
pt_status pt_inertial_step(const pt_grid *grid, const void *coeff, pt_dtype dtype, int64_t np,
                           double dt, double tau, double *pos, void *vel, const double *disp,
                           int32_t *ids, int sort, void *ws, size_t ws_bytes,
                           hipStream_t stream);

/* Adjoint of pt_interp_uvw (not in the paper).  With gu = dL/d(u,v,w):
 *   g_pos[d][p]  += sum_c gu[c][p] du_c/dx_d (p)          (may be NULL)
 *   g_coeff[c][.] += b_i c_j d_k gu[c][p] over each stencil (may be NULL),
 * g_coeff is FP32 in the padded layout whatever the coefficient dtype (a
 * BF16 coefficient is treated as its FP32 value: straight-through).  The
 * scatter uses FP32 atomics, so its summation order is not fixed. */
pt_status pt_interp_uvw_bwd(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                            int64_t np, const double *pos, const float *g_out,
                            double *g_pos, float *g_coeff, hipStream_t stream);

/* Adjoint of pt_spline_coeffs.  Each padded coefficient gradient is folded
 * onto the grid line it copies, then the transposed line solves are applied
 * (the 1-4-1 periodic matrix is symmetric, so they are the same solves; they
 * commute): fold, y and x in one pass where rows have 256, 512 or 1024 points
 * and the y lines split into whole chunks, else x (fused with the fold) and
 * y; then z.  g_coeff float [3][nz+3][ny+3][nx+3] in (not modified; must not
 * overlap g_field, which also holds intermediate values during the call);
 * g_field float [3][nz][ny][nx] out (overwritten). */
pt_status pt_spline_coeffs_bwd(const pt_grid *grid, const float *g_coeff, float *g_field,
                               void *ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint of one pt_rk2_step.  pos_n: the positions the step started from
 * (in the step's input order); sort: as given to the forward step (with
 * PT_SORTED, pos_n in cell order and g_pos in that order).
 * g_pos: on entry dL/d(output positions) in the step's output order, on exit
 * dL/d(pos_n) in the input order.  g_coeff (may be NULL) accumulates dL/dS.
 *   x*b = J(x*)^T (dt/2) lam;  u0b = dt/2 lam + dt x*b;
 *   x^n b = lam + x*b + J(x^n)^T u0b;  g_coeff += W(x*)^T (dt/2) lam + W(x^n)^T u0b. */
pt_status pt_rk2_step_bwd(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                          int64_t np, double dt, const double *pos_n, int sort,
                          double *g_pos, float *g_coeff, void *ws, size_t ws_bytes,
                          hipStream_t stream);

/* The Heun step of eq. (dxdt) (Sec. 4.3) on particles in cell order, as
 * pt_rk2_step_out with PT_SORTED, that also keeps what its adjoint needs, for
 * a caller that runs the adjoint after it (not in the paper): the velocity
 * u0 = u(x_n) and the velocity gradients du_c/dx_d (the 64-term sums of
 * Operation 3 of Sec. 2.2) at x_n and at the predictor x* = x_n + dt u0.
 * The forward then evaluates values and gradients at both stage points and
 * pt_rk2_step_bwd_saved needs no gather of its own.  pos_out equals the
 * output of pt_rk2_step_out to rounding (the same formulas; the values come
 * from the gradient evaluation).  PT_F32 and PT_BF16 coefficients only
 * (PT_ERR_UNSUPPORTED for PT_F64).
 *   pos_in   in   double [3][np], in cell order
 *   pos_out  out  double [3][np]; may be pos_in, else must not overlap it
 *   saved    out  float [21][np]: rows 0-2 u0; row 3 + 3c + d du_c/dx_d at
 *                 x_n; row 12 + 3c + d du_c/dx_d at x*; must not overlap
 *                 pos_in or pos_out
 *   ws            >= pt_workspace_bytes(PT_OP_RK2, ...) bytes */
pt_status pt_rk2_step_save(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                           int64_t np, double dt, const double *pos_in, double *pos_out,
                           float *saved, void *ws, size_t ws_bytes, hipStream_t stream);

/* The Heun step of eq. (dxdt) (Sec. 4.3) on particles in cell order, as
 * pt_rk2_step_out with PT_SORTED, that also returns (u, v, w) and the nine
 * velocity gradients at x_n (Operations 2 and 3 of Sec. 2.2: the velocity
 * gradients need the twice-differentiable interpolant) from the same pass
 * over the coefficients, as pt_interp_sorted with nout = 12 would.  pos_out
 * equals the output of pt_rk2_step_out to rounding.  PT_F32 and PT_BF16
 * coefficients only (PT_ERR_UNSUPPORTED for PT_F64).
 *   pos_in   in   double [3][np], in cell order
 *   pos_out  out  double [3][np]; may be pos_in, else must not overlap it
 *   out      out  float [12][np]: rows u, v, w, then du_c/dx_d at 3 + 3c + d;
 *                 must not overlap pos_in or pos_out
 *   ws            >= pt_workspace_bytes(PT_OP_RK2, ...) bytes */
pt_status pt_rk2_step_grad(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                           int64_t np, double dt, const double *pos_in, double *pos_out,
                           float *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint of pt_rk2_step_save from what it kept: the arithmetic of
 * pt_rk2_step_bwd with PT_SORTED (same formulas, with J(x^n) and J(x*) read
 * from saved instead of gathered); no coefficients are read.
 *   pos_n   in      double [3][np]: pos_in of the forward call (cell order)
 *   saved   in      float [21][np] written by that call
 *   g_pos   in/out  double [3][np]: dL/d(pos_out) in, dL/d(pos_n) out
 *   g_coeff in/out  float [3][nz+3][ny+3][nx+3], accumulates dL/dS (may be NULL)
 *   ws              >= pt_workspace_bytes(PT_OP_RK2_BWD, grid, PT_F32, np) bytes */
pt_status pt_rk2_step_bwd_saved(const pt_grid *grid, int64_t np, double dt,
                                const double *pos_n, const float *saved, double *g_pos,
                                float *g_coeff, void *ws, size_t ws_bytes, hipStream_t stream);

/* pt_rk2_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same step, with the same kernels and results, without a caller
 * workspace.  Its scratch is a static device array of the library, 64 MiB per
 * device (PT_NOALLOC_SCRATCH_BYTES), held until the process ends; the call
 * itself allocates nothing (with kernel timing, pt_timing_enable, off).
 *   sort  PT_UNSORTED (scratch: 12 bytes per particle, 24 for PT_F64) or
 *         PT_SORTED (scratch: the particle table, 8 bytes per particle and the
 *         work items); PT_SORT needs the sort's workspace: PT_ERR_ARG
 *   pos   in/out double [3][np]
 * Returns PT_ERR_WORKSPACE when the step needs more scratch than the array
 * holds (more than about 5.5M particles unsorted in FP32, or about 7M sorted
 * on a 1024^3 grid).  Every call on a device uses that device's one array: calls that
 * overlap on one device (several streams, several host threads) race; calls
 * in one stream order are safe, since each call writes every scratch word it
 * reads before reading it. */
#define PT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pt_status pt_rk2_step_noalloc(const pt_grid *grid, const void *coeff, pt_dtype dtype,
                              int64_t np, double dt, double *pos, int sort,
                              hipStream_t stream);

/* One device's part of the particle migration between sub-domains
 * (Sec. 4.3): with the grid split into z-slabs, the particles that left this
 * device's slab [z0, z0 + nzl) (cells modulo nz) are separated from the ones
 * that stay, with all their attributes, and the gaps are closed.  The output
 * is one stable partition [stay | lower | upper]: each particle's group comes
 * from its shadow z cell c (as in pt_sort_particles), rel = (c - z0) mod nz;
 * rel < nzl stays, otherwise it goes to the neighbouring slab below if
 * nz - rel <= rel - nzl + 1 (the nearer side, ties below), else above.
 * Inside each group the input order is kept.
 *   pos      in   double [3][np];  ids  in int32 [np] or NULL
 *   z0, nzl  in   0 <= z0 < nz, 1 <= nzl <= nz
 *   pos_out  out  double [3][np], must not overlap pos
 *   ids_out  out  int32 [np] (not read when ids is NULL)
 *   counts   out  int64 [3] in device memory: stay, lower, upper
 *   ws            >= pt_workspace_bytes(PT_OP_SLAB_PARTITION, ...) bytes
 * A non-finite position keeps its particle in the slab and sets the flag
 * pt_last_device_error() reports. */
pt_status pt_slab_partition(const pt_grid *grid, int64_t np, const double *pos,
                            const int32_t *ids, int32_t z0, int32_t nzl, double *pos_out,
                            int32_t *ids_out, int64_t *counts, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* Diagnostics: the number of particles (PT_OP_RK2, PT_OP_INERTIAL,
 * PT_OP_INTERP_SORTED) or of particles plus stencils (PT_OP_RK2_BWD, whose
 * list is reused by the scatter) that the last column-tiled call on this
 * workspace sent to the global-memory path (a predicted point outside its
 * column's tile).  Synchronises the device; grid, dtype and np as given to
 * that call.  Other ops return PT_ERR_ARG. */
pt_status pt_tiled_deferred(int op, const pt_grid *grid, pt_dtype dtype, int64_t np,
                            const void *ws, int64_t *count);

/* Synchronises `stream`, then returns PT_ERR_NONFINITE if any kernel on the
 * current device met a non-finite position since the previous call (and
 * clears the flag), PT_ERR_HIP on a runtime error, else PT_OK. */
pt_status pt_last_device_error(hipStream_t stream);

/* Static description of a status code. */
const char *pt_status_string(pt_status status);

/* Kernel timing (diagnostics, not on the hot path).  While enabled, the
 * library brackets each launch of its main kernels with a pair of HIP events
 * recorded on the launch stream.  pt_timing_read synchronises on the events
 * of `kernel`, returns their summed elapsed time and count, and forgets them.
 * Kernel names: "spline_x", "spline_y", "spline_z", "spline_x_pad" (the x
 * pass that writes the padded coefficients), "spline_x_fold" (the adjoint's
 * x pass that reads the padded gradient), "spline_y_carry" and
 * "spline_yx_pad" (the forward's fused y + x pass and the y pass that feeds
 * it its carries), "spline_fold_y_carry" and "spline_fyx" (the adjoint's
 * fused fold + y + x pass and the folded y pass that feeds it its carries),
 * "tile_rk2_fwd_save" and "rk2_bwd_saved" (pt_rk2_step_save and the first
 * kernel of pt_rk2_step_bwd_saved), "tile_rk2_fwd_grad" (pt_rk2_step_grad),
 * "sort_keys", "sort_pass", "sort_permute",
 * "sorted_table" (the particle table of PT_SORTED), "slab_partition",
 * "tile_rk2_fwd",
 * "tile_rk2_bwd_gather", "tile_scatter", "tile_tv_stage1", "tile_tv_stage2",
 * "tile_inertial", "tile_interp", "tile_interp_grad", "inertial_direct",
 * "interp", "rk2_direct_stage2", "rk2_direct_bwd", "rk2_direct_bwd_gather". */
pt_status pt_timing_enable(int on);
pt_status pt_timing_read(const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* PT_SPLINE_H */
