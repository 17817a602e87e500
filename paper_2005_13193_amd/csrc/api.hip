// C ABI entry points: host-side argument validation, workspace carving and
// dispatch to the kernels of solve.hip, sort.hip, gather.hip and tile.hip.
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "pt_common.h"
#include "pt_inertial.h"

namespace pt {

// solve.hip
size_t spline_ws_floats(const pt_grid* g, pt_dtype dtype);
size_t spline_slab_ws_floats(const pt_grid* g, int nzl, int W, pt_dtype dtype);
pt_status spline_slab_fwd(const pt_grid* g, int nzl, int W, const float* field, void* coeff,
                          pt_dtype dtype, float* ws, hipStream_t s);
pt_status spline_fwd(const pt_grid* g, const float* field, void* coeff, pt_dtype dtype, float* ws,
                     hipStream_t s);
pt_status spline_bwd(const pt_grid* g, const float* gcoeff, float* gfield, float* ws,
                     hipStream_t s);
// sort.hip
int key_bits(const pt_grid* g);
size_t sort_ws_bytes(const pt_grid* g, int64_t np);
pt_status presorted_table(const pt_grid* g, int64_t np, const double* pos, int32_t* lstart,
                          hipStream_t s);
pt_status sort_particles(const pt_grid* g, int64_t np, const double* pos, double* pos_sorted,
                         int32_t* perm, uint64_t* keys_out, int32_t* lstart, void* ws,
                         hipStream_t s);
pt_status permute_ids(int64_t np, const int32_t* in, const int32_t* perm, int32_t* out,
                      hipStream_t s);
pt_status permute_rows(int64_t np, const void* in, int elem_bytes, const int32_t* perm, void* out,
                       hipStream_t s);
// gather.hip (value arrays: float, or double for PT_F64)
pt_status interp_fwd(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np,
                     const double* pos, void* out, int nout, hipStream_t s);
pt_status rk2_advance(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np, double dt,
                      const double* x, double* x_out, void* u0, hipStream_t s);
pt_status inertial_advance(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np,
                           const InertialCoef& k, const double* x, const void* v,
                           const double* disp, double* x_out, void* v_out, hipStream_t s);
pt_status interp_bwd(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np,
                     const double* pos, const float* gout, double* gpos, float* gcoeff,
                     hipStream_t s);
pt_status rk2_backward(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np, double dt,
                       const double* x, const double* lam, double* out, float* gcoeff, void* u0,
                       double* xbs, hipStream_t s);
pt_status scatter_back(int64_t np, const double* in, const int32_t* perm, double* out,
                       hipStream_t s);
pt_status rk2_bwd_gather(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np,
                        double dt, const double* x, const double* lam, double* xbn, float* u0f,
                        float* ub0f, float* ub1f, int* umax, hipStream_t s);
pt_status rk2_correct(const pt_grid* g, const void* coeff, pt_dtype dtype, int64_t np, double dt,
                      const double* x, const void* u0, double* x_out, hipStream_t s);
// tile.hip
int64_t tile_nlayers(const pt_grid* g);
pt_status tile_rk2_fwd(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                       int64_t np, double dt, const double* x, double* x_out, void* defer,
                       void* items_ws, bool check, hipStream_t s);
size_t tile_items_bytes(const pt_grid* g, int64_t np, bool scatter);
pt_status tile_rk2_fwd_save(const pt_grid* g, const void* coeff, pt_dtype dtype,
                            const int32_t* ls, int64_t np, double dt, const double* x,
                            double* x_out, float* saved, void* defer, void* items_ws, bool check,
                            hipStream_t s);
pt_status tile_rk2_fwd_grad(const pt_grid* g, const void* coeff, pt_dtype dtype,
                            const int32_t* ls, int64_t np, double dt, const double* x,
                            double* x_out, float* out, void* defer, void* items_ws, bool check,
                            hipStream_t s);
pt_status tile_rk2_bwd_saved(const pt_grid* g, const int32_t* ls, int64_t np, double dt,
                             const double* x, const float* saved, double* lam, float* ub0,
                             float* ub1, float* gcoeff, void* defer, void* items_ws,
                             hipStream_t s);
pt_status tile_rk2_bwd(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                       int64_t np, double dt, const double* x, const double* lam, double* xbn,
                       float* u0, float* ub0, float* ub1, float* gcoeff, void* defer,
                       void* items_ws, bool check, hipStream_t s);
size_t tile_defer_bytes(int64_t np);
pt_status tile_defer_reset(void* defer, hipStream_t s);
int* tile_umax_slots(void* defer);
pt_status tile_scatter_only(const pt_grid* g, const int32_t* ls, int64_t np, double dt,
                            const double* x, float* u0, float* ub0, float* ub1, float* gcoeff,
                            void* defer, void* items_ws, bool check, hipStream_t s);
pt_status tile_interp(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                      int64_t np, const double* x, int nout, float* out, void* defer,
                      void* items_ws, hipStream_t s);
pt_status tile_inertial(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                        int64_t np, const InertialCoef& k, const double* x, const float* v,
                        const double* disp, double* x_out, float* v_out, void* defer,
                        void* items_ws, bool check, hipStream_t s);
// migrate.hip
size_t slab_partition_ws_bytes(int64_t np);
pt_status slab_partition(const pt_grid* grid, int64_t np, const double* pos, const int32_t* ids,
                         int z0, int nzl, double* pos_out, int32_t* ids_out, int64_t* counts,
                         void* ws, hipStream_t s);
pt_status tile_tv_stage1(const pt_grid* g, const void* coeff, pt_dtype dtype, const int32_t* ls,
                         int64_t np, const double* x, double* x_out, float* u_n, void* defer,
                         void* items_ws, hipStream_t s);
pt_status tile_tv_stage2(const pt_grid* g, const void* coeff, pt_dtype dtype, int32_t* ls,
                         int64_t np, double dt, const double* x, const float* u_n, double* x_out,
                         void* defer, void* items_ws, hipStream_t s);

// One non-finite-position flag per device, in the library's static device
// memory; kernels receive its device address.
static __device__ int g_error_flag;

constexpr int kMaxDevices = 64;
static int* g_flag_ptr[kMaxDevices];
static std::mutex g_flag_mu;

int* device_error_flag() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_flag_mu);
  if (!g_flag_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_error_flag)) != hipSuccess) return nullptr;
    g_flag_ptr[dev] = (int*)p;
  }
  return g_flag_ptr[dev];
}

// ------------------------------------------------- no-allocation scratch ---
// Scratch of pt_rk2_step_noalloc: one array per device in the library's
// static device memory, held until the process ends.  Host code must not pass
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): its device address is looked up once per device, with that device
// current, and kept here.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static void* g_scratch_ptr[kMaxDevices];

static void* noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_flag_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// ------------------------------------------------------------- timing ---
struct TimingRec {
  std::string name;
  hipEvent_t start, stop;
};
static std::mutex g_time_mu;
static bool g_time_on = false;
static std::vector<TimingRec> g_time_recs;

bool timing_on() {
  std::lock_guard<std::mutex> lock(g_time_mu);
  return g_time_on;
}

void timing_record(const char* name, hipEvent_t start, hipEvent_t stop) {
  std::lock_guard<std::mutex> lock(g_time_mu);
  g_time_recs.push_back({name, start, stop});
}

static inline size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// Coefficients of the inertial step (pt_inertial.h) for h > 0, tau >= 0.
// With r = h / tau: p1 = (1 - e^-r)/r from expm1 (no cancellation), and
// 1/2 - p2 = 1/2 - (1 - p1)/r, which cancels for small r, from its Taylor
// series sum_{j>=1} (-1)^(j+1) r^j / (j+2)! there (Horner, 18 terms: below
// 1e-20 relative for r < 0.5).
InertialCoef inertial_coef(double h, double tau) {
  InertialCoef k;
  if (tau == 0.0) {
    k.cv = 0.0; k.cu = h; k.cc = 0.5 * h; k.E = 0.0; k.bu0 = 0.0; k.b = 1.0;
    return k;
  }
  const double r = h / tau;
  const double E = exp(-r);
  const double p1 = r > 0.0 ? -expm1(-r) / r : 1.0;
  double half_minus_p2;
  if (r < 0.5) {
    // sum_{j=1..18} (-1)^(j+1) r^j / (j+2)!, from the highest term down
    double acc = 0.0;
    for (int j = 18; j >= 1; --j) {
      double f = 1.0;  // 1 / (j+2)!
      for (int q = 2; q <= j + 2; ++q) f /= (double)q;
      acc = acc * r + ((j & 1) ? f : -f);
    }
    half_minus_p2 = acc * r;
  } else {
    half_minus_p2 = 0.5 - (1.0 - p1) / r;
  }
  k.cv = h * p1;
  k.cu = h * (1.0 - p1);
  k.cc = h * half_minus_p2;
  k.E = E;
  k.bu0 = p1 - E;
  k.b = 1.0 - p1;
  return k;
}

static pt_status check_grid(const pt_grid* g) {
  if (!g) return PT_ERR_NULL;
  const int n[3] = {g->nx, g->ny, g->nz};
  const double L[3] = {g->lx, g->ly, g->lz};
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 4) return PT_ERR_SIZE;
    if (!(L[d] > 0.0) || !isfinite(L[d])) return PT_ERR_SIZE;
  }
  for (int d = 0; d < 3; ++d)
    if (n[d] > 8192) return PT_ERR_UNSUPPORTED;
  return PT_OK;
}

static pt_status check_np(int64_t np) {
  if (np < 0 || np > (int64_t)0x7fffffff) return PT_ERR_SIZE;
  return PT_OK;
}

// The column-tiled kernels count deferred stencils (up to 2 np) in 32-bit
// signed words, so they take fewer than 2^30 particles per call.
static pt_status check_tiled_np(int64_t np) {
  return np >= ((int64_t)1 << 30) ? PT_ERR_UNSUPPORTED : PT_OK;
}

static pt_status check_dtype(pt_dtype d) {
  return (d == PT_F32 || d == PT_BF16 || d == PT_F64) ? PT_OK : PT_ERR_DTYPE;
}

// The column-tiled kernels stage FP32 or BF16 coefficients; FP64 storage
// takes the one-thread-per-particle gathers on the sorted particles.
static bool tiled(pt_dtype d) { return d != PT_F64; }

static pt_status ready() { return device_error_flag() ? PT_OK : PT_ERR_HIP; }

#define PT_TRY(expr)                  \
  do {                                \
    pt_status st_ = (expr);           \
    if (st_ != PT_OK) return st_;     \
  } while (0)

// ------------------------------------------------------ workspace sizes ---
static size_t lstart_bytes(const pt_grid* g) { return 4 * (size_t)(tile_nlayers(g) + 1); }

struct Rk2Ws {
  void* sort;
  double* pos_sorted;
  int32_t* perm;
  int32_t* ids_tmp;
  void* u0;          // 3 np values (float, double for PT_F64)
  int32_t* lstart;
  void* defer;
  void* items;
  void* vel_sorted;  // inertial step: 3 np values
  double* disp_sorted;  // inertial step: 3 np doubles
};

static size_t rk2_ws_bytes(const pt_grid* g, int64_t np, pt_dtype dt) {
  return a256(sort_ws_bytes(g, np)) + a256(24 * (size_t)np) + 2 * a256(4 * (size_t)np) +
         a256(3 * value_bytes(dt) * (size_t)np) + a256(lstart_bytes(g)) +
         a256(tile_defer_bytes(np)) + a256(tile_items_bytes(g, np, false));
}

static size_t inertial_ws_bytes(const pt_grid* g, int64_t np, pt_dtype dt) {
  return rk2_ws_bytes(g, np, dt) + a256(3 * value_bytes(dt) * (size_t)np) +
         a256(24 * (size_t)np);
}

static Rk2Ws carve_rk2(const pt_grid* g, int64_t np, pt_dtype dt, void* ws) {
  char* p = (char*)ws;
  Rk2Ws w;
  w.sort = p; p += a256(sort_ws_bytes(g, np));
  w.pos_sorted = (double*)p; p += a256(24 * (size_t)np);
  w.perm = (int32_t*)p; p += a256(4 * (size_t)np);
  w.ids_tmp = (int32_t*)p; p += a256(4 * (size_t)np);
  w.u0 = p; p += a256(3 * value_bytes(dt) * (size_t)np);
  w.lstart = (int32_t*)p; p += a256(lstart_bytes(g));
  w.defer = p; p += a256(tile_defer_bytes(np));
  w.items = p; p += a256(tile_items_bytes(g, np, false));
  // inertial step only (inertial_ws_bytes)
  w.vel_sorted = p; p += a256(3 * value_bytes(dt) * (size_t)np);
  w.disp_sorted = (double*)p;
  return w;
}

struct Rk2BwdWs {
  void* sort;
  double* pos_sorted;
  int32_t* perm;
  double* xbn;
  double* xbs;   // direct path; the tiled paths keep ub1 (12 bytes/particle) here
  void* u0;      // 3 np values (float, double for PT_F64)
  float* ub0;
  int32_t* lstart;
  void* defer;
  void* items;
};

static size_t rk2_bwd_ws_bytes(const pt_grid* g, int64_t np, pt_dtype dt) {
  return a256(sort_ws_bytes(g, np)) + 3 * a256(24 * (size_t)np) + a256(4 * (size_t)np) +
         a256(3 * value_bytes(dt) * (size_t)np) + a256(12 * (size_t)np) + a256(lstart_bytes(g)) +
         a256(tile_defer_bytes(np)) + a256(tile_items_bytes(g, np, false)) +
         a256(tile_items_bytes(g, np, true));
}

static Rk2BwdWs carve_rk2_bwd(const pt_grid* g, int64_t np, pt_dtype dt, void* ws) {
  char* p = (char*)ws;
  Rk2BwdWs w;
  w.sort = p; p += a256(sort_ws_bytes(g, np));
  w.pos_sorted = (double*)p; p += a256(24 * (size_t)np);
  w.xbn = (double*)p; p += a256(24 * (size_t)np);
  w.xbs = (double*)p; p += a256(24 * (size_t)np);
  w.perm = (int32_t*)p; p += a256(4 * (size_t)np);
  w.u0 = p; p += a256(3 * value_bytes(dt) * (size_t)np);
  w.ub0 = (float*)p; p += a256(12 * (size_t)np);
  w.lstart = (int32_t*)p; p += a256(lstart_bytes(g));
  w.defer = p; p += a256(tile_defer_bytes(np));
  w.items = p;
  return w;
}

}  // namespace pt

using namespace pt;

extern "C" {

pt_status pt_workspace_bytes(int op, const pt_grid* grid, pt_dtype dtype, int64_t np,
                             size_t* bytes) {
  if (!bytes) return PT_ERR_NULL;
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  if (op != PT_OP_SPLINE && op != PT_OP_SPLINE_BWD) PT_TRY(check_np(np));
  if (op == PT_OP_SPLINE_SLAB && (np < 6 || np > 8192)) return PT_ERR_SIZE;
  const size_t n3 = (size_t)grid->nx * grid->ny * grid->nz;
  switch (op) {
    case PT_OP_SPLINE: *bytes = a256(4 * spline_ws_floats(grid, dtype)); break;
    case PT_OP_SPLINE_BWD: *bytes = a256(4 * n3); break;
    case PT_OP_SORT: *bytes = a256(sort_ws_bytes(grid, np)) + a256(4 * (size_t)np); break;
    case PT_OP_RK2: *bytes = a256(rk2_ws_bytes(grid, np, dtype)); break;
    case PT_OP_RK2_BWD: *bytes = a256(rk2_bwd_ws_bytes(grid, np, dtype)); break;
    case PT_OP_INERTIAL: *bytes = a256(inertial_ws_bytes(grid, np, dtype)); break;
    case PT_OP_INTERP_SORTED:
      *bytes = a256(lstart_bytes(grid)) + a256(tile_defer_bytes(np)) +
               a256(tile_items_bytes(grid, np, false));
      break;
    // np = input planes of the slab, nzl + 3 + 2 W
    case PT_OP_SPLINE_SLAB:
      *bytes = a256(4 * spline_slab_ws_floats(grid, (int)np - 3, 0, dtype));
      break;
    case PT_OP_SLAB_PARTITION: *bytes = a256(slab_partition_ws_bytes(np)); break;
    default: return PT_ERR_ARG;
  }
  return PT_OK;
}

pt_status pt_key_layout(const pt_grid* grid, int32_t* tile_x, int32_t* tile_y, int32_t* bits) {
  PT_TRY(check_grid(grid));
  if (!tile_x || !tile_y || !bits) return PT_ERR_NULL;
  *tile_x = kTileX;
  *tile_y = kTileY;
  *bits = key_bits(grid);
  return PT_OK;
}

pt_status pt_spline_coeffs(const pt_grid* grid, const float* field, void* coeff, pt_dtype dtype,
                           void* ws, size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  if (!field || !coeff) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_SPLINE, grid, dtype, 0, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  return spline_fwd(grid, field, coeff, dtype, (float*)ws, stream);
}

pt_status pt_spline_coeffs_slab(const pt_grid* grid, int32_t nzl, int32_t halo,
                                const float* field, void* coeff, pt_dtype dtype, void* ws,
                                size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  if (nzl < 1 || nzl > grid->nz || halo < 1 || halo > 64) return PT_ERR_SIZE;
  const int64_t nzi = (int64_t)nzl + 3 + 2 * (int64_t)halo;
  if (nzi > 8192) return PT_ERR_UNSUPPORTED;
  if (!field || !coeff) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_SPLINE_SLAB, grid, dtype, nzi, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  return spline_slab_fwd(grid, nzl, halo, field, coeff, dtype, (float*)ws, stream);
}

pt_status pt_spline_coeffs_bwd(const pt_grid* grid, const float* g_coeff, float* g_field, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  if (!g_coeff || !g_field) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_SPLINE_BWD, grid, PT_F32, 0, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  return spline_bwd(grid, g_coeff, g_field, (float*)ws, stream);
}

pt_status pt_sort_particles(const pt_grid* grid, int64_t np, const double* pos, double* pos_sorted,
                            int32_t* perm, int32_t* ids, uint64_t* keys_out, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_np(np));
  if (np == 0) return PT_OK;
  if (!pos || !perm) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_SORT, grid, PT_F32, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  PT_TRY(sort_particles(grid, np, pos, pos_sorted, perm, keys_out, nullptr, ws, stream));
  if (!ids) return PT_OK;
  // the labels' staging buffer sits after the sort's own workspace
  int32_t* ids_tmp = (int32_t*)((char*)ws + a256(sort_ws_bytes(grid, np)));
  PT_TRY(permute_ids(np, ids, perm, ids_tmp, stream));
  PT_HIP_CHECK(hipMemcpyAsync(ids, ids_tmp, 4 * (size_t)np, hipMemcpyDeviceToDevice, stream));
  return PT_OK;
}

pt_status pt_slab_partition(const pt_grid* grid, int64_t np, const double* pos,
                            const int32_t* ids, int32_t z0, int32_t nzl, double* pos_out,
                            int32_t* ids_out, int64_t* counts, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_np(np));
  if (z0 < 0 || z0 >= grid->nz || nzl < 1 || nzl > grid->nz) return PT_ERR_ARG;
  if (!counts) return PT_ERR_NULL;
  if (np > 0 && (!pos || !pos_out || (ids && !ids_out))) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_SLAB_PARTITION, grid, PT_F32, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  if (np > 0 && pos_out < pos + 3 * np && pos < pos_out + 3 * np) return PT_ERR_ARG;
  PT_TRY(ready());
  return slab_partition(grid, np, pos, ids, z0, nzl, pos_out, ids_out, counts, ws, stream);
}

pt_status pt_interp_uvw(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                        const double* pos, void* out, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (np == 0) return PT_OK;
  if (!coeff || !pos || !out) return PT_ERR_NULL;
  PT_TRY(ready());
  return interp_fwd(grid, coeff, dtype, np, pos, out, 3, stream);
}

pt_status pt_interp_grad(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                         const double* pos, void* out, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (np == 0) return PT_OK;
  if (!coeff || !pos || !out) return PT_ERR_NULL;
  PT_TRY(ready());
  return interp_fwd(grid, coeff, dtype, np, pos, out, 12, stream);
}

pt_status pt_interp_sorted(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                           const double* pos, int nout, void* out, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (nout != 3 && nout != 12) return PT_ERR_ARG;
  PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!coeff || !pos || !out) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_INTERP_SORTED, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  if (!tiled(dtype)) return interp_fwd(grid, coeff, dtype, np, pos, out, nout, stream);
  char* p = (char*)ws;
  int32_t* lstart = (int32_t*)p;
  void* defer = p + a256(lstart_bytes(grid));
  void* items = (char*)defer + a256(tile_defer_bytes(np));
  PT_TRY(presorted_table(grid, np, pos, lstart, stream));
  return tile_interp(grid, coeff, dtype, lstart, np, pos, nout, (float*)out, defer, items,
                     stream);
}

pt_status pt_rk2_step(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                      double dt, double* pos, int32_t* ids, int sort, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!isfinite(dt)) return PT_ERR_ARG;
  if (sort != PT_UNSORTED && sort != PT_SORT && sort != PT_SORTED) return PT_ERR_ARG;
  if (sort != PT_UNSORTED) PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!coeff || !pos) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_RK2, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  Rk2Ws w = carve_rk2(grid, np, dtype, ws);
  if (sort == PT_SORT) {
    PT_TRY(sort_particles(grid, np, pos, w.pos_sorted, w.perm, nullptr, w.lstart, w.sort,
                          stream));
    if (ids) {
      PT_TRY(permute_ids(np, ids, w.perm, w.ids_tmp, stream));
      PT_HIP_CHECK(hipMemcpyAsync(ids, w.ids_tmp, 4 * (size_t)np, hipMemcpyDeviceToDevice, stream));
    }
    if (!tiled(dtype))
      return rk2_advance(grid, coeff, dtype, np, dt, w.pos_sorted, pos, w.u0, stream);
    return tile_rk2_fwd(grid, coeff, dtype, w.lstart, np, dt, w.pos_sorted, pos, w.defer, w.items,
                        false, stream);
  }
  if (sort == PT_SORTED && tiled(dtype)) {
    PT_TRY(presorted_table(grid, np, pos, w.lstart, stream));
    return tile_rk2_fwd(grid, coeff, dtype, w.lstart, np, dt, pos, pos, w.defer, w.items, true,
                        stream);
  }
  return rk2_advance(grid, coeff, dtype, np, dt, pos, pos, w.u0, stream);
}

pt_status pt_rk2_step_out(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                          double dt, const double* pos_in, double* pos_out, int sort, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!isfinite(dt)) return PT_ERR_ARG;
  if (sort != PT_UNSORTED && sort != PT_SORTED) return PT_ERR_ARG;
  if (sort == PT_SORTED) PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!coeff || !pos_in || !pos_out) return PT_ERR_NULL;
  if (pos_out != pos_in && pos_out < pos_in + 3 * np && pos_in < pos_out + 3 * np)
    return PT_ERR_ARG;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_RK2, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  Rk2Ws w = carve_rk2(grid, np, dtype, ws);
  if (sort == PT_SORTED && tiled(dtype)) {
    PT_TRY(presorted_table(grid, np, pos_in, w.lstart, stream));
    return tile_rk2_fwd(grid, coeff, dtype, w.lstart, np, dt, pos_in, pos_out, w.defer,
                        w.items, true, stream);
  }
  return rk2_advance(grid, coeff, dtype, np, dt, pos_in, pos_out, w.u0, stream);
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char *pa = (const char*)a, *pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

pt_status pt_rk2_step_save(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                           double dt, const double* pos_in, double* pos_out, float* saved,
                           void* ws, size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!isfinite(dt)) return PT_ERR_ARG;
  PT_TRY(check_tiled_np(np));
  if (!tiled(dtype)) return PT_ERR_UNSUPPORTED;
  if (np == 0) return PT_OK;
  if (!coeff || !pos_in || !pos_out || !saved) return PT_ERR_NULL;
  const size_t pb = 24 * (size_t)np, sb = 84 * (size_t)np;
  if ((pos_out != pos_in && overlaps(pos_out, pb, pos_in, pb)) ||
      overlaps(saved, sb, pos_in, pb) || overlaps(saved, sb, pos_out, pb))
    return PT_ERR_ARG;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_RK2, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  Rk2Ws w = carve_rk2(grid, np, dtype, ws);
  PT_TRY(presorted_table(grid, np, pos_in, w.lstart, stream));
  return tile_rk2_fwd_save(grid, coeff, dtype, w.lstart, np, dt, pos_in, pos_out, saved, w.defer,
                           w.items, true, stream);
}

pt_status pt_rk2_step_grad(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                           double dt, const double* pos_in, double* pos_out, float* out,
                           void* ws, size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!isfinite(dt)) return PT_ERR_ARG;
  PT_TRY(check_tiled_np(np));
  if (!tiled(dtype)) return PT_ERR_UNSUPPORTED;
  if (np == 0) return PT_OK;
  if (!coeff || !pos_in || !pos_out || !out) return PT_ERR_NULL;
  const size_t pb = 24 * (size_t)np, ob = 48 * (size_t)np;
  if ((pos_out != pos_in && overlaps(pos_out, pb, pos_in, pb)) ||
      overlaps(out, ob, pos_in, pb) || overlaps(out, ob, pos_out, pb))
    return PT_ERR_ARG;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_RK2, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  Rk2Ws w = carve_rk2(grid, np, dtype, ws);
  PT_TRY(presorted_table(grid, np, pos_in, w.lstart, stream));
  return tile_rk2_fwd_grad(grid, coeff, dtype, w.lstart, np, dt, pos_in, pos_out, out, w.defer,
                           w.items, true, stream);
}

pt_status pt_rk2_step_bwd_saved(const pt_grid* grid, int64_t np, double dt, const double* pos_n,
                                const float* saved, double* g_pos, float* g_coeff, void* ws,
                                size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_np(np));
  if (!isfinite(dt)) return PT_ERR_ARG;
  PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!pos_n || !saved || !g_pos) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_RK2_BWD, grid, PT_F32, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  Rk2BwdWs w = carve_rk2_bwd(grid, np, PT_F32, ws);
  PT_TRY(presorted_table(grid, np, pos_n, w.lstart, stream));
  return tile_rk2_bwd_saved(grid, w.lstart, np, dt, pos_n, saved, g_pos, w.ub0, (float*)w.xbs,
                            g_coeff, w.defer, w.items, stream);
}

pt_status pt_rk2_stage1(const pt_grid* grid, const void* coeff_n, pt_dtype dtype, int64_t np,
                        double* pos, int32_t* ids, int sort, void* u_n, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (sort) PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!coeff_n || !pos || !u_n) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_RK2, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  Rk2Ws w = carve_rk2(grid, np, dtype, ws);
  if (sort) {
    PT_TRY(sort_particles(grid, np, pos, w.pos_sorted, w.perm, nullptr, w.lstart, w.sort,
                          stream));
    if (ids) {
      PT_TRY(permute_ids(np, ids, w.perm, w.ids_tmp, stream));
      PT_HIP_CHECK(hipMemcpyAsync(ids, w.ids_tmp, 4 * (size_t)np, hipMemcpyDeviceToDevice, stream));
    }
    if (!tiled(dtype)) {
      PT_HIP_CHECK(hipMemcpyAsync(pos, w.pos_sorted, 24 * (size_t)np, hipMemcpyDeviceToDevice,
                                  stream));
      return interp_fwd(grid, coeff_n, dtype, np, pos, u_n, 3, stream);
    }
    return tile_tv_stage1(grid, coeff_n, dtype, w.lstart, np, w.pos_sorted, pos, (float*)u_n,
                          w.defer, w.items, stream);
  }
  return interp_fwd(grid, coeff_n, dtype, np, pos, u_n, 3, stream);
}

pt_status pt_rk2_stage2(const pt_grid* grid, const void* coeff_np1, pt_dtype dtype, int64_t np,
                        double dt, double* pos, const void* u_n, int sorted, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!isfinite(dt)) return PT_ERR_ARG;
  if (sorted) PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!coeff_np1 || !pos || !u_n) return PT_ERR_NULL;
  PT_TRY(ready());
  if (!sorted || !tiled(dtype))
    return rk2_correct(grid, coeff_np1, dtype, np, dt, pos, u_n, pos, stream);
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_RK2, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  Rk2Ws w = carve_rk2(grid, np, dtype, ws);
  return tile_tv_stage2(grid, coeff_np1, dtype, w.lstart, np, dt, pos, (const float*)u_n, pos,
                        w.defer, w.items, stream);
}

pt_status pt_interp_uvw_bwd(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                            const double* pos, const float* g_out, double* g_pos, float* g_coeff,
                            hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (np == 0 || (!g_pos && !g_coeff)) return PT_OK;
  if (!coeff || !pos || !g_out) return PT_ERR_NULL;
  PT_TRY(ready());
  return interp_bwd(grid, coeff, dtype, np, pos, g_out, g_pos, g_coeff, stream);
}

pt_status pt_rk2_step_bwd(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                          double dt, const double* pos_n, int sort, double* g_pos, float* g_coeff,
                          void* ws, size_t ws_bytes, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!isfinite(dt)) return PT_ERR_ARG;
  if (sort != PT_UNSORTED && sort != PT_SORT && sort != PT_SORTED) return PT_ERR_ARG;
  if (sort != PT_UNSORTED) PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!coeff || !pos_n || !g_pos) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_RK2_BWD, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  Rk2BwdWs w = carve_rk2_bwd(grid, np, dtype, ws);
  if (sort != PT_UNSORTED && !tiled(dtype)) {
    // FP64 storage: the gather half one thread per particle in FP64, then the
    // column-tiled scatter on the same (sorted) order
    const double* x = pos_n;
    double* xbn = g_pos;  // PT_SORTED: in place
    if (sort == PT_SORT) {
      PT_TRY(sort_particles(grid, np, pos_n, w.pos_sorted, w.perm, nullptr, w.lstart, w.sort,
                            stream));
      x = w.pos_sorted;
      xbn = w.xbn;
    } else {
      PT_TRY(presorted_table(grid, np, pos_n, w.lstart, stream));
    }
    PT_TRY(tile_defer_reset(w.defer, stream));
    PT_TRY(rk2_bwd_gather(grid, coeff, dtype, np, dt, x, g_pos, xbn, (float*)w.u0, w.ub0,
                          (float*)w.xbs, tile_umax_slots(w.defer), stream));
    if (g_coeff)
      PT_TRY(tile_scatter_only(grid, w.lstart, np, dt, x, (float*)w.u0, w.ub0, (float*)w.xbs,
                               g_coeff, w.defer, w.items, sort == PT_SORTED, stream));
    return sort == PT_SORT ? scatter_back(np, w.xbn, w.perm, g_pos, stream) : PT_OK;
  }
  if (sort == PT_SORT) {
    PT_TRY(sort_particles(grid, np, pos_n, w.pos_sorted, w.perm, nullptr, w.lstart, w.sort,
                          stream));
    if (!tiled(dtype))
      PT_TRY(rk2_backward(grid, coeff, dtype, np, dt, w.pos_sorted, g_pos, w.xbn, g_coeff, w.u0,
                          w.xbs, stream));
    else
      PT_TRY(tile_rk2_bwd(grid, coeff, dtype, w.lstart, np, dt, w.pos_sorted, g_pos, w.xbn,
                          (float*)w.u0, w.ub0, (float*)w.xbs, g_coeff, w.defer, w.items, false,
                          stream));
    return scatter_back(np, w.xbn, w.perm, g_pos, stream);
  }
  if (sort == PT_SORTED && tiled(dtype)) {
    // the order is kept, so dL/dx_n goes straight into g_pos
    PT_TRY(presorted_table(grid, np, pos_n, w.lstart, stream));
    return tile_rk2_bwd(grid, coeff, dtype, w.lstart, np, dt, pos_n, g_pos, g_pos, (float*)w.u0,
                        w.ub0, (float*)w.xbs, g_coeff, w.defer, w.items, true, stream);
  }
  return rk2_backward(grid, coeff, dtype, np, dt, pos_n, g_pos, g_pos, g_coeff, w.u0, w.xbs,
                      stream);
}

pt_status pt_inertial_step(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                           double dt, double tau, double* pos, void* vel, const double* disp,
                           int32_t* ids, int sort, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!(dt > 0.0) || !isfinite(dt) || !(tau >= 0.0) || !isfinite(tau)) return PT_ERR_ARG;
  if (sort != PT_UNSORTED && sort != PT_SORT && sort != PT_SORTED) return PT_ERR_ARG;
  if (sort != PT_UNSORTED) PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!coeff || !pos || (tau > 0.0 && !vel)) return PT_ERR_NULL;
  size_t need = 0;
  PT_TRY(pt_workspace_bytes(PT_OP_INERTIAL, grid, dtype, np, &need));
  if (!ws || ws_bytes < need) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  if (tau == 0.0) vel = nullptr;  // the tracer: no velocity is carried
  const InertialCoef k = inertial_coef(dt, tau);
  Rk2Ws w = carve_rk2(grid, np, dtype, ws);
  const size_t vb = value_bytes(dtype);
  if (sort == PT_SORT) {
    PT_TRY(sort_particles(grid, np, pos, w.pos_sorted, w.perm, nullptr, w.lstart, w.sort,
                          stream));
    if (ids) {
      PT_TRY(permute_ids(np, ids, w.perm, w.ids_tmp, stream));
      PT_HIP_CHECK(hipMemcpyAsync(ids, w.ids_tmp, 4 * (size_t)np, hipMemcpyDeviceToDevice, stream));
    }
    const void* vs = nullptr;
    if (vel) {
      PT_TRY(permute_rows(np, vel, (int)vb, w.perm, w.vel_sorted, stream));
      vs = w.vel_sorted;
    }
    const double* ds = nullptr;
    if (disp) {
      PT_TRY(permute_rows(np, disp, 8, w.perm, w.disp_sorted, stream));
      ds = w.disp_sorted;
    }
    if (!tiled(dtype))
      return inertial_advance(grid, coeff, dtype, np, k, w.pos_sorted, vs, ds, pos, vel, stream);
    return tile_inertial(grid, coeff, dtype, w.lstart, np, k, w.pos_sorted, (const float*)vs, ds,
                         pos, (float*)vel, w.defer, w.items, false, stream);
  }
  if (sort == PT_SORTED && tiled(dtype)) {
    PT_TRY(presorted_table(grid, np, pos, w.lstart, stream));
    return tile_inertial(grid, coeff, dtype, w.lstart, np, k, pos, (const float*)vel, disp, pos,
                         (float*)vel, w.defer, w.items, true, stream);
  }
  return inertial_advance(grid, coeff, dtype, np, k, pos, vel, disp, pos, vel, stream);
}

pt_status pt_rk2_step_noalloc(const pt_grid* grid, const void* coeff, pt_dtype dtype, int64_t np,
                              double dt, double* pos, int sort, hipStream_t stream) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!isfinite(dt)) return PT_ERR_ARG;
  if (sort != PT_UNSORTED && sort != PT_SORTED) return PT_ERR_ARG;
  if (sort == PT_SORTED) PT_TRY(check_tiled_np(np));
  if (np == 0) return PT_OK;
  if (!coeff || !pos) return PT_ERR_NULL;
  const bool tile = sort == PT_SORTED && tiled(dtype);
  // scratch layout: the particle table, the deferred list and the work items
  // (tiled), or the stage-1 velocities (one thread per particle)
  const size_t need = tile ? a256(lstart_bytes(grid)) + a256(tile_defer_bytes(np)) +
                                 a256(tile_items_bytes(grid, np, false))
                           : a256(3 * value_bytes(dtype) * (size_t)np);
  if (need > kNoAllocScratchBytes) return PT_ERR_WORKSPACE;
  PT_TRY(ready());
  char* sp = (char*)noalloc_scratch();
  if (!sp) return PT_ERR_HIP;
  if (!tile) return rk2_advance(grid, coeff, dtype, np, dt, pos, pos, sp, stream);
  int32_t* lstart = (int32_t*)sp;
  void* defer = sp + a256(lstart_bytes(grid));
  void* items = (char*)defer + a256(tile_defer_bytes(np));
  // every scratch word the kernels read is written first in this call: the
  // table by presorted_table, the deferred-list header and item counters by
  // the launch's own clearing kernels
  PT_TRY(presorted_table(grid, np, pos, lstart, stream));
  return tile_rk2_fwd(grid, coeff, dtype, lstart, np, dt, pos, pos, defer, items, true, stream);
}

pt_status pt_tiled_deferred(int op, const pt_grid* grid, pt_dtype dtype, int64_t np,
                            const void* ws, int64_t* count) {
  PT_TRY(check_grid(grid));
  PT_TRY(check_dtype(dtype));
  PT_TRY(check_np(np));
  if (!ws || !count) return PT_ERR_NULL;
  const void* defer = nullptr;
  if (op == PT_OP_RK2 || op == PT_OP_INERTIAL) {
    defer = carve_rk2(grid, np, dtype, (void*)ws).defer;
  } else if (op == PT_OP_RK2_BWD) {
    defer = carve_rk2_bwd(grid, np, dtype, (void*)ws).defer;
  } else if (op == PT_OP_INTERP_SORTED) {
    defer = (const char*)ws + a256(lstart_bytes(grid));
  } else {
    return PT_ERR_ARG;
  }
  int v = 0;
  PT_HIP_CHECK(hipDeviceSynchronize());
  PT_HIP_CHECK(hipMemcpy(&v, defer, sizeof(int), hipMemcpyDeviceToHost));
  *count = v;
  return PT_OK;
}

pt_status pt_last_device_error(hipStream_t stream) {
  int* flag = device_error_flag();
  if (!flag) return PT_ERR_HIP;
  PT_HIP_CHECK(hipStreamSynchronize(stream));
  int v = 0;
  PT_HIP_CHECK(hipMemcpy(&v, flag, sizeof(int), hipMemcpyDeviceToHost));
  if (v) {
    const int zero = 0;
    PT_HIP_CHECK(hipMemcpy(flag, &zero, sizeof(int), hipMemcpyHostToDevice));
    return PT_ERR_NONFINITE;
  }
  return PT_OK;
}

pt_status pt_timing_enable(int on) {
  std::lock_guard<std::mutex> lock(g_time_mu);
  g_time_on = on != 0;
  return PT_OK;
}

pt_status pt_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return PT_ERR_NULL;
  std::lock_guard<std::mutex> lock(g_time_mu);
  double sum = 0.0;
  int64_t n = 0;
  pt_status st = PT_OK;
  std::vector<TimingRec> keep;
  for (auto& r : g_time_recs) {
    if (r.name != kernel) {
      keep.push_back(r);
      continue;
    }
    float ms = 0.0f;
    if (hipEventSynchronize(r.stop) != hipSuccess ||
        hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
      st = PT_ERR_HIP;
    sum += ms;
    ++n;
    if (hipEventDestroy(r.start) != hipSuccess || hipEventDestroy(r.stop) != hipSuccess)
      st = PT_ERR_HIP;
  }
  g_time_recs.swap(keep);
  *total_ms = sum;
  *launches = n;
  return st;
}

const char* pt_status_string(pt_status s) {
  switch (s) {
    case PT_OK: return "ok";
    case PT_ERR_NULL: return "required pointer is NULL";
    case PT_ERR_SIZE: return "invalid grid size, box length or particle count";
    case PT_ERR_DTYPE: return "unknown coefficient dtype";
    case PT_ERR_WORKSPACE: return "workspace missing or too small";
    case PT_ERR_NONFINITE: return "non-finite particle position";
    case PT_ERR_HIP: return "HIP runtime error";
    case PT_ERR_UNSUPPORTED: return "unsupported size";
    case PT_ERR_ARG: return "invalid argument";
  }
  return "unknown status";
}

}  // extern "C"
