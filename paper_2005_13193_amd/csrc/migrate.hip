// One device's part of the particle migration between sub-domains (Sec. 4.3):
// after a step each process finds the particles that have left its
// sub-domain, copies them with their attributes into outgoing buffers and
// closes the gaps among the ones that stay, before the exchange with the
// neighbours.  Here the sub-domains are z-slabs, so a departing particle goes
// to the slab below or the one above, and the three groups are written as one
// stable partition [stay | lower | upper] of the positions (and labels).
//
// Three launches over blocks of 1024 particles: per-block counts of each
// group, one exclusive scan over the (group, block) counts in group-major
// order, and the scatter, in which each block ranks its particles within
// their group with wave ballots.  Every particle's group is formed from its
// shadow z cell exactly as the cell sort forms it, so the partition is
// bit-exact.
#include "pt_common.h"

namespace pt {

constexpr int kMigTB = 1024;
constexpr int kMigWaves = kMigTB / 64;

// 0: stays (its shadow z cell lies in [z0, z0 + nzl) modulo nz); 1: lower
// neighbour; 2: upper neighbour, whichever side of the slab is nearer
// periodically (ties go to the lower one).
__device__ __forceinline__ int slab_group(const GridDev& g, double z, int z0, int nzl,
                                          bool* bad) {
  double t;
  const int c = cell_1d(z, g.cs[2], g.nz, &t, bad);
  int rel = c - z0;
  if (rel < 0) rel += g.nz;
  if (rel < nzl) return 0;
  const int up = rel - nzl + 1;  // cells above the slab's top layer
  const int down = g.nz - rel;   // cells below its bottom layer
  return down <= up ? 1 : 2;
}

__global__ __launch_bounds__(kMigTB) void mig_count(GridDev g, int64_t np,
                                                    const double* __restrict__ z, int z0,
                                                    int nzl, uint32_t* __restrict__ counts,
                                                    int64_t nb, int* err) {
  __shared__ uint32_t s_cnt[3];
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kMigTB + threadIdx.x;
  bool bad = false;
  const int grp = i < np ? slab_group(g, z[i], z0, nzl, &bad) : -1;
  if (bad) *err = 1;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint64_t m = __ballot(grp == k);
    if (lane == 0 && m) atomicAdd(&s_cnt[k], (uint32_t)__popcll(m));
  }
  __syncthreads();
  if (threadIdx.x < 3) counts[(int64_t)threadIdx.x * nb + blockIdx.x] = s_cnt[threadIdx.x];
}

// Exclusive scan in place over n = 3 nb counts (one workgroup), and the group
// totals into totals[3].
__global__ __launch_bounds__(kMigTB) void mig_scan(uint32_t* __restrict__ data, int64_t nb,
                                                   int64_t* __restrict__ totals) {
  __shared__ uint32_t s_wave[kMigWaves];
  __shared__ uint32_t s_carry;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int64_t n = 3 * nb;
  for (int64_t base = 0; base < n; base += kMigTB) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = i < n ? data[i] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t woff = s_carry;
    for (int w = 0; w < wave; ++w) woff += s_wave[w];
    if (i < n) data[i] = woff + incl - v;
    __syncthreads();
    if (threadIdx.x == kMigTB - 1) s_carry = woff + incl;
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    // group k starts at data[k nb] (the scan of all earlier groups)
    const int k = threadIdx.x;
    const uint32_t start = nb > 0 ? data[k * nb] : 0u;
    const uint32_t end = k < 2 ? (nb > 0 ? data[(k + 1) * nb] : 0u) : s_carry;
    totals[k] = (int64_t)(end - start);
  }
}

__global__ __launch_bounds__(kMigTB) void mig_scatter(GridDev g, int64_t np,
                                                      const double* __restrict__ pos,
                                                      const int32_t* __restrict__ ids, int z0,
                                                      int nzl,
                                                      const uint32_t* __restrict__ offsets,
                                                      int64_t nb, double* __restrict__ pos_out,
                                                      int32_t* __restrict__ ids_out) {
  __shared__ uint32_t s_wcnt[3][kMigWaves];
  const int64_t i = (int64_t)blockIdx.x * kMigTB + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool bad = false;
  const int grp = i < np ? slab_group(g, pos[2 * np + i], z0, nzl, &bad) : -1;
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t rank = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint64_t m = __ballot(grp == k);
    if (lane == 0) s_wcnt[k][wave] = (uint32_t)__popcll(m);
    if (grp == k) rank = (uint32_t)__popcll(m & below);
  }
  __syncthreads();
  if (grp < 0) return;
  uint32_t woff = 0;
  for (int w = 0; w < wave; ++w) woff += s_wcnt[grp][w];
  const int64_t dst = (int64_t)offsets[(int64_t)grp * nb + blockIdx.x] + woff + rank;
#pragma unroll
  for (int c = 0; c < 3; ++c) pos_out[c * np + dst] = pos[c * np + i];
  if (ids) ids_out[dst] = ids[i];
}

size_t slab_partition_ws_bytes(int64_t np) {
  const int64_t nb = (np + kMigTB - 1) / kMigTB;
  return 4 * (size_t)(3 * nb) + 256;
}

// ws: slab_partition_ws_bytes(np) bytes; counts: device int64 [3].
pt_status slab_partition(const pt_grid* grid, int64_t np, const double* pos, const int32_t* ids,
                         int z0, int nzl, double* pos_out, int32_t* ids_out, int64_t* counts,
                         void* ws, hipStream_t s) {
  const GridDev g = make_grid_dev(grid);
  const int64_t nb = (np + kMigTB - 1) / kMigTB;
  uint32_t* cnt = (uint32_t*)ws;
  if (nb > 0) {
    hipLaunchKernelGGL(mig_count, dim3((unsigned)nb), dim3(kMigTB), 0, s, g, np, pos + 2 * np,
                       z0, nzl, cnt, nb, device_error_flag());
    PT_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(mig_scan, dim3(1), dim3(kMigTB), 0, s, cnt, nb, counts);
  PT_LAUNCH_CHECK();
  if (nb > 0) {
    TimedLaunch t("slab_partition", s);
    hipLaunchKernelGGL(mig_scatter, dim3((unsigned)nb), dim3(kMigTB), 0, s, g, np, pos, ids, z0,
                       nzl, cnt, nb, pos_out, ids_out);
  }
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
