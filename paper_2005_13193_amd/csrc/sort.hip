// Particle ordering by spline cell (the one-device counterpart of the
// position-based particle-to-process mapping of Sec. 3): cell keys in FP64,
// a stable least-significant-digit radix sort of (key, index) with 8-bit
// digits (a lone top bit joins the last digit: 33-bit keys take passes of 8,
// 8, 8 and 9 bits), and the permutation of the particle arrays.
//
// Radix pass structure: the input is cut into block tiles of kSortTile
// consecutive elements (8 waves x 16 rounds x 64 lanes).  A histogram kernel
// counts the digits of every tile, an exclusive scan over the digit-major
// count table gives every (digit, tile) its output offset, and a scatter
// kernel re-reads each tile, ranks equal digits in input order (wave ballots
// within a round, running per-wave counts across rounds, wave prefixes
// across the tile), reorders the tile by digit in LDS, and writes each
// digit's run contiguously (about 32 elements per 8-bit digit and tile).
#include <hip/hip_runtime.h>

#include "pt_common.h"

namespace pt {

constexpr int kSortThreads = 512;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortRounds = 16;
constexpr int kWaveItems = 64 * kSortRounds;            // elements per wave
constexpr int kSortTile = kSortThreads * kSortRounds;   // elements per tile
constexpr int kScanItems = 8;             // per thread in the scan kernels
constexpr int kScanBlock = 256 * kScanItems;

// Cell key of particle i (see pt_key_layout): column, layer, row, column
// offset; *bad is set for a non-finite coordinate.
template <typename K>
__device__ __forceinline__ K cell_key(const GridDev& g, int64_t np,
                                      const double* __restrict__ pos, int64_t i, bool* bad) {
  double t;
  const int a = cell_1d(pos[i], g.cs[0], g.nx, &t, bad);
  const int b = cell_1d(pos[np + i], g.cs[1], g.ny, &t, bad);
  const int c = cell_1d(pos[2 * np + i], g.cs[2], g.nz, &t, bad);
  const K ncx = (K)((g.nx + kTileX - 1) / kTileX);
  return ((((K)(b / kTileY) * ncx + (K)(a / kTileX)) * (K)g.nz + (K)c) * (K)kTileY +
          (K)(b % kTileY)) * (K)kTileX + (K)(a % kTileX);
}

template <typename K>
__global__ __launch_bounds__(256) void cell_key_kernel(GridDev g, int64_t np,
                                                       const double* __restrict__ pos,
                                                       K* __restrict__ keys,
                                                       uint32_t* __restrict__ vals, int* err) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  bool bad = false;
  keys[i] = cell_key<K>(g, np, pos, i, &bad);
  vals[i] = (uint32_t)i;
  if (bad) *err = 1;
}

// The half-layer (column, layer, upper or lower 16 rows) of a key: the
// particle table's index.
constexpr int kHalfLayerShift = 9;  // log2(kTileX * kTileY / 2)
static_assert(kTileX * kTileY == (2 << kHalfLayerShift), "half-layer shift");

// Particle table straight from positions taken to be in cell order: entry
// L is the first particle of half-layer L or later (np past the last one).
// Thread i compares the half-layers of particles i - 1 and i (each thread
// forms one, the neighbour's comes through LDS; the first thread of a block
// forms its predecessor's itself).  For positions not in order some entries
// are left as they were; the table's users check it before trusting it.
template <typename K>
__global__ __launch_bounds__(256) void sorted_layer_table(GridDev g, int64_t np,
                                                          const double* __restrict__ pos,
                                                          int64_t nlayers,
                                                          int32_t* __restrict__ ls, int* err) {
  __shared__ int64_t s_half[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool bad = false;
  const int64_t lcur =
      i < np ? (int64_t)(cell_key<K>(g, np, pos, i, &bad) >> kHalfLayerShift) : nlayers;
  s_half[threadIdx.x] = lcur;
  __syncthreads();
  if (i > np) return;
  int64_t lprev = -1;
  if (i > 0) {
    lprev = threadIdx.x > 0 ? s_half[threadIdx.x - 1]
                            : (int64_t)(cell_key<K>(g, np, pos, i - 1, &bad) >> kHalfLayerShift);
  }
  if (bad) *err = 1;
  for (int64_t L = lprev + 1; L <= lcur && L <= nlayers; ++L) ls[L] = (int32_t)i;
}

// Lanes holding the same DB-bit digit: AND of the ballots of each bit (or of
// their complements), restricted to the valid lanes.
template <int DB>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
  uint64_t peers = valid;
#pragma unroll
  for (int b = 0; b < DB; ++b) {
    const int bit = (d >> b) & 1;
    const uint64_t bal = __ballot(bit);
    peers &= bit ? bal : ~bal;
  }
  return peers;
}

// Digit counts of one tile: counts[d * ntiles + tile].
template <typename K, int DB>
__global__ __launch_bounds__(kSortThreads) void radix_hist(const K* __restrict__ keys, int64_t n,
                                                           int shift,
                                                           uint32_t* __restrict__ counts,
                                                           int64_t ntiles) {
  constexpr int kBins = 1 << DB;
  __shared__ uint32_t h[kSortWaves][kBins];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = lane; i < kBins; i += 64) h[wave][i] = 0;
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kSortTile + (int64_t)wave * kWaveItems;
  const uint64_t lt = (1ull << lane) - 1;
  uint32_t d[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t idx = base + r * 64 + lane;
    d[r] = idx < n ? (uint32_t)((keys[idx] >> shift) & (kBins - 1)) : (uint32_t)kBins;
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool ok = d[r] < (uint32_t)kBins;
    const uint64_t peers = match_digit<DB>(d[r] & (kBins - 1), __ballot(ok));
    if (ok && (peers & lt) == 0) h[wave][d[r]] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  for (int dd = tid; dd < kBins; dd += kSortThreads) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) c += h[w][dd];
    counts[(int64_t)dd * ntiles + tile] = c;
  }
}

// LDS of the scatter kernel: the tile's keys and values, per-wave digit
// counts, per digit its start in the reordered tile and its global offset,
// and the wave sums of the digit scan.
template <typename K, int DB>
constexpr size_t radix_scatter_lds() {
  return (size_t)kSortTile * (sizeof(K) + 4) +
         4 * ((size_t)kSortWaves * (1 << DB) + 2 * (size_t)(1 << DB) + kSortWaves);
}

// Stable scatter of one tile to the offsets of the scanned count table.
template <typename K, int DB>
__global__ __launch_bounds__(kSortThreads) void radix_scatter(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, const uint32_t* __restrict__ offsets,
    int64_t ntiles) {
  constexpr int kBins = 1 << DB;
  // the scan over digits: a scan thread takes a contiguous run of kDpt
  constexpr int kDpt = kBins > kSortThreads ? kBins / kSortThreads : 1;
  constexpr int kScanThreads = kBins / kDpt;
  extern __shared__ __align__(16) unsigned char smem[];
  K* tk = (K*)smem;                                          // [kSortTile]
  uint32_t* tv = (uint32_t*)(tk + kSortTile);                // [kSortTile]
  uint32_t* h = tv + kSortTile;                              // [kSortWaves][kBins]
  uint32_t* dstart = h + kSortWaves * kBins;                 // [kBins]
  uint32_t* goff = dstart + kBins;                           // [kBins]
  uint32_t* wsum = goff + kBins;                             // [kSortWaves]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t tile = blockIdx.x;
  const int64_t tbase = tile * kSortTile;
  const int tile_n = (int)min((int64_t)kSortTile, n - tbase);
  const int64_t base = tbase + (int64_t)wave * kWaveItems;
  for (int i = lane; i < kBins; i += 64) h[wave * kBins + i] = 0;
  for (int dd = tid; dd < kBins; dd += kSortThreads)
    goff[dd] = offsets[(int64_t)dd * ntiles + tile];

  K k[kSortRounds];
  uint32_t v[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t idx = base + r * 64 + lane;
    const bool ok = idx < n;
    k[r] = ok ? kin[idx] : (K)0;
    v[r] = ok ? vin[idx] : 0u;
  }
  // wave-local ranks: rank = earlier rounds' count of the digit + lanes below
  const uint64_t lt = (1ull << lane) - 1;
  uint32_t dr[kSortRounds];  // digit << 16 | wave-local rank
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool ok = base + r * 64 + lane < n;
    const uint32_t d = (uint32_t)((k[r] >> shift) & (kBins - 1));
    const uint64_t peers = match_digit<DB>(d, __ballot(ok));
    const uint32_t start = ok ? h[wave * kBins + d] : 0u;
    dr[r] = (d << 16) | (start + (uint32_t)__popcll(peers & lt));
    // the lowest lane of each digit group advances the running count; its
    // new value depends on the value it read, so the read completes first
    if (ok && (peers & lt) == 0) h[wave * kBins + d] = start + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: exclusive prefixes over the waves, then over the digits
  uint32_t tot[kDpt];
  uint32_t mine = 0;
  if (tid < kScanThreads) {
#pragma unroll
    for (int q = 0; q < kDpt; ++q) {
      const int dd = tid * kDpt + q;
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t c = h[w * kBins + dd];
        h[w * kBins + dd] = run;
        run += c;
      }
      tot[q] = run;
      mine += run;
    }
  }
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  if (tid < kScanThreads) {
    uint32_t off = incl - mine;  // exclusive within the wave
    for (int w = 0; w < wave; ++w) off += wsum[w];
#pragma unroll
    for (int q = 0; q < kDpt; ++q) {
      dstart[tid * kDpt + q] = off;
      off += tot[q];
    }
  }
  __syncthreads();
  // reorder the tile by digit in LDS
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    if (base + r * 64 + lane < n) {
      const uint32_t d = dr[r] >> 16;
      const uint32_t lp = dstart[d] + h[wave * kBins + d] + (dr[r] & 0xffffu);
      tk[lp] = k[r];
      tv[lp] = v[r];
    }
  }
  __syncthreads();
  // each digit's run goes to consecutive global positions
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int i = r * kSortThreads + tid;
    if (i < tile_n) {
      const K key = tk[i];
      const uint32_t d = (uint32_t)((key >> shift) & (kBins - 1));
      const uint32_t dst = goff[d] + ((uint32_t)i - dstart[d]);
      if (dst < (uint64_t)n) {  // always true for consistent counts; guards the store
        kout[dst] = key;
        vout[dst] = tv[i];
      }
    }
  }
}

// ------------------------------------------------- exclusive scan (u32) ---
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__global__ __launch_bounds__(256) void scan_blocks(uint32_t* __restrict__ data, int64_t n,
                                                   uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)tid * kScanItems;
  uint32_t v[kScanItems];
  uint32_t tot = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? data[base + i] : 0u;
    tot += v[i];
  }
  const uint32_t incl = wave_incl_scan(tot, lane);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (int w = 0; w < wave; ++w) woff += wsum[w];
  uint32_t run = woff + incl - tot;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) data[base + i] = run;
    run += v[i];
  }
  if (tid == 255) block_sums[blockIdx.x] = woff + incl;
}

__global__ __launch_bounds__(256) void scan_add(uint32_t* __restrict__ data, int64_t n,
                                                const uint32_t* __restrict__ block_offsets) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  const uint32_t off = block_offsets[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) data[base + i] += off;
}

static size_t scan_scratch_words(int64_t n) {
  size_t w = 0;
  while (n > 1) {
    n = (n + kScanBlock - 1) / kScanBlock;
    w += (size_t)n + 64;
  }
  return w + 64;
}

static pt_status exclusive_scan(uint32_t* data, int64_t n, uint32_t* scratch, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(scan_blocks, dim3((unsigned)nb), dim3(256), 0, s, data, n, scratch);
  PT_LAUNCH_CHECK();
  if (nb > 1) {
    pt_status st = exclusive_scan(scratch, nb, scratch + nb + 64, s);
    if (st != PT_OK) return st;
    hipLaunchKernelGGL(scan_add, dim3((unsigned)nb), dim3(256), 0, s, data, n, scratch);
    PT_LAUNCH_CHECK();
  }
  return PT_OK;
}

// -------------------------------------------------------------- permute ---
__global__ __launch_bounds__(256) void permute_pos(int64_t np, const double* __restrict__ pos,
                                                   const int32_t* __restrict__ perm,
                                                   double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const int64_t p = perm[i];
  if ((uint64_t)p >= (uint64_t)np) return;
  out[i] = pos[p];
  out[np + i] = pos[np + p];
  out[2 * np + i] = pos[2 * np + p];
}

__global__ __launch_bounds__(256) void permute_i32(int64_t np, const int32_t* __restrict__ in,
                                                   const int32_t* __restrict__ perm,
                                                   int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const int64_t p = perm[i];
  if ((uint64_t)p < (uint64_t)np) out[i] = in[p];
}

// out[r][i] = in[r][perm[i]] for the three rows of a [3][np] array.
template <typename T>
__global__ __launch_bounds__(256) void permute_rows3(int64_t np, const T* __restrict__ in,
                                                     const int32_t* __restrict__ perm,
                                                     T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const int64_t p = perm[i];
  if ((uint64_t)p >= (uint64_t)np) return;
  out[i] = in[p];
  out[np + i] = in[np + p];
  out[2 * np + i] = in[2 * np + p];
}

template <typename K>
__global__ __launch_bounds__(256) void widen_keys(int64_t np, const K* __restrict__ k,
                                                  uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < np) out[i] = (uint64_t)k[i];
}

// ------------------------------------------------------------ host side ---

int key_bits(const pt_grid* g) {
  const uint64_t ncx = (uint64_t)((g->nx + kTileX - 1) / kTileX);
  const uint64_t ncy = (uint64_t)((g->ny + kTileY - 1) / kTileY);
  const uint64_t range = ncx * ncy * (uint64_t)g->nz * kTileX * kTileY;
  int bits = 0;
  while (bits < 64 && ((range - 1) >> bits) != 0) ++bits;
  return bits < 1 ? 1 : bits;
}

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int64_t tile_nlayers(const pt_grid* g);  // tile.hip: half-layers of the particle table

struct SortWs {
  void* keys[2];
  uint32_t* vals0;
  uint32_t* counts;
  uint32_t* scan;
};

static int64_t sort_tiles(int64_t np) { return (np + kSortTile - 1) / kSortTile; }

// Digits of the radix passes: 8 bits each; a lone top bit (bits % 8 == 1,
// bits > 8) joins the last digit, which then has 9 bits (one pass fewer).
static int sort_passes(int bits, int* last_db) {
  const int passes = (bits + 7) / 8;
  if (passes > 1 && bits % 8 == 1) {
    *last_db = 9;
    return passes - 1;
  }
  *last_db = 8;
  return passes;
}

size_t sort_ws_bytes(const pt_grid* g, int64_t np) {
  const size_t kb = key_bits(g) > 32 ? 8 : 4;
  int last_db = 8;
  sort_passes(key_bits(g), &last_db);
  const size_t ncount = (size_t)sort_tiles(np) << last_db;
  return 2 * align256(kb * (size_t)np) + align256(4 * (size_t)np) + align256(4 * ncount) +
         align256(4 * scan_scratch_words((int64_t)ncount));
}

static SortWs carve_sort_ws(const pt_grid* g, int64_t np, void* ws) {
  const size_t kb = key_bits(g) > 32 ? 8 : 4;
  const int64_t nt = sort_tiles(np);
  char* p = (char*)ws;
  SortWs w;
  w.keys[0] = p; p += align256(kb * (size_t)np);
  w.keys[1] = p; p += align256(kb * (size_t)np);
  w.vals0 = (uint32_t*)p; p += align256(4 * (size_t)np);
  int last_db = 8;
  sort_passes(key_bits(g), &last_db);
  w.counts = (uint32_t*)p; p += align256(4 * ((size_t)nt << last_db));
  w.scan = (uint32_t*)p;
  return w;
}

pt_status build_layer_table(const pt_grid* g, int64_t np, const void* keys, int key_bytes,
                            int32_t* ls, hipStream_t s);

// One radix pass of DB-bit digits at bit `shift`, keys and values from
// buffer src to the other.
template <typename K, int DB>
static pt_status radix_pass(K* const kbuf[2], uint32_t* const vbuf[2], int src, int shift,
                            int64_t np, const SortWs& w, hipStream_t s) {
  const int64_t nt = sort_tiles(np);
  constexpr size_t lds = radix_scatter_lds<K, DB>();
  static_assert(lds <= 160 * 1024, "radix_scatter LDS");
  if (hipFuncSetAttribute((const void*)radix_scatter<K, DB>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return PT_ERR_HIP;
  const int dst = src ^ 1;
  TimedLaunch t("sort_pass", s);
  hipLaunchKernelGGL((radix_hist<K, DB>), dim3((unsigned)nt), dim3(kSortThreads), 0, s,
                     kbuf[src], np, shift, w.counts, nt);
  PT_LAUNCH_CHECK();
  pt_status st = exclusive_scan(w.counts, nt << DB, w.scan, s);
  if (st != PT_OK) return st;
  hipLaunchKernelGGL((radix_scatter<K, DB>), dim3((unsigned)nt), dim3(kSortThreads), lds, s,
                     kbuf[src], vbuf[src], kbuf[dst], vbuf[dst], np, shift, w.counts, nt);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

template <typename K>
static pt_status sort_impl(const pt_grid* g, int64_t np, const double* pos, int32_t* perm,
                           uint64_t* keys_out, int32_t* lstart, void* ws, hipStream_t s) {
  const GridDev gd = make_grid_dev(g);
  SortWs w = carve_sort_ws(g, np, ws);
  const int bits = key_bits(g);
  int last_db = 8;
  const int passes = sort_passes(bits, &last_db);
  K* kbuf[2] = {(K*)w.keys[0], (K*)w.keys[1]};
  // pass i writes value buffer (passes - 1 - i) & 1: 0 = perm, 1 = scratch,
  // so that the last pass lands in perm.
  uint32_t* vbuf[2] = {(uint32_t*)perm, w.vals0};
  const int first_dst = (passes - 1) & 1;
  const int src0 = first_dst ^ 1;
  {
    TimedLaunch t("sort_keys", s);
    hipLaunchKernelGGL(cell_key_kernel<K>, dim3(grid_1d(np, 256)), dim3(256), 0, s, gd, np, pos,
                       kbuf[src0], vbuf[src0], device_error_flag());
  }
  PT_LAUNCH_CHECK();
  int src = src0;
  for (int p = 0; p < passes; ++p) {
    const pt_status st = p + 1 == passes && last_db == 9
                             ? radix_pass<K, 9>(kbuf, vbuf, src, 8 * p, np, w, s)
                             : radix_pass<K, 8>(kbuf, vbuf, src, 8 * p, np, w, s);
    if (st != PT_OK) return st;
    src ^= 1;
  }
  if (keys_out) {
    hipLaunchKernelGGL(widen_keys<K>, dim3(grid_1d(np, 256)), dim3(256), 0, s, np, kbuf[src],
                       keys_out);
    PT_LAUNCH_CHECK();
  }
  if (lstart) return build_layer_table(g, np, kbuf[src], (int)sizeof(K), lstart, s);
  return PT_OK;
}

// The particle table of positions that should already be in cell order,
// built from the positions in one pass.  For positions that are not in order
// the table is not a partition; its users check it on the device before
// trusting it.
pt_status presorted_table(const pt_grid* g, int64_t np, const double* pos, int32_t* lstart,
                          hipStream_t s) {
  const GridDev gd = make_grid_dev(g);
  const int64_t nl = tile_nlayers(g);
  TimedLaunch t("sorted_table", s);
  if (key_bits(g) > 32)
    hipLaunchKernelGGL(sorted_layer_table<uint64_t>, dim3(grid_1d(np + 1, 256)), dim3(256), 0, s,
                       gd, np, pos, nl, lstart, device_error_flag());
  else
    hipLaunchKernelGGL(sorted_layer_table<uint32_t>, dim3(grid_1d(np + 1, 256)), dim3(256), 0, s,
                       gd, np, pos, nl, lstart, device_error_flag());
  PT_LAUNCH_CHECK();
  return PT_OK;
}

pt_status sort_particles(const pt_grid* g, int64_t np, const double* pos, double* pos_sorted,
                         int32_t* perm, uint64_t* keys_out, int32_t* lstart, void* ws,
                         hipStream_t s) {
  pt_status st = key_bits(g) > 32
                     ? sort_impl<uint64_t>(g, np, pos, perm, keys_out, lstart, ws, s)
                     : sort_impl<uint32_t>(g, np, pos, perm, keys_out, lstart, ws, s);
  if (st != PT_OK) return st;
  if (pos_sorted) {
    TimedLaunch t("sort_permute", s);
    hipLaunchKernelGGL(permute_pos, dim3(grid_1d(np, 256)), dim3(256), 0, s, np, pos, perm,
                       pos_sorted);
    PT_LAUNCH_CHECK();
  }
  return PT_OK;
}

// [3][np] rows of 4- or 8-byte elements permuted as the particles.
pt_status permute_rows(int64_t np, const void* in, int elem_bytes, const int32_t* perm, void* out,
                       hipStream_t s) {
  if (elem_bytes == 8)
    hipLaunchKernelGGL(permute_rows3<double>, dim3(grid_1d(np, 256)), dim3(256), 0, s, np,
                       (const double*)in, perm, (double*)out);
  else
    hipLaunchKernelGGL(permute_rows3<float>, dim3(grid_1d(np, 256)), dim3(256), 0, s, np,
                       (const float*)in, perm, (float*)out);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

pt_status permute_ids(int64_t np, const int32_t* in, const int32_t* perm, int32_t* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(permute_i32, dim3(grid_1d(np, 256)), dim3(256), 0, s, np, in, perm, out);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
