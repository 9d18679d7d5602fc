// Particle binning for the block-tiled transfers (not a step of the paper's
// method; it orders the work so that each grid block's particles are
// contiguous): key = grid block of the particle's base cell, a stable LSD
// radix sort of (key, index) with 8-bit digits, a gather of the particle SoA
// into key order, per-block [begin, end) ranges, the list of occupied blocks,
// the transfer work items (runs of at most s.item_particles particles of one
// block) and the list of active blocks (each occupied block with the
// neighbours its tile reaches). Also the host<->SoA marshalling kernels and
// the diagnostic stress kernel.
//
// Every buffer is cleared with fill kernels (no memset nodes), so the whole
// pipeline can be captured in a HIP graph.
#include "mpm_device.h"
#include "mpm_internal.h"

namespace mpm {

constexpr int kSortWG = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortWG * kSortItems;  // keys per workgroup
constexpr int kRadix = 256;
constexpr int kScanWG = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanWG * kScanItems;

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return;
  int64_t wgs = (n + 255) / 256;
  if (wgs > 4096) wgs = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)wgs), dim3(256), 0, st, p, n, v);
}

// ------------------------------------------------------------------ scan
// Exclusive prefix sum of a u32 array, three passes: per-tile sums, a scan of
// the tile sums in one workgroup, then per-tile scans offset by it.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // Hillis-Steele over kScanWG thread values in LDS.
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanWG; off <<= 1) {
    const uint32_t add = (t >= off) ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  *total = sh[kScanWG - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanWG) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                         uint32_t* __restrict__ partial) {
  __shared__ uint32_t sh[kScanWG];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in[base + k];
  uint32_t total;
  block_exclusive_scan(s, sh, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanWG) void k_scan_partials(uint32_t* partial, int n_part,
                                                           uint32_t* total_out) {
  __shared__ uint32_t sh[kScanWG];
  const int per = (n_part + kScanWG - 1) / kScanWG;
  const int lo = threadIdx.x * per;
  uint32_t s = 0;
  for (int k = 0; k < per; ++k)
    if (lo + k < n_part) s += partial[lo + k];
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, sh, &total);
  for (int k = 0; k < per; ++k)
    if (lo + k < n_part) {
      const uint32_t x = partial[lo + k];
      partial[lo + k] = run;
      run += x;
    }
  if (threadIdx.x == 0 && total_out) *total_out = total;
}

__global__ __launch_bounds__(kScanWG) void k_scan_down(const uint32_t* __restrict__ in, int64_t n,
                                                       const uint32_t* __restrict__ partial,
                                                       uint32_t* __restrict__ out) {
  __shared__ uint32_t sh[kScanWG];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t vals[kScanItems];
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    vals[k] = (base + k < n) ? in[base + k] : 0u;
    s += vals[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, sh, &total) + partial[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) {
      out[base + k] = run;
      run += vals[k];
    }
}

// out may alias in. partial needs ceil(n / kScanTile) entries.
static void exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partial,
                           uint32_t* total_out, hipStream_t st) {
  const int n_part = (int)((n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(n_part), dim3(kScanWG), 0, st, in, n, partial);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanWG), 0, st, partial, n_part, total_out);
  hipLaunchKernelGGL(k_scan_down, dim3(n_part), dim3(kScanWG), 0, st, in, n, partial, out);
}

// ------------------------------------------------------------------ keys
// Scene of the particle with original index o: the last scene whose offset is
// <= o (scene_off holds n_scenes + 1 ascending offsets).
__device__ __forceinline__ uint32_t scene_of(const uint32_t* __restrict__ scene_off, int n_scenes, uint32_t o) {
  int lo = 0, hi = n_scenes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (scene_off[mid] <= o)
      lo = mid;
    else
      hi = mid - 1;
  }
  return (uint32_t)lo;
}

// Half (0 or 1) of the base cell that an offset r - 0.5 - floor(r - 0.5) in
// [0, 1) falls in. Halves rather than finer classes: a lattice of two
// particles per cell and axis sits at offsets near 1/4 and 3/4, away from the
// boundary, so slow material keeps its classes and the next sort its order.
__device__ __forceinline__ uint32_t sub_cell_half(float frac) { return frac >= 0.5f ? 1u : 0u; }

// Binning keys: the block of the base cell (scene-major) in the high bits,
// then 6 bits from the particle's sub-cell class (its half of the base cell
// per axis) and the base cell's z layer in the block. Within a class,
// consecutive particles (the lanes of one wave) sit in different base cells,
// so their LDS atomics hit different nodes: at up to 8 particles per cell a
// class holds about one particle of each cell. A block that fits in one work
// item is ordered class first (a class then spans all of the block's cells);
// a larger one z layer first, so that each of its work items covers a few
// layers of the tile. Block sizes come from the previous sort (prev_begin /
// prev_end); blocks above kDenseBlock particles, and blocks without a count
// (at the first sort, the order given), keep their order. In a denser block
// a class still holds many particles of a cell; its work items deal
// particles to lanes 8 apart (item_lane), which spreads particles given in a
// lattice or random order better. Invalid particles get `sentinel`, which
// sorts after every block.
__global__ void k_keygen(const float* __restrict__ part, const uint32_t* __restrict__ id,
                         const uint32_t* __restrict__ scene_off, int64_t cap, int64_t N, SimK s,
                         const uint32_t* __restrict__ prev_begin, const uint32_t* __restrict__ prev_end,
                         uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t sentinel,
                         Status* st) {
  unsigned dom = 0, nf = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t key = sentinel;
    int cell[3];
    uint32_t cls = 0;
    bool ok = true, fin = true;
    for (int a = 0; a < 3; ++a) {
      const float r = part[(FX + a) * cap + i] * s.inv_dx;
      fin = fin && isfinite(r);
      const float b = floorf(r - 0.5f);
      ok = ok && (b >= 0.0f) && (b + 2.0f <= (float)(s.n - 1));
      cell[a] = ok ? (int)b : 0;
      cls |= ok ? sub_cell_half(r - 0.5f - b) << a : 0u;
    }
    if (ok && fin) {
      const uint32_t scene = s.n_scenes > 1 ? scene_of(scene_off, s.n_scenes, id[i]) : 0u;
      const uint32_t blk = scene * s.nb3 + (uint32_t)(((cell[2] >> kTileLog2) * s.nb + (cell[1] >> kTileLog2)) * s.nb +
                                                      (cell[0] >> kTileLog2));
      // work tile: the block, or (4-cell tiles) its sub-block sx + 2 sy + 4 sz
      uint32_t unit = blk;
      if (s.unit_shift)
        unit = (blk << 3) | (uint32_t)(((cell[0] >> 2) & 1) | (((cell[1] >> 2) & 1) << 1) | (((cell[2] >> 2) & 1) << 2));
      const uint32_t prev = prev_end[unit] - prev_begin[unit];
      const uint32_t z = (uint32_t)(cell[2] & (s.tile - 1));
      const uint32_t dense = 8u * (uint32_t)(s.tile * s.tile * s.tile);
      uint32_t sub = 0u;  // dense or new tile: keep the order
      if (prev > 0u && prev <= s.item_particles)
        sub = (cls << 3) | z;  // one work item: class first, so a class spans the tile's cells
      else if (prev > 0u && prev <= dense)
        sub = (z << 3) | cls;  // several items: z layers first, so an item covers a few layers
      key = (unit << kClassBits) | sub;
    } else if (!fin) {
      nf++;
    } else {
      dom++;
    }
    keys[i] = key;
    vals[i] = (uint32_t)i;
  }
  if (dom) atomicAdd(&st->n_domain, (unsigned long long)dom);
  if (nf) atomicAdd(&st->n_nonfinite, (unsigned long long)nf);
}

// ------------------------------------------------------------------ radix sort
// Lanes of one wave whose digit equals this lane's (a match over 8 ballots).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const unsigned lane = threadIdx.x & 63u;
  return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// Per tile digit counts; hist is digit-major: hist[d * n_tiles + tile].
__global__ __launch_bounds__(kSortWG) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t N,
                                                        int shift, uint32_t* __restrict__ hist,
                                                        int n_tiles) {
  __shared__ uint32_t cnt[kSortWG / 64][kRadix];
  const int wave = threadIdx.x >> 6;
  for (int w = 0; w < kSortWG / 64; ++w) cnt[w][threadIdx.x] = 0u;
  __syncthreads();
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  // All of this thread's keys are loaded before the rounds, so the loads
  // are in flight together.
  uint32_t kr[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = tile0 + (int64_t)r * kSortWG + threadIdx.x;
    kr[r] = i < N ? keys[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = tile0 + (int64_t)r * kSortWG + threadIdx.x;
    const bool valid = i < N;
    const uint32_t d = valid ? ((kr[r] >> shift) & (kRadix - 1)) : 0u;
    const uint64_t peers = match_digit(d, valid);
    if (valid && (peers & lanemask_lt()) == 0ull) cnt[wave][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  uint32_t s = 0;
  for (int w = 0; w < kSortWG / 64; ++w) s += cnt[w][threadIdx.x];
  hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = s;
}

// Stable scatter of a tile: keys keep their order within a digit.
__global__ __launch_bounds__(kSortWG) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint32_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout, int64_t N,
                                                           int shift, const uint32_t* __restrict__ offs,
                                                           int n_tiles) {
  __shared__ uint32_t run[kRadix];
  __shared__ uint32_t wcnt[kSortWG / 64][kRadix];
  const int wave = threadIdx.x >> 6;
  run[threadIdx.x] = offs[(int64_t)threadIdx.x * n_tiles + blockIdx.x];
  for (int w = 0; w < kSortWG / 64; ++w) wcnt[w][threadIdx.x] = 0u;
  __syncthreads();
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  // All of this thread's keys and values are loaded before the rounds, so
  // the loads are in flight together.
  uint32_t kr[kSortItems], vr[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = tile0 + (int64_t)r * kSortWG + threadIdx.x;
    kr[r] = i < N ? kin[i] : 0u;
    vr[r] = i < N ? vin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = tile0 + (int64_t)r * kSortWG + threadIdx.x;
    const bool valid = i < N;
    const uint32_t k = kr[r];
    const uint32_t v = vr[r];
    const uint32_t d = (k >> shift) & (kRadix - 1);
    const uint64_t peers = match_digit(d, valid);
    const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
    if (valid && rank == 0u) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kSortWG / 64; ++w) {
      add += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0u;
    }
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ permutation, ranges
// Gathers the particle SoA into key order: x, F, E (when stored) and, with
// VC, v and C (between fused substeps they are not live). The field loops
// are unrolled so that a lane's loads are all in flight before its stores.
// Without VC, particles with the sentinel key (stencil outside the grid or
// state not finite) still carry their v and C: no transfer kernel visits
// them, so the values in memory are the ones read back for them.
template <bool VC, bool HAS_E>
__global__ void k_permute(const float* __restrict__ src, float* __restrict__ dst,
                          const uint32_t* __restrict__ id_src, uint32_t* __restrict__ id_dst,
                          const uint32_t* __restrict__ perm, const uint32_t* __restrict__ keys,
                          uint32_t sentinel, int64_t cap, int64_t N) {
  constexpr int kLo = VC ? FX : FF;  // fields [FX, FX + 3) and [kLo, kEnd)
  constexpr int kEnd = HAS_E ? kFields : kFields - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t j = perm[i];
    float x[3], r[kEnd - kLo];
#pragma unroll
    for (int f = 0; f < 3; ++f) x[f] = src[(FX + f) * cap + j];
#pragma unroll
    for (int f = kLo; f < kEnd; ++f)
      if (f >= FV) r[f - kLo] = src[f * cap + j];
    const uint32_t id = id_src[j];
#pragma unroll
    for (int f = 0; f < 3; ++f) dst[(FX + f) * cap + i] = x[f];
#pragma unroll
    for (int f = kLo; f < kEnd; ++f)
      if (f >= FV) dst[f * cap + i] = r[f - kLo];
    if constexpr (!VC) {
      if (keys[i] >= sentinel)
        for (int f = FV; f < FF; ++f) dst[f * cap + i] = src[f * cap + j];
    }
    id_dst[i] = id;
  }
}

__global__ void k_ranges(const uint32_t* __restrict__ keys, int64_t N, uint32_t n_blocks, int shift,
                         uint32_t* __restrict__ begin, uint32_t* __restrict__ end) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[i] >> shift;
    if (k >= n_blocks) continue;
    if (i == 0 || (keys[i - 1] >> shift) != k) begin[k] = (uint32_t)i;
    if (i == N - 1 || (keys[i + 1] >> shift) != k) end[k] = (uint32_t)(i + 1);
  }
}

__global__ void k_flag_occupied(const uint32_t* __restrict__ begin, const uint32_t* __restrict__ end,
                                uint32_t n_blocks, uint32_t* __restrict__ flags) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks; b += gridDim.x * blockDim.x)
    flags[b] = end[b] > begin[b] ? 1u : 0u;
}

// Grid blocks that the LDS tile of an occupied work tile touches, within the
// same scene: the tile of edge T at cell origin o spans nodes [o, o + T + 1]
// per axis.
__global__ void k_mark_dilated(const uint32_t* __restrict__ begin, const uint32_t* __restrict__ end,
                               int nb, uint32_t nb3, uint32_t n_units, int tile, int unit_shift,
                               uint32_t* __restrict__ mark) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_units; u += gridDim.x * blockDim.x) {
    if (!(end[u] > begin[u])) continue;
    const uint32_t b = u >> unit_shift;
    const uint32_t scene = b / nb3, lb = b - scene * nb3;
    int o[3] = {(int)(lb % nb) * kTile, (int)((lb / nb) % nb) * kTile, (int)(lb / (nb * nb)) * kTile};
    if (unit_shift)
      for (int a = 0; a < 3; ++a) o[a] += (int)((u >> a) & 1u) * tile;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = o[a] >> kTileLog2;
      hi[a] = min((o[a] + tile + 1) >> kTileLog2, nb - 1);
    }
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) mark[scene * nb3 + (uint32_t)((k * nb + j) * nb + i)] = 1u;
  }
}

__global__ void k_flag_marked(const uint32_t* __restrict__ mark, uint32_t n_blocks,
                              uint32_t* __restrict__ flags) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks; b += gridDim.x * blockDim.x)
    flags[b] = mark[b] == 1u ? 1u : 0u;
}

// Work items of each block (one per `item` particles or part of it).
__global__ void k_item_counts(const uint32_t* __restrict__ begin, const uint32_t* __restrict__ end,
                              uint32_t n_blocks, uint32_t item, uint32_t* __restrict__ counts) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks; b += gridDim.x * blockDim.x)
    counts[b] = end[b] > begin[b] ? (end[b] - begin[b] + item - 1) / item : 0u;
}

// work[off[b] + j] = {b, begin[b] + j item}, with kDenseFlag in b when the
// block holds more than `dense` particles.
__global__ void k_emit_items(const uint32_t* __restrict__ begin, const uint32_t* __restrict__ end,
                             const uint32_t* __restrict__ off, uint32_t n_blocks, uint32_t item, uint32_t dense,
                             uint2* __restrict__ work) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks; b += gridDim.x * blockDim.x) {
    if (!(end[b] > begin[b])) continue;
    uint32_t o = off[b];
    const uint32_t tag = (end[b] - begin[b] > dense) ? kDenseFlag : 0u;
    for (uint32_t p = begin[b]; p < end[b]; p += item) work[o++] = make_uint2(b | tag, p);
  }
}

// Work items of each XCD's range (the contiguous eighth of the list that
// the transfer kernels' walk gives an XCD) from `src` to `dst` in decreasing
// size, in buckets of item_particles / 64 particles and in list (spatial)
// order within a bucket: the workgroups of an XCD take its first items and
// then claim the rest in order, so the items claimed last, at the end of a
// launch, are the small ones (longest first). One workgroup per range; tiles
// of the range in order, each item ranked among the tile's items of its
// bucket before it, keep the order within a bucket.
constexpr int kOrderWG = 256;
constexpr int kSizeBuckets = 64;
__global__ __launch_bounds__(kOrderWG) void k_order_items(const uint2* __restrict__ src, uint2* __restrict__ dst,
                                                          const uint32_t* __restrict__ blk_end, const Status* st,
                                                          uint32_t item, int bucket_shift) {
  __shared__ uint32_t cnt[kSizeBuckets], start[kSizeBuckets];
  __shared__ uint8_t tb[kOrderWG];
  const uint32_t n = st->n_work, chunk = (n + kXcds - 1) / kXcds;
  const uint32_t lo = min(blockIdx.x * chunk, n), hi = min(lo + chunk, n);
  auto bucket = [&](uint2 it) -> uint32_t {
    const uint32_t c = min(item, blk_end[it.x & ~kDenseFlag] - it.y);
    return (kSizeBuckets - 1) - min((uint32_t)(kSizeBuckets - 1), c >> bucket_shift);
  };
  if (threadIdx.x < kSizeBuckets) cnt[threadIdx.x] = 0u;
  __syncthreads();
  for (uint32_t i = lo + threadIdx.x; i < hi; i += kOrderWG) atomicAdd(&cnt[bucket(src[i])], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = lo;
    for (int k = 0; k < kSizeBuckets; ++k) {
      start[k] = s;
      s += cnt[k];
    }
  }
  __syncthreads();
  for (uint32_t t0 = lo; t0 < hi; t0 += kOrderWG) {
    const uint32_t i = t0 + threadIdx.x;
    const bool has = i < hi;
    const uint2 it = has ? src[i] : make_uint2(0u, 0u);
    const uint32_t bk = has ? bucket(it) : (uint32_t)kSizeBuckets;
    tb[threadIdx.x] = (uint8_t)bk;
    __syncthreads();
    if (has) {
      uint32_t rank = 0u;
      for (uint32_t j = 0; j < threadIdx.x; ++j) rank += tb[j] == bk;
      dst[start[bk] + rank] = it;
    }
    __syncthreads();
    if (threadIdx.x < kSizeBuckets) {
      uint32_t c = 0u;
      for (int j = 0; j < kOrderWG; ++j) c += tb[j] == threadIdx.x;
      start[threadIdx.x] += c;
    }
    __syncthreads();
  }
}

// list[pos[b]] = b for flagged blocks; flags and pos may not alias.
__global__ void k_compact(const uint32_t* __restrict__ mark_or_range_b,
                          const uint32_t* __restrict__ range_e, const uint32_t* __restrict__ pos,
                          uint32_t n_blocks, int mode, uint32_t* __restrict__ list) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_blocks; b += gridDim.x * blockDim.x) {
    const bool take = (mode == 0) ? (range_e[b] > mark_or_range_b[b]) : (mark_or_range_b[b] == 1u);
    if (take) list[pos[b]] = b;
  }
}

__global__ void k_reset_epoch(Status* st) {
  st->ovf_count[0] = 0u;
  st->ovf_count[1] = 0u;
  st->fb_at_sort = st->n_fallback;
}

static unsigned grid_for(int64_t n, int wg) {
  int64_t g = (n + wg - 1) / wg;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Stable LSD radix sort of (b.keys[0], b.vals[0]), 8 bits per pass; returns
// which ping-pong half holds the result.
static int radix_sort(Buffers& b, int64_t N, int key_bits, hipStream_t st) {
  int src = 0;
  if (N > 0) {
    const int n_tiles = (int)((N + kSortTile - 1) / kSortTile);
    for (int shift = 0; shift < key_bits; shift += 8) {
      hipLaunchKernelGGL(k_radix_hist, dim3(n_tiles), dim3(kSortWG), 0, st, b.keys[src], N, shift,
                         b.hist, n_tiles);
      exclusive_scan(b.hist, b.hist, (int64_t)kRadix * n_tiles, b.scan_tmp, nullptr, st);
      hipLaunchKernelGGL(k_radix_scatter, dim3(n_tiles), dim3(kSortWG), 0, st, b.keys[src], b.vals[src],
                         b.keys[src ^ 1], b.vals[src ^ 1], N, shift, b.hist, n_tiles);
      src ^= 1;
    }
  }
  return src;
}

// Tile counts of particles in memory order, for the binning of new
// particles: the keys and their sort as in launch_binning, then the tile
// ranges of the sorted keys in blk_begin / blk_end; the particles stay where
// they are and no list is built. The binning that follows reads the counts.
void launch_tile_counts(Buffers& b, int64_t N, const SimK& s, int key_bits, hipStream_t st) {
  const uint32_t n_blocks = s.nb3 * (uint32_t)s.n_scenes;
  const uint32_t n_units = n_blocks << s.unit_shift;
  const uint32_t sentinel = n_units << kClassBits;
  hipLaunchKernelGGL(k_keygen, dim3(grid_for(N, 256)), dim3(256), 0, st, b.part[b.cur], b.id[b.cur],
                     b.scene_off, b.cap, N, s, b.blk_begin, b.blk_end, b.keys[0], b.vals[0], sentinel, b.status);
  const int src = radix_sort(b, N, key_bits + kClassBits, st);
  fill_u32(b.blk_begin, n_units, 0u, st);
  fill_u32(b.blk_end, n_units, 0u, st);
  hipLaunchKernelGGL(k_ranges, dim3(grid_for(N, 256)), dim3(256), 0, st, b.keys[src], N, n_units, kClassBits,
                     b.blk_begin, b.blk_end);
}

void launch_binning(Buffers& b, int64_t N, const SimK& s, int key_bits, bool with_vc, hipStream_t st) {
  const uint32_t n_blocks = s.nb3 * (uint32_t)s.n_scenes;
  const uint32_t n_units = n_blocks << s.unit_shift;  // work tiles
  const uint32_t sentinel = n_units << kClassBits;
  // 1. keys: scene-major work tile ids, then sub-cell classes
  hipLaunchKernelGGL(k_keygen, dim3(grid_for(N, 256)), dim3(256), 0, st, b.part[b.cur], b.id[b.cur],
                     b.scene_off, b.cap, N, s, b.blk_begin, b.blk_end, b.keys[0], b.vals[0], sentinel, b.status);
  // 2. stable LSD radix sort, 8 bits per pass (key_bits: bits of a work tile id or the sentinel)
  const int src = radix_sort(b, N, key_bits + kClassBits, st);
  // 3. gather the particle state into key order
  const dim3 pg(grid_for(N, 256)), pb(256);
  const float* ps = b.part[b.cur];
  float* pd = b.part[b.cur ^ 1];
  const uint32_t* kk = b.keys[src];
  if (with_vc && s.has_E)
    hipLaunchKernelGGL((k_permute<true, true>), pg, pb, 0, st, ps, pd, b.id[b.cur], b.id[b.cur ^ 1], b.vals[src], kk,
                       sentinel, b.cap, N);
  else if (with_vc)
    hipLaunchKernelGGL((k_permute<true, false>), pg, pb, 0, st, ps, pd, b.id[b.cur], b.id[b.cur ^ 1], b.vals[src], kk,
                       sentinel, b.cap, N);
  else if (s.has_E)
    hipLaunchKernelGGL((k_permute<false, true>), pg, pb, 0, st, ps, pd, b.id[b.cur], b.id[b.cur ^ 1], b.vals[src], kk,
                       sentinel, b.cap, N);
  else
    hipLaunchKernelGGL((k_permute<false, false>), pg, pb, 0, st, ps, pd, b.id[b.cur], b.id[b.cur ^ 1], b.vals[src], kk,
                       sentinel, b.cap, N);
  b.cur ^= 1;
  // 4. per-tile ranges
  fill_u32(b.blk_begin, n_units, 0u, st);
  fill_u32(b.blk_end, n_units, 0u, st);
  hipLaunchKernelGGL(k_ranges, dim3(grid_for(N, 256)), dim3(256), 0, st, b.keys[src], N, n_units, kClassBits,
                     b.blk_begin, b.blk_end);
  // 5. occupied list (ascending tile id: spatially ordered, x fastest)
  hipLaunchKernelGGL(k_flag_occupied, dim3(grid_for(n_units, 256)), dim3(256), 0, st, b.blk_begin,
                     b.blk_end, n_units, b.flags);
  exclusive_scan(b.flags, b.flags, n_units, b.scan_tmp, &b.status->n_occ, st);
  hipLaunchKernelGGL(k_compact, dim3(grid_for(n_units, 256)), dim3(256), 0, st, b.blk_begin, b.blk_end,
                     b.flags, n_units, 0, b.occ_list);
  // 5b. transfer work items (ascending tile id, then particle runs); tiles
  // above 8 particles per cell are dense
  const uint32_t dense = 8u * (uint32_t)(s.tile * s.tile * s.tile);
  hipLaunchKernelGGL(k_item_counts, dim3(grid_for(n_units, 256)), dim3(256), 0, st, b.blk_begin, b.blk_end,
                     n_units, s.item_particles, b.flags);
  exclusive_scan(b.flags, b.flags, n_units, b.scan_tmp, &b.status->n_work, st);
  hipLaunchKernelGGL(k_emit_items, dim3(grid_for(n_units, 256)), dim3(256), 0, st, b.blk_begin, b.blk_end,
                     b.flags, n_units, s.item_particles, dense, b.work_tmp);
  // 5c. largest items first within each XCD's range
  int bucket_shift = 0;
  while (((uint32_t)kSizeBuckets << (bucket_shift + 1)) <= (uint32_t)s.item_particles) ++bucket_shift;
  hipLaunchKernelGGL(k_order_items, dim3(kXcds), dim3(kOrderWG), 0, st, (const uint2*)b.work_tmp, b.work,
                     (const uint32_t*)b.blk_end, (const Status*)b.status, (uint32_t)s.item_particles, bucket_shift);
  // 6. active list: the grid blocks the occupied tiles' LDS tiles touch
  fill_u32(b.mark, n_blocks, 0u, st);
  hipLaunchKernelGGL(k_mark_dilated, dim3(grid_for(n_units, 256)), dim3(256), 0, st, b.blk_begin,
                     b.blk_end, s.nb, s.nb3, n_units, s.tile, s.unit_shift, b.mark);
  hipLaunchKernelGGL(k_flag_marked, dim3(grid_for(n_blocks, 256)), dim3(256), 0, st, b.mark, n_blocks,
                     b.flags);
  exclusive_scan(b.flags, b.flags, n_blocks, b.scan_tmp, &b.status->n_act, st);
  hipLaunchKernelGGL(k_compact, dim3(grid_for(n_blocks, 256)), dim3(256), 0, st, b.mark, nullptr,
                     b.flags, n_blocks, 1, b.act_list);
  hipLaunchKernelGGL(k_reset_epoch, dim3(1), dim3(1), 0, st, b.status);
}

// ------------------------------------------------------------------ rollout order
// Keys of particles held as an AoS x (N x 3) in the caller's order: the block
// of the base cell (one scene), or the sentinel when the stencil leaves the
// grid or x is not finite.
__global__ void k_order_keys(const float* __restrict__ x, int64_t N, SimK s, uint32_t sentinel,
                             uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    int cell[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
      const float r = x[3 * i + a] * s.inv_dx;
      const float c = floorf(r - 0.5f);
      ok = ok && (c >= 0.0f) && (c + 2.0f <= (float)(s.n - 1));  // false for NaN
      cell[a] = ok ? (int)c : 0;
    }
    keys[i] = ok ? (uint32_t)(((cell[2] >> kTileLog2) * s.nb + (cell[1] >> kTileLog2)) * s.nb + (cell[0] >> kTileLog2))
                 : sentinel;
    vals[i] = (uint32_t)i;
  }
}

// First sorted position holding the sentinel key (left at N when there is
// none).
__global__ void k_first_sentinel(const uint32_t* __restrict__ keys, int64_t N, uint32_t sentinel,
                                 uint32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    if (keys[i] >= sentinel && (i == 0 || keys[i - 1] < sentinel)) *out = (uint32_t)i;
}

hipError_t launch_order(Buffers& b, int64_t N, const SimK& s, const float* x, int key_bits, uint32_t item,
                        uint32_t* order, uint32_t* begin, uint32_t* end, uint2* work, uint32_t* info,
                        hipStream_t st) {
  const uint32_t n_blocks = s.nb3;
  hipLaunchKernelGGL(k_order_keys, dim3(grid_for(N, 256)), dim3(256), 0, st, x, N, s, n_blocks, b.keys[0],
                     b.vals[0]);
  const int src = radix_sort(b, N, key_bits, st);
  fill_u32(begin, n_blocks, 0u, st);
  fill_u32(end, n_blocks, 0u, st);
  hipLaunchKernelGGL(k_ranges, dim3(grid_for(N, 256)), dim3(256), 0, st, b.keys[src], N, n_blocks, 0, begin, end);
  hipLaunchKernelGGL(k_item_counts, dim3(grid_for(n_blocks, 256)), dim3(256), 0, st, begin, end, n_blocks, item,
                     b.flags);
  exclusive_scan(b.flags, b.flags, n_blocks, b.scan_tmp, &info[0], st);
  hipLaunchKernelGGL(k_emit_items, dim3(grid_for(n_blocks, 256)), dim3(256), 0, st, begin, end, b.flags, n_blocks,
                     item, 0xffffffffu, work);  // never flagged
  fill_u32(&info[1], 1, (uint32_t)N, st);
  hipLaunchKernelGGL(k_first_sentinel, dim3(grid_for(N, 256)), dim3(256), 0, st, b.keys[src], N, n_blocks,
                     &info[1]);
  if (N == 0) return hipSuccess;
  return hipMemcpyAsync(order, b.vals[src], sizeof(uint32_t) * (size_t)N, hipMemcpyDeviceToDevice, st);
}

// ------------------------------------------------------------------ diagnostics
__global__ void k_count_active_nodes(const uint32_t* __restrict__ node_cnt, const uint32_t* __restrict__ act_list,
                                     const uint32_t* __restrict__ ovf_list, const Status* st, int parity,
                                     unsigned long long* out) {
  __shared__ unsigned long long sh[256];
  const unsigned n_act = st->n_act, total = n_act + st->ovf_count[parity];
  unsigned long long s = 0;
  for (unsigned i = threadIdx.x; i < total; i += blockDim.x)
    s += node_cnt[i < n_act ? act_list[i] : ovf_list[i - n_act]];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

void launch_count_active_nodes(Buffers& b, int parity, unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_count_active_nodes, dim3(1), dim3(256), 0, st, b.node_cnt, b.act_list,
                     b.ovf_list[parity], b.status, parity, out);
}

// Impulse totals of one scene: the per-block sums of its nb^3 blocks. Thread
// (r, c) of kSumRows x 27 adds component c of blocks r, r + kSumRows, ...
constexpr int kSumRows = 8;
__global__ void k_sum_impulses(const float* __restrict__ blocks, uint32_t first, uint32_t count,
                               double* __restrict__ out) {
  __shared__ double part[kSumRows][kImpulseRows * 3];
  const int c = threadIdx.x % (kImpulseRows * 3), r = threadIdx.x / (kImpulseRows * 3);
  double s = 0.0;
  for (uint32_t i = r; i < count; i += kSumRows) s += (double)blocks[(size_t)(first + i) * (kImpulseRows * 3) + c];
  part[r][c] = s;
  __syncthreads();
  if (r == 0) {
    double t = 0.0;
    for (int k = 0; k < kSumRows; ++k) t += part[k][c];
    out[c] = t;
  }
}

void launch_clear_impulses(Buffers& b, const SimK& s, hipStream_t st) {
  fill_u32((uint32_t*)b.imp_blocks, (int64_t)s.nb3 * s.n_scenes * kImpulseRows * 3, 0u, st);
}

void launch_sum_impulses(Buffers& b, const SimK& s, int scene, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_impulses, dim3(1), dim3(kSumRows * kImpulseRows * 3), 0, st, b.imp_blocks,
                     (uint32_t)scene * s.nb3, s.nb3, out);
}

// ------------------------------------------------------------------ marshalling
__global__ void k_load(float* __restrict__ part, uint32_t* __restrict__ id, int64_t cap, int64_t N,
                       const float* __restrict__ x, const float* __restrict__ v,
                       const float* __restrict__ C, const float* __restrict__ F,
                       const float* __restrict__ E) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    for (int a = 0; a < 3; ++a) {
      part[(FX + a) * cap + i] = x[3 * i + a];
      part[(FV + a) * cap + i] = v ? v[3 * i + a] : 0.0f;
    }
    for (int k = 0; k < 9; ++k) {
      part[(FC + k) * cap + i] = C ? C[9 * i + k] : 0.0f;
      part[(FF + k) * cap + i] = F ? F[9 * i + k] : ((k % 4 == 0) ? 1.0f : 0.0f);
    }
    if (E) part[FE * cap + i] = E[i];
    id[i] = (uint32_t)i;
  }
}

void launch_load_particles(Buffers& b, int64_t N, const float* x, const float* v, const float* C,
                           const float* F, const float* E, hipStream_t st) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_load, dim3(grid_for(N, 256)), dim3(256), 0, st, b.part[b.cur], b.id[b.cur], b.cap, N,
                     x, v, C, F, E);
}

__global__ void k_unpermute(const float* __restrict__ part, const uint32_t* __restrict__ id, int64_t cap,
                            int64_t N, float* __restrict__ x, float* __restrict__ v,
                            float* __restrict__ C, float* __restrict__ F) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = id[i];
    for (int a = 0; a < 3; ++a) {
      if (x) x[3 * o + a] = part[(FX + a) * cap + i];
      if (v) v[3 * o + a] = part[(FV + a) * cap + i];
    }
    for (int k = 0; k < 9; ++k) {
      if (C) C[9 * o + k] = part[(FC + k) * cap + i];
      if (F) F[9 * o + k] = part[(FF + k) * cap + i];
    }
  }
}

void launch_unpermute(const Buffers& b, int64_t N, float* x, float* v, float* C, float* F, hipStream_t st) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_unpermute, dim3(grid_for(N, 256)), dim3(256), 0, st, b.part[b.cur], b.id[b.cur], b.cap,
                     N, x, v, C, F);
}

__global__ void k_eval_stress(int64_t n, const float* __restrict__ F, const float* __restrict__ E,
                              float c_mu, float c_la, float* __restrict__ tau) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float f[9], t[9];
    for (int k = 0; k < 9; ++k) f[k] = F[9 * i + k];
    bool inv;
    kirchhoff(f, c_mu * E[i], c_la * E[i], t, &inv);
    for (int k = 0; k < 9; ++k) tau[9 * i + k] = t[k];
  }
}

void launch_eval_stress(int64_t n, const float* F, const float* E, float nu, float* tau, hipStream_t st) {
  if (n <= 0) return;
  const double dnu = nu;
  const float c_mu = (float)(1.0 / (2.0 * (1.0 + dnu)));
  const float c_la = (float)(dnu / ((1.0 + dnu) * (1.0 - 2.0 * dnu)));
  hipLaunchKernelGGL(k_eval_stress, dim3(grid_for(n, 256)), dim3(256), 0, st, n, F, E, c_mu, c_la, tau);
}

}  // namespace mpm
