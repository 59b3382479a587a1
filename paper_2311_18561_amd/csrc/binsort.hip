// Tile binning and depth ordering (Sec. 3.1: Gaussians sorted by camera depth,
// rendered per 16x16 tile) on gfx950.
//
// The instance order is the lexicographic order of (tile, depth bits, index).
// It is built as a least-significant-digit radix sort whose depth digits are
// hoisted in front of the duplication:
//   1. compact the visible Gaussians (index order) with their depth bits;
//   2. stable LSD radix sort of (depth bits, index) over the visible ones only;
//   3. scan the tile counts in that order and emit, for each Gaussian, one
//      instance per tile of its rectangle (row-major) - instances now appear
//      in (depth, index) order;
//   4. stable LSD radix sort of the instances by tile id (ceil(bits/8) passes);
//   5. per-tile [first, last+1) ranges.
// Step 4's stability keeps (depth, index) order inside a tile, so the result
// equals a full sort of (tile, depth, index) keys, while the passes over the
// instance array move 8 bytes per instance instead of 12.
//
// With tile culling on, step 3 lists a Gaussian only in the tiles it can
// reach (alpha >= 1/255 at some pixel).  Those form one column interval per
// tile row of its rectangle, so the culled emission works on rows: count the
// rectangle rows, compute every row's interval once (a thread per Gaussian,
// at most one loop over its rows), scan the interval lengths into instance
// offsets and write each row's interval (a thread per row).  Fewer instances
// then reach the tile sort, the ranges and the compositing loops.
//
// Every radix pass is the classic three-kernel form: per-block digit
// histograms in LDS (atomics on LDS counters), an exclusive scan of each
// digit's row of block counts, and a scatter whose in-block ranks come from
// wave ballots (lanes with equal digits) and per-wave LDS counters, which keeps
// the sort stable.  Counts live on the device; kernels sized for a capacity
// exit early past the live count, so no host synchronisation is needed.
#include <mutex>

#include "pvg_math.hpp"

namespace pvg {

constexpr int kThreads = 256;
constexpr int kScanItems = 4;                       // items per thread in the scans / compaction
constexpr int kScanBlock = kThreads * kScanItems;   // 1024
constexpr int kRsItems = 16;                        // items per thread in a tile pass
constexpr int kRsBlock = kThreads * kRsItems;       // 4096
// Items per thread in a depth pass: 1024 keys a block, so that the visible
// Gaussians of one view (0.58M in the benchmark) fill the chip: with 4096 the
// passes had 142 blocks for 256 CUs, and their scatter ran at 0.5 TB/s.
constexpr int kDepthItems = 4;
constexpr int kDepthBlock = kThreads * kDepthItems;  // 1024
// Digits of the depth passes.  Three passes of 11 bits measured slower than
// four of 8 on the benchmark's 0.58M visible Gaussians (2048-digit block
// scans and 11 ballots per key outweigh the saved pass).
constexpr int kDepthBits = 8;
constexpr int kDepthPasses = (32 + kDepthBits - 1) / kDepthBits;

// ------------------------------------------------------------------ helpers
template <class T>
__device__ __forceinline__ T wave_incl_scan(T x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over a 256-thread block.
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T* lds5, T& total) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const T x = wave_incl_scan<T>(v, lane);
  if (lane == 63) lds5[wid] = x;
  __syncthreads();
  if (tid == 0) {
    T s = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      const T t = lds5[w];
      lds5[w] = s;
      s += t;
    }
    lds5[4] = s;
  }
  __syncthreads();
  const T r = lds5[wid] + x - v;
  total = lds5[4];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t live_count(const uint32_t* n_dev, int64_t n_host) {
  return n_dev ? static_cast<int64_t>(*n_dev) : n_host;
}
__device__ __forceinline__ int64_t live_count64(const int64_t* n_dev, int64_t n_host) {
  return n_dev ? *n_dev : n_host;
}

// ------------------------------------------------------------------ step 1: compaction
__global__ void __launch_bounds__(kThreads) k_vis_count(const uint32_t* __restrict__ tiles, const int64_t* n_live,
                                                        int64_t n_host, unsigned long long* partials) {
  __shared__ unsigned long long lds[5];
  const int64_t n = live_count64(n_live, n_host);
  if (static_cast<int64_t>(blockIdx.x) * kScanBlock >= n) return;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x * kScanItems;
  unsigned long long c = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n && tiles[base + k] > 0u) ++c;
  unsigned long long tot;
  block_excl_scan<unsigned long long>(c, lds, tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Exclusive scan of `count` block partials in place (one block), unless
// *skip is set.  The total goes to *total_out; with cap >= 0 it is checked
// against the capacity: over it, *total_out = 0 and *over_flag = 1.
// sat_out (optional) receives the total saturated to 32 bits.
__global__ void __launch_bounds__(1024) k_scan_partials(unsigned long long* partials, const uint32_t* count_dev,
                                                        const int64_t* count_dev64, int64_t count_host,
                                                        int per_block, uint32_t* total_out, int64_t cap,
                                                        uint32_t* over_flag, uint32_t* sat_out,
                                                        const uint32_t* skip) {
  __shared__ unsigned long long wsum[17];
  if (skip && *skip) return;
  const int64_t items = count_dev64 ? *count_dev64 : live_count(count_dev, count_host);
  const int64_t count = (items + per_block - 1) / per_block;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  unsigned long long carry = 0;
  for (int64_t base = 0; base < count; base += 1024) {
    const int64_t i = base + tid;
    const unsigned long long v = i < count ? partials[i] : 0ull;
    const unsigned long long x = wave_incl_scan<unsigned long long>(v, lane);
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (tid == 0) {
      unsigned long long s = 0;
      for (int w = 0; w < 16; ++w) {
        const unsigned long long t = wsum[w];
        wsum[w] = s;
        s += t;
      }
      wsum[16] = s;
    }
    __syncthreads();
    if (i < count) partials[i] = carry + wsum[wid] + x - v;
    carry += wsum[16];
    __syncthreads();
  }
  if (tid == 0) {
    const bool over = cap >= 0 && carry > static_cast<unsigned long long>(cap);
    *total_out = over ? 0u : static_cast<uint32_t>(carry);
    if (over) *over_flag = 1u;
    if (sat_out) *sat_out = carry > 0xffffffffull ? 0xffffffffu : static_cast<uint32_t>(carry);
  }
}

__global__ void __launch_bounds__(kThreads) k_vis_compact(const uint32_t* __restrict__ tiles,
                                                          const float* __restrict__ depth, const int64_t* n_live,
                                                          int64_t n_host,
                                                          const unsigned long long* __restrict__ partials,
                                                          uint32_t* keys, uint32_t* vals) {
  __shared__ unsigned long long lds[5];
  const int64_t n = live_count64(n_live, n_host);
  if (static_cast<int64_t>(blockIdx.x) * kScanBlock >= n) return;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x * kScanItems;
  bool f[kScanItems];
  unsigned long long c = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    f[k] = base + k < n && tiles[base + k] > 0u;
    c += f[k] ? 1 : 0;
  }
  unsigned long long tot;
  unsigned long long pos = block_excl_scan<unsigned long long>(c, lds, tot) + partials[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (f[k]) {
      keys[pos] = __float_as_uint(depth[base + k]);
      vals[pos] = static_cast<uint32_t>(base + k);
      ++pos;
    }
  }
}

// ------------------------------------------------------------------ radix passes
// kMaxBits: the widest digit a kernel instance handles (8 for the tile
// passes, 11 for the depth passes: 32 bits in three passes); `bits` <= it.
template <int kMaxBits, int kPer>
__global__ void __launch_bounds__(kThreads) k_rs_hist(const uint32_t* __restrict__ keys, const uint32_t* n_dev,
                                                      int64_t n_host, int shift, int bits, uint32_t* hist,
                                                      int64_t cols) {
  constexpr int kR = 1 << kMaxBits;
  constexpr int kBlock = kThreads * kPer;
  __shared__ uint32_t h[kR];
  const int64_t n = live_count(n_dev, n_host);
  const int64_t nb = (n + kBlock - 1) / kBlock;
  const int radix = 1 << bits;
  const uint32_t mask = static_cast<uint32_t>(radix - 1);
  for (int64_t lb = blockIdx.x; lb < nb; lb += gridDim.x) {
    for (int d = threadIdx.x; d < radix; d += kThreads) h[d] = 0;
    __syncthreads();
    const int64_t base = lb * kBlock + threadIdx.x;
#pragma unroll 4
    for (int k = 0; k < kPer; ++k) {
      const int64_t i = base + k * kThreads;
      if (i < n) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < radix; d += kThreads) hist[d * cols + lb] = h[d];
    __syncthreads();
  }
}

// One block per digit: exclusive scan of that digit's block counts (blocks
// of `block` keys).
__global__ void __launch_bounds__(kThreads) k_rs_rowscan(uint32_t* hist, int64_t cols, const uint32_t* n_dev,
                                                         int64_t n_host, int64_t block, uint32_t* rowtot) {
  __shared__ uint32_t lds[5];
  const int64_t n = live_count(n_dev, n_host);
  const int64_t nb = (n + block - 1) / block;
  uint32_t* row = hist + blockIdx.x * cols;
  uint32_t carry = 0;
  for (int64_t base = 0; base < nb; base += kThreads * 4) {
    const int64_t i0 = base + threadIdx.x * 4;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = i0 + k < nb ? row[i0 + k] : 0u;
      s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<uint32_t>(s, lds, tot) + carry;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < nb) row[i0 + k] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = carry;
}

// Scatter of one stable LSD pass.  Each wave ranks its own contiguous 1024
// keys (wave ballots find lanes with equal digits; a wave-private LDS counter
// per digit carries ranks across its 16 sub-tiles), the block combines the
// four waves per digit, stages the block's 4096 pairs locally sorted in LDS and
// writes each digit's run contiguously.  A thread owns kPerT consecutive
// digits in the block-wide digit scans.
template <int kMaxBits, int kPer>
__global__ void __launch_bounds__(kThreads) k_rs_scatter(const uint32_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin, uint32_t* kout,
                                                         uint32_t* vout, const uint32_t* n_dev, int64_t n_host,
                                                         int shift, int bits, const uint32_t* __restrict__ hist,
                                                         int64_t cols, const uint32_t* __restrict__ rowtot) {
  constexpr int kR = 1 << kMaxBits;
  constexpr int kPerT = kR / kThreads > 0 ? kR / kThreads : 1;  // digits per thread in the digit scans
  constexpr int kBlock = kThreads * kPer;        // items per block
  constexpr int kWaveItems = 64 * kPer;          // contiguous items per wave
  __shared__ uint32_t s_cnt[kThreads / 64][kR];  // per-wave digit counts, then per-wave digit bases
  __shared__ uint32_t s_off[kR];                 // block-local first slot of each digit
  __shared__ uint32_t s_gbase[kR];               // global first slot of each digit for this block
  __shared__ uint32_t s_k[kBlock];
  __shared__ uint32_t s_v[kBlock];
  __shared__ uint32_t lds[5];
  const int64_t n = live_count(n_dev, n_host);
  const int64_t nb = (n + kBlock - 1) / kBlock;
  if (static_cast<int64_t>(blockIdx.x) >= nb) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int radix = 1 << bits;
  const uint32_t mask = static_cast<uint32_t>(radix - 1);
  const uint64_t lt = (1ull << lane) - 1ull;
  // digit_base[j]: first global slot of digit tid * kPerT + j
  uint32_t digit_base[kPerT];
  {
    uint32_t t[kPerT], sum = 0;
#pragma unroll
    for (int j = 0; j < kPerT; ++j) {
      const int d = tid * kPerT + j;
      t[j] = d < radix ? rowtot[d] : 0u;
      sum += t[j];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<uint32_t>(sum, lds, tot);
#pragma unroll
    for (int j = 0; j < kPerT; ++j) {
      digit_base[j] = run;
      run += t[j];
    }
  }
  for (int64_t lb = blockIdx.x; lb < nb; lb += gridDim.x) {
    for (int w = 0; w < kThreads / 64; ++w)
      for (int d = tid; d < radix; d += kThreads) s_cnt[w][d] = 0;
#pragma unroll
    for (int j = 0; j < kPerT; ++j) {
      const int d = tid * kPerT + j;
      if (d < radix) s_gbase[d] = digit_base[j] + hist[d * cols + lb];
    }
    __syncthreads();
    // phase 1: wave-local stable ranks
    const int64_t wbase = lb * kBlock + static_cast<int64_t>(wid) * kWaveItems;
    uint32_t key[kPer], val[kPer], rank[kPer];
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int64_t i = wbase + it * 64 + lane;
      const bool valid = i < n;
      key[it] = valid ? kin[i] : 0u;
      val[it] = valid ? vin[i] : 0u;
      const uint32_t dig = (key[it] >> shift) & mask;
      uint64_t peers = __ballot(valid);
      for (int b = 0; b < bits; ++b) {
        const bool bit = (dig >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
      }
      uint32_t old = 0;
      if (valid) old = s_cnt[wid][dig];
      rank[it] = old + static_cast<uint32_t>(__popcll(peers & lt));
      __builtin_amdgcn_wave_barrier();
      if (valid && (peers & lt) == 0) s_cnt[wid][dig] = old + static_cast<uint32_t>(__popcll(peers));
      __builtin_amdgcn_wave_barrier();
      if (!valid) rank[it] = 0xffffffffu;
    }
    __syncthreads();
    // phase 2: per digit, combine the waves and scan over digits
    {
      uint32_t c[kPerT][kThreads / 64], tot[kPerT], sum = 0;
#pragma unroll
      for (int j = 0; j < kPerT; ++j) {
        const int d = tid * kPerT + j;
        tot[j] = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
          c[j][w] = d < radix ? s_cnt[w][d] : 0u;
          tot[j] += c[j][w];
        }
        sum += tot[j];
      }
      uint32_t all;
      uint32_t off = block_excl_scan<uint32_t>(sum, lds, all);
#pragma unroll
      for (int j = 0; j < kPerT; ++j) {
        const int d = tid * kPerT + j;
        if (d < radix) {
          s_off[d] = off;
          uint32_t run = off;
          for (int w = 0; w < kThreads / 64; ++w) {
            s_cnt[w][d] = run;
            run += c[j][w];
          }
        }
        off += tot[j];
      }
    }
    __syncthreads();
    // phase 3: stage locally sorted
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      if (rank[it] != 0xffffffffu) {
        const uint32_t dig = (key[it] >> shift) & mask;
        const uint32_t p = s_cnt[wid][dig] + rank[it];
        s_k[p] = key[it];
        s_v[p] = val[it];
      }
    }
    __syncthreads();
    // phase 4: coalesced runs out
    const int64_t live = min(static_cast<int64_t>(kBlock), n - lb * kBlock);
    for (int p = tid; p < live; p += kThreads) {
      const uint32_t k = s_k[p];
      const uint32_t dig = (k >> shift) & mask;
      const uint32_t o = s_gbase[dig] + (static_cast<uint32_t>(p) - s_off[dig]);
      kout[o] = k;
      vout[o] = s_v[p];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ step 3: tile counts and emission
__global__ void __launch_bounds__(kThreads) k_tile_count(const uint32_t* __restrict__ order,
                                                         const uint32_t* __restrict__ tiles, const uint32_t* n_dev,
                                                         int64_t n_host, unsigned long long* partials) {
  __shared__ unsigned long long lds[5];
  const int64_t n = live_count(n_dev, n_host);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x * kScanItems;
  if (static_cast<int64_t>(blockIdx.x) * kScanBlock >= n) return;
  unsigned long long c = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) c += tiles[order[base + k]];
  unsigned long long tot;
  block_excl_scan<unsigned long long>(c, lds, tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__device__ __forceinline__ int32_t clamp_tile_e(float v, int32_t hi) {
  const float f = floorf(v);
  if (f < 0.0f) return 0;
  if (f > static_cast<float>(hi)) return hi;
  return static_cast<int32_t>(f);
}

// First instance of each visible Gaussian in depth order: the exclusive scan
// of the tile counts (block partials already scanned).
__global__ void __launch_bounds__(kThreads) k_tile_offsets(const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ tiles,
                                                           const uint32_t* n_dev, int64_t n_host,
                                                           const unsigned long long* __restrict__ partials,
                                                           const uint32_t* __restrict__ counters,
                                                           uint32_t* offsets, uint32_t* first) {
  __shared__ unsigned long long lds[5];
  if (counters[2]) return;  // over capacity: offsets would not fit 32 bits, nothing is emitted
  const int64_t n = live_count(n_dev, n_host);
  if (static_cast<int64_t>(blockIdx.x) * kScanBlock >= n) return;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x * kScanItems;
  uint32_t c[kScanItems];
  unsigned long long sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    c[k] = base + k < n ? tiles[order[base + k]] : 0u;
    sum += c[k];
  }
  unsigned long long tot;
  unsigned long long r = block_excl_scan<unsigned long long>(sum, lds, tot) + partials[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) {
      offsets[base + k] = static_cast<uint32_t>(r);
      if (first) first[order[base + k]] = static_cast<uint32_t>(r);
    }
    r += c[k];
  }
}

// Last k in [0, n) with a[k] <= x, for non-decreasing a with a[0] <= x, by a
// 64-way search of the whole wave (each round shrinks the interval 64x).
__device__ __forceinline__ int64_t wave_last_le(const uint32_t* __restrict__ a, int64_t n, uint32_t x, int lane) {
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int64_t p = lo + (((hi - lo) * (lane + 1)) >> 6);
    const bool ok = p <= lo || (p < hi && a[p] <= x);
    const int L = __popcll(__ballot(ok));  // ok holds for a prefix of the lanes
    const int64_t nlo = L > 0 ? __shfl(p, L - 1, 64) : lo;
    const int64_t nhi = __shfl(p, L, 64);
    lo = nlo > lo ? nlo : lo;
    hi = nhi;
  }
  return lo;
}

constexpr int kEmitChunk = 2048;  // instances per block iteration

// Instance emission balanced by instances: a block writes a fixed chunk of
// the instance array, finds the Gaussians that own it with a wave search over
// the offsets, stages their rectangles in LDS and fills the chunk (coalesced),
// so a few huge near-camera splats cannot serialise one block.
__global__ void __launch_bounds__(kThreads) k_emit(ViewSet vs, const uint32_t* __restrict__ order,
                                                   const float* __restrict__ xy, const int32_t* __restrict__ radius,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint32_t* __restrict__ counters, uint32_t* keys,
                                                   uint32_t* vals) {
  __shared__ uint32_t s_off[kEmitChunk];
  __shared__ uint32_t s_g[kEmitChunk];
  __shared__ uint32_t s_base[kEmitChunk];
  __shared__ uint32_t s_wg[kEmitChunk];  // rectangle width (low 16) | tile grid width (high 16)
  __shared__ int64_t s_k[2];
  if (counters[2]) return;
  const int64_t M = counters[0];
  const int64_t nvis = counters[1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t nchunks = (M + kEmitChunk - 1) / kEmitChunk;
  for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const int64_t j0 = chunk * kEmitChunk;
    const int64_t j1 = min(M, j0 + kEmitChunk);
    if (wid < 2) {
      const int64_t k = wave_last_le(offsets, nvis, static_cast<uint32_t>(wid == 0 ? j0 : j1 - 1), lane);
      if (lane == 0) s_k[wid] = k;
    }
    __syncthreads();
    const int64_t k0 = s_k[0];
    const int cnt = static_cast<int>(s_k[1] - k0 + 1);  // <= kEmitChunk: each owner starts in the chunk
    for (int q = tid; q < cnt; q += kThreads) {
      const int64_t k = k0 + q;
      const uint32_t g = order[k];
      const View& v = view_at(vs, view_of_gauss(vs, g));
      const float2 m = reinterpret_cast<const float2*>(xy)[g];
      const float rr = static_cast<float>(radius[g]);
      const int32_t x0 = clamp_tile_e((m.x - rr) / 16.0f, v.GX);
      const int32_t y0 = clamp_tile_e((m.y - rr) / 16.0f, v.GY);
      const int32_t x1 = clamp_tile_e(((m.x + rr) + 15.0f) / 16.0f, v.GX);
      s_off[q] = offsets[k];
      s_g[q] = g;
      s_base[q] = static_cast<uint32_t>(v.tile_off + static_cast<int64_t>(y0) * v.GX + x0);
      s_wg[q] = static_cast<uint32_t>(x1 - x0) | (static_cast<uint32_t>(v.GX) << 16);
    }
    __syncthreads();
    for (int64_t j = j0 + tid; j < j1; j += kThreads) {
      int lo = 0, hi = cnt - 1;
      const uint32_t uj = static_cast<uint32_t>(j);
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= uj) lo = mid; else hi = mid - 1;
      }
      const uint32_t q = uj - s_off[lo];
      const uint32_t wg = s_wg[lo];
      const uint32_t w = wg & 0xffffu, gx = wg >> 16;
      const uint32_t dy = q / w, dx = q - dy * w;
      keys[j] = s_base[lo] + dy * gx + dx;
      vals[j] = s_g[lo];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ step 3 with tile culling
// Rectangle of Gaussian g (in its view) and the view.
__device__ __forceinline__ const View& rect_of(const ViewSet& vs, const float* __restrict__ xy,
                                               const int32_t* __restrict__ radius, uint32_t g, float2& m,
                                               int32_t rect[4]) {
  const View& v = view_at(vs, view_of_gauss(vs, g));
  m = reinterpret_cast<const float2*>(xy)[g];
  tile_rect(m.x, m.y, radius[g], v.GX, v.GY, rect);
  return v;
}

// The row kernels take one visible Gaussian per thread (a row loop is at
// most one image height of tiles long, and near splats sort first).
constexpr int kRowBlock = kThreads;

// Block sums of the rectangle row counts in depth order.
__global__ void __launch_bounds__(kThreads) k_row_count(ViewSet vs, const uint32_t* __restrict__ order,
                                                        const float* __restrict__ xy,
                                                        const int32_t* __restrict__ radius, const uint32_t* n_dev,
                                                        int64_t n_host, unsigned long long* partials) {
  __shared__ unsigned long long lds[5];
  const int64_t n = live_count(n_dev, n_host);
  if (static_cast<int64_t>(blockIdx.x) * kRowBlock >= n) return;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kRowBlock + threadIdx.x;
  unsigned long long c = 0;
  if (k < n) {
    float2 m;
    int32_t rect[4];
    rect_of(vs, xy, radius, order[k], m, rect);
    c = static_cast<unsigned long long>(rect[3] - rect[1]);
  }
  unsigned long long tot;
  block_excl_scan<unsigned long long>(c, lds, tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Index of each visible Gaussian's first rectangle row (row_off[k]) and, for
// the adjoint, row_base[g] = row_off[k] - y0 (mod 2^32).
__global__ void __launch_bounds__(kThreads) k_row_base(ViewSet vs, const uint32_t* __restrict__ order,
                                                       const float* __restrict__ xy,
                                                       const int32_t* __restrict__ radius, const uint32_t* n_dev,
                                                       int64_t n_host,
                                                       const unsigned long long* __restrict__ row_partials,
                                                       const uint32_t* __restrict__ counters, uint32_t* row_off,
                                                       uint32_t* row_base) {
  __shared__ unsigned long long lds[5];
  if (counters[2]) return;
  const int64_t n = live_count(n_dev, n_host);
  if (static_cast<int64_t>(blockIdx.x) * kRowBlock >= n) return;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kRowBlock + threadIdx.x;
  uint32_t g = 0;
  int32_t rect[4] = {0, 0, 0, 0};
  if (k < n) {
    float2 m;
    g = order[k];
    rect_of(vs, xy, radius, g, m, rect);
  }
  unsigned long long tot;
  const unsigned long long r0 =
      block_excl_scan<unsigned long long>(static_cast<unsigned long long>(rect[3] - rect[1]), lds, tot) +
      row_partials[blockIdx.x];
  if (k < n) {
    row_off[k] = static_cast<uint32_t>(r0);
    if (row_base) row_base[g] = static_cast<uint32_t>(r0) - static_cast<uint32_t>(rect[1]);
  }
}

// One thread per rectangle row, 256 consecutive rows per block iteration.
// The rows' owners (at most 256, consecutive in depth order) are found by a
// wave search over row_off and staged in LDS with their ellipse.  Writes
// rows[i] = (g, first reached column | count << 16, global tile id of that
// column, row index within the Gaussian) and the block's reached-tile sums.
__global__ void __launch_bounds__(kThreads) k_row_intervals(ViewSet vs, const uint32_t* __restrict__ order,
                                                            const float* __restrict__ xy,
                                                            const float* __restrict__ conic_op,
                                                            const int32_t* __restrict__ radius,
                                                            const uint32_t* __restrict__ row_off,
                                                            const uint32_t* __restrict__ num_rows,
                                                            const uint32_t* __restrict__ counters, uint4* rows,
                                                            unsigned long long* tile_partials) {
  __shared__ uint32_t s_off[kRowBlock];
  __shared__ uint32_t s_g[kRowBlock];
  __shared__ int32_t s_rect[kRowBlock][4];  // x0, x1, y0, y1
  __shared__ int32_t s_view[kRowBlock][3];  // H, GX, tile_off (32 bits)
  __shared__ ReachRows s_rr[kRowBlock];
  __shared__ int64_t s_k[2];
  __shared__ unsigned long long lds[5];
  if (counters[2]) return;
  const int64_t R = *num_rows;
  const int64_t nvis = counters[1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t nblocks = (R + kRowBlock - 1) / kRowBlock;
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int64_t i0 = blk * kRowBlock;
    const int64_t i1 = min(R, i0 + kRowBlock);
    if (wid < 2) {
      const int64_t k = wave_last_le(row_off, nvis, static_cast<uint32_t>(wid == 0 ? i0 : i1 - 1), lane);
      if (lane == 0) s_k[wid] = k;
    }
    __syncthreads();
    const int64_t k0 = s_k[0];
    // <= kRowBlock as every Gaussian has a row; the bound only matters for
    // records that changed since k_row_count (a caller's race), as does the
    // row check below: such input yields wrong lists, never a write out of bounds
    const int cnt = static_cast<int>(min<int64_t>(kRowBlock, s_k[1] - k0 + 1));
    if (tid < cnt) {
      const uint32_t g = order[k0 + tid];
      float2 m;
      int32_t rect[4];
      const View& v = rect_of(vs, xy, radius, g, m, rect);
      const float4 co = reinterpret_cast<const float4*>(conic_op)[g];
      s_off[tid] = row_off[k0 + tid];
      s_g[tid] = g;
      s_rect[tid][0] = rect[0];
      s_rect[tid][1] = rect[2];
      s_rect[tid][2] = rect[1];
      s_rect[tid][3] = rect[3];
      s_view[tid][0] = v.H;
      s_view[tid][1] = v.GX;
      s_view[tid][2] = static_cast<int32_t>(v.tile_off);
      s_rr[tid] = reach_rows_init(m.x, m.y, co.x, co.y, co.z, co.w);
    }
    __syncthreads();
    const int64_t i = i0 + tid;
    uint32_t len = 0;
    if (i < i1) {
      int lo = 0, hi = cnt - 1;
      const uint32_t ui = static_cast<uint32_t>(i);
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= ui) lo = mid; else hi = mid - 1;
      }
      const uint32_t r = ui - s_off[lo];
      const int ty = s_rect[lo][2] + static_cast<int>(r);
      int c0 = 0, c1 = -1;
      if (ty < s_rect[lo][3]) reach_row(s_rr[lo], ty, s_view[lo][0], s_rect[lo][0], s_rect[lo][1], c0, c1);
      len = c1 >= c0 ? static_cast<uint32_t>(c1 - c0 + 1) : 0u;
      const uint32_t tile = static_cast<uint32_t>(s_view[lo][2]) +
                            static_cast<uint32_t>(ty) * static_cast<uint32_t>(s_view[lo][1]) +
                            static_cast<uint32_t>(c0);
      rows[i] = make_uint4(s_g[lo], static_cast<uint32_t>(c0) | (len << 16), tile, r);
    }
    unsigned long long tot;
    block_excl_scan<unsigned long long>(len, lds, tot);
    if (tid == 0) tile_partials[blk] = tot;
  }
}

// One thread per row again (same blocks): instance offset of each row from
// the scanned block sums and a block scan, the adjoint's row records
// brows[i] = (offset, first column | count << 16), first[g], and the block's
// instances, which are consecutive in the output, written 256 at a time.
// Each instance's row is found 4096 instances at a time: every non-empty row
// marks its first instance in the chunk (the row holding the chunk's first
// instance marks slot 0), and a max-scan carries the marks forward (rows
// start in increasing order), so an instance finds its row with one LDS read
// instead of a binary search over the block's 256 row starts.
constexpr int kEmitRun = 4096;  // instances per chunk of the owner scan
__global__ void __launch_bounds__(kThreads) k_row_emit(const uint4* __restrict__ rows,
                                                       const uint32_t* __restrict__ num_rows,
                                                       const unsigned long long* __restrict__ tile_partials,
                                                       const uint32_t* __restrict__ counters, uint2* brows,
                                                       uint32_t* first, uint32_t* keys, uint32_t* vals) {
  constexpr int kPerT = kEmitRun / kThreads;  // 16 owner slots per thread in the scan
  __shared__ uint32_t s_start[kRowBlock];
  __shared__ uint32_t s_tile[kRowBlock];
  __shared__ uint32_t s_g[kRowBlock];
  __shared__ int s_own[kEmitRun];
  __shared__ int s_wmax[kThreads / 64];
  __shared__ unsigned long long lds[5];
  if (counters[2]) return;
  const int64_t R = *num_rows;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t nblocks = (R + kRowBlock - 1) / kRowBlock;
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int64_t i = blk * kRowBlock + tid;
    uint4 rec = make_uint4(0u, 0u, 0u, 1u);
    if (i < R) rec = rows[i];
    const uint32_t len = rec.y >> 16;
    unsigned long long tot;
    const uint32_t pre = static_cast<uint32_t>(block_excl_scan<unsigned long long>(len, lds, tot));
    const uint32_t base = static_cast<uint32_t>(tile_partials[blk]);
    if (i < R) {
      if (brows) brows[i] = make_uint2(base + pre, rec.y);
      if (first && rec.w == 0u) first[rec.x] = base + pre;
    }
    s_start[tid] = pre;
    s_tile[tid] = rec.z;
    s_g[tid] = rec.x;
    const uint32_t total = static_cast<uint32_t>(tot);
    for (uint32_t c0 = 0; c0 < total; c0 += kEmitRun) {
      const uint32_t n = min(static_cast<uint32_t>(kEmitRun), total - c0);
      for (int k = tid; k < kEmitRun; k += kThreads) s_own[k] = 0;
      __syncthreads();
      if (len > 0 && pre < c0 + n && pre + len > c0)  // this row has instances in the chunk
        s_own[pre > c0 ? pre - c0 : 0] = tid;
      __syncthreads();
      // inclusive max-scan of s_own[0 .. kEmitRun): 16 slots per thread, then
      // the threads' maxima across the block
      int run = 0;
#pragma unroll
      for (int k = 0; k < kPerT; ++k) run = max(run, s_own[kPerT * tid + k]);
      int incl = run;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl = max(incl, y);
      }
      if (lane == 63) s_wmax[wid] = incl;
      __syncthreads();
      int carry = __shfl_up(incl, 1, 64);
      if (lane == 0) carry = 0;
      for (int w = 0; w < wid; ++w) carry = max(carry, s_wmax[w]);
#pragma unroll
      for (int k = 0; k < kPerT; ++k) {
        carry = max(carry, s_own[kPerT * tid + k]);
        s_own[kPerT * tid + k] = carry;
      }
      __syncthreads();
      for (uint32_t u = tid; u < n; u += kThreads) {
        const int o = s_own[u];
        const uint32_t t = c0 + u;
        keys[base + t] = s_tile[o] + (t - s_start[o]);
        vals[base + t] = s_g[o];
      }
      __syncthreads();
    }
  }
}

// Four keys a thread (one 16-byte read, plus the keys either side): the
// tile of each is a range's first entry where the key before differs, its
// last where the key after does.
__global__ void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ counters,
                         uint32_t* ranges, int64_t ntiles) {
  const int64_t n = counters[0];
  const int64_t n4 = (n + 3) / 4;
  const bool vec = (reinterpret_cast<uintptr_t>(keys) & 15u) == 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t j0 = 4 * i;
    uint32_t k[6];  // keys j0 - 1 .. j0 + 4 (the outer two only where they exist)
    if (vec && j0 + 4 <= n) {
      const uint4 q = reinterpret_cast<const uint4*>(keys)[i];
      k[1] = q.x; k[2] = q.y; k[3] = q.z; k[4] = q.w;
    } else {
      for (int c = 0; c < 4; ++c) k[1 + c] = j0 + c < n ? keys[j0 + c] : 0u;
    }
    k[0] = j0 > 0 ? keys[j0 - 1] : 0u;
    k[5] = j0 + 4 < n ? keys[j0 + 4] : 0u;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t j = j0 + c;
      const uint32_t t = k[1 + c];
      if (j >= n || static_cast<int64_t>(t) >= ntiles) continue;  // only records changed under a running sort
      if (j == 0 || k[c] != t) ranges[2 * static_cast<int64_t>(t)] = static_cast<uint32_t>(j);
      if (j == n - 1 || k[2 + c] != t) ranges[2 * static_cast<int64_t>(t) + 1] = static_cast<uint32_t>(j + 1);
    }
  }
}

// ------------------------------------------------------------------ host pipeline
static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

BinPlan plan_bins(int64_t n, int64_t tiles, int64_t capacity) {
  BinPlan p{};
  p.n = n;
  p.tiles = tiles;
  p.capacity = capacity;
  int bits = 0;
  while ((int64_t{1} << bits) < tiles) ++bits;
  p.tile_bits = bits;
  p.tile_passes = static_cast<int>(cdiv(bits, 8));
  p.hist_cols = std::max<int64_t>(1, cdiv(capacity, kRsBlock));
  p.hist_cols_depth = std::max<int64_t>(1, cdiv(n, kDepthBlock));
  size_t off = 0;
  p.off_vis_keys = off; off = align256(off + sizeof(uint32_t) * 2 * std::max<int64_t>(n, 1));
  p.off_vis_vals = off; off = align256(off + sizeof(uint32_t) * 2 * std::max<int64_t>(n, 1));
  p.off_offsets = off;  off = align256(off + sizeof(uint32_t) * std::max<int64_t>(n, 1));
  const int64_t nparts = std::max<int64_t>(1, cdiv(n, kThreads));  // blocks of the row kernels (the most)
  p.off_partials = off; off = align256(off + sizeof(unsigned long long) * (nparts + 1));
  p.off_hist = off;
  off = align256(off + sizeof(uint32_t) * std::max<int64_t>((int64_t{1} << kDepthBits) * p.hist_cols_depth,
                                                            256 * p.hist_cols));
  p.off_rowtot = off;   off = align256(off + sizeof(uint32_t) * (1 << kDepthBits));
  p.off_partials2 = off;
  off = align256(off + sizeof(unsigned long long) * (std::max<int64_t>(1, cdiv(capacity, kThreads)) + 1));
  p.off_rows = off;     off = align256(off + sizeof(uint4) * std::max<int64_t>(capacity, 1));
  p.off_num_rows = off; off = align256(off + sizeof(uint32_t) * 4);
  p.total = off;
  return p;
}

// One stable LSD pass of `bits` bits at `shift` from (kin, vin) to (kout, vout).
constexpr int64_t kMaxGrid = 8192;  // physical blocks of a grid-stride pass

template <int kMaxBits, int kPer>
static hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                             const uint32_t* n_dev, int64_t n_grid, int shift, int bits, uint32_t* hist,
                             int64_t cols, uint32_t* rowtot, hipStream_t s) {
  if (bits < 1 || bits > kMaxBits) return hipErrorInvalidValue;
  constexpr int64_t kBlock = int64_t{kThreads} * kPer;
  const unsigned nb = static_cast<unsigned>(std::min(kMaxGrid, std::max<int64_t>(1, cdiv(n_grid, kBlock))));
  auto hist_kernel = k_rs_hist<kMaxBits, kPer>;
  auto scatter_kernel = k_rs_scatter<kMaxBits, kPer>;
  hipLaunchKernelGGL(hist_kernel, dim3(nb), dim3(kThreads), 0, s, kin, n_dev, n_grid, shift, bits, hist, cols);
  hipLaunchKernelGGL(k_rs_rowscan, dim3(1u << bits), dim3(kThreads), 0, s, hist, cols, n_dev, n_grid, kBlock,
                     rowtot);
  hipLaunchKernelGGL(scatter_kernel, dim3(nb), dim3(kThreads), 0, s, kin, vin, kout, vout, n_dev, n_grid,
                     shift, bits, hist, cols, rowtot);
  return hipGetLastError();
}

int run_bin_sort(const ViewSet& vs, const Geom& geom, pvg_bins* bins, void* tmp, const BinPlan& plan,
                 int sync_count, hipStream_t s) {
  char* base = static_cast<char*>(tmp);
  uint32_t* vkeys = reinterpret_cast<uint32_t*>(base + plan.off_vis_keys);
  uint32_t* vvals = reinterpret_cast<uint32_t*>(base + plan.off_vis_vals);
  unsigned long long* partials = reinterpret_cast<unsigned long long*>(base + plan.off_partials);
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + plan.off_hist);
  uint32_t* rowtot = reinterpret_cast<uint32_t*>(base + plan.off_rowtot);
  uint32_t* offsets = reinterpret_cast<uint32_t*>(base + plan.off_offsets);
  uint32_t* counters = bins->counters;
  const int64_t n = plan.n;
  const int64_t cap = plan.capacity;
  const int64_t nvis_stride = std::max<int64_t>(n, 1);

  PVG_HIP(launch_fill_u32(counters, 0u, 4, s));
  if (n > 0) {
    StageScope sc(PVG_STAGE_COMPACT, s);
    const unsigned nb = static_cast<unsigned>(cdiv(n, kScanBlock));
    hipLaunchKernelGGL(k_vis_count, dim3(nb), dim3(kThreads), 0, s, geom.tiles, vs.live, n, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, static_cast<const uint32_t*>(nullptr),
                       vs.live, n, kScanBlock, counters + 1, int64_t{-1}, static_cast<uint32_t*>(nullptr),
                       static_cast<uint32_t*>(nullptr), static_cast<const uint32_t*>(nullptr));
    // into buffer 1 when the depth passes are odd in number, so they end in buffer 0
    const int64_t start = (kDepthPasses & 1) * nvis_stride;
    hipLaunchKernelGGL(k_vis_compact, dim3(nb), dim3(kThreads), 0, s, geom.tiles, geom.depth, vs.live, n, partials,
                       vkeys + start, vvals + start);
    PVG_HIP(hipGetLastError());
  }
  // depth sort of the visible Gaussians: kDepthPasses LSD passes, ending in buffer 0
  if (n > 0) {
    StageScope sc(PVG_STAGE_DEPTH_SORT, s);
    const auto depth_pass = radix_pass<kDepthBits, kDepthItems>;
    for (int pass = 0; pass < kDepthPasses; ++pass) {
      const int src = ((kDepthPasses & 1) + pass) & 1, dst = src ^ 1;
      const int shift = kDepthBits * pass;
      PVG_HIP(depth_pass(vkeys + src * nvis_stride, vvals + src * nvis_stride, vkeys + dst * nvis_stride,
                                     vvals + dst * nvis_stride, counters + 1, n, shift,
                                     std::min(kDepthBits, 32 - shift), hist, plan.hist_cols_depth, rowtot, s));
    }
  }
  const uint32_t* order = vvals;  // buffer 0 after the depth passes
  const bool cull = bins->tile_cull != 0;
  unsigned long long* partials2 = reinterpret_cast<unsigned long long*>(base + plan.off_partials2);
  uint4* rows = reinterpret_cast<uint4*>(base + plan.off_rows);
  uint32_t* num_rows = reinterpret_cast<uint32_t*>(base + plan.off_num_rows);
  const unsigned nbv_max = static_cast<unsigned>(std::max<int64_t>(1, cdiv(n, kScanBlock)));
  // instance counts in depth order and the capacity check: rectangle tiles, or
  // (culled) rectangle rows, their reached intervals and the reached tiles
  if (n > 0) {
    StageScope sc(PVG_STAGE_SCAN_EMIT, s);
    if (!cull) {
      hipLaunchKernelGGL(k_tile_count, dim3(nbv_max), dim3(kThreads), 0, s, order, geom.tiles, counters + 1, n,
                         partials);
      hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, counters + 1,
                         static_cast<const int64_t*>(nullptr), n, kScanBlock, counters, cap, counters + 2,
                         counters + 3, static_cast<const uint32_t*>(nullptr));
    } else {
      PVG_HIP(launch_fill_u32(num_rows, 0u, 1, s));
      const unsigned nbr = static_cast<unsigned>(cdiv(n, kRowBlock));
      const unsigned nrb = static_cast<unsigned>(std::min(kMaxGrid, std::max<int64_t>(1, cdiv(cap, kRowBlock))));
      hipLaunchKernelGGL(k_row_count, dim3(nbr), dim3(kThreads), 0, s, vs, order, geom.xy, geom.radius,
                         counters + 1, n, partials);
      hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, counters + 1,
                         static_cast<const int64_t*>(nullptr), n, kRowBlock, num_rows, cap, counters + 2,
                         counters + 3, static_cast<const uint32_t*>(nullptr));
      hipLaunchKernelGGL(k_row_base, dim3(nbr), dim3(kThreads), 0, s, vs, order, geom.xy, geom.radius, counters + 1,
                         n, partials, counters, offsets, bins->row_base);
      hipLaunchKernelGGL(k_row_intervals, dim3(nrb), dim3(kThreads), 0, s, vs, order, geom.xy, geom.conic_op,
                         geom.radius, offsets, num_rows, counters, rows, partials2);
      hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials2, num_rows,
                         static_cast<const int64_t*>(nullptr), int64_t{0}, kRowBlock, counters, cap, counters + 2,
                         counters + 3, counters + 2);
    }
    PVG_HIP(hipGetLastError());
  }
  int64_t m_grid = cap;
  int64_t vis_grid = n;
  int64_t row_grid = cap;
  if (sync_count) {
    uint32_t host_counts[4], host_rows = 0;
    PVG_HIP(hipMemcpyAsync(host_counts, counters, sizeof(host_counts), hipMemcpyDeviceToHost, s));
    if (cull && n > 0) PVG_HIP(hipMemcpyAsync(&host_rows, num_rows, sizeof(host_rows), hipMemcpyDeviceToHost, s));
    PVG_HIP(hipStreamSynchronize(s));
    bins->num_instances = host_counts[3] == 0xffffffffu ? int64_t{0xffffffff} : int64_t{host_counts[3]};
    bins->num_visible = host_counts[1];
    if (host_counts[2]) {
      set_error("instance capacity %lld is smaller than the %lld %s of this render", static_cast<long long>(cap),
                static_cast<long long>(bins->num_instances),
                cull && host_rows == 0 ? "rectangle rows" : "instances");
      return PVG_ERR_CAPACITY;
    }
    m_grid = host_counts[0];
    vis_grid = host_counts[1];
    row_grid = host_rows;
  }
  const int passes = plan.tile_passes;
  const int start = passes & 1;  // so that the last pass lands in buffer 0
  // culled lists: the row pass also writes the adjoint's row records and
  // first[], so it runs whenever there are rows, even with nothing listed
  if (n > 0 && vis_grid > 0 && (cull ? row_grid > 0 : m_grid > 0)) {
    StageScope sc(PVG_STAGE_SCAN_EMIT, s);
    const unsigned nbv = static_cast<unsigned>(cdiv(vis_grid, kScanBlock));
    if (!cull) {
      hipLaunchKernelGGL(k_tile_offsets, dim3(nbv), dim3(kThreads), 0, s, order, geom.tiles, counters + 1, n,
                         partials, counters, offsets, bins->first);
      const unsigned nbe = static_cast<unsigned>(std::min(kMaxGrid, cdiv(m_grid, kEmitChunk)));
      hipLaunchKernelGGL(k_emit, dim3(nbe), dim3(kThreads), 0, s, vs, order, geom.xy, geom.radius, offsets,
                         counters, bins->keys + start * cap, bins->vals + start * cap);
    } else {
      const unsigned nre = static_cast<unsigned>(std::min(kMaxGrid, std::max<int64_t>(1, cdiv(row_grid, kRowBlock))));
      hipLaunchKernelGGL(k_row_emit, dim3(nre), dim3(kThreads), 0, s, rows, num_rows, partials2, counters,
                         reinterpret_cast<uint2*>(bins->rows), bins->first, bins->keys + start * cap,
                         bins->vals + start * cap);
    }
    PVG_HIP(hipGetLastError());
  }
  if (passes > 0 && m_grid > 0) {
    StageScope sc(PVG_STAGE_TILE_SORT, s);
    const auto tile_pass = radix_pass<8, kRsItems>;
    const int per = (plan.tile_bits + passes - 1) / passes;
    for (int pass = 0; pass < passes; ++pass) {
      const int src = (start + pass) & 1, dst = src ^ 1;
      const int shift = per * pass;
      const int bits = std::min(per, plan.tile_bits - shift);
      PVG_HIP(tile_pass(bins->keys + src * cap, bins->vals + src * cap, bins->keys + dst * cap,
                            bins->vals + dst * cap, counters, m_grid, shift, bits, hist, plan.hist_cols, rowtot, s));
    }
  }
  {
    StageScope sc(PVG_STAGE_RANGES, s);
    PVG_HIP(launch_fill_u32(bins->ranges, 0u, 2 * plan.tiles, s));
    if (m_grid > 0) {
      hipLaunchKernelGGL(k_ranges, dim3(static_cast<unsigned>(std::min(kMaxGrid * 4, cdiv(m_grid, 1024)))),
                         dim3(256), 0, s, bins->keys, counters, bins->ranges, static_cast<int64_t>(plan.tiles));
      PVG_HIP(hipGetLastError());
    }
  }
  return PVG_OK;
}

// ------------------------------------------------- library-held bin_sort scratch
// The scratch of pvg_bin_sort_noalloc, for callers that cannot allocate device
// memory.  Each device the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, never a
// device address: host code uses only the address hipGetSymbolAddress returns,
// looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[PVG_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

}  // namespace pvg
