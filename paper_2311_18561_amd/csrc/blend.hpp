// Device helpers shared by the compositing kernels (Sec. 3.1, Eq. (3)) of
// the colour and channel path and of the N-channel feature path: the
// XCD-banded tile order, wave reductions, the base-2 pair exponent and the
// gathers of the adjoint's per-(Gaussian, tile) records.
#pragma once
#include "pvg_math.hpp"

namespace pvg {

// Tiles are dealt to the eight XCDs (which receive workgroups round-robin)
// in chunks of xcd_chunk(total) consecutive tiles, about one tile row of a
// 1920-pixel view: chunk k goes to XCD k mod 8.  Each XCD then sees the
// image's whole mix of light and heavy tiles (with one band of rows per XCD,
// the XCDs holding the densest rows kept working long after the others),
// while a chunk's tiles, which share many Gaussians, stay in one XCD's L2.
// `total` is the launch's tile capacity (the same on host and device); the
// grid is render_grid(total) blocks, and blocks whose tile is past the live
// count return at once.
__host__ __device__ __forceinline__ int64_t xcd_chunk(int64_t total) {
  const int64_t c = total / 80;
  return c < 1 ? 1 : (c > 120 ? 120 : c);
}
__host__ __device__ __forceinline__ int64_t render_grid(int64_t total) {
  const int64_t span = 8 * xcd_chunk(total);
  return (total + span - 1) / span * span;
}
__host__ __device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t total) {
  const int64_t c = xcd_chunk(total);
  const int64_t q = b >> 3, x = b & 7;
  return ((q / c) * 8 + x) * c + q % c;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sums ten per-lane values over the wave by halving: a half-wave swap adds
// two values at once (lanes 0-31 keep the sums of the even-indexed values,
// 32-63 of the odd ones), a row swap does the same between the two 16-lane
// rows of each half, and DPP folds the last three values within each row.
// Afterwards every lane of row r (lanes 16r .. 16r+15) holds, in out[k], the
// wave total of value 4k + 2(r & 1) + (r >> 1) (indices >= 10 are padding).
__device__ __forceinline__ float swap_sum32(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_sum16(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float dpp_add(float x, int ctrl) {
  switch (ctrl) {  // the control word must be a compile-time constant
    case 0x128: return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xf, 0xf, true));
    case 0x124: return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xf, 0xf, true));
    case 0x4e: return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4e, 0xf, 0xf, true));
    default: return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xb1, 0xf, 0xf, true));
  }
}
__device__ __forceinline__ void wave_sum10(const float a[10], float out[3]) {
  float h[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) h[m] = swap_sum32(a[2 * m], a[2 * m + 1]);
  out[0] = swap_sum16(h[0], h[1]);
  out[1] = swap_sum16(h[2], h[3]);
  out[2] = swap_sum16(h[4], 0.0f);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out[k] = dpp_add(out[k], 0x128);  // row_ror:8
    out[k] = dpp_add(out[k], 0x124);  // row_ror:4
    out[k] = dpp_add(out[k], 0x4e);   // quad_perm [2,3,0,1]
    out[k] = dpp_add(out[k], 0xb1);   // quad_perm [1,0,3,2]
  }
}

// The same for sixteen values: out[k] (k < 4) of the lanes of row r holds the
// wave total of value 4k + 2(r & 1) + (r >> 1).
__device__ __forceinline__ void wave_sum16(const float a[16], float out[4]) {
  float h[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) h[m] = swap_sum32(a[2 * m], a[2 * m + 1]);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = swap_sum16(h[2 * k], h[2 * k + 1]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    out[k] = dpp_add(out[k], 0x128);  // row_ror:8
    out[k] = dpp_add(out[k], 0x124);  // row_ror:4
    out[k] = dpp_add(out[k], 0x4e);   // quad_perm [2,3,0,1]
    out[k] = dpp_add(out[k], 0xb1);   // quad_perm [1,0,3,2]
  }
}

// Wave totals of kN per-lane values (any count), sixteen or ten at a time
// with wave_sum16 / wave_sum10; lanes with lane % 16 == 0 store value q's
// total in dst[q] (q < kN), so dst must hold kN floats visible to the wave.
// With kGap > 0 the values from kSplit on go kGap slots further (dst[q +
// kGap]), leaving a gap the caller fills.
template <int kN, int kSplit = kN, int kGap = 0>
__device__ __forceinline__ void wave_sum_store(const float* a, int lane, float* dst) {
#pragma unroll
  for (int b = 0; b < kN; b += 16) {
    const int r = lane >> 4;
    if (kN - b > 10) {
      float x[16], red[4];
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = b + i < kN ? a[b + i] : 0.0f;
      wave_sum16(x, red);
      if ((lane & 15) == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int q = b + 4 * k + 2 * (r & 1) + (r >> 1);
          if (q < kN) dst[q < kSplit ? q : q + kGap] = red[k];
        }
      }
    } else {
      float x[10], red[3];
#pragma unroll
      for (int i = 0; i < 10; ++i) x[i] = b + i < kN ? a[b + i] : 0.0f;
      wave_sum10(x, red);
      if ((lane & 15) == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int q = b + 4 * k + 2 * (r & 1) + (r >> 1);
          if (q < kN) dst[q < kSplit ? q : q + kGap] = red[k];
        }
      }
    }
  }
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

// The pair exponent in base 2.  With the conic (A, B, C) scaled once per
// Gaussian into q = -log2(e) (A / 2, B, C / 2), the exponent of Eq. (3)'s
// 2D Gaussian at offset (dx, dy) is power = ln 2 * p2 with
//   p2 = q.x dx^2 + q.y dx dy + q.z dy^2 = (q.z dy + q.y dx) dy + q.x dx^2,
// so alpha = o 2^p2 takes the hardware base-2 exponential directly.  A lane
// forms c1 = q.y dx and c0 = q.x dx^2 once per Gaussian (its four pixels
// share dx) and then two FMAs per pixel.  The rounding differs from the
// natural-base form by a few ulps relative to the terms' magnitudes; a skip
// or stop decision can then go the other way only where its exact value sits
// within that of a threshold.  The forward and the adjoint share this
// function, so they take every decision alike.
constexpr float kLog2e = 1.44269504088896341f;

__device__ __forceinline__ float4 pair_coefs(float A, float B, float C, float o) {
  return make_float4(-0.5f * kLog2e * A, -kLog2e * B, -0.5f * kLog2e * C, o);
}

__device__ __forceinline__ float pair_exp2(float qz, float c1, float c0, float dy) {
  return fmaf(fmaf(qz, dy, c1), dy, c0);
}

constexpr int kPix = 4;  // pixels per lane

// The forward walks a batch's pairs in groups of kGroup (a batch is padded
// with pairs no pixel uses up to a whole group).
constexpr int kGroup = 4;
__device__ __forceinline__ int pad_to(int cnt) { return (cnt + kGroup - 1) / kGroup * kGroup; }

// The index range [e0, e0 + cnt) of a visible Gaussian's pairs in emission
// order: first[g] and the listed count (its rectangle's tiles, or, for
// culled lists, up to the end of its last row).  Lists of an overflowed sort
// hold nothing; a range outside the record slots comes back empty.
template <bool kCulled>
__device__ __forceinline__ void record_range(const ViewSet& vs, const Geom& geom, const Lists& lists, int64_t gi,
                                             uint32_t& e0, uint32_t& cnt) {
  e0 = lists.first[gi];
  cnt = 0;
  if (kCulled) {
    const View& v = view_at(vs, view_of_gauss(vs, gi));
    const float2 m = reinterpret_cast<const float2*>(geom.xy)[gi];
    int32_t rect[4];
    tile_rect(m.x, m.y, geom.radius[gi], v.GX, v.GY, rect);
    const uint32_t ri = lists.row_base[gi] + static_cast<uint32_t>(rect[3] - 1);
    if (static_cast<int64_t>(ri) < lists.capacity) {
      const uint2 rw = lists.rows[ri];
      cnt = rw.x + (rw.y >> 16) - e0;
    }
  } else {
    cnt = geom.tiles[gi];
  }
  const uint64_t cap = static_cast<uint64_t>(lists.capacity);
  if (static_cast<uint64_t>(e0) > cap || static_cast<uint64_t>(cnt) > cap - e0) cnt = 0;
}

// Emission-order index of the pair (Gaussian g with 2D mean m, tile (tx,
// ty)): for rectangle lists first[g] plus the tile's row-major index in the
// Gaussian's rectangle; for culled lists the tile's rank among the reached
// tiles, rows[row_base[g] + ty].x + tx - (the row's first column).  Indices
// >= capacity (only for lists these records do not belong to) are skipped
// by the caller.
template <bool kCulled>
__device__ __forceinline__ uint32_t record_index(const Lists& lists, const Geom& geom, const View& v, uint32_t g,
                                                 float2 m, int tx, int ty) {
  if (kCulled) {
    const uint32_t ri = lists.row_base[g] + static_cast<uint32_t>(ty);
    if (static_cast<int64_t>(ri) >= lists.capacity) return static_cast<uint32_t>(min<int64_t>(lists.capacity, 0xffffffffll));
    const uint2 rw = lists.rows[ri];
    return rw.x + static_cast<uint32_t>(tx - static_cast<int>(rw.y & 0xffffu));
  }
  int32_t rect[4];
  tile_rect(m.x, m.y, geom.radius[g], v.GX, v.GY, rect);
  return lists.first[g] + static_cast<uint32_t>((ty - rect[1]) * (rect[2] - rect[0]) + (tx - rect[0]));
}

// acc[q] += r[q], q < kSums; records of a multiple of four floats (the
// record array 16-byte aligned) are read 16 bytes at a time.
template <int kSums>
__device__ __forceinline__ void add_record(const float* __restrict__ r, float* acc) {
  if constexpr (kSums % 4 == 0) {
#pragma unroll
    for (int q = 0; q < kSums / 4; ++q) {
      const float4 x = reinterpret_cast<const float4*>(r)[q];
      acc[4 * q] += x.x;
      acc[4 * q + 1] += x.y;
      acc[4 * q + 2] += x.z;
      acc[4 * q + 3] += x.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kSums; ++q) acc[q] += r[q];
  }
}

// Sum of one Gaussian's flagged records in [e0, e0 + cnt) by one thread,
// reading the flags 16 at a time.  The emission order keeps a Gaussian's
// pairs contiguous.
// kAcc (>= kSums) is the width of acc, which is cleared first.
template <int kSums, int kAcc = 16>
__device__ __forceinline__ void gather_range(uint32_t e0, uint32_t cnt, const float* __restrict__ rec,
                                             const uint8_t* __restrict__ vis, float acc[kAcc]) {
  static_assert(kSums <= kAcc, "accumulator narrower than a record");
#pragma unroll
  for (int c = 0; c < kAcc; ++c) acc[c] = 0.0f;
  const uint32_t e1 = e0 + cnt;
  for (uint32_t b = e0 & ~15u; b < e1; b += 16) {
    const uint4 w = *reinterpret_cast<const uint4*>(vis + b);
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t e = b + static_cast<uint32_t>(j);
      if (((words[j >> 2] >> (8 * (j & 3))) & 0xffu) && e >= e0 && e < e1) {
        const float* r = rec + kSums * static_cast<int64_t>(e);  // records are kSums floats apart
        add_record<kSums>(r, acc);
      }
    }
  }
}

constexpr uint32_t kShortRange = 48;  // Gaussians with more listed pairs are gathered by a whole wave
// Gaussians with more listed pairs than this (near-camera splats reach most
// of the frame's 9,600 tiles, and a splat in front is flagged in nearly all of
// them) are gathered by the whole block, each wave taking every fourth
// round of 1,024 pairs: one wave alone took about 90 us over the largest,
// while the rest of the gather needed 48 us.
constexpr uint32_t kHugeRange = 2048;

// Sum of one Gaussian's flagged records in [e0, e0 + cnt) by a whole wave:
// each round, lane l reads the 16 flags at b + 16 l (1024 pairs per round),
// the wave compacts the flagged indices into its LDS list `idx` (a wave
// prefix sum of the lanes' counts gives each lane its slots), and the lanes
// then take the listed records 64 at a time.  A near-camera splat with
// thousands of listed tiles thus needs a few rounds instead of one round per
// 64 flags.  Every lane returns its partial sums; the caller reduces them.
template <int kSums, int kAcc = 16>
__device__ __forceinline__ void gather_range_wave(uint32_t e0, uint32_t cnt, int lane,
                                                  const float* __restrict__ rec,
                                                  const uint8_t* __restrict__ vis, uint32_t* idx,
                                                  float acc[kAcc]) {
  static_assert(kSums <= kAcc, "accumulator narrower than a record");
#pragma unroll
  for (int c = 0; c < kAcc; ++c) acc[c] = 0.0f;
  const uint32_t e1 = e0 + cnt;
  for (uint32_t b = e0 & ~15u; b < e1; b += 1024) {
    const uint32_t mb = b + 16u * static_cast<uint32_t>(lane);
    uint32_t words[4] = {0u, 0u, 0u, 0u};
    if (mb < e1) {
      const uint4 w = *reinterpret_cast<const uint4*>(vis + mb);
      words[0] = w.x; words[1] = w.y; words[2] = w.z; words[3] = w.w;
    }
    uint32_t bits = 0;  // bit j: pair mb + j is flagged and inside the range
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t e = mb + static_cast<uint32_t>(j);
      if (((words[j >> 2] >> (8 * (j & 3))) & 0xffu) && e >= e0 && e < e1) bits |= 1u << j;
    }
    const int c = __popc(bits);
    int incl = c;  // inclusive prefix over the lanes
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    const int total = __shfl(incl, 63, 64);
    int slot = incl - c;
    while (bits) {
      const int j = __ffs(bits) - 1;
      bits &= bits - 1u;
      idx[slot++] = mb + static_cast<uint32_t>(j);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int k = lane; k < total; k += 64) {
      const float* r = rec + kSums * static_cast<int64_t>(idx[k]);
      add_record<kSums>(r, acc);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}


}  // namespace pvg
