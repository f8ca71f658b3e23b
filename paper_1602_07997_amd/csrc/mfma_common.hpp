// Helpers shared by the MFMA step kernels (gfx950 matrix cores): operand
// types, the FP32 operand-array swizzle, 16-bit splits and the split products.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

namespace dgw {
namespace mfma {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int rup(int x, int m) { return (x + m - 1) / m * m; }

// ---- host side: splitting a short last round of workgroups ----------------

// Workgroups of `kernel` (launched with `threads` threads) resident on the
// current device at once: its occupancy times the compute units, cached per
// device in `cache` (one array per kernel); 0 when unknown.
template <int kDevices>
inline int resident_workgroups(const void* kernel, int threads, std::atomic<int> (&cache)[kDevices]) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (dev >= 0 && dev < kDevices) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int occ = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int slots = occ > 0 && cus > 0 ? occ * cus : 0;
  if (slots > 0 && dev >= 0 && dev < kDevices) cache[dev].store(slots, std::memory_order_relaxed);
  return slots;
}

// Launch plan of `tiles` tiles on `slots` resident workgroups: the tiles of
// the last, partial round (all tiles when they do not fill one round) are
// each shared by `parts` workgroups, as many as the free slots of that round
// allow, up to max_parts; the workgroup for part j of such a tile takes its
// pairs [j P / parts, (j + 1) P / parts).  parts = 1: one workgroup per tile.
struct TailSplit {
  int64_t grid;  // workgroups to launch
  int64_t from;  // first split tile (= tiles when none is split)
  int parts;
};

inline TailSplit plan_tail_split(int64_t tiles, int slots, int max_parts) {
  TailSplit t{tiles, tiles, 1};
  if (max_parts <= 1 || slots <= 0 || tiles <= 0) return t;
  const int64_t full = ((tiles - 1) / slots) * slots;
  const int64_t tail = tiles - full;
  const int64_t fit = slots / tail;
  const int parts = static_cast<int>(fit < max_parts ? fit : max_parts);
  if (parts > 1) t = TailSplit{full + tail * parts, full, parts};
  return t;
}

// Device side: the tile and pair range [p0, p1) of workgroup blockIdx.x of a
// launch planned by plan_tail_split (split_parts <= 1: whole tiles).
__device__ __forceinline__ int64_t split_tile(int64_t whole_tile, int64_t split_from, int split_parts, int pairs,
                                              int& p0, int& p1) {
  const int64_t b = blockIdx.x;
  p0 = 0;
  p1 = pairs;
  if (split_parts <= 1 || b < split_from) return whole_tile;
  const int64_t t = b - split_from;
  const int j = static_cast<int>(t % split_parts);
  p0 = j * pairs / split_parts;
  p1 = (j + 1) * pairs / split_parts;
  return split_from + t / split_parts;
}

// Column swizzle of the FP32 [row][E] operand arrays: a bijection on [0, E)
// per row that keeps the fragment reads conflict-free and spreads the
// row-consecutive staging writes over the banks.
template <int E>
__device__ __forceinline__ int swz(int m, int e) {
  if constexpr (E == 16)
    return e ^ ((m >> 1) & 15);
  else
    return (((e >> 4) ^ (m & 1)) << 4) + ((e & 15) ^ ((m >> 1) & 15));
}

// Round to nearest even: float -> bfloat16 bits.
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// x = hi + lo in the 16-bit format of PREC (bit patterns).
template <int PREC>
__device__ __forceinline__ void split16(float x, uint16_t& hi, uint16_t& lo) {
  if constexpr (PREC == 1) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
  } else {
    const _Float16 h = static_cast<_Float16>(x);
    const _Float16 l = static_cast<_Float16>(x - static_cast<float>(h));
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  }
}

struct Frag16 {
  shortx4 hi, lo;
};

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int PREC>
__device__ __forceinline__ floatx4 mfma16(shortx4 a, shortx4 b, floatx4 c) {
  if constexpr (PREC == 1) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(halfx4, a), __builtin_bit_cast(halfx4, b), c,
                                                 0, 0, 0);
  }
}

// acc += A B with the split products (small terms first)
template <int PREC>
__device__ __forceinline__ floatx4 mfma_split(const Frag16& a, const Frag16& b, floatx4 c) {
  c = mfma16<PREC>(a.lo, b.hi, c);
  c = mfma16<PREC>(a.hi, b.lo, c);
  return mfma16<PREC>(a.hi, b.hi, c);
}

// gfx950 16x16x32 products: lane l holds row (A) / column (B) l%16 at
// k = 8 (l/16) + t, t = 0..7; the accumulator layout is that of 16x16x16.
// Twice the work of a 16x16x16 instruction at the same issue cost.
struct Frag32 {
  shortx8 hi, lo;
};

template <int PREC>
__device__ __forceinline__ floatx4 mfma32(shortx8 a, shortx8 b, floatx4 c) {
  if constexpr (PREC == 1) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, a), __builtin_bit_cast(halfx8, b), c,
                                                  0, 0, 0);
  }
}

template <int PREC>
__device__ __forceinline__ floatx4 mfma_split(const Frag32& a, const Frag32& b, floatx4 c) {
  c = mfma32<PREC>(a.lo, b.hi, c);
  c = mfma32<PREC>(a.hi, b.lo, c);
  return mfma32<PREC>(a.hi, b.hi, c);
}

// Register sets of a software-pipelined operator stream.
template <class T, int A, int B>
struct Ring {
  T v[A][B];
};

// Software pipeline over NK k-steps in groups of PD: the operator fragments
// of the next group are read into the other of two register sets before the
// products of the current group (the scheduling barriers keep that order),
// so that their latency overlaps PD k-steps of products.  load(r, g) fills r
// with group g (clamping past the end), compute(r, g, cnt) runs the first cnt
// k-steps of group g.
// UNROLL unrolls the group loop completely (group indices then fold to
// constants, e.g. to pick an accumulator per face).
template <int NK, int PD, class R, bool UNROLL = false, class Load, class Compute>
__device__ __forceinline__ void pipelined(Load&& load, Compute&& compute) {
  constexpr int NGT = (NK + PD - 1) / PD, LAST = NK - (NGT - 1) * PD;
  R ra, rb;
  load(ra, 0);
  auto two = [&](int g) {
    load(rb, g + 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(ra, g, PD);
    load(ra, g + 2);
    __builtin_amdgcn_sched_barrier(0);
    compute(rb, g + 1, PD);
  };
  if constexpr (UNROLL) {
#pragma unroll
    for (int g = 0; g + 2 < NGT; g += 2) two(g);
  } else {
#pragma unroll 1
    for (int g = 0; g + 2 < NGT; g += 2) two(g);
  }
  if constexpr (NGT % 2 == 1) {
    compute(ra, NGT - 1, LAST);
  } else {
    load(rb, NGT - 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(ra, NGT - 2, PD);
    compute(rb, NGT - 1, LAST);
  }
}

}  // namespace mfma
}  // namespace dgw
