// Host packing of the reference operators into MFMA fragment order, and the
// 16-bit splits of the mixed-precision variants.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "mfma_pack.hpp"

namespace dgw {

uint16_t bf16_round(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

float bf16_float(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

// IEEE binary16, round to nearest even (subnormals included, overflow to inf).
uint16_t f16_round(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t sign = (u >> 16) & 0x8000u;
  const int32_t e8 = static_cast<int32_t>((u >> 23) & 0xff);
  uint32_t mant = u & 0x7fffffu;
  if (e8 == 0xff) return static_cast<uint16_t>(sign | 0x7c00u | (mant ? 0x200u : 0u));
  const int32_t e = e8 - 127 + 15;
  if (e >= 31) return static_cast<uint16_t>(sign | 0x7c00u);
  if (e <= 0) {
    if (e < -10) return static_cast<uint16_t>(sign);
    mant |= 0x800000u;
    const int shift = 14 - e;
    uint32_t m = mant >> shift;
    const uint32_t rem = mant & ((1u << shift) - 1u), half = 1u << (shift - 1);
    if (rem > half || (rem == half && (m & 1u))) ++m;
    return static_cast<uint16_t>(sign | m);
  }
  uint32_t h = sign | (static_cast<uint32_t>(e) << 10) | (mant >> 13);
  const uint32_t rem = mant & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;  // a carry into the exponent is correct rounding
  return static_cast<uint16_t>(h);
}

float f16_float(uint16_t h) {
  const uint32_t sign = static_cast<uint32_t>(h & 0x8000u) << 16;
  const uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
  uint32_t u;
  if (e == 0) {
    if (m == 0) {
      u = sign;
    } else {  // subnormal: m * 2^-24
      const float v = std::ldexp(static_cast<float>(m), -24);
      std::memcpy(&u, &v, 4);
      u |= sign;
    }
  } else if (e == 31) {
    u = sign | 0x7f800000u | (m << 13);
  } else {
    u = sign | ((e - 15 + 127) << 23) | (m << 13);
  }
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

static int source_column(const ColMap* colmap, int col) {
  if (!colmap) return col;
  return col < static_cast<int>(colmap->size()) ? (*colmap)[col] : -1;
}

ColMap face_block_columns(int Nfp, int KF) {
  if (KF < Nfp) return ColMap();  // no face blocks (merged layout)
  ColMap m(static_cast<size_t>(4) * KF, -1);
  for (int f = 0; f < 4; ++f)
    for (int j = 0; j < Nfp; ++j) m[static_cast<size_t>(f) * KF + j] = f * Nfp + j;
  return m;
}

void pack_fp32(const double* A, int rows, int cols, int MB, int KP, std::vector<float>& out, const ColMap* colmap) {
  const size_t base = out.size();
  out.resize(base + static_cast<size_t>(MB) * (KP / 4) * 64, 0.0f);
  for (int mb = 0; mb < MB; ++mb)
    for (int kk = 0; kk < KP / 4; ++kk)
      for (int l = 0; l < 64; ++l) {
        const int row = mb * 16 + l % 16, col = source_column(colmap, kk * 4 + l / 16);
        if (row < rows && col >= 0 && col < cols)
          out[base + (static_cast<size_t>(mb) * (KP / 4) + kk) * 64 + l] =
              static_cast<float>(A[static_cast<size_t>(row) * cols + col]);
      }
}

void pack_split16(const double* A, int rows, int cols, int MB, int K, int KW, bool bf16, std::vector<uint16_t>& hi,
                  std::vector<uint16_t>& lo, const ColMap* colmap) {
  const int KB = 4 * KW;  // k per fragment
  const size_t base = hi.size();
  const size_t n = static_cast<size_t>(MB) * (K / KB) * 64 * KW;
  hi.resize(base + n, 0);
  lo.resize(base + n, 0);
  for (int mb = 0; mb < MB; ++mb)
    for (int kk = 0; kk < K / KB; ++kk)
      for (int l = 0; l < 64; ++l)
        for (int t = 0; t < KW; ++t) {
          const int row = mb * 16 + l % 16, col = source_column(colmap, kk * KB + KW * (l / 16) + t);
          if (row >= rows || col < 0 || col >= cols) continue;
          const double x = A[static_cast<size_t>(row) * cols + col];
          const size_t idx = base + ((static_cast<size_t>(mb) * (K / KB) + kk) * 64 + l) * KW + t;
          if (bf16) {
            const uint16_t h = bf16_round(static_cast<float>(x));
            hi[idx] = h;
            lo[idx] = bf16_round(static_cast<float>(x - static_cast<double>(bf16_float(h))));
          } else {
            const uint16_t h = f16_round(static_cast<float>(x));
            hi[idx] = h;
            lo[idx] = f16_round(static_cast<float>(x - static_cast<double>(f16_float(h))));
          }
        }
}

}  // namespace dgw
