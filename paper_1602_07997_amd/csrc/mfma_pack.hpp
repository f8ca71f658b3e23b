// Host packing of operators into MFMA fragment order (see mfma_pack.cpp).
#pragma once

#include <cstdint>
#include <vector>

namespace dgw {

uint16_t bf16_round(float x);
float bf16_float(uint16_t h);
uint16_t f16_round(float x);
float f16_float(uint16_t h);

// Fragment column k reads source column colmap[k] of A (-1: zero); a null
// map is the identity.
using ColMap = std::vector<int>;

// A (rows x cols, row-major) as 16x4 FP32 fragments, lane l holding
// A[mb*16 + l%16][c(4 kk + l/16)] with c the column map; appended to out as
// [MB][KP/4][64].
void pack_fp32(const double* A, int rows, int cols, int MB, int KP, std::vector<float>& out,
               const ColMap* colmap = nullptr);

// A as 16 x (4 KW) fragments of 16-bit pairs x = hi + lo (KW = 4: the
// 16x16x16 instructions, KW = 8: 16x16x32), lane l holding
// A[mb*16 + l%16][c(4 KW kk + KW (l/16) + t)], t < KW; appended as
// [MB][K/(4 KW)][64][KW] to hi and lo.
void pack_split16(const double* A, int rows, int cols, int MB, int K, int KW, bool bf16, std::vector<uint16_t>& hi,
                  std::vector<uint16_t>& lo, const ColMap* colmap = nullptr);

// Column map of the per-face LIFT: face f's Nfp columns start at K = f*KF
// (the rest of each face block zero); empty when KF < Nfp.
ColMap face_block_columns(int Nfp, int KF);

}  // namespace dgw
