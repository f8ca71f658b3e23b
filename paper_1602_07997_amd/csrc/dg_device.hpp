// Device-side helpers shared by the step kernels (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgw {
namespace dev {

template <int N>
struct Deg {
  static constexpr int NP = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int NFP = (N + 1) * (N + 2) / 2;
};

template <int PHYS>
struct Phys;
template <>
struct Phys<0> {  // acoustic: p, v1, v2, v3
  static constexpr int NF = 4, NT = 2, NAUX = 3, CB = 8;
};
template <>
struct Phys<1> {  // elastic: v1, v2, v3, s11, s22, s33, s23, s13, s12
  static constexpr int NF = 9, NT = 6, NAUX = 9, CB = 16;
};
template <>
struct Phys<2> {  // anisotropic elastic: the elastic fields, a general stiffness per element
  static constexpr int NF = 9, NT = 6, NAUX = 9, CB = 32;
};

// Offset of the Voigt stiffness entry C_ab (a <= b) among the 21 entries of
// the upper triangle stored row by row.
__host__ __device__ __forceinline__ constexpr int upper6(int a, int b) { return a * 6 - a * (a - 1) / 2 + (b - a); }

constexpr int kThreads = 256;

// Voigt index of the symmetric stress component (i, j).
__device__ __forceinline__ constexpr int voigt(int i, int j) {
  return (i == j) ? i : (3 + (3 - i - j));  // (1,2)->3, (0,2)->4, (0,1)->5
}

// Outward unit normal and Fscale of reference face f from G (row-major 3x3):
// n ~ G nref_f with nref = (0,0,-1), (0,-1,0), (1,1,1), (-1,0,0) for f = 0..3,
// Fscale = |G nref_f|.  The reference normal is formed with 0/1 weights rather
// than a chain of selects: hipcc (ROCm 7.2) turned such a chain into branches
// that left face 3 with the face-1 value.
__device__ __forceinline__ void face_normal(const float* G, int f, float n[3], float& fs) {
  const float is0 = static_cast<float>(f == 0), is1 = static_cast<float>(f == 1);
  const float is2 = static_cast<float>(f == 2), is3 = static_cast<float>(f == 3);
  const float w0 = is2 - is3, w1 = is2 - is1, w2 = is2 - is0;
  float v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = G[3 * i + 0] * w0 + G[3 * i + 1] * w1 + G[3 * i + 2] * w2;
  const float ss = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const float inv = __builtin_amdgcn_rsqf(ss);
  fs = ss * inv;
  n[0] = v[0] * inv;
  n[1] = v[1] * inv;
  n[2] = v[2] * inv;
}

// Per-(element, face) constants of the upwind penalty, computed once per face
// instead of at every face node.  Record layout (FaceRec<PHYS>::W floats):
//   acoustic: n0 n1 n2 Z+ fp fv wall 0      with, at a face node,
//             alpha = [[p]] - Z+ [[v.n]],  Pp = fp * alpha,  Pv = fv * alpha,
//             fp = Fscale rho c^2 k_c, fv = -Fscale c k_c, k_c = 2/(Z- + Z+)
//   elastic:  n0 n1 n2 Zp+ Zs+ Fscale k_p k_s wall 0 0 0
//   anisotropic: n0 n1 n2 at av bt bv wall   with S = Z- + Z+ and, at a face
//             node with full jumps [v] = v+ - v-, [t] = t+ - t-,
//             velocity lift  at [t] + av [v],  at = Fscale Z-/(S rho),
//             av = Fscale Z- Z+/(S rho);  strain lift  bt [t] + bv [v],
//             bt = Fscale/S,  bv = Fscale Z+/S
// (wall = 1 for an unpaired face: the mirror ghost state applies there).
template <int PHYS>
struct FaceRec;
template <>
struct FaceRec<0> {
  static constexpr int W = 8, WALL = 6;
};
template <>
struct FaceRec<1> {
  static constexpr int W = 12, WALL = 8;
};
template <>
struct FaceRec<2> {
  static constexpr int W = 8, WALL = 7;
};

template <int PHYS>
__device__ __forceinline__ void face_record(const float* __restrict__ G, const float* __restrict__ cf, int f,
                                            int word, float* __restrict__ out) {
  float n[3], fs;
  face_normal(G, f, n, fs);
  const bool wall = (word & 7) == 7;
  out[0] = n[0];
  out[1] = n[1];
  out[2] = n[2];
  if constexpr (PHYS == 0) {
    const float ZM = cf[2];
    const float ZP = wall ? ZM : cf[4 + f];
    const float kc = 2.0f * __builtin_amdgcn_rcpf(ZM + ZP);
    out[3] = ZP;
    out[4] = fs * cf[0] * kc;
    out[5] = -fs * cf[3] * kc;
    out[6] = wall ? 1.0f : 0.0f;
    out[7] = 0.0f;
  } else if constexpr (PHYS == 2) {
    const float ZM = cf[22];
    const float ZP = wall ? ZM : cf[24 + f];
    const float iS = __builtin_amdgcn_rcpf(ZM + ZP);
    const float irho = cf[21];
    out[3] = fs * ZM * iS * irho;
    out[4] = fs * ZM * ZP * iS * irho;
    out[5] = fs * iS;
    out[6] = fs * ZP * iS;
    out[7] = wall ? 1.0f : 0.0f;
  } else {
    const float ZpM = cf[3], ZsM = cf[4];
    const float ZpP = wall ? ZpM : cf[8 + f];
    const float ZsP = wall ? ZsM : cf[12 + f];
    out[3] = ZpP;
    out[4] = ZsP;
    out[5] = fs;
    out[6] = 2.0f * __builtin_amdgcn_rcpf(ZpM + ZpP);
    out[7] = 2.0f * __builtin_amdgcn_rcpf(ZsM + ZsP);
    out[8] = wall ? 1.0f : 0.0f;
    out[9] = out[10] = out[11] = 0.0f;
  }
}

// Face node of the neighbour's face that meets own face node j under the
// relative orientation o (0..5): own node j <-> (a, b) with b the outer index
// of the face lattice, barycentric beta = (N - a - b, a, b) on the own face's
// vertices; own vertex p is the neighbour's vertex P_o[p] for the six
// permutations P = (012, 021, 102, 120, 201, 210), so the neighbour's
// (a', b') = (beta[p1], beta[p2]) with P_o[p1] = 1, P_o[p2] = 2.  The same
// numbering as the host-built permutation rows, computed in registers.
__host__ __device__ __forceinline__ int face_perm_node(int N, int o, int j) {
  // row b of the face lattice starts at S(b) = b (N + 1) - b (b - 1) / 2
  int b = 0;
  for (int bb = 1; bb <= N; ++bb) b += (j >= bb * (N + 1) - bb * (bb - 1) / 2) ? 1 : 0;
  const int a = j - (b * (N + 1) - b * (b - 1) / 2);
  const int beta0 = N - a - b, beta1 = a, beta2 = b;
  // p1, p2 per orientation: (1,2) (2,1) (0,2) (0,1) (2,0) (1,0)
  const int p1 = (o == 0 || o == 5) ? 1 : ((o == 1 || o == 4) ? 2 : 0);
  const int p2 = (o == 0 || o == 2) ? 2 : ((o == 1 || o == 3) ? 1 : 0);
  const int a2 = p1 == 0 ? beta0 : (p1 == 1 ? beta1 : beta2);
  const int b2 = p2 == 0 ? beta0 : (p2 == 1 ? beta1 : beta2);
  return b2 * (N + 1) - b2 * (b2 - 1) / 2 + a2;
}

__device__ __forceinline__ int64_t tile_of_block(int xcd_remap) {
  const int64_t b = blockIdx.x;
  if (!xcd_remap) return b;
  // Workgroups are dealt to the 8 XCDs round-robin; this option gives each
  // XCD a contiguous range of tiles so that neighbours share an L2 (off by
  // default: keeping the tiles in flight one contiguous window of the
  // arrays measured faster).
  const int64_t per = gridDim.x / 8;  // grid is a multiple of 8 when remapping
  return (b % 8) * per + b / 8;
}

}  // namespace dev
}  // namespace dgw
