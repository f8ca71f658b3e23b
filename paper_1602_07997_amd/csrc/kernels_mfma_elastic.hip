// MFMA variants of the fused DG step, isotropic elastic system (Sec. 2.1 and
// the elastic right-hand side of Sec. 3.2), gfx950 matrix cores.
//
// With the element as the GEMM column, for a tile of E = 16 NBLK elements:
//   Dv_il = D_l v_i                 (9 products, K = Np)
//   dS_i  = sum_l D_l S_il,  S_il = sum_a g_al s_ia   (K = Np, S formed per k-step)
//   a_c   = L_f A_c                 (5 products per face, K = Nfp, L_f the
//                                    face-f block of the lift matrix)
// with the penalty scalars of Sec. 2.1 at face f's nodes (jumps halved)
//   A1 = Fs k_p (s_nn + Zp+ v_n), A2 = Fs k_s (s_nn + Zs+ v_n), A3 = Fs (s n + Zs+ v).
// The face normal, k_s and the element's coefficients are constant over an
// affine face, so they are applied after the product:
//   Lv_i  = sum_f n_i (c_p a1 - c_s a2) + k_s c_s a3_i
//   Ls_ij = sum_f 2 mu (a1 - a2) n_i n_j + mu k_s (n_i a3_j + a3_i n_j) + delta_ij lambda a1
// and the right-hand side is
//   r_v_i = (1/rho) dS_i + Lv_i,
//   r_s_ij = mu (dv_i/dx_j + dv_j/dx_i) + delta_ij lambda div v + Ls_ij,
//   dv_i/dx_j = sum_l g_jl Dv_il.
// Precisions as in the acoustic kernel: FP32 16x16x4, or BF16 / FP16
// 16x16x16 with both operands split hi + lo and three products accumulated in
// FP32.  Workgroups of 8 wavefronts (4 for the 16-bit products at N = 5,
// 12 for FP32 at N = 6, with 32-element tiles, and N = 8); phases:
//   A1  every global read indexed by the tile alone, issued together;
//       constants into LDS;
//   A2  neighbour traces; face records; the five LIFT operands of every face
//       node into LDS;
//   C2  LIFT products per face, combined into the nine contributions and
//       kept in registers;
//   B1  the tile's nine fields into the same LDS region;
//   C1  volume products and the epilogue (transpose through a per-wave LDS
//       scratch, AB3 update, q / r writes, own traces), pair by pair.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_device.hpp"
#include "kernels.hpp"
#include "mfma_common.hpp"

namespace dgw {

namespace {

using namespace dev;
using namespace mfma;

// eight wavefronts per workgroup; four for the split 16-bit products at
// N = 5, whose tile has only four (node block, element block) pairs, so that
// no wavefront idles through the products and two workgroups share a compute
// unit (measured: ~20% faster there, neutral or slower elsewhere); twelve for
// the FP32 products at N = 8, whose eleven pairs then take one round instead
// of two (5% faster despite a few spilled registers; neutral for 16-bit),
// and for FP32 at N = 6 with 32-element tiles, whose twelve pairs take one
// wavefront each (7% faster than 16-element tiles on eight wavefronts)
template <int N, int PREC>
constexpr int elastic_threads() {
  return (N == 5 && PREC != 0) ? 256 : (((N == 8 || N == 6) && PREC == 0) ? 768 : 512);
}

// Waves per SIMD the register allocation must allow.  The default follows
// from the workgroup size (threads / 256); FP32 at N = 5 sits at the edge of
// 168 VGPRs (3 waves) and is held there: at 2 waves it runs about 30% slower.
template <int N, int PREC>
constexpr int elastic_min_waves() {
  return (N == 5 && PREC == 0) ? 3 : (elastic_threads<N, PREC>() + 255) / 256;
}

template <int N, int PREC, int PHYS = 1>
struct EShape {
  static constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP;
  static constexpr int KS = PREC == 0 ? 4 : 16;
  static constexpr int MB = (NP + 15) / 16;
  static constexpr int KP = rup(NP, KS);
  static constexpr int KF = rup(NFP, KS);  // LIFT K of one face, zero padded
  static constexpr int KL = 4 * KF;        // LIFT K, face blocks of KF
  // 32-element tiles for FP32 at N = 6: twelve pairs, one per wavefront
  static constexpr int NBLK = (N == 1) ? 4 : (N <= 3 ? 2 : ((N == 6 && PREC == 0) ? 2 : 1));
  static constexpr int E = 16 * NBLK;
  static constexpr int PAIRS = MB * NBLK;
  static constexpr int NSV = 9;  // volume operand sets (the fields)
  // LIFT operand sets (the lifted penalty scalars): five for the isotropic
  // flux, six for the anisotropic one (velocity correction, strain vector)
  static constexpr int NSL = PHYS == 1 ? 5 : 6;
  static constexpr int THREADS = elastic_threads<N, PREC>();
  // 4-byte words: the LIFT sets, then (reused) the volume sets
  static constexpr int REGION = (NSV * KP > NSL * KL ? NSV * KP : NSL * KL) * E;
};

// Operand region, sets of STRIDE rows (KL for the LIFT operands, KP for the
// fields): set s, row k, column e.
//   FP32 sets (PREC 0, and the volume sets of every precision):
//     PREC 0:  word (s*STRIDE + k)*E + swz(k, e)
//     else:    word s*STRIDE*E + ((k/4)*E + e)*4 + k%4   (4 consecutive k contiguous)
//   16-bit split sets (LIFT operands of PREC 1, 2): hi at unit
//     s*STRIDE*E + ((k/4)*E + e)*4 + k%4, lo REGION units later.
template <int N, int PREC, int STRIDE, int PHYS = 1>
struct ERegion {
  using S = EShape<N, PREC, PHYS>;
  float* w;
  __device__ __forceinline__ int f32_word(int s, int k, int e) const {
    if constexpr (PREC == 0)
      return (s * STRIDE + k) * S::E + swz<S::E>(k, e);
    else
      return s * STRIDE * S::E + ((k >> 2) * S::E + e) * 4 + (k & 3);
  }
  __device__ __forceinline__ void put_f32(int s, int k, int e, float x) const { w[f32_word(s, k, e)] = x; }
  __device__ __forceinline__ void put_split(int s, int k, int e, float x) const {
    if constexpr (PREC == 0) {
      put_f32(s, k, e, x);
    } else {
      uint16_t* u = reinterpret_cast<uint16_t*>(w);
      uint16_t hi, lo;
      split16<PREC>(x, hi, lo);
      const int idx = s * STRIDE * S::E + ((k >> 2) * S::E + e) * 4 + (k & 3);
      u[idx] = hi;
      u[S::REGION + idx] = lo;
    }
  }
};

template <int PREC>
__device__ __forceinline__ Frag16 split4(const float4& x) {
  uint16_t h0, l0, h1, l1, h2, l2, h3, l3;
  split16<PREC>(x.x, h0, l0);
  split16<PREC>(x.y, h1, l1);
  split16<PREC>(x.z, h2, l2);
  split16<PREC>(x.w, h3, l3);
  Frag16 f;
  f.hi = shortx4{static_cast<short>(h0), static_cast<short>(h1), static_cast<short>(h2), static_cast<short>(h3)};
  f.lo = shortx4{static_cast<short>(l0), static_cast<short>(l1), static_cast<short>(l2), static_cast<short>(l3)};
  return f;
}

template <int N, int PREC, int PHYS>
// Pairs [p0, p1) of the tile's (node block, element block) pairs: all of
// them, or a part of a tile split over several workgroups (every workgroup
// of a split tile stages the whole tile and writes only its pairs' nodes)
__device__ __forceinline__ void step_mfma_elastic_tile(const StepArgs& a, int64_t tile, int p0, int p1) {
  static_assert(PHYS == 1 || (PHYS == 2 && PREC == 0), "anisotropic: FP32 products only");
  using S = EShape<N, PREC, PHYS>;
  constexpr int NP = S::NP, NFP = S::NFP, MB = S::MB, KP = S::KP, KL = S::KL, KF = S::KF, E = S::E;
  constexpr int NF = 9, NT = 6, CB = Phys<PHYS>::CB;
  constexpr int NSL = S::NSL;
  constexpr int FW = FaceRec<PHYS>::W;
  constexpr int TH = S::THREADS;
  constexpr int NW = TH / 64;
  constexpr int NIT = (E * KP + TH - 1) / TH;
  constexpr int FIT = (E * KL + TH - 1) / TH;
  constexpr int SCR = 16 * 17;
  constexpr int PPW = (S::PAIRS + NW - 1) / NW;

  __shared__ __attribute__((aligned(16))) float s_B[S::REGION];
  __shared__ float s_g[E * 9];
  __shared__ float s_cf[E * CB];
  __shared__ float s_face[E * 4 * FW];
  __shared__ float s_scr[NW * SCR];

  const int64_t e0 = a.e_begin + tile * E;
  if (e0 >= a.K) return;  // whole workgroup exits together
  const int ne = static_cast<int>((a.K - e0) < E ? (a.K - e0) : E);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int kq = lane >> 4, nl = lane & 15;
  const bool step = (a.mode == kStepMode);
  const ERegion<N, PREC, KL, PHYS> lreg{s_B};  // LIFT operands
  const ERegion<N, PREC, KP, PHYS> vreg{s_B};  // fields (after the LIFT products)

  // ---- A1: every global read indexed by the tile alone, issued together ----
  // Loads are unconditional at clamped (in-range) addresses and unused values
  // are dropped by selects, so that none waits behind a branch or behind
  // another item's load.
  constexpr int GIT = (E * 9 + TH - 1) / TH;
  constexpr int CIT = (E * CB + TH - 1) / TH;
  constexpr int PIT = (6 * NFP + TH - 1) / TH;
  static_assert(6 * NFP <= NW * SCR, "the permutation table borrows the transpose scratch");
  static_assert(E * 4 <= TH, "one face record per thread");
  int* s_perm = reinterpret_cast<int*>(s_scr);  // free until the epilogue
  float gv[GIT], cv[CIT];
  int pv[PIT];
#pragma unroll
  for (int t = 0; t < GIT; ++t) {
    const int i = tid + t * TH;
    gv[t] = a.geo[e0 * 9 + (i < ne * 9 ? i : 0)];
  }
#pragma unroll
  for (int t = 0; t < CIT; ++t) {
    const int i = tid + t * TH;
    cv[t] = a.cf[e0 * CB + (i < ne * CB ? i : 0)];
  }
#pragma unroll
  for (int t = 0; t < PIT; ++t) {
    const int i = tid + t * TH;
    pv[t] = a.perm[i < 6 * NFP ? i : 0];
  }
  const int rec_e = tid >> 2, rec_f = tid & 3;
  const int rec_word = a.conn[(e0 + (rec_e < ne ? rec_e : 0)) * 4 + rec_f];
  // face-slot items i = e*KL + slot, slot = f*KF + j, a face node while j < NFP:
  // connectivity word and own trace (v and s n of the fields read this step)
  int cw[FIT];
  float ot[FIT][NT];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * TH;
    const int e = i / KL, slot = i - e * KL;
    const int fs = slot / KF, js = slot - fs * KF;
    const bool ok = e < ne && js < NFP;
    const int ec = ok ? e : 0, f = ok ? fs : 0, j = ok ? js : 0;
    cw[t] = a.conn[(e0 + ec) * 4 + f];
    const float* own = a.qf_in + ((e0 + ec) * 4 + f) * NT * NFP + j;
#pragma unroll
    for (int c = 0; c < NT; ++c) ot[t][c] = own[c * NFP];
  }
#pragma unroll
  for (int t = 0; t < GIT; ++t) {
    const int i = tid + t * TH;
    if (i < ne * 9) s_g[i] = gv[t];
  }
#pragma unroll
  for (int t = 0; t < CIT; ++t) {
    const int i = tid + t * TH;
    if (i < ne * CB) s_cf[i] = cv[t];
  }
#pragma unroll
  for (int t = 0; t < PIT; ++t) {
    const int i = tid + t * TH;
    if (i < 6 * NFP) s_perm[i] = pv[t];
  }
  __syncthreads();

  // ---- A2: neighbour traces; face records; LIFT operands at every face slot --
  float nt[FIT][NT];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * TH;
    const int e = i / KL, slot = i - e * KL;
    const int fs = slot / KF, js = slot - fs * KF;
    const bool ok = e < ne && js < NFP;
    const int ec = ok ? e : 0, f = ok ? fs : 0, j = ok ? js : 0;
    const int w = cw[t];
    const bool wall = (w & 7) == 7;
    // a wall reads its own trace (in range, value unused)
    const int64_t kn = wall ? e0 + ec : static_cast<int64_t>(w >> 5);
    const int fnb = wall ? f : (w >> 3) & 3;
    const int jn = wall ? j : s_perm[(w & 7) * NFP + j];
    const float* tr = a.qf_in + (kn * 4 + fnb) * NT * NFP + jn;
#pragma unroll
    for (int c = 0; c < NT; ++c) nt[t][c] = tr[c * NFP];
  }
  if (rec_e < ne) face_record<PHYS>(s_g + 9 * rec_e, s_cf + CB * rec_e, rec_f, rec_word, s_face + tid * FW);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * TH;
    if (i >= E * KL) continue;
    const int e = i / KL, slot = i - e * KL;
    // the five lifted scalars of Sec. 2.1's elastic penalty (jumps halved):
    // A1 = Fs k_p (s_nn + Zp+ v_n), A2 = Fs k_s (s_nn + Zs+ v_n),
    // A3 = Fs (s n + Zs+ v); the normal and the coefficients are applied
    // after the per-face LIFT products
    float b[NSL];
#pragma unroll
    for (int c = 0; c < NSL; ++c) b[c] = 0.0f;
    const int f = slot / KF;
    if (e < ne && slot - f * KF < NFP) {
      const float* rec = s_face + (e * 4 + f) * FW;
      const float n0 = rec[0], n1 = rec[1], n2 = rec[2];
      const bool wall = (cw[t] & 7) == 7;
      const float gw = (cw[t] & 8) ? 0.0f : 1.0f;  // absorbing wall: zero exterior state
      float vM[3], tM[3], vP[3], tP[3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        vM[ii] = ot[t][ii];
        tM[ii] = ot[t][3 + ii];
        // traction-free wall: mirror state v+ = v-, (s n)+ = -(s n)-;
        // otherwise the neighbour stored s n with its own normal
        vP[ii] = wall ? gw * vM[ii] : nt[t][ii];
        tP[ii] = wall ? -gw * tM[ii] : -nt[t][3 + ii];
      }
      if constexpr (PHYS == 2) {
        // one-impedance Riemann solution per side: the velocity correction
        // (t* - t-)/rho and the vector v* - v-, both times Fscale (full jumps)
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          const float jv = vP[ii] - vM[ii], jt = tP[ii] - tM[ii];
          b[ii] = rec[3] * jt + rec[4] * jv;
          b[3 + ii] = rec[5] * jt + rec[6] * jv;
        }
      } else {
        float jv[3], jt[3];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          jv[ii] = 0.5f * (vP[ii] - vM[ii]);
          jt[ii] = 0.5f * (tP[ii] - tM[ii]);
        }
        const float jvn = jv[0] * n0 + jv[1] * n1 + jv[2] * n2;
        const float jsnn = jt[0] * n0 + jt[1] * n1 + jt[2] * n2;
        const float ZpP = rec[3], ZsP = rec[4], fs = rec[5], kp = rec[6], ks = rec[7];
        b[0] = fs * kp * (jsnn + ZpP * jvn);
        b[1] = fs * ks * (jsnn + ZsP * jvn);
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) b[2 + ii] = fs * (jt[ii] + ZsP * jv[ii]);
      }
    }
#pragma unroll
    for (int c = 0; c < NSL; ++c) lreg.put_split(c, slot, e, b[c]);
  }
  __syncthreads();

  // isotropic, N = 5 and 8: the first batch of the field staging below is read now,
  // so that its latency hides behind the LIFT products (4 % / 1 % faster;
  // 2 % slower at N = 6, where the registers it holds cost spills)
  constexpr int BB = 3;
  constexpr bool B1PRE = PHYS == 1 && (N == 5 || N == 8);
  float xpre[B1PRE ? BB : 1][9];
  if constexpr (B1PRE) {
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int i = tid + u * TH;
      const int e = i / KP, n = i - e * KP;
      const bool ok = u < NIT && i < E * KP && e < ne && n < NP;
      const float* qe = a.q_in + (e0 + (ok ? e : 0)) * NF * NP + (ok ? n : 0);
#pragma unroll
      for (int c = 0; c < 9; ++c) xpre[u][c] = qe[c * NP];
    }
  }

  // ---- C2: LIFT products per face, combined into the nine right-hand-side
  // contributions (kept in registers) ------------------------------------------
  // For face f with normal n and the element's lambda, mu, c_p, c_s and the
  // face's k_s, the lifted scalars a1 = L_f A1, a2 = L_f A2, a3 = L_f A3 give
  //   velocity  n (c_p a1 - c_s a2) + k_s c_s a3
  //   stress    2 mu (a1 - a2) n n^T + mu k_s (n a3^T + a3 n^T) + lambda a1 I.
  floatx4 LL[PPW][9];
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
#pragma unroll
    for (int c = 0; c < 9; ++c) LL[q][c] = floatx4{0, 0, 0, 0};
    const int p = p0 + wave + NW * q;
    if (p >= p1) continue;
    const int mb = p % MB, nb = p / MB;
    const int col = nb * 16 + nl;
    const int ecol = col < ne ? col : 0;
    floatx4 LA[NSL];
#pragma unroll
    for (int c = 0; c < NSL; ++c) LA[c] = floatx4{0, 0, 0, 0};
    auto combine = [&](int f) {
      const float* rec = s_face + (ecol * 4 + f) * FW;
      if constexpr (PHYS == 2) {
        // velocity: the lifted corrections as they are; rows 3..8 collect
        // the engineering strain of n (x) w, to which the stiffness is
        // applied once, with the volume strain, before the update
        const float n0 = rec[0], n1 = rec[1], n2 = rec[2];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float w0 = LA[3][r], w1 = LA[4][r], w2 = LA[5][r];
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) LL[q][ii][r] += LA[ii][r];
          LL[q][3][r] += n0 * w0;
          LL[q][4][r] += n1 * w1;
          LL[q][5][r] += n2 * w2;
          LL[q][6][r] += n1 * w2 + n2 * w1;
          LL[q][7][r] += n0 * w2 + n2 * w0;
          LL[q][8][r] += n0 * w1 + n1 * w0;
        }
      } else {
        const float* cf = s_cf + ecol * CB;
        const float nn[3] = {rec[0], rec[1], rec[2]};
        const float ks = rec[7];
        const float lam = cf[0], mu = cf[1], cp = cf[5], cs = cf[6];
        const int vi[6] = {0, 1, 2, 1, 0, 0};
        const int vj[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float a1 = LA[0][r], a2 = LA[1][r];
          const float a3[3] = {LA[2][r], LA[3][r], LA[4][r]};
          const float t = cp * a1 - cs * a2;
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) LL[q][ii][r] += nn[ii] * t + ks * cs * a3[ii];
          const float b2 = 2.0f * mu * (a1 - a2), c3 = mu * ks;
#pragma unroll
          for (int v = 0; v < 6; ++v) {
            const int ii = vi[v], jj = vj[v];
            float x = b2 * nn[ii] * nn[jj] + c3 * (nn[ii] * a3[jj] + a3[ii] * nn[jj]);
            if (ii == jj) x += lam * a1;
            LL[q][3 + v][r] += x;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < NSL; ++c) LA[c] = floatx4{0, 0, 0, 0};
    };
    // operator fragments stream through two register sets (pipelined, fully
    // unrolled so that each k-step's face is known at compile time)
    if constexpr (PREC == 0) {
      const float* Lp = a.Lpack + static_cast<int64_t>(mb) * (KL / 4) * 64 + lane;
      constexpr int NK = KL / 4, NKF = KF / 4, PD = NK < 8 ? NK : 8;
      using R = Ring<float, PD, 1>;
      auto load = [&](R& r, int g) {
#pragma unroll
        for (int i = 0; i < PD; ++i) r.v[i][0] = Lp[(g * PD + i < NK ? g * PD + i : NK - 1) * 64];
      };
      auto compute = [&](const R& r, int g, int cnt) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          if (i >= cnt) break;
          const int kk = g * PD + i;
          const int k = kk * 4 + kq;
#pragma unroll
          for (int c = 0; c < NSL; ++c) LA[c] = mfma_f32(r.v[i][0], s_B[lreg.f32_word(c, k, col)], LA[c]);
          if (kk % NKF == NKF - 1) combine(kk / NKF);
        }
      };
      pipelined<NK, PD, R, true>(load, compute);
    } else {
      const uint16_t* u = reinterpret_cast<const uint16_t*>(s_B);
      constexpr int LO = S::REGION;  // 16-bit units
      const shortx4* Lh = reinterpret_cast<const shortx4*>(a.L16h) + static_cast<int64_t>(mb) * (KL / 16) * 64 + lane;
      const shortx4* Ll = reinterpret_cast<const shortx4*>(a.L16l) + static_cast<int64_t>(mb) * (KL / 16) * 64 + lane;
      constexpr int NK = KL / 16, NKF = KF / 16, PD = NK < 2 ? NK : 2;
      using R = Ring<Frag16, PD, 1>;
      auto load = [&](R& r, int g) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          const int kk = g * PD + i < NK ? g * PD + i : NK - 1;
          r.v[i][0] = Frag16{Lh[kk * 64], Ll[kk * 64]};
        }
      };
      auto compute = [&](const R& r, int g, int cnt) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          if (i >= cnt) break;
          const int kk = g * PD + i;
          const int off = ((kk * 4 + kq) * E + col) * 4;
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            Frag16 b;
            b.hi = *reinterpret_cast<const shortx4*>(u + c * KL * E + off);
            b.lo = *reinterpret_cast<const shortx4*>(u + LO + c * KL * E + off);
            LA[c] = mfma_split<PREC>(r.v[i][0], b, LA[c]);
          }
          if (kk % NKF == NKF - 1) combine(kk / NKF);
        }
      };
      pipelined<NK, PD, R, true>(load, compute);
    }
  }
  __syncthreads();

  // ---- B1: the nine fields (FP32) -------------------------------------------
  // reads in batches of up to three node items, at clamped addresses (the
  // first batch possibly before the LIFT products, above)
#pragma unroll
  for (int t0 = 0; t0 < NIT; t0 += BB) {
    float x[BB][9];
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int i = tid + (t0 + u) * TH;
      const int e = i / KP, n = i - e * KP;
      const bool ok = t0 + u < NIT && i < E * KP && e < ne && n < NP;
      const float* qe = a.q_in + (e0 + (ok ? e : 0)) * NF * NP + (ok ? n : 0);
#pragma unroll
      for (int c = 0; c < 9; ++c) x[u][c] = (B1PRE && t0 == 0) ? xpre[B1PRE ? u : 0][c] : qe[c * NP];
    }
#pragma unroll
    for (int u = 0; u < BB; ++u) {
      const int i = tid + (t0 + u) * TH;
      if (t0 + u >= NIT || i >= E * KP) continue;
      const int e = i / KP, n = i - e * KP;
      const bool ok = e < ne && n < NP;
#pragma unroll
      for (int c = 0; c < 9; ++c) vreg.put_f32(c, n, e, ok ? x[u][c] : 0.0f);
    }
  }
  __syncthreads();

  // ---- C1: volume products and the epilogue, pair by pair -------------------
  float* scr = s_scr + wave * SCR;
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
    const int p = p0 + wave + NW * q;
    if (p >= p1) continue;
    const int mb = p % MB, nb = p / MB;
    const int col = nb * 16 + nl;
    const int ec = col < ne ? col : 0;
    float G[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) G[t] = s_g[9 * ec + t];
    floatx4 Dv[3][3], dS[3];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) {
      dS[ii] = floatx4{0, 0, 0, 0};
#pragma unroll
      for (int l = 0; l < 3; ++l) Dv[ii][l] = floatx4{0, 0, 0, 0};
    }
    if constexpr (PREC == 0) {
      const float* Dp = a.Dpack + static_cast<int64_t>(mb) * (KP / 4) * 64 + lane;
      constexpr int JS = MB * (KP / 4) * 64;
      // prefetch depth 2 at N = 8 keeps the twelve-wavefront workgroup free
      // of register spills (157 registers; 1% faster than depth 4 with 52
      // bytes of scratch per lane); at N = 6 depth 4 with 16 bytes of spills
      // measured 3% faster than the spill-free depth 2
      constexpr int PDV = N == 8 ? 2 : 4;
      constexpr int NK = KP / 4, PD = NK < PDV ? NK : PDV;
      using R = Ring<float, PD, 3>;
      auto load = [&](R& r, int g) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          const int kk = g * PD + i < NK ? g * PD + i : NK - 1;
#pragma unroll
          for (int l = 0; l < 3; ++l) r.v[i][l] = Dp[l * JS + kk * 64];
        }
      };
      auto compute = [&](const R& r, int g, int cnt) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          if (i >= cnt) break;
          const int k = (g * PD + i) * 4 + kq;
          float x[9];
#pragma unroll
          for (int c = 0; c < 9; ++c) x[c] = s_B[vreg.f32_word(c, k, col)];
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) {
            const float si0 = x[3 + voigt(ii, 0)], si1 = x[3 + voigt(ii, 1)], si2 = x[3 + voigt(ii, 2)];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
              Dv[ii][l] = mfma_f32(r.v[i][l], x[ii], Dv[ii][l]);
              const float ax = G[0 * 3 + l] * si0 + G[1 * 3 + l] * si1 + G[2 * 3 + l] * si2;
              dS[ii] = mfma_f32(r.v[i][l], ax, dS[ii]);
            }
          }
        }
      };
      pipelined<NK, PD, R>(load, compute);
    } else {
      constexpr int JS = MB * (KP / 16) * 64;
      const shortx4* Dh = reinterpret_cast<const shortx4*>(a.D16h) + static_cast<int64_t>(mb) * (KP / 16) * 64 + lane;
      const shortx4* Dl = reinterpret_cast<const shortx4*>(a.D16l) + static_cast<int64_t>(mb) * (KP / 16) * 64 + lane;
      constexpr int NK = KP / 16, PD = 1;
      using R = Ring<Frag16, PD, 3>;
      auto load = [&](R& r, int g) {
#pragma unroll
        for (int l = 0; l < 3; ++l) r.v[0][l] = Frag16{Dh[l * JS + g * 64], Dl[l * JS + g * 64]};
      };
      auto compute = [&](const R& r, int kk, int) {
        float4 x[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) x[c] = *reinterpret_cast<const float4*>(s_B + vreg.f32_word(c, kk * 16 + 4 * kq, col));
        const Frag16* d = r.v[0];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          const Frag16 vb = split4<PREC>(x[ii]);
          const float4 s0 = x[3 + voigt(ii, 0)], s1 = x[3 + voigt(ii, 1)], s2 = x[3 + voigt(ii, 2)];
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            Dv[ii][l] = mfma_split<PREC>(d[l], vb, Dv[ii][l]);
            const float g0 = G[0 * 3 + l], g1 = G[1 * 3 + l], g2 = G[2 * 3 + l];
            float4 ax;
            ax.x = g0 * s0.x + g1 * s1.x + g2 * s2.x;
            ax.y = g0 * s0.y + g1 * s1.y + g2 * s2.y;
            ax.z = g0 * s0.z + g1 * s1.z + g2 * s2.z;
            ax.w = g0 * s0.w + g1 * s1.w + g2 * s2.w;
            dS[ii] = mfma_split<PREC>(d[l], split4<PREC>(ax), dS[ii]);
          }
        }
      };
      pipelined<NK, PD, R>(load, compute);
    }
    // right-hand sides in the accumulator layout (rows 4 kq + r, column nl)
    const float* cf = s_cf + ec * CB;
    float rr[9][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float gv[3][3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          gv[ii][jj] = G[3 * jj + 0] * Dv[ii][0][r] + G[3 * jj + 1] * Dv[ii][1][r] + G[3 * jj + 2] * Dv[ii][2][r];
      if constexpr (PHYS == 2) {
        // stiffness times the volume strain plus the faces' strain
        const float irho = cf[21];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) rr[ii][r] = irho * dS[ii][r] + LL[q][ii][r];
        const float ev[6] = {gv[0][0] + LL[q][3][r], gv[1][1] + LL[q][4][r], gv[2][2] + LL[q][5][r],
                             gv[1][2] + gv[2][1] + LL[q][6][r], gv[0][2] + gv[2][0] + LL[q][7][r],
                             gv[0][1] + gv[1][0] + LL[q][8][r]};
#pragma unroll
        for (int va = 0; va < 6; ++va) {
          float x = 0.0f;
#pragma unroll
          for (int vb = 0; vb < 6; ++vb) x += cf[va <= vb ? upper6(va, vb) : upper6(vb, va)] * ev[vb];
          rr[3 + va][r] = x;
        }
      } else {
        const float lam = cf[0], mu = cf[1], irho = cf[2];
        const float divv = gv[0][0] + gv[1][1] + gv[2][2];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) rr[ii][r] = irho * dS[ii][r] + LL[q][ii][r];
        const int vi[6] = {0, 1, 2, 1, 0, 0};
        const int vj[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          const int ii = vi[v], jj = vj[v];
          float x = mu * (gv[ii][jj] + gv[jj][ii]) + LL[q][3 + v][r];
          if (ii == jj) x += lam * divv;
          rr[3 + v][r] = x;
        }
      }
    }
    // transpose, update and write field by field; lane -> (node mb*16 + nl,
    // element nb*16 + kq + 4 it); the fields q^m come from the operand region
    // (the FP32 volume sets are exact copies, still in place), the history
    // is read three fields at a time, each batch issued together at clamped
    // addresses
    const int n = mb * 16 + nl;
    const int ncl = n < NP ? n : NP - 1;
    int nfs[3] = {-1, -1, -1};
    if (step) {
#pragma unroll
      for (int s = 0; s < 3; ++s) nfs[s] = a.nodeface[ncl * 3 + s];
    }
    const float* p1 = a.c1 != 0.0f ? a.r1 : a.q_in;  // history read only where it is used
    const float* p2 = a.c2 != 0.0f ? a.r2 : a.q_in;
    const float w1 = a.c1 != 0.0f ? 1.0f : 0.0f, w2 = a.c2 != 0.0f ? 1.0f : 0.0f;
    float qn[9][4];
#pragma unroll
    for (int c0 = 0; c0 < NF; c0 += 3) {
      float qo[3][4], h1[3][4], h2[3][4];
      if (step) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int e = nb * 16 + kq + 4 * it;
          const int64_t base = (e0 + (e < ne ? e : ne - 1)) * NF * NP + ncl;
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            qo[u][it] = s_B[vreg.f32_word(c0 + u, ncl, e < ne ? e : ne - 1)];
            h1[u][it] = p1[base + (c0 + u) * NP];
            h2[u][it] = p2[base + (c0 + u) * NP];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int c = c0 + u;
#pragma unroll
        for (int r = 0; r < 4; ++r) scr[nl * 17 + 4 * kq + r] = rr[c][r];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        float rt[4];
#pragma unroll
        for (int it = 0; it < 4; ++it) rt[it] = scr[(kq + 4 * it) * 17 + nl];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int e = nb * 16 + kq + 4 * it;
          qn[c][it] = step ? qo[u][it] + a.c0 * rt[it] + a.c1 * (w1 * h1[u][it]) + a.c2 * (w2 * h2[u][it]) : 0.0f;
          if (e >= ne || n >= NP) continue;
          const int64_t base = (e0 + e) * NF * NP + c * NP + n;
          a.r_out[base] = rt[it];
          if (step) a.q_out[base] = qn[c][it];
        }
      }
    }
    if (!step) continue;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int e = nb * 16 + kq + 4 * it;
      if (e >= ne || n >= NP) continue;
      const float* fr = s_face + e * 4 * FW;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int fj = nfs[s];
        if (fj < 0) break;
        const int f = fj / NFP, j = fj - f * NFP;
        const float n0 = fr[f * FW + 0], n1 = fr[f * FW + 1], n2 = fr[f * FW + 2];
        float* tr = a.qf_out + ((e0 + e) * 4 + f) * NT * NFP + j;
        tr[0] = qn[0][it];
        tr[NFP] = qn[1][it];
        tr[2 * NFP] = qn[2][it];
        // s n with Voigt (11, 22, 33, 23, 13, 12)
        tr[3 * NFP] = qn[3][it] * n0 + qn[8][it] * n1 + qn[7][it] * n2;
        tr[4 * NFP] = qn[8][it] * n0 + qn[4][it] * n1 + qn[6][it] * n2;
        tr[5 * NFP] = qn[7][it] * n0 + qn[6][it] * n1 + qn[5][it] * n2;
      }
    }
  }
}

// PHYS = 1: isotropic elasticity; PHYS = 2: anisotropic (FP32 products only)
template <int N, int PREC, int PHYS>
__global__ void __launch_bounds__((elastic_threads<N, PREC>()), (elastic_min_waves<N, PREC>()))
dg_step_mfma_elastic(StepArgs a) {
  int p0, p1;
  const int64_t tile = split_tile(tile_of_block(a.xcd_remap), a.split_from, a.split_parts,
                                  EShape<N, PREC, PHYS>::PAIRS, p0, p1);
  step_mfma_elastic_tile<N, PREC, PHYS>(a, tile, p0, p1);
}

template <int N, int PREC, int PHYS>
__global__ void __launch_bounds__((elastic_threads<N, PREC>()), (elastic_min_waves<N, PREC>()))
dg_step_mfma_elastic_batch(const StepArgs* __restrict__ args, const int2* __restrict__ work, int phase) {
  const int2 w = work[blockIdx.x];
  if (w.x < 0) return;  // padding entry of the work list
  const StepArgs a = args[w.x * kBatchPhases + phase];
  step_mfma_elastic_tile<N, PREC, PHYS>(a, w.y, 0, EShape<N, PREC, PHYS>::PAIRS);
}

// A short last round of tiles is split over up to ceil(pairs / 4)
// workgroups per tile, so that each part runs at most one pair's products
// per SIMD (tiles in launch order only).
template <int N, int PREC, int PHYS = 1>
hipError_t emfma_impl(const StepArgs& a, hipStream_t s) {
  constexpr int E = EShape<N, PREC, PHYS>::E, P = EShape<N, PREC, PHYS>::PAIRS;
  int64_t tiles = (a.K - a.e_begin + E - 1) / E;
  if (a.xcd_remap) tiles = ((tiles + 7) / 8) * 8;
  StepArgs b = a;
  TailSplit plan{tiles, tiles, 1};
  if (a.tail_split && !a.xcd_remap) {
    static std::atomic<int> slots_cache[16];
    const int slots = resident_workgroups(reinterpret_cast<const void*>(&dg_step_mfma_elastic<N, PREC, PHYS>),
                                          elastic_threads<N, PREC>(), slots_cache);
    plan = plan_tail_split(tiles, slots, (P + 3) / 4);
  }
  b.split_from = plan.from;
  b.split_parts = plan.parts;
  if (plan.grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_mfma_elastic<N, PREC, PHYS>), dim3(static_cast<unsigned>(plan.grid)),
                     dim3(elastic_threads<N, PREC>()), 0, s, b);
  return hipGetLastError();
}

template <int N, int PREC, int PHYS = 1>
hipError_t emfma_batch_impl(const StepArgs* args, const int2* work, int64_t ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_mfma_elastic_batch<N, PREC, PHYS>), dim3(static_cast<unsigned>(ntiles)),
                     dim3(elastic_threads<N, PREC>()), 0, s, args, work, phase);
  return hipGetLastError();
}

}  // namespace

#define DGW_EMFMA_DISPATCH(CALL)                                                         \
  switch (mfma_precision(variant)) {                                                     \
    case 0:                                                                              \
      switch (N) {                                                                       \
        case 1: return CALL(1, 0); case 2: return CALL(2, 0); case 3: return CALL(3, 0); \
        case 4: return CALL(4, 0); case 5: return CALL(5, 0); case 6: return CALL(6, 0); \
        case 7: return CALL(7, 0); case 8: return CALL(8, 0);                            \
      }                                                                                  \
      break;                                                                             \
    case 1:                                                                              \
      switch (N) {                                                                       \
        case 1: return CALL(1, 1); case 2: return CALL(2, 1); case 3: return CALL(3, 1); \
        case 4: return CALL(4, 1); case 5: return CALL(5, 1); case 6: return CALL(6, 1); \
        case 7: return CALL(7, 1); case 8: return CALL(8, 1);                            \
      }                                                                                  \
      break;                                                                             \
    case 2:                                                                              \
      switch (N) {                                                                       \
        case 1: return CALL(1, 2); case 2: return CALL(2, 2); case 3: return CALL(3, 2); \
        case 4: return CALL(4, 2); case 5: return CALL(5, 2); case 6: return CALL(6, 2); \
        case 7: return CALL(7, 2); case 8: return CALL(8, 2);                            \
      }                                                                                  \
      break;                                                                             \
  }

int mfma_elastic_tile_elements(int N, int variant) {
#define CALL(n, p) EShape<n, p>::E
  DGW_EMFMA_DISPATCH(CALL)
#undef CALL
  return -1;
}

MfmaPacking mfma_elastic_packing(int N, int variant) {
#define CALL(n, p) MfmaPacking{EShape<n, p>::MB, EShape<n, p>::KP, EShape<n, p>::KL, EShape<n, p>::KS, EShape<n, p>::E, EShape<n, p>::KF}
  DGW_EMFMA_DISPATCH(CALL)
#undef CALL
  return MfmaPacking{};
}

// the anisotropic kernels: FP32 products only
#define DGW_AMFMA_DISPATCH(CALL)                                                          \
  if (mfma_precision(variant) == 0) {                                                      \
    switch (N) {                                                                           \
      case 1: return CALL(1, 0); case 2: return CALL(2, 0); case 3: return CALL(3, 0);     \
      case 4: return CALL(4, 0); case 5: return CALL(5, 0); case 6: return CALL(6, 0);     \
      case 7: return CALL(7, 0); case 8: return CALL(8, 0);                                \
    }                                                                                      \
  }

hipError_t launch_step_mfma_elastic(int physics, int N, int variant, const StepArgs& a, hipStream_t s) {
  if (physics == 2) {
#define CALL(n, p) emfma_impl<n, p, 2>(a, s)
    DGW_AMFMA_DISPATCH(CALL)
#undef CALL
    return hipErrorInvalidValue;
  }
#define CALL(n, p) emfma_impl<n, p>(a, s)
  DGW_EMFMA_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_step_batch_mfma_elastic(int physics, int N, int variant, const StepArgs* args, const int2* work,
                                          int64_t ntiles, int phase, hipStream_t s) {
  if (physics == 2) {
#define CALL(n, p) emfma_batch_impl<n, p, 2>(args, work, ntiles, phase, s)
    DGW_AMFMA_DISPATCH(CALL)
#undef CALL
    return hipErrorInvalidValue;
  }
#define CALL(n, p) emfma_batch_impl<n, p>(args, work, ntiles, phase, s)
  DGW_EMFMA_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

#undef DGW_AMFMA_DISPATCH

#undef DGW_EMFMA_DISPATCH

}  // namespace dgw
