// MFMA variants of the fused DG step (acoustic), gfx950 matrix cores.
//
// The volume and LIFT products of eqs. (5)-(6) become small GEMMs with the
// element as the column index.  For a tile of E = 16 NBLK elements:
//   T_j = D_j p,   dv = sum_j D_j U_j  (U_j = sum_i g_ij v_i)        K = Np
//   lp  = sum_f L_f Pp_f,   lv_i = sum_f n_f,i L_f Pv_f              K = Nfp per face
// with L_f the face-f block of the lift matrix (Np x Nfp), and Pp = Fscale
// rho c^2 k_c alpha, Pv = -Fscale c k_c alpha the upwind penalties of
// Sec. 2.1 at face f's nodes.  The face normal is constant on an affine
// face, so it multiplies the lifted scalar Pv after the product: two lifted
// operands instead of four.  Three precisions:
//   PREC 0  FP32 v_mfma_f32_16x16x4_f32;
//   PREC 1  BF16 v_mfma_f32_16x16x32_bf16 (gfx950) with FP32 accumulation
//           and the split x = x_hi + x_lo of both operands, D x ~ D_hi x_hi +
//           D_hi x_lo + D_lo x_hi (the dropped D_lo x_lo is ~2^-16 |D||x|);
//   PREC 2  FP16 v_mfma_f32_16x16x32_f16 with the same three products
//           (~2^-22 |D||x| dropped).
// Operators are split and packed on the host in fragment order (the LIFT in
// face blocks of KF columns); the right-hand operands (p, U_j, the
// penalties) are formed and split once per tile in LDS.  Fields, r and the
// update stay FP32.
//
// Phases of one workgroup (4 wavefronts; 6 at N = 6, 8 at N = 7 and for the
// 16-bit products at N = 8):
//   A1  every global read indexed by the tile alone (constants, connectivity
//       words, own traces, fields), issued together; constants into LDS;
//   A2  neighbour traces and the upwind alpha of every face node (kept in
//       registers); face records; p and U_j of every node into LDS;
//   C1  volume products, one (16-node block, 16-element block) pair per
//       wavefront in turn;
//   B2  the two penalty operands into the same LDS region;
//   C2  LIFT products per face, then the epilogue: the pair's right-hand
//       sides are combined in the accumulator layout, transposed through a
//       per-wave LDS scratch so that every global access is a run of 16
//       consecutive nodes, and the AB3 update, q / r writes and own-trace
//       emission follow.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_device.hpp"
#include "kernels.hpp"
#include "mfma_common.hpp"

namespace dgw {

namespace {

using namespace dev;
using namespace mfma;

// k-steps of operator prefetch in the FP32 products (the LIFT stream takes
// twice as many) and in the 16-bit ones; the shallower FP32 depth at
// N = 5..7 leaves registers for more resident wavefronts (measured 1-4%
// faster there, 3% slower at N = 8)
constexpr int prefetch_fp32(int N) { return (N >= 5 && N <= 7) ? 2 : 4; }
constexpr int kPrefetch16 = 1;

// wavefronts per workgroup: one per (node block, element block) pair where
// that fits the tile (N = 4 FP32: three pairs, N = 6: six, N = 7: eight),
// which also leaves fewer accumulators per wavefront and so more resident
// wavefronts (N = 4: eight workgroups per compute unit instead of six, 2%
// faster); at N = 8 the split 16-bit products take eight wavefronts for
// eleven pairs, the FP32 ones keep four (measured faster each way)
constexpr int acoustic_waves(int N, int PREC) {
  return (N == 4 && PREC == 0) ? 3 : (N == 6 ? 6 : (N == 7 ? 8 : ((N == 8 && PREC != 0) ? 8 : 4)));
}

// resident wavefronts per SIMD that the register allocation must allow: the
// staging phases of N = 4, 5 are latency-bound, and the compiler fits them
// in 78 / 96 registers without spilling when asked (six / five workgroups
// per compute unit instead of four: 2-8% faster); the FP16 split products
// would spill, so they keep the default.  FP32 at N = 6 (six wavefronts per
// workgroup) and the split products at N = 3 sit just above the 80 / 168
// register edges of 6 / 3 waves and are held below them, without spilling
constexpr int acoustic_min_waves(int N, int PREC) {
  return (N == 4 && PREC == 0) ? 6
         : ((N == 4 || N == 5) && PREC != 2) ? 5
         : (N == 6 && PREC == 0) ? 6
         : (N == 3 && PREC != 0) ? 3
         : 1;
}

// Tile configuration CFG = precision (0 FP32, 1 BF16, 2 FP16) + 4 for the
// alternative FP32 tile that the autotuner may pick per mesh: twice the
// elements per tile and twice the wavefronts from N = 4 (pairs per wavefront
// unchanged), half the elements per tile below (more, smaller tiles).
constexpr int cfg_prec(int CFG) { return CFG & 3; }
constexpr bool cfg_wide(int CFG) { return CFG >= 4; }

template <int N, int CFG>
struct MShape {
  static constexpr int P = cfg_prec(CFG);        // precision of the products
  static constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP;
  static constexpr int KS = P == 0 ? 4 : 32;     // k per instruction
  static constexpr int MB = (NP + 15) / 16;      // 16-row node blocks
  static constexpr int KP = rup(NP, KS);         // volume K, zero padded
  static constexpr int KF = rup(NFP, KS);        // LIFT K of one face, zero padded
  static constexpr int KL = 4 * KF;              // LIFT K, face blocks of KF
  static constexpr int NBLK0 = (N <= 2) ? 4 : (N == 3 ? 2 : 1);
  static constexpr int NBLK = !cfg_wide(CFG) ? NBLK0 : (N <= 3 ? NBLK0 / 2 : 2);
  static constexpr int E = 16 * NBLK;            // elements per tile
  static constexpr int PAIRS = MB * NBLK;
  // wavefronts per workgroup (the wide N = 4 tile keeps eight: six spill)
  static constexpr int NW = (cfg_wide(CFG) && N >= 4) ? 2 * (N == 4 ? 4 : acoustic_waves(N, P)) : acoustic_waves(N, P);
  static constexpr int THREADS = 64 * NW;
  // 4-byte words of B operands: four volume sets of KP rows, then (reused)
  // two penalty sets of KL rows
  static constexpr int REGION = (4 * KP > 2 * KL ? 4 * KP : 2 * KL) * E;
};

// B operand region, sets of STRIDE rows (KP for the volume operands, KL for
// the penalties): set s, row k, column e.
//   FP32:   word (s*STRIDE + k)*E + swz(k, e)
//   16-bit: hi at unit s*STRIDE*E + ((k/8)*E + e)*8 + k%8, lo REGION units later
template <int N, int CFG, int STRIDE>
struct BRegion {
  using S = MShape<N, CFG>;
  float* w;
  __device__ __forceinline__ void put(int s, int k, int e, float x) const {
    if constexpr (S::P == 0) {
      w[(s * STRIDE + k) * S::E + swz<S::E>(k, e)] = x;
    } else {
      uint16_t* u = reinterpret_cast<uint16_t*>(w);
      uint16_t hi, lo;
      split16<S::P>(x, hi, lo);
      const int idx = s * STRIDE * S::E + ((k >> 3) * S::E + e) * 8 + (k & 7);
      u[idx] = hi;
      u[S::REGION + idx] = lo;
    }
  }
};

// Pairs [p0, p1) of the tile's (node block, element block) pairs: all of
// them, or a part of a tile split over several workgroups (every workgroup
// of a split tile stages the whole tile and writes only its pairs' nodes)
template <int N, int CFG>
__device__ __forceinline__ void step_mfma_tile(const StepArgs& a, int64_t tile, int p0, int p1) {
  using S = MShape<N, CFG>;
  constexpr int PREC = S::P;
  constexpr int NP = S::NP, NFP = S::NFP, MB = S::MB, KP = S::KP, KL = S::KL, KF = S::KF, E = S::E;
  constexpr int NF = 4, NT = 2, CB = 8;
  constexpr int FW = FaceRec<0>::W;
  constexpr int NW = S::NW, TH = S::THREADS;
  constexpr int NIT = (E * KP + TH - 1) / TH;  // node items (incl. padding) per thread
  constexpr int FIT = (E * KL + TH - 1) / TH;  // face-slot items (incl. padding) per thread
  constexpr int SCR = 16 * 17;                 // per-wave transpose scratch
  constexpr int PPW = (S::PAIRS + NW - 1) / NW;  // pairs per wavefront (at most)

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
  const bool step = (a.mode == kStepMode);
  const BRegion<N, CFG, KP> breg{s_B};   // volume operands
  const BRegion<N, CFG, KL> lreg{s_B};    // penalty operands (after the volume products)
  // tile-local arrays: uniform 64-bit bases, 32-bit offsets within the tile
  const float* tq = a.q_in + e0 * NF * NP;
  const float* ttr = a.qf_in + e0 * 4 * NT * NFP;
  const int32_t* tconn = a.conn + e0 * 4;

  // ---- A1: every global read of the tile's inputs, issued together --------
  // Each load is unconditional at a clamped, in-range address and unused
  // values are dropped by selects, so that no load waits behind a branch or
  // behind another item's load: the phase costs one memory round trip.
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
    gv[t] = (a.geo + e0 * 9)[i < ne * 9 ? i : ne * 9 - 1];
  }
#pragma unroll
  for (int t = 0; t < CIT; ++t) {
    const int i = tid + t * TH;
    cv[t] = (a.cf + e0 * CB)[i < ne * CB ? i : ne * CB - 1];
  }
#pragma unroll
  for (int t = 0; t < PIT; ++t) {
    const int i = tid + t * TH;
    pv[t] = a.perm[i < 6 * NFP ? i : 6 * NFP - 1];
  }
  // connectivity word of this thread's face record (e, f) = (tid / 4, tid % 4)
  const int rec_e = tid >> 2, rec_f = tid & 3;
  const int rec_word = tconn[(rec_e < ne ? rec_e : ne - 1) * 4 + rec_f];
  // face-slot items i = e*KL + slot, slot = f*KF + j, a face node while j < NFP:
  // connectivity word and own trace (p, v.n of the fields read this step);
  // the own trace waits for the neighbour's round at the highest degrees
  // (register budget)
  constexpr bool LATE_OWN = N >= 7;
  int cw[FIT];
  float pM[FIT], vnM[FIT];
  auto load_own = [&](int t) {
    const int i = tid + t * TH;
    const int e = i / KL, slot = i - e * KL;
    const int fs = slot / KF, js = slot - fs * KF;
    const bool ok = e < ne && js < NFP;
    const int ec = ok ? e : 0, f = ok ? fs : 0, j = ok ? js : 0;
    const float* own = ttr + (ec * 4 + f) * NT * NFP + j;
    pM[t] = own[0];
    vnM[t] = own[NFP];
  };
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * TH;
    const int e = i / KL, slot = i - e * KL;
    const int fs = slot / KF;
    const bool ok = e < ne && slot - fs * KF < NFP;
    cw[t] = tconn[(ok ? e : 0) * 4 + (ok ? fs : 0)];
    if (!LATE_OWN) load_own(t);
  }
  // node items i = e*KP + n (n < KP, so that the zero padding is written
  // too): the fields of the first NIT1 items now, the rest with the
  // neighbour traces (register budget)
  constexpr int NIT1 = (PREC == 0 && N >= 7) ? NIT : (NIT < 6 ? NIT : 6);
  float qv[NIT][NF];
  auto load_node = [&](int t) {
    const int i = tid + t * TH;
    const int e = i / KP, n = i - e * KP;
    const bool ok = i < E * KP && e < ne && n < NP;
    const float* qe = tq + ((ok ? e : 0) * NF * NP + (ok ? n : 0));
#pragma unroll
    for (int c = 0; c < NF; ++c) qv[t][c] = qe[c * NP];
  };
#pragma unroll
  for (int t = 0; t < NIT1; ++t) load_node(t);
  // FP32 at the highest degrees (register budget): the first items' raw
  // fields go straight into the operand region (p final, v converted to U_j
  // after the barrier by the same thread)
  constexpr bool RAW = PREC == 0 && N >= 7;
  if constexpr (RAW) {
#pragma unroll
    for (int t = 0; t < NIT1; ++t) {
      const int i = tid + t * TH;
      if (i >= E * KP) continue;
      const int e = i / KP, n = i - e * KP;
      const bool ok = e < ne && n < NP;
#pragma unroll
      for (int c = 0; c < NF; ++c) breg.put(c, n, e, ok ? qv[t][c] : 0.0f);
    }
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

  // ---- A2: neighbour traces; face records; volume operands p, U_j ---------
#pragma unroll
  for (int t = NIT1; t < NIT; ++t) load_node(t);
  // upwind alpha at the face slots from the own and neighbour traces
  // (rigid wall: mirror state p+ = p-, v.n+ = -v.n-; absorbing wall: zero
  // exterior state; Z+ = Z- on both)
  float alpha[FIT];
  constexpr int FCH = LATE_OWN ? (FIT + 1) / 2 : FIT;  // items per round (register budget)
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    if (LATE_OWN && t % FCH == 0) {
      if (t > 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = t; u < t + FCH && u < FIT; ++u) load_own(u);
    }
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
    const float pP = tr[0];
    const float vnP = -tr[NFP];  // the neighbour stored v.n with its own normal
    const float ZP = wall ? s_cf[ec * CB + 2] : s_cf[ec * CB + 4 + f];
    // absorbing wall (bit 3 of a wall's word): zero exterior state
    const float gw = (w & 8) ? 0.0f : 1.0f;
    const float pp = wall ? gw * pM[t] : pP;
    const float vp = wall ? -gw * vnM[t] : vnP;
    alpha[t] = ok ? 0.5f * (pp - pM[t]) - ZP * 0.5f * (vp - vnM[t]) : 0.0f;
  }
  // materialise alpha here: otherwise the compiler sinks its arithmetic to
  // the penalty phase and keeps the four trace values per item live across
  // the volume products
#pragma unroll
  for (int t = 0; t < FIT; ++t) __asm__ volatile("" : "+v"(alpha[t]));
  if (rec_e < ne) face_record<0>(s_g + 9 * rec_e, s_cf + CB * rec_e, rec_f, rec_word, s_face + tid * FW);
#pragma unroll
  for (int t = 0; t < NIT; ++t) {
    const int i = tid + t * TH;
    if (i >= E * KP) continue;
    const int e = i / KP, n = i - e * KP;
    float v0, v1, v2;
    if (RAW && t < NIT1) {  // raw fields staged before the barrier (p is in place)
      v0 = s_B[(1 * KP + n) * E + swz<E>(n, e)];
      v1 = s_B[(2 * KP + n) * E + swz<E>(n, e)];
      v2 = s_B[(3 * KP + n) * E + swz<E>(n, e)];
    } else {
      v0 = qv[t][1];
      v1 = qv[t][2];
      v2 = qv[t][3];
    }
    float p = 0.f, u0 = 0.f, u1 = 0.f, u2 = 0.f;
    if (e < ne && n < NP) {
      const float* G = s_g + 9 * e;
      p = qv[t][0];
      u0 = G[0] * v0 + G[3] * v1 + G[6] * v2;
      u1 = G[1] * v0 + G[4] * v1 + G[7] * v2;
      u2 = G[2] * v0 + G[5] * v1 + G[8] * v2;
    }
    if (!(RAW && t < NIT1)) breg.put(0, n, e, p);
    breg.put(1, n, e, u0);
    breg.put(2, n, e, u1);
    breg.put(3, n, e, u2);
  }
  __syncthreads();

  // ---- C1: volume products ---------------------------------------------------
  const int kq = lane >> 4;  // row quad of the accumulator / k group of the operands
  floatx4 T0[PPW], T1[PPW], T2[PPW], DV[PPW];
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
    const int p = p0 + wave + NW * q;
    T0[q] = T1[q] = T2[q] = DV[q] = floatx4{0, 0, 0, 0};
    if (p >= p1) continue;
    const int mb = p % MB, nb = p / MB;
    const int col = nb * 16 + (lane & 15);
    if constexpr (PREC == 0) {
      const float* Dp = a.Dpack + static_cast<int64_t>(mb) * (KP / 4) * 64 + lane;
      constexpr int JS = MB * (KP / 4) * 64;
      // Operator fragments stream from L2 through two register sets: the
      // loads of the next group of PD k-steps are issued before the products
      // of the current group (the scheduling barrier keeps them there), so
      // their latency overlaps PD k-steps of products.
      constexpr int NK = KP / 4, PD = NK < prefetch_fp32(N) ? NK : prefetch_fp32(N);
      using R = Ring<float, PD, 3>;
      auto load = [&](R& r, int g) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          const int kk = g * PD + i < NK ? g * PD + i : NK - 1;  // clamped; the extra reads are unused
          r.v[i][0] = Dp[kk * 64];
          r.v[i][1] = Dp[JS + kk * 64];
          r.v[i][2] = Dp[2 * JS + kk * 64];
        }
      };
      auto compute = [&](const R& r, int g, int cnt) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          if (i >= cnt) break;
          const int k = (g * PD + i) * 4 + kq;
          const int c = swz<E>(k, col);
          const float bp = s_B[(0 * KP + k) * E + c];
          const float b0 = s_B[(1 * KP + k) * E + c];
          const float b1 = s_B[(2 * KP + k) * E + c];
          const float b2 = s_B[(3 * KP + k) * E + c];
          T0[q] = mfma_f32(r.v[i][0], bp, T0[q]);
          T1[q] = mfma_f32(r.v[i][1], bp, T1[q]);
          T2[q] = mfma_f32(r.v[i][2], bp, T2[q]);
          DV[q] = mfma_f32(r.v[i][0], b0, DV[q]);
          DV[q] = mfma_f32(r.v[i][1], b1, DV[q]);
          DV[q] = mfma_f32(r.v[i][2], b2, DV[q]);
        }
      };
      pipelined<NK, PD, R>(load, compute);
    } else {
      const uint16_t* u = reinterpret_cast<const uint16_t*>(s_B);
      constexpr int LO = S::REGION;  // 16-bit units
      constexpr int JS = MB * (KP / 32) * 64;  // fragments between D_0, D_1, D_2
      const shortx8* Dh = reinterpret_cast<const shortx8*>(a.D16h) + static_cast<int64_t>(mb) * (KP / 32) * 64 + lane;
      const shortx8* Dl = reinterpret_cast<const shortx8*>(a.D16l) + static_cast<int64_t>(mb) * (KP / 32) * 64 + lane;
      // operator fragments through two register sets, as in the FP32 path
      constexpr int NK = KP / 32, PD = NK < kPrefetch16 ? NK : kPrefetch16;
      using R = Ring<Frag32, PD, 3>;
      auto load = [&](R& r, int g) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          const int kk = g * PD + i < NK ? g * PD + i : NK - 1;  // clamped; the extra reads are unused
#pragma unroll
          for (int j = 0; j < 3; ++j) r.v[i][j] = Frag32{Dh[j * JS + kk * 64], Dl[j * JS + kk * 64]};
        }
      };
      auto compute = [&](const R& r, int g, int cnt) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          if (i >= cnt) break;
          const int kk = g * PD + i;
          const int off = ((kk * 4 + kq) * E + col) * 8;
          Frag32 bp, b0, b1, b2;
          bp.hi = *reinterpret_cast<const shortx8*>(u + 0 * KP * E + off);
          bp.lo = *reinterpret_cast<const shortx8*>(u + LO + 0 * KP * E + off);
          b0.hi = *reinterpret_cast<const shortx8*>(u + 1 * KP * E + off);
          b0.lo = *reinterpret_cast<const shortx8*>(u + LO + 1 * KP * E + off);
          b1.hi = *reinterpret_cast<const shortx8*>(u + 2 * KP * E + off);
          b1.lo = *reinterpret_cast<const shortx8*>(u + LO + 2 * KP * E + off);
          b2.hi = *reinterpret_cast<const shortx8*>(u + 3 * KP * E + off);
          b2.lo = *reinterpret_cast<const shortx8*>(u + LO + 3 * KP * E + off);
          T0[q] = mfma_split<PREC>(r.v[i][0], bp, T0[q]);
          T1[q] = mfma_split<PREC>(r.v[i][1], bp, T1[q]);
          T2[q] = mfma_split<PREC>(r.v[i][2], bp, T2[q]);
          DV[q] = mfma_split<PREC>(r.v[i][0], b0, DV[q]);
          DV[q] = mfma_split<PREC>(r.v[i][1], b1, DV[q]);
          DV[q] = mfma_split<PREC>(r.v[i][2], b2, DV[q]);
        }
      };
      pipelined<NK, PD, R>(load, compute);
    }
  }
  __syncthreads();

  // ---- B2: penalty operands (the region is reused) -------------------------
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * TH;
    if (i >= E * KL) continue;
    const int e = i / KL, slot = i - e * KL;
    float fp = 0.f, fv = 0.f;
    const int f = slot / KF;
    if (e < ne && slot - f * KF < NFP) {
      const float* rec = s_face + (e * 4 + f) * FW;
      fp = rec[4] * alpha[t];
      fv = rec[5] * alpha[t];
    }
    lreg.put(0, slot, e, fp);
    lreg.put(1, slot, e, fv);
  }
  __syncthreads();

  // ---- C2: LIFT products and the epilogue, pair by pair ---------------------
  float* scr = s_scr + wave * SCR;
  const int nl = lane & 15, eg = lane >> 4;
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
    const int p = p0 + wave + NW * q;
    if (p >= p1) continue;
    const int mb = p % MB, nb = p / MB;
    const int col = nb * 16 + nl;
    // per-face LIFT of the two penalty scalars; k-steps never straddle a
    // face block (KF is a multiple of the instruction's K), and the fully
    // unrolled stream resolves each k-step's face at compile time
    floatx4 lp = {0, 0, 0, 0}, LV[4];  // p penalty summed over faces; v penalty per face
#pragma unroll
    for (int f = 0; f < 4; ++f) LV[f] = floatx4{0, 0, 0, 0};
    if constexpr (PREC == 0) {
      const float* Lp = a.Lpack + static_cast<int64_t>(mb) * (KL / 4) * 64 + lane;
      constexpr int NK = KL / 4, PD = NK < 2 * prefetch_fp32(N) ? NK : 2 * prefetch_fp32(N);
      using R = Ring<float, PD, 1>;
      auto load = [&](R& r, int g) {
#pragma unroll
        for (int i = 0; i < PD; ++i) r.v[i][0] = Lp[(g * PD + i < NK ? g * PD + i : NK - 1) * 64];
      };
      auto compute = [&](const R& r, int g, int cnt) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          if (i >= cnt) break;
          const int kk = g * PD + i, f = kk / (KF / 4);
          const int k = kk * 4 + kq;
          const int c = swz<E>(k, col);
          lp = mfma_f32(r.v[i][0], s_B[(0 * KL + k) * E + c], lp);
          LV[f] = mfma_f32(r.v[i][0], s_B[(1 * KL + k) * E + c], LV[f]);
        }
      };
      pipelined<NK, PD, R, true>(load, compute);
    } else {
      const uint16_t* u = reinterpret_cast<const uint16_t*>(s_B);
      constexpr int LO = S::REGION;  // 16-bit units
      const shortx8* Lh = reinterpret_cast<const shortx8*>(a.L16h) + static_cast<int64_t>(mb) * (KL / 32) * 64 + lane;
      const shortx8* Ll = reinterpret_cast<const shortx8*>(a.L16l) + static_cast<int64_t>(mb) * (KL / 32) * 64 + lane;
      constexpr int NK = KL / 32, PD = NK < 2 * kPrefetch16 ? NK : 2 * kPrefetch16;
      using R = Ring<Frag32, PD, 1>;
      auto load = [&](R& r, int g) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          const int kk = g * PD + i < NK ? g * PD + i : NK - 1;
          r.v[i][0] = Frag32{Lh[kk * 64], Ll[kk * 64]};
        }
      };
      auto compute = [&](const R& r, int g, int cnt) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
          if (i >= cnt) break;
          const int kk = g * PD + i, f = kk / (KF / 32);
          const int off = ((kk * 4 + kq) * E + col) * 8;
          Frag32 b;
          b.hi = *reinterpret_cast<const shortx8*>(u + 0 * KL * E + off);
          b.lo = *reinterpret_cast<const shortx8*>(u + LO + 0 * KL * E + off);
          lp = mfma_split<PREC>(r.v[i][0], b, lp);
          b.hi = *reinterpret_cast<const shortx8*>(u + 1 * KL * E + off);
          b.lo = *reinterpret_cast<const shortx8*>(u + LO + 1 * KL * E + off);
          LV[f] = mfma_split<PREC>(r.v[i][0], b, LV[f]);
        }
      };
      pipelined<NK, PD, R, true>(load, compute);
    }
    const int n = mb * 16 + nl;
    const int ncl = n < NP ? n : NP - 1;
    // right-hand sides in the accumulator layout: row 4*kq + r, column nl
    float rr[4][4];
    {
      const int ec = col < ne ? col : 0;
      const float* G = s_g + 9 * ec;
      const float rc2 = s_cf[ec * CB + 0], irho = s_cf[ec * CB + 1];
      const float* fr = s_face + ec * 4 * FW;  // the element's face normals
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float lv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
          lv[i] = fr[0 * FW + i] * LV[0][r] + fr[1 * FW + i] * LV[1][r] + fr[2 * FW + i] * LV[2][r] +
                  fr[3 * FW + i] * LV[3][r];
        rr[0][r] = -rc2 * DV[q][r] + lp[r];
        rr[1][r] = -irho * (G[0] * T0[q][r] + G[1] * T1[q][r] + G[2] * T2[q][r]) + lv[0];
        rr[2][r] = -irho * (G[3] * T0[q][r] + G[4] * T1[q][r] + G[5] * T2[q][r]) + lv[1];
        rr[3][r] = -irho * (G[6] * T0[q][r] + G[7] * T1[q][r] + G[8] * T2[q][r]) + lv[2];
      }
    }
    // transpose field by field through the wave's scratch:
    // lane -> (node mb*16 + nl, element nb*16 + eg + 4 it)
    float rt[4][4];  // [field][it]
#pragma unroll
    for (int c = 0; c < NF; ++c) {
#pragma unroll
      for (int r = 0; r < 4; ++r) scr[nl * 17 + 4 * kq + r] = rr[c][r];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int it = 0; it < 4; ++it) rt[c][it] = scr[(eg + 4 * it) * 17 + nl];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    // AB3 update: fields and history read in two halves (register budget),
    // each half's reads issued together at clamped addresses
    float qn[4][4];
    int nfs[3] = {-1, -1, -1};
    if (step) {
      // history read only where it is used
      const float* t1 = (a.c1 != 0.0f ? a.r1 : a.q_in) + e0 * NF * NP;
      const float* t2 = (a.c2 != 0.0f ? a.r2 : a.q_in) + e0 * NF * NP;
      const float w1 = a.c1 != 0.0f ? 1.0f : 0.0f, w2 = a.c2 != 0.0f ? 1.0f : 0.0f;
#pragma unroll
      for (int s = 0; s < 3; ++s) nfs[s] = a.nodeface[ncl * 3 + s];
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        float qo[4][2], h1[4][2], h2[4][2];
#pragma unroll
        for (int ih = 0; ih < 2; ++ih) {
          const int e = nb * 16 + eg + 4 * (2 * half + ih);
          const int off = (e < ne ? e : ne - 1) * NF * NP + ncl;
#pragma unroll
          for (int c = 0; c < NF; ++c) {
            qo[c][ih] = tq[off + c * NP];
            h1[c][ih] = t1[off + c * NP];
            h2[c][ih] = t2[off + c * NP];
          }
        }
#pragma unroll
        for (int ih = 0; ih < 2; ++ih)
#pragma unroll
          for (int c = 0; c < NF; ++c) {
            const int it = 2 * half + ih;
            qn[c][it] = qo[c][ih] + a.c0 * rt[c][it] + a.c1 * (w1 * h1[c][ih]) + a.c2 * (w2 * h2[c][ih]);
          }
      }
    }
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int e = nb * 16 + eg + 4 * it;
      if (e >= ne || n >= NP) continue;
      const int off = e * NF * NP + n;
#pragma unroll
      for (int c = 0; c < NF; ++c) (a.r_out + e0 * NF * NP)[off + c * NP] = rt[c][it];
      if (!step) continue;
#pragma unroll
      for (int c = 0; c < NF; ++c) (a.q_out + e0 * NF * NP)[off + c * NP] = qn[c][it];
      const float* fr = s_face + e * 4 * FW;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int fj = nfs[s];
        if (fj < 0) break;
        const int f = fj / NFP, j = fj - f * NFP;
        float* tr = a.qf_out + e0 * 4 * NT * NFP + ((e * 4 + f) * NT * NFP + j);
        tr[0] = qn[0][it];
        tr[NFP] = fr[f * FW + 0] * qn[1][it] + fr[f * FW + 1] * qn[2][it] + fr[f * FW + 2] * qn[3][it];
      }
    }
  }
}

template <int N, int CFG>
__global__ void __launch_bounds__((MShape<N, CFG>::THREADS), (acoustic_min_waves(N, cfg_prec(CFG))))
dg_step_mfma_acoustic(StepArgs a) {
  int p0, p1;
  const int64_t tile = split_tile(tile_of_block(a.xcd_remap), a.split_from, a.split_parts, MShape<N, CFG>::PAIRS, p0, p1);
  step_mfma_tile<N, CFG>(a, tile, p0, p1);
}

template <int N, int CFG>
__global__ void __launch_bounds__((MShape<N, CFG>::THREADS), (acoustic_min_waves(N, cfg_prec(CFG))))
dg_step_mfma_acoustic_batch(const StepArgs* __restrict__ args, const int2* __restrict__ work, int phase) {
  const int2 w = work[blockIdx.x];
  if (w.x < 0) return;  // padding entry of the work list
  const StepArgs a = args[w.x * kBatchPhases + phase];
  step_mfma_tile<N, CFG>(a, w.y, 0, MShape<N, CFG>::PAIRS);
}

template <int N, int CFG>
hipError_t mfma_batch_impl(const StepArgs* args, const int2* work, int64_t ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_mfma_acoustic_batch<N, CFG>), dim3(static_cast<unsigned>(ntiles)), dim3(MShape<N, CFG>::THREADS), 0,
                     s, args, work, phase);
  return hipGetLastError();
}

// A short last round of tiles is split over up to ceil(pairs / 4)
// workgroups per tile, so that each part runs at most one pair's products
// per SIMD (tiles in launch order only).
template <int N, int CFG>
hipError_t mfma_impl(const StepArgs& a, hipStream_t s) {
  using S = MShape<N, CFG>;
  int64_t tiles = (a.K - a.e_begin + S::E - 1) / S::E;
  if (a.xcd_remap) tiles = ((tiles + 7) / 8) * 8;
  StepArgs b = a;
  TailSplit plan{tiles, tiles, 1};
  if (a.tail_split && !a.xcd_remap) {
    static std::atomic<int> slots_cache[16];
    const int slots =
        resident_workgroups(reinterpret_cast<const void*>(&dg_step_mfma_acoustic<N, CFG>), S::THREADS, slots_cache);
    plan = plan_tail_split(tiles, slots, (S::PAIRS + 3) / 4);
  }
  b.split_from = plan.from;
  b.split_parts = plan.parts;
  if (plan.grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_mfma_acoustic<N, CFG>), dim3(static_cast<unsigned>(plan.grid)), dim3(S::THREADS), 0, s, b);
  return hipGetLastError();
}

template <int N, int CFG>
MfmaPacking packing_of() {
  using S = MShape<N, CFG>;
  return MfmaPacking{S::MB, S::KP, S::KL, S::KS, S::E, S::KF};
}

}  // namespace

int mfma_precision(int variant) {
  return (variant == kVariantMfma || variant == kVariantMfmaWide)
             ? 0
             : (variant == kVariantMfmaBf16 ? 1 : (variant == kVariantMfmaF16 ? 2 : -1));
}

// tile configuration of an acoustic MFMA variant (see MShape)
static int mfma_config(int variant) { return variant == kVariantMfmaWide ? 4 : mfma_precision(variant); }

#define DGW_MFMA_DISPATCH(CALL)                                                          \
  switch (mfma_config(variant)) {                                                        \
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
    case 4:                                                                              \
      switch (N) {                                                                       \
        case 1: return CALL(1, 4); case 2: return CALL(2, 4); case 3: return CALL(3, 4); \
        case 4: return CALL(4, 4); case 5: return CALL(5, 4); case 6: return CALL(6, 4); \
        case 7: return CALL(7, 4); case 8: return CALL(8, 4);                            \
      }                                                                                  \
      break;                                                                             \
  }

MfmaPacking mfma_packing(int physics, int N, int variant) {
  if (physics != 0) return mfma_elastic_packing(N, variant);
#define CALL(n, p) packing_of<n, p>()
  DGW_MFMA_DISPATCH(CALL)
#undef CALL
  return MfmaPacking{};
}

hipError_t launch_step_mfma(int physics, int N, int variant, const StepArgs& a, hipStream_t s) {
  if (physics != 0) return hipErrorInvalidValue;
#define CALL(n, p) mfma_impl<n, p>(a, s)
  DGW_MFMA_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_step_batch_mfma(int physics, int N, int variant, const StepArgs* args, const int2* work,
                                  int64_t ntiles, int phase, hipStream_t s) {
  if (physics != 0) return hipErrorInvalidValue;
#define CALL(n, p) mfma_batch_impl<n, p>(args, work, ntiles, phase, s)
  DGW_MFMA_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

#undef DGW_MFMA_DISPATCH

}  // namespace dgw
