// MFMA variant of the fused DG step (acoustic), FP32 matrix cores on gfx950.
//
// The volume and LIFT products of eqs. (5)-(6) become small GEMMs with the
// element as the column index: for a tile of E = 16*NBLK elements
//   T_j   = D_j p                       (3 products [Np x Np][Np x E])
//   div   = sum_j D_j U_j,  U_j = sum_i g_ij v_i      (same D_j fragments)
//   Lp    = L Pp            (merged LIFT of the pressure penalty, all faces)
//   Lv_f  = L_f Pv_f        (LIFT of the scalar velocity penalty, per face;
//                            the face normal is applied afterwards)
// on v_mfma_f32_16x16x4_f32.  A operands (D_j, L) are packed on the host in
// 16x4 fragment order so that every A load is one coalesced 256-byte access;
// B operands come from LDS laid out [field][node][element] with the element
// fastest.  Each (16-row node block, 16-element column block) pair of the
// tile is owned by one wave, whose accumulators hold all four fields of its
// nodes: the epilogue combines them with the element's geometry and
// coefficients, applies the AB3 update and writes q, r and the own traces,
// exactly as the node-per-thread variant does.
#include <hip/hip_runtime.h>

#include "dg_device.hpp"
#include "kernels.hpp"

namespace dgw {

namespace {

using namespace dev;

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int N>
struct MfmaShape {
  static constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP;
  static constexpr int MB = (NP + 15) / 16;       // 16-row node blocks
  static constexpr int KP = (NP + 3) / 4 * 4;     // K padding of the volume products
  static constexpr int NFPP = (NFP + 3) / 4 * 4;  // each face's block padded to whole k-steps
  static constexpr int KL = 4 * NFPP;             // K of the LIFT product
  // 16-element column blocks per workgroup: enough (node block, column block)
  // pairs for four waves while the LDS tile stays small.
  static constexpr int NBLK = (N <= 4) ? 4 : (N == 6 ? 2 : 1);
  static constexpr int E = 16 * NBLK;
  static constexpr int ES = E;  // LDS row stride of the B operands
};

// Column swizzle of the [row][element] B-operand arrays (row stride E): a
// bijection on [0, E) per row chosen so that the 16x4 fragment reads (lanes
// split over four consecutive rows) and the staging writes (consecutive rows,
// one element) both touch 32 distinct LDS banks.
template <int E>
__device__ __forceinline__ int swz(int m, int e) {
  if constexpr (E == 16)
    return e ^ ((m >> 1) & 15);
  else
    return (((e >> 4) ^ (m & 1)) << 4) + ((e & 15) ^ ((m >> 1) & 15));
}

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int N>
__device__ __forceinline__ void step_mfma_tile(const StepArgs& a, int64_t tile) {
  using S = MfmaShape<N>;
  constexpr int NP = S::NP, NFP = S::NFP, NFN = 4 * NFP;
  constexpr int MB = S::MB, KP = S::KP, NFPP = S::NFPP, KL = S::KL;
  constexpr int NBLK = S::NBLK, E = S::E, ES = S::ES;
  constexpr int NF = 4, NT = 2, CB = 8;
  constexpr int FIT = (E * NFN + kThreads - 1) / kThreads;

  __shared__ float s_q[NF * KP * ES];  // [c][m][e]
  __shared__ float s_fl[2 * KL * ES];  // [scalar][f*NFPP + j][e]
  __shared__ float s_g[E * 9];
  __shared__ float s_cf[E * CB];
  constexpr int FW = FaceRec<0>::W;
  __shared__ float s_face[E * 4 * FW];

  const int64_t e0 = tile * E;
  if (e0 >= a.K) return;  // whole workgroup exits together
  const int ne = static_cast<int>((a.K - e0) < E ? (a.K - e0) : E);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const bool step = (a.mode == kStepMode);

  // ---- phase A: neighbour traces, zero padding, tile staging --------------
  int word[FIT];
  float nbt[FIT][NT];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * kThreads;
    word[t] = 7;
    nbt[t][0] = nbt[t][1] = 0.0f;
    if (i < ne * NFN) {
      const int e = i / NFN, fn = i - e * NFN;
      const int f = fn / NFP, j = fn - f * NFP;
      const int w = a.conn[(e0 + e) * 4 + f];
      word[t] = w;
      if ((w & 7) != 7) {
        const int64_t kn = static_cast<int64_t>(w >> 5);
        const int fnb = (w >> 3) & 3;
        const int jn = a.perm[(w & 7) * NFP + j];
        const float* tr = a.qf_in + (kn * 4 + fnb) * NT * NFP + jn;
        nbt[t][0] = tr[0];
        nbt[t][1] = tr[NFP];
      }
    }
  }
  // padded rows (m >= NP) and padded columns (e >= ne) of the B operands are 0
  for (int i = tid; i < NF * KP * ES; i += kThreads) {
    const int row = i / ES, m = row % KP, e = i % ES;
    if (m >= NP || e >= ne) s_q[row * ES + swz<E>(m, e)] = 0.0f;
  }
  for (int i = tid; i < 2 * KL * ES; i += kThreads) s_fl[i] = 0.0f;
  {
    const float* src = a.q_in + e0 * NF * NP;
    for (int i = tid; i < ne * NF * NP; i += kThreads) {
      const int e = i / (NF * NP), rem = i - e * (NF * NP);
      const int c = rem / NP, m = rem - c * NP;
      s_q[(c * KP + m) * ES + swz<E>(m, e)] = src[i];
    }
    for (int i = tid; i < ne * 9; i += kThreads) s_g[i] = a.geo[e0 * 9 + i];
    for (int i = tid; i < ne * CB; i += kThreads) s_cf[i] = a.cf[e0 * CB + i];
    for (int i = tid; i < ne * 4; i += kThreads) {
      const int e = i >> 2, f = i & 3;
      face_record<0>(a.geo + (e0 + e) * 9, a.cf + (e0 + e) * CB, f, a.conn[(e0 + e) * 4 + f], s_face + i * FW);
    }
  }
  __syncthreads();

  // ---- phase B: upwind penalties times Fscale at the real face nodes -------
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * kThreads;
    if (i >= ne * NFN) continue;
    const int e = i / NFN, fn = i - e * NFN;
    const int f = fn / NFP, j = fn - f * NFP;
    const float* rec = s_face + (e * 4 + f) * FW;
    const float nrm[3] = {rec[0], rec[1], rec[2]};
    const int vn = a.fmask[f * NFP + j];
    const bool wall = (word[t] & 7) == 7;
    const int cv = swz<E>(vn, e);
    const float pM = s_q[(0 * KP + vn) * ES + cv];
    const float vnM = nrm[0] * s_q[(1 * KP + vn) * ES + cv] + nrm[1] * s_q[(2 * KP + vn) * ES + cv] +
                      nrm[2] * s_q[(3 * KP + vn) * ES + cv];
    // rigid wall: mirror state p+ = p-, v.n+ = -v.n-
    const float pP = wall ? pM : nbt[t][0];
    const float vnP = wall ? -vnM : -nbt[t][1];  // neighbour stored v.n with its own normal
    const float alpha = 0.5f * (pP - pM) - rec[3] * 0.5f * (vnP - vnM);
    const int slot = f * NFPP + j;
    const int cs = swz<E>(slot, e);
    s_fl[(0 * KL + slot) * ES + cs] = rec[4] * alpha;
    s_fl[(1 * KL + slot) * ES + cs] = rec[5] * alpha;
  }
  __syncthreads();

  // ---- phase C: one (node block, column block) pair per wave --------------
  const int kq = lane >> 4;  // k offset of this lane in a 16x4 fragment / row quad of C
  for (int p = wave; p < MB * NBLK; p += 4) {
    const int mb = p % MB, nb = p / MB;
    const int el = nb * 16 + (lane & 15);  // this lane's element (column)
    const bool live = el < ne;
    float G[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) G[t] = live ? s_g[el * 9 + t] : 0.0f;
    // AB3 history of this lane's four nodes, issued before the products
    float h1[4][NF], h2[4][NF];
    const bool use1 = step && (a.c1 != 0.0f), use2 = step && (a.c2 != 0.0f);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = mb * 16 + 4 * kq + r;
      const bool ok = live && n < NP;
      const int64_t base = (e0 + el) * NF * NP + n;
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        h1[r][c] = (ok && use1) ? a.r1[base + c * NP] : 0.0f;
        h2[r][c] = (ok && use2) ? a.r2[base + c * NP] : 0.0f;
      }
    }
    floatx4 T0 = {0, 0, 0, 0}, T1 = T0, T2 = T0, d0 = T0, d1 = T0, d2 = T0;
    const float* Dp = a.Dpack + static_cast<int64_t>(mb) * (KP / 4) * 64 + lane;
    constexpr int JS = MB * (KP / 4) * 64;  // stride between D_0, D_1, D_2
    // fully unrolled so that the A fragments of all k-steps are requested
    // before the first product needs them
#pragma unroll
    for (int kk = 0; kk < KP / 4; ++kk) {
      const int m = kk * 4 + kq;
      const int cm = swz<E>(m, el);
      const float bp = s_q[(0 * KP + m) * ES + cm];
      const float v0 = s_q[(1 * KP + m) * ES + cm];
      const float v1 = s_q[(2 * KP + m) * ES + cm];
      const float v2 = s_q[(3 * KP + m) * ES + cm];
      const float u0 = G[0] * v0 + G[3] * v1 + G[6] * v2;
      const float u1 = G[1] * v0 + G[4] * v1 + G[7] * v2;
      const float u2 = G[2] * v0 + G[5] * v1 + G[8] * v2;
      const float a0 = Dp[kk * 64], a1 = Dp[JS + kk * 64], a2 = Dp[2 * JS + kk * 64];
      T0 = mfma4(a0, bp, T0);
      d0 = mfma4(a0, u0, d0);
      T1 = mfma4(a1, bp, T1);
      d1 = mfma4(a1, u1, d1);
      T2 = mfma4(a2, bp, T2);
      d2 = mfma4(a2, u2, d2);
    }
    floatx4 lp = {0, 0, 0, 0}, lv0 = lp, lv1 = lp, lv2 = lp, lv3 = lp;
    const float* Lp = a.Lpack + static_cast<int64_t>(mb) * (KL / 4) * 64 + lane;
#define DGW_LIFT_FACE(F, ACC)                                                   \
  _Pragma("unroll") for (int kf = 0; kf < NFPP / 4; ++kf) {                     \
    const int kl = (F) * (NFPP / 4) + kf;                                       \
    const int slot = kl * 4 + kq;                                               \
    const int csl = swz<E>(slot, el);                                           \
    const float bfp = s_fl[(0 * KL + slot) * ES + csl];                         \
    const float bfv = s_fl[(1 * KL + slot) * ES + csl];                         \
    const float al = Lp[kl * 64];                                               \
    lp = mfma4(al, bfp, lp);                                                    \
    ACC = mfma4(al, bfv, ACC);                                                  \
  }
    DGW_LIFT_FACE(0, lv0)
    DGW_LIFT_FACE(1, lv1)
    DGW_LIFT_FACE(2, lv2)
    DGW_LIFT_FACE(3, lv3)
#undef DGW_LIFT_FACE
    if (!live) continue;
    const float* cf = s_cf + el * CB;
    const float rc2 = cf[0], irho = cf[1];
    const float* fr = s_face + el * 4 * FW;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = mb * 16 + 4 * kq + r;
      if (n >= NP) continue;
      float rr[NF];
      rr[0] = -rc2 * (d0[r] + d1[r] + d2[r]) + lp[r];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
        rr[1 + ii] = -irho * (G[3 * ii + 0] * T0[r] + G[3 * ii + 1] * T1[r] + G[3 * ii + 2] * T2[r]) +
                     (fr[0 * FW + ii] * lv0[r] + fr[1 * FW + ii] * lv1[r] + fr[2 * FW + ii] * lv2[r] +
                      fr[3 * FW + ii] * lv3[r]);
      const int64_t base = (e0 + el) * NF * NP + n;
      if (!step) {
#pragma unroll
        for (int c = 0; c < NF; ++c) a.r_out[base + c * NP] = rr[c];
        continue;
      }
      float qn[NF];
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        qn[c] = s_q[(c * KP + n) * ES + swz<E>(n, el)] + a.c0 * rr[c] + a.c1 * h1[r][c] + a.c2 * h2[r][c];
        a.q_out[base + c * NP] = qn[c];
        a.r_out[base + c * NP] = rr[c];
      }
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int fj = a.nodeface[n * 3 + s];
        if (fj < 0) break;
        const int f = fj / NFP, j = fj - f * NFP;
        float* tr = a.qf_out + ((e0 + el) * 4 + f) * NT * NFP + j;
        tr[0] = qn[0];
        tr[NFP] = fr[f * FW + 0] * qn[1] + fr[f * FW + 1] * qn[2] + fr[f * FW + 2] * qn[3];
      }
    }
  }
}

template <int N>
__global__ void __launch_bounds__(kThreads)
dg_step_mfma_acoustic(StepArgs a) {
  step_mfma_tile<N>(a, tile_of_block(a.xcd_remap));
}

template <int N>
__global__ void __launch_bounds__(kThreads)
dg_step_mfma_acoustic_batch(const StepArgs* __restrict__ args, const int2* __restrict__ work, int phase) {
  const int2 w = work[blockIdx.x];
  if (w.x < 0) return;  // padding entry of the work list
  const StepArgs a = args[w.x * kBatchPhases + phase];
  step_mfma_tile<N>(a, w.y);
}

template <int N>
hipError_t mfma_batch_impl(const StepArgs* args, const int2* work, int64_t ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_mfma_acoustic_batch<N>), dim3(static_cast<unsigned>(ntiles)), dim3(kThreads), 0, s,
                     args, work, phase);
  return hipGetLastError();
}

template <int N>
hipError_t mfma_impl(const StepArgs& a, hipStream_t s) {
  constexpr int E = MfmaShape<N>::E;
  int64_t tiles = (a.K + E - 1) / E;
  if (a.xcd_remap) tiles = ((tiles + 7) / 8) * 8;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_mfma_acoustic<N>), dim3(static_cast<unsigned>(tiles)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

int mfma_tile_elements(int N) {
  switch (N) {
    case 1: return MfmaShape<1>::E; case 2: return MfmaShape<2>::E; case 3: return MfmaShape<3>::E;
    case 4: return MfmaShape<4>::E; case 5: return MfmaShape<5>::E; case 6: return MfmaShape<6>::E;
    case 7: return MfmaShape<7>::E; case 8: return MfmaShape<8>::E;
  }
  return -1;
}

hipError_t launch_step_batch_mfma(int physics, int N, const StepArgs* args, const int2* work, int64_t ntiles,
                                  int phase, hipStream_t s) {
  if (physics != 0) return hipErrorInvalidValue;
  switch (N) {
    case 1: return mfma_batch_impl<1>(args, work, ntiles, phase, s);
    case 2: return mfma_batch_impl<2>(args, work, ntiles, phase, s);
    case 3: return mfma_batch_impl<3>(args, work, ntiles, phase, s);
    case 4: return mfma_batch_impl<4>(args, work, ntiles, phase, s);
    case 5: return mfma_batch_impl<5>(args, work, ntiles, phase, s);
    case 6: return mfma_batch_impl<6>(args, work, ntiles, phase, s);
    case 7: return mfma_batch_impl<7>(args, work, ntiles, phase, s);
    case 8: return mfma_batch_impl<8>(args, work, ntiles, phase, s);
  }
  return hipErrorInvalidValue;
}

int mfma_mblocks(int N) { return (((N + 1) * (N + 2) * (N + 3) / 6) + 15) / 16; }
int mfma_kpad(int N) { return (((N + 1) * (N + 2) * (N + 3) / 6) + 3) / 4 * 4; }
int mfma_face_pad(int N) { return (((N + 1) * (N + 2) / 2) + 3) / 4 * 4; }

hipError_t launch_step_mfma(int physics, int N, const StepArgs& a, hipStream_t s) {
  if (physics != 0) return hipErrorInvalidValue;
  switch (N) {
    case 1: return mfma_impl<1>(a, s);
    case 2: return mfma_impl<2>(a, s);
    case 3: return mfma_impl<3>(a, s);
    case 4: return mfma_impl<4>(a, s);
    case 5: return mfma_impl<5>(a, s);
    case 6: return mfma_impl<6>(a, s);
    case 7: return mfma_impl<7>(a, s);
    case 8: return mfma_impl<8>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dgw
