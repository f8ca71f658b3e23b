// HIP kernels of the nodal DG wave step for gfx950.
//
// One fused kernel per time step (Sec. 3.2's volume, surface and update
// kernels merged): a workgroup owns a tile of KT consecutive elements and
//   A  issues every global load at once: the neighbour traces of its
//      face-node items (gathered through the packed connectivity word and the
//      face-node permutation), the AB3 history of its node items, and the
//      tile's fields, inverse Jacobians and coefficients (into LDS);
//   B  forms the per-node geometric combinations of the volume term
//      (acoustic U_j = sum_i g_ij v_i, eq. (5); elastic S_il = sum_j g_jl s_ij)
//      and, at every face node, the upwind penalty of Sec. 2.1 times Fscale;
//   C  node per thread: the six (acoustic) or eighteen (elastic) Np x Np
//      matrix-vector products with D_j, the merged LIFT product, the
//      coefficient combinations of eqs. (5)-(6) / the elastic right-hand
//      side, and the AB3 update of eq. (4); writes q^{m+1}, r^m and the own
//      traces (acoustic p and n.v, elastic v and s n) of the faces the node
//      lies on into the other trace buffer.
// Traces are double-buffered, so no element reads a trace written in the
// same launch; every element's fields are read and written only by its own
// workgroup.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <type_traits>

#include "dg_device.hpp"
#include "kernels.hpp"

// Partial sums of the allocation-free energy entry point.  Each device that
// loads the library holds its own copy until the process ends.  In host code
// this name is only a stand-in for the symbol: the device address comes from
// hipGetSymbolAddress (static_energy_partials below) and is what kernels get.
static __device__ __align__(256) double scratch[dgw::kStaticEnergyPartials];

namespace dgw {

namespace {

using namespace dev;

// Elements per workgroup, chosen so that KT*NP fills ~256 threads; the
// elastic fields at N = 1 take 32 elements (measured: at N = 2 the full 25
// is 5% faster than 20 and 14% faster than 16; at N = 3, 4 fewer elements
// than 256 / Np measured slower, and so did other counts for the acoustic
// fields at N = 1..3).
template <int N, int PHYS>
struct Tile {
  static constexpr int NP = Deg<N>::NP;
  static constexpr int raw = 256 / NP;
  static constexpr int KT = (N == 8 && PHYS == 0) ? 3 : (PHYS != 0 && N == 1 ? 32 : (raw < 1 ? 1 : raw));
};

// Number of lifted scalars per face node: acoustic (Fscale*penalty for p,
// scalar velocity penalty along n), elastic (k_p a_p, k_s a_s, vector a_s),
// anisotropic (the velocity correction vector, and the vector w whose strain
// n (x) w the stiffness takes), each times Fscale.  The normal and the
// per-face / per-element constants are applied after the lift, so the merged
// LIFT product runs on 2 / 5 / 6 columns per element instead of 4 / 9 / 9.
template <int PHYS>
struct LiftCols;
template <>
struct LiftCols<0> {
  static constexpr int NL = 2;
};
template <>
struct LiftCols<1> {
  static constexpr int NL = 5;
};
template <>
struct LiftCols<2> {
  static constexpr int NL = 6;
};

template <int N, int PHYS>
__device__ __forceinline__ void step_valu_tile(const StepArgs& a, int64_t tile) {
  constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP, NFN = 4 * NFP;
  constexpr int NF = Phys<PHYS>::NF, NT = Phys<PHYS>::NT, NAUX = Phys<PHYS>::NAUX;
  constexpr int CB = Phys<PHYS>::CB;
  constexpr int NL = LiftCols<PHYS>::NL;
  constexpr int KT = Tile<N, PHYS>::KT;
  constexpr int NIT = (KT * NP + kThreads - 1) / kThreads;   // node items per thread
  constexpr int FIT = (KT * NFN + kThreads - 1) / kThreads;  // face-node items per thread

  __shared__ float s_q[KT * NF * NP];
  __shared__ float s_aux[KT * NAUX * NP];
  __shared__ float s_lift[KT * NL * NFN];
  __shared__ float s_g[KT * 9];
  __shared__ float s_cf[KT * CB];
  constexpr int FW = FaceRec<PHYS>::W;
  __shared__ float s_face[KT * 4 * FW];
  // Up to N = 4 the operators (3 Np^2 + 4 Nfp Np floats, at most 23 KB) are
  // staged in LDS with the tile, so that the node loops read them at LDS
  // latency instead of waiting on the cache for every k.
  constexpr bool OPS_LDS = N <= 4;
  constexpr int NDT = 3 * NP * NP, NLT = NFN * NP;
  __shared__ float s_ops[OPS_LDS ? NDT + NLT : 1];

  const int64_t e0 = a.e_begin + tile * KT;
  if (e0 >= a.K) return;  // whole workgroup exits together
  const int ne = static_cast<int>((a.K - e0) < KT ? (a.K - e0) : KT);
  const int tid = threadIdx.x;
  const bool step = (a.mode == kStepMode);

  // ---- phase A: issue every global load before the first barrier ----------
  // Loads are unconditional at clamped (in-range) addresses and unused values
  // are dropped by selects, so that no load waits behind a branch or behind
  // another item's load.  Two dependent rounds: (1) everything indexed by
  // the tile alone, then, once the connectivity words are in and the face-node
  // permutation is formed in registers (2), (3) the neighbour traces.
  constexpr int QV = (KT * NF * NP + 4 * kThreads - 1) / (4 * kThreads);  // float4 per thread
  constexpr int GIT = (KT * 9 + kThreads - 1) / kThreads;
  constexpr int CIT = (KT * CB + kThreads - 1) / kThreads;
  static_assert(KT * 4 <= kThreads, "one face record per thread");
  // (1) connectivity words of the face-node items
  int word[FIT];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * kThreads;
    const bool ok = i < ne * NFN;
    const int e = ok ? i / NFN : 0, f = ok ? (i - e * NFN) / NFP : 0;
    word[t] = a.conn[(e0 + e) * 4 + f];
  }
  // (1) AB3 history of this thread's node items (read only where it is used)
  float h1[NIT][NF], h2[NIT][NF];
  {
    const bool use1 = step && (a.c1 != 0.0f), use2 = step && (a.c2 != 0.0f);
    const float* p1 = use1 ? a.r1 : a.q_in;
    const float* p2 = use2 ? a.r2 : a.q_in;
#pragma unroll
    for (int t = 0; t < NIT; ++t) {
      const int i = tid + t * kThreads;
      const int ic = i < ne * NP ? i : 0;
      const int e = ic / NP, n = ic - e * NP;
      const int64_t base = (e0 + e) * NF * NP + n;
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        const float x1 = p1[base + c * NP], x2 = p2[base + c * NP];
        h1[t][c] = use1 ? x1 : 0.0f;
        h2[t][c] = use2 ? x2 : 0.0f;
      }
    }
  }
  // (1) the tile's fields, inverse Jacobians, coefficients and face-record words
  const int cnt = ne * NF * NP;
  const bool vec4 = ((e0 * NF * NP) & 3) == 0;
  const int nfull = vec4 ? cnt >> 2 : 0;  // whole float4 of the aligned copy
  float4 qv[QV];
  float qtail;
  {
    const float* src = a.q_in + e0 * NF * NP;
    // the aligned copy's last cnt % 4 values, one per thread
    qtail = src[4 * nfull + tid < cnt ? 4 * nfull + tid : 0];
#pragma unroll
    for (int t = 0; t < QV; ++t) {
      const int i4 = tid + t * kThreads;
      if (vec4) {
        qv[t] = reinterpret_cast<const float4*>(src)[i4 < nfull ? i4 : 0];
      } else {
        float x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ii = 4 * i4 + u;
          x[u] = src[ii < cnt ? ii : 0];
        }
        qv[t] = make_float4(x[0], x[1], x[2], x[3]);
      }
    }
  }
  float gv[GIT], cv[CIT];
#pragma unroll
  for (int t = 0; t < GIT; ++t) {
    const int i = tid + t * kThreads;
    gv[t] = a.geo[e0 * 9 + (i < ne * 9 ? i : 0)];
  }
#pragma unroll
  for (int t = 0; t < CIT; ++t) {
    const int i = tid + t * kThreads;
    cv[t] = a.cf[e0 * CB + (i < ne * CB ? i : 0)];
  }
  const int rec_e = tid >> 2, rec_f = tid & 3;
  const int rec_word = a.conn[(e0 + (rec_e < ne ? rec_e : 0)) * 4 + rec_f];
  constexpr int OIT = OPS_LDS ? (NDT + NLT + kThreads - 1) / kThreads : 0;
  float ov[OIT > 0 ? OIT : 1];
#pragma unroll
  for (int t = 0; t < OIT; ++t) {
    const int i = tid + t * kThreads;
    ov[t] = i < NDT ? a.DT[i] : a.LT[i < NDT + NLT ? i - NDT : 0];
  }
  // volume node of each face-node item; face slots of each node item
  int vnode[FIT], nfs[NIT][3];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * kThreads;
    const bool ok = i < ne * NFN;
    const int e = ok ? i / NFN : 0, fn = ok ? i - e * NFN : 0;
    vnode[t] = a.fmask[fn];
  }
#pragma unroll
  for (int t = 0; t < NIT; ++t) {
    const int i = tid + t * kThreads;
    const int ic = i < ne * NP ? i : 0;
    const int n = ic - (ic / NP) * NP;
#pragma unroll
    for (int s = 0; s < 3; ++s) nfs[t][s] = a.nodeface[n * 3 + s];
  }
  // (2) permuted face node on the neighbour's side (arithmetic, no load)
  int jn[FIT];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * kThreads;
    const bool ok = i < ne * NFN;
    const int e = ok ? i / NFN : 0, fn = ok ? i - e * NFN : 0;
    const int j = fn - (fn / NFP) * NFP;
    const int o = (word[t] & 7) == 7 ? 0 : (word[t] & 7);
    jn[t] = face_perm_node(N, o, j);
  }
  // (3) neighbour traces (a wall reads its own, in range and unused)
  float nbt[FIT][NT];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * kThreads;
    const bool ok = i < ne * NFN;
    const int e = ok ? i / NFN : 0, fn = ok ? i - e * NFN : 0;
    const int f = fn / NFP, j = fn - f * NFP;
    const int w = word[t];
    const bool wall = (w & 7) == 7;
    const int64_t kn = wall ? e0 + e : static_cast<int64_t>(w >> 5);
    const int fnb = wall ? f : (w >> 3) & 3;
    const float* tr = a.qf_in + (kn * 4 + fnb) * NT * NFP + (wall ? j : jn[t]);
#pragma unroll
    for (int c = 0; c < NT; ++c) nbt[t][c] = tr[c * NFP];
  }
  // stage the tile into LDS
#pragma unroll
  for (int t = 0; t < QV; ++t) {
    const int i4 = tid + t * kThreads;
    const float x[4] = {qv[t].x, qv[t].y, qv[t].z, qv[t].w};
    const int lim = vec4 ? 4 * nfull : cnt;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (4 * i4 + u < lim) s_q[4 * i4 + u] = x[u];
  }
  if (vec4 && 4 * nfull + tid < cnt) s_q[4 * nfull + tid] = qtail;
#pragma unroll
  for (int t = 0; t < OIT; ++t) {
    const int i = tid + t * kThreads;
    if (i < NDT + NLT) s_ops[i] = ov[t];
  }
#pragma unroll
  for (int t = 0; t < GIT; ++t) {
    const int i = tid + t * kThreads;
    if (i < ne * 9) s_g[i] = gv[t];
  }
#pragma unroll
  for (int t = 0; t < CIT; ++t) {
    const int i = tid + t * kThreads;
    if (i < ne * CB) s_cf[i] = cv[t];
  }
  __syncthreads();
  // per-face constants, once per face
  if (rec_e < ne) face_record<PHYS>(s_g + 9 * rec_e, s_cf + CB * rec_e, rec_f, rec_word, s_face + tid * FW);

  // ---- phase B: volume combinations and upwind penalties -----------------
  for (int i = tid; i < ne * NP; i += kThreads) {
    const int e = i / NP, n = i - e * NP;
    const float* G = s_g + 9 * e;
    const float* qe = s_q + e * NF * NP;
    float* ax = s_aux + e * NAUX * NP;
    if constexpr (PHYS == 0) {
      const float v0 = qe[1 * NP + n], v1 = qe[2 * NP + n], v2 = qe[3 * NP + n];
#pragma unroll
      for (int j = 0; j < 3; ++j) ax[j * NP + n] = G[0 * 3 + j] * v0 + G[1 * 3 + j] * v1 + G[2 * 3 + j] * v2;
    } else {
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        const float si0 = qe[(3 + voigt(ii, 0)) * NP + n];
        const float si1 = qe[(3 + voigt(ii, 1)) * NP + n];
        const float si2 = qe[(3 + voigt(ii, 2)) * NP + n];
#pragma unroll
        for (int l = 0; l < 3; ++l)
          ax[(ii * 3 + l) * NP + n] = G[0 * 3 + l] * si0 + G[1 * 3 + l] * si1 + G[2 * 3 + l] * si2;
      }
    }
  }
  __syncthreads();  // face records
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = tid + t * kThreads;
    if (i >= ne * NFN) continue;
    const int e = i / NFN, fn = i - e * NFN;
    const int f = fn / NFP;
    const float* rec = s_face + (e * 4 + f) * FW;
    const float nrm[3] = {rec[0], rec[1], rec[2]};
    const int vn = vnode[t];
    const float* qe = s_q + e * NF * NP;
    const bool wall = (word[t] & 7) == 7;
    // reflecting wall: mirror ghost state (gw = 1); absorbing wall (bit 3 of
    // a wall's word): zero exterior state (gw = 0)
    const float gw = (word[t] & 8) ? 0.0f : 1.0f;
    float* lf = s_lift + e * NL * NFN + fn;
    if constexpr (PHYS == 0) {
      const float pM = qe[vn];
      const float vnM = nrm[0] * qe[NP + vn] + nrm[1] * qe[2 * NP + vn] + nrm[2] * qe[3 * NP + vn];
      // rigid wall: mirror state p+ = p-, v.n+ = -v.n-
      const float pP = wall ? gw * pM : nbt[t][0];
      const float vnP = wall ? -gw * vnM : -nbt[t][1];  // neighbour stored v.n with its own normal
      const float alpha = 0.5f * (pP - pM) - rec[3] * 0.5f * (vnP - vnM);
      lf[0] = rec[4] * alpha;    // lifted into r^p
      lf[NFN] = rec[5] * alpha;  // lifted, then times n, into r^v
    } else {
      float vM[3], tM[3], vP[3], tP[3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) vM[ii] = qe[ii * NP + vn];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
        tM[ii] = qe[(3 + voigt(ii, 0)) * NP + vn] * nrm[0] + qe[(3 + voigt(ii, 1)) * NP + vn] * nrm[1] +
                 qe[(3 + voigt(ii, 2)) * NP + vn] * nrm[2];
      // traction-free wall: mirror state v+ = v-, (s n)+ = -(s n)-
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        vP[ii] = wall ? gw * vM[ii] : nbt[t][ii];
        tP[ii] = wall ? -gw * tM[ii] : -nbt[t][3 + ii];  // neighbour stored s n with its own normal
      }
      if constexpr (PHYS == 2) {
        // one-impedance Riemann solution per side: the velocity correction
        // (t* - t-)/rho and the vector v* - v-, both times Fscale
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          const float jv = vP[ii] - vM[ii], jt = tP[ii] - tM[ii];
          lf[ii * NFN] = rec[3] * jt + rec[4] * jv;
          lf[(3 + ii) * NFN] = rec[5] * jt + rec[6] * jv;
        }
      } else {
        const float ZpP = rec[3], ZsP = rec[4], fs = rec[5];
        float jv[3], jt[3];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          jv[ii] = 0.5f * (vP[ii] - vM[ii]);
          jt[ii] = 0.5f * (tP[ii] - tM[ii]);
        }
        const float jvn = jv[0] * nrm[0] + jv[1] * nrm[1] + jv[2] * nrm[2];
        const float jsnn = jt[0] * nrm[0] + jt[1] * nrm[1] + jt[2] * nrm[2];
        lf[0] = fs * rec[6] * (jsnn + ZpP * jvn);    // k_p alpha_p
        lf[NFN] = fs * rec[7] * (jsnn + ZsP * jvn);  // k_s alpha_s
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) lf[(2 + ii) * NFN] = fs * (jt[ii] + ZsP * jv[ii]);  // vector alpha_s
      }
    }
  }
  __syncthreads();

  // ---- phase C: node per thread: D_j products, LIFT, combinations, AB3 ----
#pragma unroll
  for (int t = 0; t < NIT; ++t) {
    const int i = tid + t * kThreads;
    if (i >= ne * NP) continue;
    const int e = i / NP, n = i - e * NP;
    const float* G = s_g + 9 * e;
    const float* qe = s_q + e * NF * NP;
    const float* ax = s_aux + e * NAUX * NP;
    const float* lf = s_lift + e * NL * NFN;
    const float* cf = s_cf + e * CB;
    const float* fr = s_face + e * 4 * FW;  // face records of this element
    float r[NF];
    // per-face lifts of the penalty scalars
    float L[4][NL];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
      for (int c = 0; c < NL; ++c) L[f][c] = 0.0f;
#pragma unroll 4
      for (int j = 0; j < NFP; ++j) {
        const int fm = f * NFP + j;
        const float l = OPS_LDS ? s_ops[NDT + fm * NP + n] : a.LT[fm * NP + n];
#pragma unroll
        for (int c = 0; c < NL; ++c) L[f][c] += l * lf[c * NFN + fm];
      }
    }
    if constexpr (PHYS == 0) {
      float T0 = 0.f, T1 = 0.f, T2 = 0.f, dv = 0.f;
#pragma unroll 4
      for (int m = 0; m < NP; ++m) {
        const float d0 = OPS_LDS ? s_ops[(0 * NP + m) * NP + n] : a.DT[(0 * NP + m) * NP + n];
        const float d1 = OPS_LDS ? s_ops[(1 * NP + m) * NP + n] : a.DT[(1 * NP + m) * NP + n];
        const float d2 = OPS_LDS ? s_ops[(2 * NP + m) * NP + n] : a.DT[(2 * NP + m) * NP + n];
        const float pm = qe[m];
        T0 += d0 * pm;
        T1 += d1 * pm;
        T2 += d2 * pm;
        dv += d0 * ax[m] + d1 * ax[NP + m] + d2 * ax[2 * NP + m];
      }
      const float rc2 = cf[0], irho = cf[1];
      r[0] = -rc2 * dv + (L[0][0] + L[1][0] + L[2][0] + L[3][0]);
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
        r[1 + ii] = -irho * (G[3 * ii + 0] * T0 + G[3 * ii + 1] * T1 + G[3 * ii + 2] * T2) +
                    (fr[0 * FW + ii] * L[0][1] + fr[1 * FW + ii] * L[1][1] + fr[2 * FW + ii] * L[2][1] +
                     fr[3 * FW + ii] * L[3][1]);
    } else {
      float Dv[3][3], dS[3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        dS[ii] = 0.f;
#pragma unroll
        for (int l = 0; l < 3; ++l) Dv[ii][l] = 0.f;
      }
#pragma unroll 2
      for (int m = 0; m < NP; ++m) {
        float d[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) d[l] = OPS_LDS ? s_ops[(l * NP + m) * NP + n] : a.DT[(l * NP + m) * NP + n];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          const float vm = qe[ii * NP + m];
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            Dv[ii][l] += d[l] * vm;
            dS[ii] += d[l] * ax[(ii * 3 + l) * NP + m];
          }
        }
      }
      float gv[3][3];  // d v_i / d x_j = sum_l g_jl D_l v_i
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          gv[ii][jj] = G[3 * jj + 0] * Dv[ii][0] + G[3 * jj + 1] * Dv[ii][1] + G[3 * jj + 2] * Dv[ii][2];
      if constexpr (PHYS == 2) {
        // velocity: (1/rho) div s + the lifted corrections (already over rho);
        // stress: C times the engineering strain of grad v plus, per face,
        // that of n (x) w for the lifted vector w
        const float irho = cf[21];
        float ev[6] = {gv[0][0], gv[1][1], gv[2][2], gv[1][2] + gv[2][1], gv[0][2] + gv[2][0], gv[0][1] + gv[1][0]};
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) r[ii] = irho * dS[ii] + (L[0][ii] + L[1][ii] + L[2][ii] + L[3][ii]);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const float n0 = fr[f * FW + 0], n1 = fr[f * FW + 1], n2 = fr[f * FW + 2];
          const float w0 = L[f][3], w1 = L[f][4], w2 = L[f][5];
          ev[0] += n0 * w0;
          ev[1] += n1 * w1;
          ev[2] += n2 * w2;
          ev[3] += n1 * w2 + n2 * w1;
          ev[4] += n0 * w2 + n2 * w0;
          ev[5] += n0 * w1 + n1 * w0;
        }
#pragma unroll
        for (int va = 0; va < 6; ++va) {
          float acc = 0.0f;
#pragma unroll
          for (int vb = 0; vb < 6; ++vb) acc += cf[va <= vb ? upper6(va, vb) : upper6(vb, va)] * ev[vb];
          r[3 + va] = acc;
        }
      } else {
        const float lam = cf[0], mu = cf[1], irho = cf[2], cp = cf[5], cs = cf[6];
        const float divv = gv[0][0] + gv[1][1] + gv[2][2];
        // surface: velocity  sum_f [n (cp L1 - cs L2) + ks cs L3]
        //          stress    sum_f [lam L1 I + 2 mu n n^T (L1 - L2) + mu ks (n L3^T + L3 n^T)]
        float sv[3] = {0.f, 0.f, 0.f};
        float ss[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float l1sum = 0.f;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const float ks = fr[f * FW + 7];
          const float n0 = fr[f * FW + 0], n1 = fr[f * FW + 1], n2 = fr[f * FW + 2];
          const float nf[3] = {n0, n1, n2};
          const float a1 = cp * L[f][0] - cs * L[f][1];
          const float b2 = 2.0f * mu * (L[f][0] - L[f][1]);
          const float c3 = mu * ks;
          l1sum += L[f][0];
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) sv[ii] += nf[ii] * a1 + ks * cs * L[f][2 + ii];
          const int vi[6] = {0, 1, 2, 1, 0, 0};
          const int vj[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
          for (int v = 0; v < 6; ++v) {
            const int ii = vi[v], jj = vj[v];
            ss[v] += b2 * nf[ii] * nf[jj] + c3 * (nf[ii] * L[f][2 + jj] + L[f][2 + ii] * nf[jj]);
          }
        }
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) r[ii] = irho * dS[ii] + sv[ii];
        const int vi[6] = {0, 1, 2, 1, 0, 0};
        const int vj[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          const int ii = vi[v], jj = vj[v];
          float val = mu * (gv[ii][jj] + gv[jj][ii]) + ss[v];
          if (ii == jj) val += lam * (divv + l1sum);
          r[3 + v] = val;
        }
      }
    }
    const int64_t base = (e0 + e) * NF * NP + n;
    if (!step) {
#pragma unroll
      for (int c = 0; c < NF; ++c) a.r_out[base + c * NP] = r[c];
      continue;
    }
    float qn[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) {
      qn[c] = qe[c * NP + n] + a.c0 * r[c] + a.c1 * h1[t][c] + a.c2 * h2[t][c];
      a.q_out[base + c * NP] = qn[c];
      a.r_out[base + c * NP] = r[c];
    }
    // own traces of the updated fields at every face this node lies on
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int fj = nfs[t][s];
      if (fj < 0) break;
      const int f = fj / NFP, j = fj - f * NFP;
      const float n0 = fr[f * FW + 0], n1 = fr[f * FW + 1], n2 = fr[f * FW + 2];
      float* tr = a.qf_out + ((e0 + e) * 4 + f) * NT * NFP + j;
      if constexpr (PHYS == 0) {
        tr[0] = qn[0];
        tr[NFP] = n0 * qn[1] + n1 * qn[2] + n2 * qn[3];
      } else {
        tr[0] = qn[0];
        tr[NFP] = qn[1];
        tr[2 * NFP] = qn[2];
        // s n with Voigt (11, 22, 33, 23, 13, 12)
        tr[3 * NFP] = qn[3] * n0 + qn[8] * n1 + qn[7] * n2;
        tr[4 * NFP] = qn[8] * n0 + qn[4] * n1 + qn[6] * n2;
        tr[5 * NFP] = qn[7] * n0 + qn[6] * n1 + qn[5] * n2;
      }
    }
  }
}

template <int N, int PHYS>
__global__ void __launch_bounds__(kThreads)
dg_step_kernel(StepArgs a) {
  step_valu_tile<N, PHYS>(a, tile_of_block(a.xcd_remap));
}

// Many meshes of one degree in one launch: workgroup b runs tile work[b].y of
// member work[b].x with that member's arguments for this step's phase.
template <int N, int PHYS>
__global__ void __launch_bounds__(kThreads)
dg_step_kernel_batch(const StepArgs* __restrict__ args, const int2* __restrict__ work, int phase) {
  const int2 w = work[blockIdx.x];
  if (w.x < 0) return;  // padding entry of the work list
  const StepArgs a = args[w.x * kBatchPhases + phase];
  step_valu_tile<N, PHYS>(a, w.y);
}

// Own traces of a field array (initial state, right-hand-side evaluation).
template <int N, int PHYS>
__global__ void __launch_bounds__(kThreads)
dg_trace_kernel(int64_t K, const float* __restrict__ q, const float* __restrict__ geo,
                const int32_t* __restrict__ fmask, float* __restrict__ qf) {
  constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP, NFN = 4 * NFP;
  constexpr int NF = Phys<PHYS>::NF, NT = Phys<PHYS>::NT;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= K * NFN) return;
  const int64_t k = i / NFN;
  const int fn = static_cast<int>(i - k * NFN);
  const int f = fn / NFP, j = fn - f * NFP;
  float G[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) G[t] = geo[k * 9 + t];
  float nrm[3], fs;
  face_normal(G, f, nrm, fs);
  const int vn = fmask[f * NFP + j];
  const float* qe = q + k * NF * NP;
  float* tr = qf + (k * 4 + f) * NT * NFP;
  if constexpr (PHYS == 0) {
    tr[j] = qe[vn];
    tr[NFP + j] = nrm[0] * qe[NP + vn] + nrm[1] * qe[2 * NP + vn] + nrm[2] * qe[3 * NP + vn];
  } else {
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) tr[ii * NFP + j] = qe[ii * NP + vn];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
      tr[(3 + ii) * NFP + j] = qe[(3 + voigt(ii, 0)) * NP + vn] * nrm[0] +
                               qe[(3 + voigt(ii, 1)) * NP + vn] * nrm[1] +
                               qe[(3 + voigt(ii, 2)) * NP + vn] * nrm[2];
  }
}

// Traces of q + c0 r0 + c1 r1 + c2 r2 for the elements of a list (the slow
// elements next to fast ones in two-rate stepping: their state at the fast
// class's half step, from their own Adams-Bashforth history).  A term whose
// coefficient is zero is not read.
template <int N, int PHYS>
__global__ void __launch_bounds__(kThreads)
dg_trace_comb_kernel(int64_t nlist, const int32_t* __restrict__ list, const float* __restrict__ q,
                     const float* __restrict__ r0, const float* __restrict__ r1, const float* __restrict__ r2,
                     float c0, float c1, float c2, const float* __restrict__ geo,
                     const int32_t* __restrict__ fmask, float* __restrict__ qf) {
  constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP, NFN = 4 * NFP;
  constexpr int NF = Phys<PHYS>::NF, NT = Phys<PHYS>::NT;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= nlist * NFN) return;
  const int64_t item = i / NFN;
  const int fn = static_cast<int>(i - item * NFN);
  const int64_t k = list[item];
  const int f = fn / NFP, j = fn - f * NFP;
  float G[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) G[t] = geo[k * 9 + t];
  float nrm[3], fs;
  face_normal(G, f, nrm, fs);
  const int vn = fmask[f * NFP + j];
  const int64_t base = k * NF * NP + vn;
  auto val = [&](int c) {
    const int64_t at = base + static_cast<int64_t>(c) * NP;
    float v = q[at] + c0 * r0[at];
    if (c1 != 0.0f) v += c1 * r1[at];
    if (c2 != 0.0f) v += c2 * r2[at];
    return v;
  };
  float* tr = qf + (k * 4 + f) * NT * NFP;
  if constexpr (PHYS == 0) {
    tr[j] = val(0);
    tr[NFP + j] = nrm[0] * val(1) + nrm[1] * val(2) + nrm[2] * val(3);
  } else {
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) tr[ii * NFP + j] = val(ii);
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
      tr[(3 + ii) * NFP + j] = val(3 + voigt(ii, 0)) * nrm[0] + val(3 + voigt(ii, 1)) * nrm[1] +
                               val(3 + voigt(ii, 2)) * nrm[2];
  }
}

// Impedance of an anisotropic element (rho, then the 21 upper-triangle
// stiffness entries): sqrt(rho * the largest diagonal stiffness), the P
// impedance when the stiffness is isotropic.
__device__ __forceinline__ float aniso_impedance(const float* __restrict__ c) {
  float m = c[1 + upper6(0, 0)];
#pragma unroll
  for (int d = 1; d < 6; ++d) m = fmaxf(m, c[1 + upper6(d, d)]);
  return sqrtf(c[0] * m);
}

// Derived coefficients per element, including the neighbours' impedances on
// each face (own values on walls).
//   acoustic    cf = [rho c^2, 1/rho, Z, c, Z+_0..3]
//   elastic     cf = [lambda, mu, 1/rho, Zp, Zs, cp, cs, 0, Zp+_0..3, Zs+_0..3]
//   anisotropic cf = [C (21 upper-triangle entries), 1/rho, Z, 0, Z+_0..3, 0 0 0 0]
template <int PHYS>
__global__ void __launch_bounds__(kThreads)
dg_coef_kernel(int64_t K, const float* __restrict__ coef, const int32_t* __restrict__ conn,
               float* __restrict__ cf) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (k >= K) return;
  if constexpr (PHYS == 0) {
    const float rho = coef[2 * k], c = coef[2 * k + 1];
    float* o = cf + 8 * k;
    o[0] = rho * c * c;
    o[1] = 1.0f / rho;
    o[2] = rho * c;
    o[3] = c;
    for (int f = 0; f < 4; ++f) {
      const int w = conn[4 * k + f];
      int64_t kn = ((w & 7) == 7) ? k : static_cast<int64_t>(w >> 5);
      o[4 + f] = coef[2 * kn] * coef[2 * kn + 1];
    }
  } else if constexpr (PHYS == 2) {
    const float* c = coef + 22 * k;
    float* o = cf + 32 * k;
    for (int i = 0; i < 21; ++i) o[i] = c[1 + i];
    o[21] = 1.0f / c[0];
    o[22] = aniso_impedance(c);
    o[23] = 0.0f;
    for (int f = 0; f < 4; ++f) {
      const int w = conn[4 * k + f];
      const int64_t kn = ((w & 7) == 7) ? k : static_cast<int64_t>(w >> 5);
      o[24 + f] = aniso_impedance(coef + 22 * kn);
    }
    for (int i = 28; i < 32; ++i) o[i] = 0.0f;
  } else {
    const float rho = coef[3 * k], lam = coef[3 * k + 1], mu = coef[3 * k + 2];
    const float cp = sqrtf((lam + 2.0f * mu) / rho), cs = sqrtf(mu / rho);
    float* o = cf + 16 * k;
    o[0] = lam;
    o[1] = mu;
    o[2] = 1.0f / rho;
    o[3] = rho * cp;
    o[4] = rho * cs;
    o[5] = cp;
    o[6] = cs;
    o[7] = 0.0f;
    for (int f = 0; f < 4; ++f) {
      const int w = conn[4 * k + f];
      int64_t kn = ((w & 7) == 7) ? k : static_cast<int64_t>(w >> 5);
      const float rn = coef[3 * kn], ln = coef[3 * kn + 1], mn = coef[3 * kn + 2];
      o[8 + f] = rn * sqrtf((ln + 2.0f * mn) / rn);
      o[12 + f] = rn * sqrtf(mn / rn);
    }
  }
}

// Coefficient validation on the device: the smallest index of a value that
// is not positive and finite (int32: at most 3 * 2^26 coefficients).
constexpr int kNoIndex = 0x7fffffff;

__global__ void dg_flag_set_kernel(int* flag, int value) {
  if (threadIdx.x == 0) flag[0] = value;
}

__global__ void __launch_bounds__(kThreads)
dg_first_nonpositive_kernel(int64_t n, const float* __restrict__ x, int* flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) {
    const float v = x[i];
    if (!(v > 0.0f) || !(v <= 3.402823466e38f)) atomicMin(flag, static_cast<int>(i));
  }
}

// Cholesky factor of the symmetric 6x6 stiffness given by its 21 upper-
// triangle entries, in double (lower triangle of Lc, row-major); false when a
// pivot is not positive (the matrix is not positive definite) or not finite.
__device__ __forceinline__ bool stiffness_cholesky(const float* __restrict__ c21, double Lc[6][6]) {
  bool ok = true;
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j <= i; ++j) {
      double v = static_cast<double>(c21[upper6(j, i)]);
      for (int p = 0; p < j; ++p) v -= Lc[i][p] * Lc[j][p];
      if (i == j) {
        ok = ok && (v > 0.0) && (v <= 1.0e300);
        Lc[i][i] = sqrt(v > 0.0 ? v : 1.0);
      } else {
        Lc[i][j] = v / Lc[j][j];
      }
    }
  }
  return ok;
}

// Anisotropic coefficients: the smallest element index whose density is not
// positive and finite or whose stiffness is not finite and positive definite.
__global__ void __launch_bounds__(kThreads)
dg_first_bad_stiffness_kernel(int64_t K, const float* __restrict__ coef, int* flag) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (k >= K) return;
  const float* c = coef + 22 * k;
  bool ok = (c[0] > 0.0f) && (c[0] <= 3.402823466e38f);
  for (int i = 1; i < 22; ++i) ok = ok && (fabsf(c[i]) <= 3.402823466e38f);
  double Lc[6][6];
  ok = ok && stiffness_cholesky(c + 1, Lc);
  if (!ok) atomicMin(flag, static_cast<int>(k));
}

__global__ void dg_flag_none_kernel(int* flag) {
  if (threadIdx.x == 0 && flag[0] == kNoIndex) flag[0] = -1;
}

// FP64 discrete energy, partial sums per workgroup.  A workgroup takes a tile
// of KT = G*EG elements; item (g, n) forms (M q_c)_n at node n for the EG
// elements of group g, so that each mass-matrix word read from L2 serves
// EG*NF products (the matrix is read once per group, not once per element).
// Grouping pays from N = 6 (acoustic) / 7 (elastic), where the matrix no
// longer sits in L1 (measured 1.2-1.6x); below, one element per item.
template <int N, int PHYS>
struct ETile {
  static constexpr int NP = Deg<N>::NP;
  static constexpr int EG = PHYS == 0 ? (N >= 6 ? 8 : 1) : (N >= 7 ? 4 : 1);  // elements per item
  static constexpr int G = (256 / NP) < 1 ? 1 : (256 / NP);  // groups per workgroup
  static constexpr int KT = G * EG;
  // group stride in LDS words (padded to an odd count when grouping, so that
  // two groups in one wavefront read different banks)
  static constexpr int GS = EG * Phys<PHYS>::NF * NP + (EG > 1 ? 1 : 0);
};

template <int N, int PHYS>
__global__ void __launch_bounds__(kThreads)
dg_energy_kernel(int64_t K, const float* __restrict__ q, const float* __restrict__ coef,
                 const double* __restrict__ J, const double* __restrict__ M,
                 double* __restrict__ partial) {
  using T = ETile<N, PHYS>;
  constexpr int NP = T::NP, EG = T::EG, KT = T::KT, GS = T::GS;
  constexpr int NF = Phys<PHYS>::NF;
  constexpr int EW = NF * NP;  // words per element
  static_assert(NP <= kThreads, "one node per item");
  __shared__ float s_q[T::G * GS];
  __shared__ double s_red[kThreads];
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * KT;
  const int ne = static_cast<int>((K - e0) < KT ? (K - e0) : KT);
  const int tid = threadIdx.x;
  // the tile's fields (the products of items past the last element are
  // formed from stale words and dropped)
  if constexpr (EG == 1) {
    for (int i = tid; i < ne * EW; i += kThreads) s_q[i] = q[e0 * EW + i];
  } else {
    for (int i = tid; i < ne * EW; i += kThreads) {
      const int el = i / EW, r = i - el * EW;
      const int g = el / EG, e = el - g * EG;
      s_q[g * GS + e * EW + r] = q[e0 * EW + i];
    }
  }
  __syncthreads();
  double acc = 0.0;
  const int g = tid / NP, n = tid - g * NP;
  if (g < T::G) {
    const float* qg = s_q + g * GS;
    double Mq[EG][NF];
#pragma unroll
    for (int e = 0; e < EG; ++e)
#pragma unroll
      for (int c = 0; c < NF; ++c) Mq[e][c] = 0.0;
    // M is symmetric (formed as V^-T V^-1, the same sum for (n, m) and
    // (m, n)), so row n is read as column n: consecutive lanes (nodes) read
    // consecutive words
#pragma unroll 2
    for (int m = 0; m < NP; ++m) {
      const double mm = M[m * NP + n];
#pragma unroll
      for (int e = 0; e < EG; ++e)
#pragma unroll
        for (int c = 0; c < NF; ++c) Mq[e][c] += mm * static_cast<double>(qg[e * EW + c * NP + m]);
    }
#pragma unroll
    for (int e = 0; e < EG; ++e) {
      const int el = g * EG + e;
      if (el >= ne) continue;
      const int64_t k = e0 + el;
      const float* qe = qg + e * EW;
      double en;
      if constexpr (PHYS == 0) {
        const double rho = coef[2 * k], c = coef[2 * k + 1];
        en = Mq[e][0] * qe[n] / (rho * c * c);
#pragma unroll
        for (int ii = 1; ii < 4; ++ii) en += rho * Mq[e][ii] * qe[ii * NP + n];
      } else if constexpr (PHYS == 2) {
        // rho |v|^2 + s . C^-1 s, C^-1 s from the Cholesky factor
        const float* c = coef + 22 * k;
        double Lc[6][6];
        stiffness_cholesky(c + 1, Lc);
        double y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          double v = qe[(3 + i) * NP + n];
          for (int p = 0; p < i; ++p) v -= Lc[i][p] * y[p];
          y[i] = v / Lc[i][i];
        }
        for (int i = 5; i >= 0; --i) {
          double v = y[i];
          for (int p = i + 1; p < 6; ++p) v -= Lc[p][i] * y[p];
          y[i] = v / Lc[i][i];
        }
        double kin = 0.0, ss = 0.0;
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) kin += Mq[e][ii] * qe[ii * NP + n];
#pragma unroll
        for (int v = 0; v < 6; ++v) ss += Mq[e][3 + v] * y[v];
        en = static_cast<double>(c[0]) * kin + ss;
      } else {
        const double rho = coef[3 * k], lam = coef[3 * k + 1], mu = coef[3 * k + 2];
        double kin = 0.0, ss = 0.0;
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) kin += Mq[e][ii] * qe[ii * NP + n];
#pragma unroll
        for (int v = 0; v < 6; ++v) ss += (v < 3 ? 1.0 : 2.0) * Mq[e][3 + v] * qe[(3 + v) * NP + n];
        const double tr = static_cast<double>(qe[3 * NP + n]) + qe[4 * NP + n] + qe[5 * NP + n];
        const double Mtr = Mq[e][3] + Mq[e][4] + Mq[e][5];
        en = rho * kin + (ss - lam / (3.0 * lam + 2.0 * mu) * tr * Mtr) / (2.0 * mu);
      }
      acc += 0.5 * J[k] * en;
    }
  }
  s_red[tid] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) s_red[tid] += s_red[tid + w];
    __syncthreads();
  }
  if (tid == 0) partial[blockIdx.x] = s_red[0];
}

__global__ void __launch_bounds__(kThreads)
dg_sum_kernel(int64_t n, const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double s_red[kThreads];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) acc += partial[i];
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s_red[0];
}

// ---------------------------------------------------------------------------
// dispatch over (physics, degree)
// ---------------------------------------------------------------------------
template <int N, int PHYS>
hipError_t step_impl(const StepArgs& a, hipStream_t s) {
  constexpr int KT = Tile<N, PHYS>::KT;
  int64_t tiles = (a.K - a.e_begin + KT - 1) / KT;
  if (a.xcd_remap) tiles = ((tiles + 7) / 8) * 8;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_kernel<N, PHYS>), dim3(static_cast<unsigned>(tiles)), dim3(kThreads), 0, s,
                     a);
  return hipGetLastError();
}

template <int N, int PHYS>
hipError_t step_batch_impl(const StepArgs* args, const int2* work, int64_t ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_kernel_batch<N, PHYS>), dim3(static_cast<unsigned>(ntiles)), dim3(kThreads), 0, s,
                     args, work, phase);
  return hipGetLastError();
}

template <int N, int PHYS>
hipError_t trace_impl(int64_t K, const float* q, const float* geo, const int32_t* fmask, float* qf,
                      hipStream_t s) {
  const int64_t items = K * 4 * Deg<N>::NFP;
  const int64_t blocks = (items + kThreads - 1) / kThreads;
  hipLaunchKernelGGL((dg_trace_kernel<N, PHYS>), dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0,
                     s, K, q, geo, fmask, qf);
  return hipGetLastError();
}

template <int N, int PHYS>
hipError_t trace_comb_impl(int64_t nlist, const int32_t* list, const float* q, const float* r0, const float* r1,
                           const float* r2, float c0, float c1, float c2, const float* geo, const int32_t* fmask,
                           float* qf, hipStream_t s) {
  if (nlist <= 0) return hipSuccess;
  const int64_t blocks = (nlist * 4 * Deg<N>::NFP + kThreads - 1) / kThreads;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_trace_comb_kernel<N, PHYS>), dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s,
                     nlist, list, q, r0, r1, r2, c0, c1, c2, geo, fmask, qf);
  return hipGetLastError();
}

template <int N, int PHYS>
hipError_t energy_impl(int64_t K, const float* q, const float* coef, const double* J, const double* M,
                       double* partial, double* out, hipStream_t s) {
  constexpr int KT = ETile<N, PHYS>::KT;
  const int64_t blocks = (K + KT - 1) / KT;
  hipLaunchKernelGGL((dg_energy_kernel<N, PHYS>), dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0,
                     s, K, q, coef, J, M, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(dg_sum_kernel, dim3(1), dim3(kThreads), 0, s, blocks, partial, out);
  return hipGetLastError();
}

// Calls f(integral_constant<N>, integral_constant<PHYS>) for a runtime
// (physics, degree); `bad` when either is out of range.
template <int P, class R, class F>
R with_degree(int N, R bad, F&& f) {
  using P_ = std::integral_constant<int, P>;
  switch (N) {
    case 1: return f(std::integral_constant<int, 1>{}, P_{});
    case 2: return f(std::integral_constant<int, 2>{}, P_{});
    case 3: return f(std::integral_constant<int, 3>{}, P_{});
    case 4: return f(std::integral_constant<int, 4>{}, P_{});
    case 5: return f(std::integral_constant<int, 5>{}, P_{});
    case 6: return f(std::integral_constant<int, 6>{}, P_{});
    case 7: return f(std::integral_constant<int, 7>{}, P_{});
    case 8: return f(std::integral_constant<int, 8>{}, P_{});
  }
  return bad;
}

template <class R, class F>
R with_physics_degree(int physics, int N, R bad, F&& f) {
  switch (physics) {
    case 0: return with_degree<0>(N, bad, f);
    case 1: return with_degree<1>(N, bad, f);
    case 2: return with_degree<2>(N, bad, f);
  }
  return bad;
}

#define DGW_NP(n, p) decltype(n)::value, decltype(p)::value

}  // namespace

int coef_block(int physics) {
  return physics == 0 ? Phys<0>::CB : (physics == 1 ? Phys<1>::CB : Phys<2>::CB);
}
int num_traces(int physics) {
  return physics == 0 ? Phys<0>::NT : (physics == 1 ? Phys<1>::NT : Phys<2>::NT);
}

static bool is_mfma(int variant) { return mfma_precision(variant) >= 0; }

bool variant_supported(int physics, int N, int variant) {
  if (N < 1 || N > 8 || physics < 0 || physics > 2) return false;
  if (variant == kVariantValu) return true;
  if (physics == 2) return variant == kVariantMfma;  // anisotropic: node per thread and FP32 MFMA
  if (variant == kVariantMfmaWide) return physics == 0;  // acoustic tile shapes only
  if (is_mfma(variant)) return true;
  if (variant == kVariantElem) return elem_supported(physics, N);
  return false;
}

hipError_t launch_step(int physics, int N, int variant, const StepArgs& a, hipStream_t s) {
  if (!variant_supported(physics, N, variant)) return hipErrorInvalidValue;
  if (is_mfma(variant))
    return physics != 0 ? launch_step_mfma_elastic(physics, N, variant, a, s) : launch_step_mfma(physics, N, variant, a, s);
  if (variant == kVariantElem) return launch_step_elem(physics, N, a, s);
  return with_physics_degree(physics, N, hipErrorInvalidValue,
                             [&](auto n, auto p) { return step_impl<DGW_NP(n, p)>(a, s); });
}

int64_t tiles_for(int physics, int N, int variant, int64_t K) {
  const int E = tile_elements(physics, N, variant);
  return E > 0 ? (K + E - 1) / E : -1;
}

int tile_elements(int physics, int N, int variant) {
  if (!variant_supported(physics, N, variant)) return -1;
  if (is_mfma(variant)) return mfma_packing(physics, N, variant).E;
  if (variant == kVariantElem) return elem_tile_elements();
  return with_physics_degree(physics, N, -1, [&](auto n, auto p) { return Tile<DGW_NP(n, p)>::KT; });
}

hipError_t launch_step_batch(int physics, int N, int variant, const StepArgs* args, const int2* work,
                             int64_t ntiles, int phase, hipStream_t s) {
  if (!variant_supported(physics, N, variant)) return hipErrorInvalidValue;
  if (is_mfma(variant))
    return physics != 0 ? launch_step_batch_mfma_elastic(physics, N, variant, args, work, ntiles, phase, s)
                        : launch_step_batch_mfma(physics, N, variant, args, work, ntiles, phase, s);
  if (variant == kVariantElem) return launch_step_batch_elem(physics, N, args, work, ntiles, phase, s);
  return with_physics_degree(physics, N, hipErrorInvalidValue, [&](auto n, auto p) {
    return step_batch_impl<DGW_NP(n, p)>(args, work, ntiles, phase, s);
  });
}

hipError_t launch_traces(int physics, int N, int64_t K, const float* q, const float* geo,
                         const int32_t* fmask, float* qf, hipStream_t s) {
  return with_physics_degree(physics, N, hipErrorInvalidValue,
                             [&](auto n, auto p) { return trace_impl<DGW_NP(n, p)>(K, q, geo, fmask, qf, s); });
}

hipError_t launch_first_nonpositive(int64_t n, const float* x, int* flag, hipStream_t s) {
  if (n < 0 || n > kNoIndex) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dg_flag_set_kernel, dim3(1), dim3(64), 0, s, flag, kNoIndex);
  if (n > 0)
    hipLaunchKernelGGL(dg_first_nonpositive_kernel, dim3(static_cast<unsigned>((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, n, x, flag);
  hipLaunchKernelGGL(dg_flag_none_kernel, dim3(1), dim3(64), 0, s, flag);
  return hipGetLastError();
}

hipError_t launch_first_bad_stiffness(int64_t K, const float* coef, int* flag, hipStream_t s) {
  if (K < 0 || K > kNoIndex) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dg_flag_set_kernel, dim3(1), dim3(64), 0, s, flag, kNoIndex);
  if (K > 0)
    hipLaunchKernelGGL(dg_first_bad_stiffness_kernel, dim3(static_cast<unsigned>((K + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, K, coef, flag);
  hipLaunchKernelGGL(dg_flag_none_kernel, dim3(1), dim3(64), 0, s, flag);
  return hipGetLastError();
}

hipError_t launch_coef_prep(int physics, int64_t K, const float* coef, const int32_t* conn, float* cf,
                            hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((K + kThreads - 1) / kThreads)), block(kThreads);
  switch (physics) {
    case 0: hipLaunchKernelGGL(dg_coef_kernel<0>, grid, block, 0, s, K, coef, conn, cf); break;
    case 1: hipLaunchKernelGGL(dg_coef_kernel<1>, grid, block, 0, s, K, coef, conn, cf); break;
    case 2: hipLaunchKernelGGL(dg_coef_kernel<2>, grid, block, 0, s, K, coef, conn, cf); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_energy_partials(int device, double** ptr) {
  if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    int prev = 0;
    hipError_t err = hipGetDevice(&prev);
    if (err != hipSuccess) return err;
    if (prev != device && (err = hipSetDevice(device)) != hipSuccess) return err;
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) {
      const hipError_t e2 = hipSetDevice(prev);
      if (err == hipSuccess) err = e2;
    }
    if (err != hipSuccess) return err;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_trace_comb(int physics, int N, int64_t nlist, const int32_t* list, const float* q,
                             const float* r0, const float* r1, const float* r2, float c0, float c1, float c2,
                             const float* geo, const int32_t* fmask, float* qf, hipStream_t s) {
  return with_physics_degree(physics, N, hipErrorInvalidValue, [&](auto n, auto p) {
    return trace_comb_impl<DGW_NP(n, p)>(nlist, list, q, r0, r1, r2, c0, c1, c2, geo, fmask, qf, s);
  });
}

int64_t energy_blocks(int physics, int N, int64_t K) {
  return with_physics_degree(physics, N, int64_t(-1), [&](auto n, auto p) {
    constexpr int KT = ETile<DGW_NP(n, p)>::KT;
    return (K + KT - 1) / KT;
  });
}

hipError_t launch_energy(int physics, int N, int64_t K, const float* q, const float* coef, const double* J,
                         const double* mass, double* partial, double* out, hipStream_t s) {
  return with_physics_degree(physics, N, hipErrorInvalidValue, [&](auto n, auto p) {
    return energy_impl<DGW_NP(n, p)>(K, q, coef, J, mass, partial, out, s);
  });
}

#undef DGW_NP

}  // namespace dgw
