// Element-per-thread variant of the fused DG step for the lowest degrees
// (acoustic N = 1, 2; elastic N = 1): one thread owns one element, keeps its fields, history and
// neighbour traces in registers, and needs no LDS and no barrier.  At these
// degrees an element's operators are a few dozen numbers that every thread of
// a wavefront reads at the same address (scalar loads), the arithmetic per
// element is a few hundred flops, and the step is bound by the HBM traffic,
// so the kernel is written to issue every global load of an element at once:
// the fields, the AB3 history, the inverse Jacobian, the coefficients, the
// connectivity word of each face and, right after it, the neighbour's whole
// trace block of that face.  The face-node permutation between the two sides
// of a face is applied in registers: the relative orientation is a per-thread
// value, and the neighbour value at each own face node is the sum over the
// six orientations of (orientation matches) x (value at the permuted node),
// every register index being a compile-time constant.
//
// Arithmetic and conventions are those of the node-per-thread kernel: the
// right-hand sides of eqs. (5)-(6) and of the elastic system of Sec. 3.2,
// upwind penalties of Sec. 2.1 with mirror states on walls, the merged LIFT,
// the update of eq. (4) and the own traces of the updated fields.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_device.hpp"
#include "kernels.hpp"

namespace dgw {

namespace {

using namespace dev;

constexpr int kElemThreads = 256;

// Node index of the lattice point (l1, l2, l3, l4), l1 = N - l2 - l3 - l4, in
// the enumeration l4 outermost, then l3, then l2.
constexpr int node_index(int N, int l2, int l3, int l4) {
  int idx = 0;
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j + k <= N; ++j)
      for (int i = 0; i + j + k <= N; ++i) {
        if (i == l2 && j == l3 && k == l4) return idx;
        ++idx;
      }
  return -1;
}

constexpr int kFV[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
constexpr int kFP[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Face node jf of face f <-> (a, b) with b outermost; its volume node.
constexpr int face_node(int N, int f, int jf) {
  int j = 0;
  for (int b = 0; b <= N; ++b)
    for (int a = 0; a + b <= N; ++a) {
      if (j == jf) {
        int l[4] = {0, 0, 0, 0};
        l[kFV[f][0]] = N - a - b;
        l[kFV[f][1]] = a;
        l[kFV[f][2]] = b;
        return node_index(N, l[1], l[2], l[3]);
      }
      ++j;
    }
  return -1;
}

// Face node of the neighbour's face met by own face node j under
// orientation o (own face vertex p is the neighbour's vertex kFP[o][p]).
constexpr int face_perm(int N, int o, int jf) {
  int j = 0;
  for (int b = 0; b <= N; ++b)
    for (int a = 0; a + b <= N; ++a) {
      if (j == jf) {
        const int beta[3] = {N - a - b, a, b};
        int nb[3] = {0, 0, 0};
        for (int p = 0; p < 3; ++p) nb[kFP[o][p]] = beta[p];
        int jj = 0;
        for (int b2 = 0; b2 <= N; ++b2)
          for (int a2 = 0; a2 + b2 <= N; ++a2) {
            if (a2 == nb[1] && b2 == nb[2]) return jj;
            ++jj;
          }
        return -1;
      }
      ++j;
    }
  return -1;
}

// Contiguous load of CNT floats starting at p (alignment known at compile
// time from the element-major layouts) into out.
template <int CNT, int ALIGN>
__device__ __forceinline__ void load_run(const float* __restrict__ p, float* out) {
  if constexpr (ALIGN % 4 == 0 && CNT % 4 == 0) {
#pragma unroll
    for (int i = 0; i < CNT / 4; ++i) {
      const float4 v = reinterpret_cast<const float4*>(p)[i];
      out[4 * i] = v.x;
      out[4 * i + 1] = v.y;
      out[4 * i + 2] = v.z;
      out[4 * i + 3] = v.w;
    }
  } else if constexpr (ALIGN % 2 == 0 && CNT % 2 == 0) {
#pragma unroll
    for (int i = 0; i < CNT / 2; ++i) {
      const float2 v = reinterpret_cast<const float2*>(p)[i];
      out[2 * i] = v.x;
      out[2 * i + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < CNT; ++i) out[i] = p[i];
  }
}

template <int CNT, int ALIGN>
__device__ __forceinline__ void store_run(float* __restrict__ p, const float* v) {
  if constexpr (ALIGN % 4 == 0 && CNT % 4 == 0) {
#pragma unroll
    for (int i = 0; i < CNT / 4; ++i)
      reinterpret_cast<float4*>(p)[i] = float4{v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]};
  } else if constexpr (ALIGN % 2 == 0 && CNT % 2 == 0) {
#pragma unroll
    for (int i = 0; i < CNT / 2; ++i) reinterpret_cast<float2*>(p)[i] = float2{v[2 * i], v[2 * i + 1]};
  } else {
#pragma unroll
    for (int i = 0; i < CNT; ++i) p[i] = v[i];
  }
}

template <int N, int PHYS>
__device__ __forceinline__ void step_elem(const StepArgs& a, int64_t k) {
  constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP;
  constexpr int NF = Phys<PHYS>::NF, NT = Phys<PHYS>::NT, CB = Phys<PHYS>::CB;
  constexpr int NQ = NF * NP, NTR = NT * NFP;
  // element-major runs: q and r of element k start at k*NQ floats, a trace
  // block at (k*4 + f)*NTR floats
  constexpr int AQ = (NQ % 4 == 0) ? 4 : ((NQ % 2 == 0) ? 2 : 1);
  constexpr int AT = (NTR % 4 == 0) ? 4 : ((NTR % 2 == 0) ? 2 : 1);
  const bool step = (a.mode == kStepMode);

  // ---- every global load of the element --------------------------------------
  // the element's own data first (independent of the connectivity), then the
  // neighbour trace blocks, which wait for the connectivity word; a wall reads
  // its own block (in range, value unused) so that no load sits in a branch
  const int4 w4 = reinterpret_cast<const int4*>(a.conn)[k];
  const int word[4] = {w4.x, w4.y, w4.z, w4.w};
  float q[NQ];
  load_run<NQ, AQ>(a.q_in + k * NQ, q);
  float G[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i] = a.geo[k * 9 + i];
  float cf[CB];
  load_run<CB, 4>(a.cf + k * CB, cf);
  const bool use1 = step && (a.c1 != 0.0f), use2 = step && (a.c2 != 0.0f);
  // The AB3 history is read with the other loads where the registers allow
  // (acoustic: more bytes in flight pays), and only for the update where they
  // do not (elastic: fewer registers, more waves).
  constexpr bool kEarly = (PHYS == 0);
  float h1[kEarly ? NQ : 1], h2[kEarly ? NQ : 1];
  if constexpr (kEarly) {
    if (use1) load_run<NQ, AQ>(a.r1 + k * NQ, h1);
    if (use2) load_run<NQ, AQ>(a.r2 + k * NQ, h2);
  }

  float nbv[4][NTR];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const bool wall = (word[f] & 7) == 7;
    const int64_t kn = wall ? k : static_cast<int64_t>(word[f] >> 5);
    const int fnb = wall ? f : (word[f] >> 3) & 3;
    load_run<NTR, AT>(a.qf_in + (kn * 4 + fnb) * NTR, nbv[f]);
  }

  // ---- face constants and upwind penalties at the face nodes ----------------
  constexpr int NL = (PHYS == 0) ? 2 : 5;
  float pen[4][NL][NFP];
  float nrm[4][3];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    float fs;
    face_normal(G, f, nrm[f], fs);
    const bool wall = (word[f] & 7) == 7;
    const float gw = (word[f] & 8) ? 0.0f : 1.0f;  // absorbing wall: zero exterior state
    const int o = word[f] & 7;
    // neighbour trace at own face node j: sum over orientations
    float nb[NT][NFP];
#pragma unroll
    for (int j = 0; j < NFP; ++j)
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        float v = 0.0f;
#pragma unroll
        for (int oo = 0; oo < 6; ++oo) v += static_cast<float>(o == oo) * nbv[f][c * NFP + face_perm(N, oo, j)];
        nb[c][j] = v;
      }
    if constexpr (PHYS == 0) {
      const float ZM = cf[2];
      const float ZP = wall ? ZM : cf[4 + f];
      const float kc = 2.0f / (ZM + ZP);
      const float fp = fs * cf[0] * kc, fv = -fs * cf[3] * kc;
#pragma unroll
      for (int j = 0; j < NFP; ++j) {
        const int vn = face_node(N, f, j);
        const float pM = q[vn];
        const float vnM = nrm[f][0] * q[NP + vn] + nrm[f][1] * q[2 * NP + vn] + nrm[f][2] * q[3 * NP + vn];
        const float pP = wall ? gw * pM : nb[0][j];
        const float vnP = wall ? -gw * vnM : -nb[1][j];  // neighbour stored v.n with its own normal
        const float alpha = 0.5f * (pP - pM) - ZP * 0.5f * (vnP - vnM);
        pen[f][0][j] = fp * alpha;
        pen[f][1][j] = fv * alpha;
      }
    } else {
      const float ZpM = cf[3], ZsM = cf[4];
      const float ZpP = wall ? ZpM : cf[8 + f];
      const float ZsP = wall ? ZsM : cf[12 + f];
      const float kp = 2.0f / (ZpM + ZpP), ks = 2.0f / (ZsM + ZsP);
#pragma unroll
      for (int j = 0; j < NFP; ++j) {
        const int vn = face_node(N, f, j);
        float vM[3], tM[3], jv[3], jt[3];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) vM[ii] = q[ii * NP + vn];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
          tM[ii] = q[(3 + voigt(ii, 0)) * NP + vn] * nrm[f][0] + q[(3 + voigt(ii, 1)) * NP + vn] * nrm[f][1] +
                   q[(3 + voigt(ii, 2)) * NP + vn] * nrm[f][2];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          const float vP = wall ? gw * vM[ii] : nb[ii][j];
          const float tP = wall ? -gw * tM[ii] : -nb[3 + ii][j];  // neighbour stored s n with its own normal
          jv[ii] = 0.5f * (vP - vM[ii]);
          jt[ii] = 0.5f * (tP - tM[ii]);
        }
        const float jvn = jv[0] * nrm[f][0] + jv[1] * nrm[f][1] + jv[2] * nrm[f][2];
        const float jsnn = jt[0] * nrm[f][0] + jt[1] * nrm[f][1] + jt[2] * nrm[f][2];
        pen[f][0][j] = fs * kp * (jsnn + ZpP * jvn);
        pen[f][1][j] = fs * ks * (jsnn + ZsP * jvn);
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) pen[f][2 + ii][j] = fs * (jt[ii] + ZsP * jv[ii]);
      }
    }
  }

  // ---- right-hand side node by node ------------------------------------------
  float r[NQ];
#pragma unroll
  for (int n = 0; n < NP; ++n) {
    // lifts of the penalty scalars per face at node n
    float L[4][NL];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int c = 0; c < NL; ++c) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < NFP; ++j) s += a.LT[(f * NFP + j) * NP + n] * pen[f][c][j];
        L[f][c] = s;
      }
    if constexpr (PHYS == 0) {
      float T0 = 0.f, T1 = 0.f, T2 = 0.f, dv = 0.f;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const float d0 = a.DT[(0 * NP + m) * NP + n], d1 = a.DT[(1 * NP + m) * NP + n];
        const float d2 = a.DT[(2 * NP + m) * NP + n];
        const float pm = q[m];
        const float v0 = q[NP + m], v1 = q[2 * NP + m], v2 = q[3 * NP + m];
        T0 += d0 * pm;
        T1 += d1 * pm;
        T2 += d2 * pm;
        dv += d0 * (G[0] * v0 + G[3] * v1 + G[6] * v2) + d1 * (G[1] * v0 + G[4] * v1 + G[7] * v2) +
              d2 * (G[2] * v0 + G[5] * v1 + G[8] * v2);
      }
      r[n] = -cf[0] * dv + (L[0][0] + L[1][0] + L[2][0] + L[3][0]);
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
        r[(1 + ii) * NP + n] = -cf[1] * (G[3 * ii] * T0 + G[3 * ii + 1] * T1 + G[3 * ii + 2] * T2) +
                               (nrm[0][ii] * L[0][1] + nrm[1][ii] * L[1][1] + nrm[2][ii] * L[2][1] +
                                nrm[3][ii] * L[3][1]);
    } else {
      float Dv[3][3], dS[3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        dS[ii] = 0.f;
#pragma unroll
        for (int l = 0; l < 3; ++l) Dv[ii][l] = 0.f;
      }
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        float d[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) d[l] = a.DT[(l * NP + m) * NP + n];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          const float si0 = q[(3 + voigt(ii, 0)) * NP + m], si1 = q[(3 + voigt(ii, 1)) * NP + m];
          const float si2 = q[(3 + voigt(ii, 2)) * NP + m];
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            Dv[ii][l] += d[l] * q[ii * NP + m];
            dS[ii] += d[l] * (G[0 * 3 + l] * si0 + G[1 * 3 + l] * si1 + G[2 * 3 + l] * si2);
          }
        }
      }
      const float lam = cf[0], mu = cf[1], irho = cf[2], cp = cf[5], cs = cf[6];
      float gv[3][3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          gv[ii][jj] = G[3 * jj + 0] * Dv[ii][0] + G[3 * jj + 1] * Dv[ii][1] + G[3 * jj + 2] * Dv[ii][2];
      const float divv = gv[0][0] + gv[1][1] + gv[2][2];
      float sv[3] = {0.f, 0.f, 0.f};
      float ss[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float l1sum = 0.f;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const bool wall = (word[f] & 7) == 7;
        const float ZsM = cf[4], ZsP = wall ? ZsM : cf[12 + f];
        const float ks = 2.0f / (ZsM + ZsP);
        const float a1 = cp * L[f][0] - cs * L[f][1];
        const float b2 = 2.0f * mu * (L[f][0] - L[f][1]);
        const float c3 = mu * ks;
        l1sum += L[f][0];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) sv[ii] += nrm[f][ii] * a1 + ks * cs * L[f][2 + ii];
        const int vi[6] = {0, 1, 2, 1, 0, 0};
        const int vj[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          const int ii = vi[v], jj = vj[v];
          ss[v] += b2 * nrm[f][ii] * nrm[f][jj] + c3 * (nrm[f][ii] * L[f][2 + jj] + L[f][2 + ii] * nrm[f][jj]);
        }
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) r[ii * NP + n] = irho * dS[ii] + sv[ii];
      const int vi[6] = {0, 1, 2, 1, 0, 0};
      const int vj[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
      for (int v = 0; v < 6; ++v) {
        const int ii = vi[v], jj = vj[v];
        float val = mu * (gv[ii][jj] + gv[jj][ii]) + ss[v];
        if (ii == jj) val += lam * (divv + l1sum);
        r[(3 + v) * NP + n] = val;
      }
    }
  }

  // ---- update, writes, own traces -------------------------------------------
  store_run<NQ, AQ>(a.r_out + k * NQ, r);
  if (!step) return;
  if constexpr (kEarly) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      float x = q[i] + a.c0 * r[i];
      if (use1) x += a.c1 * h1[i];
      if (use2) x += a.c2 * h2[i];
      q[i] = x;
    }
  } else {
    constexpr int RUN = (AQ >= 4) ? 4 : AQ;
#pragma unroll
    for (int i0 = 0; i0 < NQ; i0 += RUN) {
      float g1[RUN], g2[RUN];
#pragma unroll
      for (int t = 0; t < RUN; ++t) g1[t] = g2[t] = 0.0f;
      if (use1) load_run<RUN, RUN>(a.r1 + k * NQ + i0, g1);
      if (use2) load_run<RUN, RUN>(a.r2 + k * NQ + i0, g2);
#pragma unroll
      for (int t = 0; t < RUN; ++t) q[i0 + t] = q[i0 + t] + a.c0 * r[i0 + t] + a.c1 * g1[t] + a.c2 * g2[t];
    }
  }
  store_run<NQ, AQ>(a.q_out + k * NQ, q);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    float tr[NTR];
#pragma unroll
    for (int j = 0; j < NFP; ++j) {
      const int vn = face_node(N, f, j);
      if constexpr (PHYS == 0) {
        tr[j] = q[vn];
        tr[NFP + j] = nrm[f][0] * q[NP + vn] + nrm[f][1] * q[2 * NP + vn] + nrm[f][2] * q[3 * NP + vn];
      } else {
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) tr[ii * NFP + j] = q[ii * NP + vn];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
          tr[(3 + ii) * NFP + j] = q[(3 + voigt(ii, 0)) * NP + vn] * nrm[f][0] +
                                   q[(3 + voigt(ii, 1)) * NP + vn] * nrm[f][1] +
                                   q[(3 + voigt(ii, 2)) * NP + vn] * nrm[f][2];
      }
    }
    store_run<NTR, AT>(a.qf_out + (k * 4 + f) * NTR, tr);
  }
}

template <int N, int PHYS>
__global__ void __launch_bounds__(kElemThreads)
dg_step_elem_kernel(StepArgs a) {
  const int64_t k = a.e_begin + tile_of_block(a.xcd_remap) * kElemThreads + threadIdx.x;
  if (k >= a.K) return;  // no barrier in this kernel
  step_elem<N, PHYS>(a, k);
}

template <int N, int PHYS>
__global__ void __launch_bounds__(kElemThreads)
dg_step_elem_kernel_batch(const StepArgs* __restrict__ args, const int2* __restrict__ work, int phase) {
  const int2 w = work[blockIdx.x];
  if (w.x < 0) return;  // padding entry of the work list
  const StepArgs a = args[w.x * kBatchPhases + phase];
  const int64_t k = a.e_begin + static_cast<int64_t>(w.y) * kElemThreads + threadIdx.x;
  if (k >= a.K) return;
  step_elem<N, PHYS>(a, k);
}

template <int N, int PHYS>
hipError_t elem_impl(const StepArgs& a, hipStream_t s) {
  int64_t tiles = (a.K - a.e_begin + kElemThreads - 1) / kElemThreads;
  if (a.xcd_remap) tiles = ((tiles + 7) / 8) * 8;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_elem_kernel<N, PHYS>), dim3(static_cast<unsigned>(tiles)), dim3(kElemThreads), 0, s,
                     a);
  return hipGetLastError();
}

template <int N, int PHYS>
hipError_t elem_batch_impl(const StepArgs* args, const int2* work, int64_t ntiles, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_step_elem_kernel_batch<N, PHYS>), dim3(static_cast<unsigned>(ntiles)), dim3(kElemThreads),
                     0, s, args, work, phase);
  return hipGetLastError();
}

}  // namespace

// Register budget: the acoustic fields, history and traces of one element fit
// in a thread's registers for N <= 2, the elastic ones for N = 1.
bool elem_supported(int physics, int N) { return physics == 0 ? (N >= 1 && N <= 2) : N == 1; }

int elem_tile_elements() { return kElemThreads; }

hipError_t launch_step_elem(int physics, int N, const StepArgs& a, hipStream_t s) {
  if (physics == 0) {
    if (N == 1) return elem_impl<1, 0>(a, s);
    if (N == 2) return elem_impl<2, 0>(a, s);
  } else {
    if (N == 1) return elem_impl<1, 1>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step_batch_elem(int physics, int N, const StepArgs* args, const int2* work, int64_t ntiles,
                                  int phase, hipStream_t s) {
  if (physics == 0) {
    if (N == 1) return elem_batch_impl<1, 0>(args, work, ntiles, phase, s);
    if (N == 2) return elem_batch_impl<2, 0>(args, work, ntiles, phase, s);
  } else {
    if (N == 1) return elem_batch_impl<1, 1>(args, work, ntiles, phase, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dgw
