// Kernels of the misfit gradient: point injection (source and adjoint
// source), receiver sampling, and the per-step accumulation of the
// coefficient gradient.
//
// The adjoint state itself is advanced by the forward step kernel: with the
// energy weight W (J M times the material block) and P = +1 on p / stresses,
// -1 on velocities, the DG operator satisfies A^T = P W A P W^{-1} (exact
// summation by parts on affine elements, symmetric upwind dissipation that
// does not couple velocities and stresses).  In the variables
// phi = P W^{-1} lambda the reverse Adams-Bashforth recursion becomes
//   phi_m = phi_{m+1} + A (dt sum_i a_i phi_{m+i}) + P W^{-1} g_m,
// an ordinary step of eq. (4) taken backwards in time.  What remains
// element-local is here.
//
// Gradient of J with respect to the coefficients theta of one element:
//   dJ/dtheta = sum_m chi_m^T P (-dW/dtheta A q_m + dB/dtheta q_m),
//   chi_m = dt (a1 phi_{m+1} + a2 phi_{m+2} + a3 phi_{m+3}),  B = W A.
// The volume part of B does not depend on theta; its surface part depends on
// the impedances of both sides of each face only.  The dW term needs
// mass-weighted products of chi and r_m = A q_m; the dB term needs, per face,
// the face traces of chi against the face-mass-weighted jumps of q_m.  The
// kernel accumulates, per element (float64):
//   acoustic: [a_p, a_v, gm_0..3, gp_0..3]
//   elastic:  [a_v, a_s, a_t, gmP_0..3, gmS_0..3, gpP_0..3, gpS_0..3]
// with gm (gp) the derivative of the face term with respect to the
// impedance on the element's own (the neighbour's) side; the finalize kernel
// adds each face's gp to the element on the other side and applies the chain
// rule to (rho, c) or (rho, lambda, mu).
#include <hip/hip_runtime.h>

#include "dg_device.hpp"
#include "kernels.hpp"
#include "mfma_common.hpp"

namespace dgw {

namespace {

using namespace dev;

constexpr int kWave = 64;

// Own traces of element k of field array q (the step kernel's convention).
template <int N, int PHYS>
__device__ __forceinline__ void element_traces(int64_t k, const float* __restrict__ q, const float* G,
                                               const int32_t* __restrict__ fmask, float* __restrict__ qf,
                                               int tid, int nthreads) {
  constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP;
  constexpr int NF = Phys<PHYS>::NF, NT = Phys<PHYS>::NT;
  const float* qe = q + k * NF * NP;
  for (int i = tid; i < 4 * NFP; i += nthreads) {
    const int f = i / NFP, j = i - f * NFP;
    float nrm[3], fs;
    face_normal(G, f, nrm, fs);
    const int vn = fmask[f * NFP + j];
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
}

// One workgroup per distinct element: q[k][field_e][:] += a_e vec_e[:] for the
// element's entries e, a_e = amp (chan < 0) or traces[chan] - data[chan];
// then the element's own traces are rewritten.
template <int N, int PHYS>
__global__ void __launch_bounds__(kWave)
dg_inject_kernel(const InjectArgs a) {
  constexpr int NP = Deg<N>::NP, NF = Phys<PHYS>::NF;
  const int u = blockIdx.x;
  const int64_t k = a.elem[u];
  const int tid = threadIdx.x;
  float* qe = a.q + k * NF * NP;
  const int e0 = a.start[u], e1 = a.start[u + 1];
  for (int n = tid; n < NP; n += kWave) {
    for (int e = e0; e < e1; ++e) {
      const int ch = a.chan[e];
      const float amp = ch < 0 ? a.amp : (a.traces[ch] - a.data[ch]);
      qe[a.field[e] * NP + n] += amp * a.vec[static_cast<int64_t>(e) * NP + n];
    }
  }
  __syncthreads();
  float G[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) G[t] = a.geo[k * 9 + t];
  element_traces<N, PHYS>(k, a.q, G, a.fmask, a.qf, tid, kWave);
}

// out[ch] = sum_n w[ch][n] q[elem[ch]][field[ch]][n]
template <int N, int PHYS>
__global__ void __launch_bounds__(256)
dg_record_kernel(int nch, const float* __restrict__ q, const int64_t* __restrict__ elem,
                 const int32_t* __restrict__ field, const float* __restrict__ w, float* __restrict__ out) {
  constexpr int NP = Deg<N>::NP, NF = Phys<PHYS>::NF;
  const int ch = blockIdx.x * 256 + threadIdx.x;
  if (ch >= nch) return;
  const float* qe = q + (elem[ch] * NF + field[ch]) * NP;
  const float* wc = w + static_cast<int64_t>(ch) * NP;
  float acc = 0.0f;
  for (int n = 0; n < NP; ++n) acc += wc[n] * qe[n];
  out[ch] = acc;
}

// One wavefront per element.  Every global load is issued up front (the
// element's accumulators, chi from the three adjoint states, r, the own and
// neighbour traces of all four faces); the mass products M r run on the
// matrix cores (M in 16x4 FP32 fragments, r from LDS, one column per field
// and, elastic, one for r_s11 + r_s22 + r_s33), the faces are processed
// together, one face node per lane, and the per-lane partial sums are added
// up through LDS.
template <int N, int PHYS>
__global__ void __launch_bounds__(kWave)
dg_grad_accum_kernel(const GradArgs a) {
  constexpr int NP = Deg<N>::NP, NFP = Deg<N>::NFP;
  constexpr int NF = Phys<PHYS>::NF, NT = Phys<PHYS>::NT, CB = Phys<PHYS>::CB;
  constexpr int NJ = (PHYS == 0) ? 2 : 6;      // jump vectors per face node
  constexpr int NACC = (PHYS == 0) ? 10 : 19;  // accumulators used
  constexpr int NQ = (PHYS == 0) ? 2 : 4;      // face quantities: gm (P, S), gp (P, S)
  constexpr int FIT = (4 * NFP + kWave - 1) / kWave;
  constexpr int MB = (NP + 15) / 16, KP = (NP + 3) / 4 * 4;  // fragments of M
  constexpr int NCOL = PHYS == 0 ? NF : NF + 1;               // columns of M r
  constexpr int NRED = PHYS == 0 ? 2 : 3;                     // volume sums before the face sums
  // r (NCOL columns, then zeros up to the last fragment's k), later the
  // per-lane partial sums [NACC][kWave + 1]
  constexpr int SR = NCOL * NP + 4, SRED = NACC * (kWave + 1);
  __shared__ float s_chi[NF * NP];
  __shared__ float s_r[SR > SRED ? SR : SRED];
  __shared__ float s_jump[4 * NJ * NFP];
  __shared__ double s_out[kGradAccStride];
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t base = k * NF * NP;
  double* acc = a.gacc + k * kGradAccStride;
  const double old = lane < NACC ? acc[lane] : 0.0;
  // every global read of the element issued together, at clamped addresses
  // (no load behind a branch): adjoint states and r, connectivity, own traces;
  // then, with the face-node permutation formed in registers, the neighbour
  // traces
  constexpr int NIT = (NF * NP + kWave - 1) / kWave;
  const float* p2 = a.c1 != 0.0f ? a.phi2 : a.phi1;  // read only where used
  const float* p3 = a.c2 != 0.0f ? a.phi3 : a.phi1;
  float x1[NIT], x2[NIT], x3[NIT], xr[NIT];
#pragma unroll
  for (int t = 0; t < NIT; ++t) {
    const int i = lane + t * kWave;
    const int64_t ic = base + (i < NF * NP ? i : 0);
    x1[t] = a.phi1[ic];
    x2[t] = p2[ic];
    x3[t] = p3[ic];
    xr[t] = a.r[ic];
  }
  int word[FIT];
  float own[FIT][NJ];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = lane + t * kWave;
    const int ic = i < 4 * NFP ? i : 0;
    const int f = ic / NFP, j = ic - f * NFP;
    word[t] = a.conn[k * 4 + f];
    const float* ow = a.tr + (k * 4 + f) * NT * NFP + j;
#pragma unroll
    for (int c = 0; c < NT; ++c) own[t][c] = ow[c * NFP];
  }
  int jn[FIT];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = lane + t * kWave;
    const int j = (i < 4 * NFP ? i : 0) % NFP;
    const int o = (word[t] & 7) == 7 ? 0 : (word[t] & 7);
    jn[t] = face_perm_node(N, o, j);
  }
  float nbv[FIT][NJ];
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = lane + t * kWave;
    const int ic = i < 4 * NFP ? i : 0;
    const int f = ic / NFP, j = ic - f * NFP;
    const bool wall = (word[t] & 7) == 7;
    const int64_t kn = wall ? k : static_cast<int64_t>(word[t] >> 5);
    const int fnb = wall ? f : (word[t] >> 3) & 3;
    const float* nb = a.tr + (kn * 4 + fnb) * NT * NFP + (wall ? j : jn[t]);
#pragma unroll
    for (int c = 0; c < NT; ++c) nbv[t][c] = nb[c * NFP];
  }
#pragma unroll
  for (int t = 0; t < NIT; ++t) {
    const int i = lane + t * kWave;
    if (i >= NF * NP) continue;
    s_chi[i] = a.c0 * x1[t] + a.c1 * x2[t] + a.c2 * x3[t];
    s_r[i] = xr[t];
  }
  float G[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) G[t] = a.geo[k * 9 + t];
  const float* cf = a.cf + k * CB;
  // jumps (halved differences, the step kernel's convention) of all faces
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = lane + t * kWave;
    if (i >= 4 * NFP) continue;
    const int f = i / NFP, j = i - f * NFP;
    const bool wall = (word[t] & 7) == 7;
    const float gw = (word[t] & 8) ? 0.0f : 1.0f;  // absorbing wall: zero exterior state
    float* sj = s_jump + f * NJ * NFP;
    if constexpr (PHYS == 0) {
      const float pM = own[t][0], vnM = own[t][1];
      const float pP = wall ? gw * pM : nbv[t][0];
      const float vnP = wall ? -gw * vnM : -nbv[t][1];
      const float jp = 0.5f * (pP - pM), jv = 0.5f * (vnP - vnM);
      sj[j] = jp - cf[4 + f] * jv;  // alpha, Z+ of this face
      sj[NFP + j] = jv;
    } else {
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        const float vM = own[t][ii], tM = own[t][3 + ii];
        const float vP = wall ? gw * vM : nbv[t][ii];
        const float tP = wall ? -gw * tM : -nbv[t][3 + ii];
        sj[ii * NFP + j] = 0.5f * (vP - vM);
        sj[(3 + ii) * NFP + j] = 0.5f * (tP - tM);
      }
    }
  }
  if (lane < 4) s_r[NCOL * NP + lane] = 0.0f;
  __syncthreads();
  if constexpr (PHYS == 1) {
    for (int m = lane; m < NP; m += kWave) s_r[NF * NP + m] = s_r[3 * NP + m] + s_r[4 * NP + m] + s_r[5 * NP + m];
    __syncthreads();
  }

  // ---- mass-weighted products of chi and r = A q ---------------------------
  // y = M [r_0 .. r_(NF-1) (, r_3 + r_4 + r_5)] node block by node block:
  // lane (kq, col) holds y[mb*16 + 4 kq + i][col], i < 4, and weighs it with
  // chi of the same node and field: acoustic p -> t0, v -> t1; elastic v ->
  // t0, s -> t1 (shear entries twice), the trace column -> t2
  float t0 = 0.f, t1 = 0.f, t2 = 0.f;
  {
    using mfma::floatx4;
    const int col = lane & 15, kq = lane >> 4;
    const int bcol = col < NCOL ? col : 0;
    const float bsel = col < NCOL ? 1.0f : 0.0f;
    const float* Mp = a.mass_pack + lane;
#pragma unroll 1
    for (int mb = 0; mb < MB; ++mb) {
      floatx4 y = floatx4{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < KP / 4; ++kk)
        y = mfma::mfma_f32(Mp[(mb * (KP / 4) + kk) * 64], bsel * s_r[bcol * NP + 4 * kk + kq], y);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = mb * 16 + 4 * kq + i;
        if (n >= NP || col >= NCOL) continue;
        if constexpr (PHYS == 0) {
          const float v = s_chi[col * NP + n] * y[i];
          if (col == 0)
            t0 += v;
          else
            t1 += v;
        } else {
          if (col < 3) {
            t0 += s_chi[col * NP + n] * y[i];
          } else if (col < 9) {
            t1 += (col < 6 ? 1.0f : 2.0f) * s_chi[col * NP + n] * y[i];
          } else {
            t2 += (s_chi[3 * NP + n] + s_chi[4 * NP + n] + s_chi[5 * NP + n]) * y[i];
          }
        }
      }
    }
  }

  // ---- face terms, one face node per lane -----------------------------------
  float nrm[4][3], fsc[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) face_normal(G, f, nrm[f], fsc[f]);
  float part[4][NQ];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[f][q] = 0.f;
#pragma unroll
  for (int t = 0; t < FIT; ++t) {
    const int i = lane + t * kWave;
    if (i >= 4 * NFP) continue;
    const int f = i / NFP, j = i - f * NFP;
    const float* sj = s_jump + f * NJ * NFP;
    float mj[NJ];  // face-mass images of the jumps at this face node
#pragma unroll
    for (int c = 0; c < NJ; ++c) mj[c] = 0.f;
    for (int jj = 0; jj < NFP; ++jj) {
      const float w = a.face_mass[jj * NFP + j];  // symmetric: contiguous across lanes
#pragma unroll
      for (int c = 0; c < NJ; ++c) mj[c] += w * sj[c * NFP + jj];
    }
    const int vn = a.fmask[f * NFP + j];
    // this item's face: select its normal with 0/1 weights (no dynamic register index)
    float n0 = 0.f, n1 = 0.f, n2 = 0.f;
#pragma unroll
    for (int ff = 0; ff < 4; ++ff) {
      const float s = static_cast<float>(f == ff);
      n0 += s * nrm[ff][0];
      n1 += s * nrm[ff][1];
      n2 += s * nrm[ff][2];
    }
    float q[NQ];
    if constexpr (PHYS == 0) {
      const float ZM = cf[2], ZP = cf[4 + f];
      const float kc = 2.0f / (ZM + ZP);
      const float yp = s_chi[vn];
      const float yvn = n0 * s_chi[NP + vn] + n1 * s_chi[2 * NP + vn] + n2 * s_chi[3 * NP + vn];
      const float at = mj[0], jvt = mj[1];
      q[0] = 0.5f * kc * kc * (-yp + ZP * yvn) * at;
      q[1] = -(yp + ZM * yvn) * (0.5f * kc * kc * at + kc * jvt);
    } else {
      const float ZpM = cf[3], ZsM = cf[4], ZpP = cf[8 + f], ZsP = cf[12 + f];
      const float kp = 2.0f / (ZpM + ZpP), ks = 2.0f / (ZsM + ZsP);
      const float nn[3] = {n0, n1, n2};
      float yv[3], Yn[3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) yv[ii] = s_chi[ii * NP + vn];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
        Yn[ii] = s_chi[(3 + voigt(ii, 0)) * NP + vn] * nn[0] + s_chi[(3 + voigt(ii, 1)) * NP + vn] * nn[1] +
                 s_chi[(3 + voigt(ii, 2)) * NP + vn] * nn[2];
      const float yvn = yv[0] * nn[0] + yv[1] * nn[1] + yv[2] * nn[2];
      const float Ynn = Yn[0] * nn[0] + Yn[1] * nn[1] + Yn[2] * nn[2];
      // face-mass images: jv (mj[0..2]), jt (mj[3..5])
      const float jvnt = mj[0] * nn[0] + mj[1] * nn[1] + mj[2] * nn[2];
      const float jsnnt = mj[3] * nn[0] + mj[4] * nn[1] + mj[5] * nn[2];
      const float apt = jsnnt + ZpP * jvnt, ast = jsnnt + ZsP * jvnt;
      float asvt[3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) asvt[ii] = mj[3 + ii] + ZsP * mj[ii];
      const float up = Ynn - ZpM * yvn, us = ZsM * yvn - Ynn;
      float w[3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) w[ii] = Yn[ii] - ZsM * yv[ii];
      const float wa = w[0] * asvt[0] + w[1] * asvt[1] + w[2] * asvt[2];
      const float base_s = ast * us + wa;
      const float yva = yv[0] * asvt[0] + yv[1] * asvt[1] + yv[2] * asvt[2];
      const float wj = w[0] * mj[0] + w[1] * mj[1] + w[2] * mj[2];
      q[0] = -0.5f * kp * kp * apt * up - kp * apt * yvn;        // gm, Zp
      q[1] = -0.5f * ks * ks * base_s + ks * (ast * yvn - yva);  // gm, Zs
      q[2] = -0.5f * kp * kp * apt * up + kp * jvnt * up;        // gp, Zp
      q[3] = -0.5f * ks * ks * base_s + ks * (jvnt * us + wj);   // gp, Zs
    }
#pragma unroll
    for (int ff = 0; ff < 4; ++ff) {
      const float s = static_cast<float>(f == ff);
#pragma unroll
      for (int c = 0; c < NQ; ++c) part[ff][c] += s * q[c];
    }
  }
  // ---- reductions and the accumulator update ---------------------------------
  // the partial sums of all lanes into LDS (the r region is free now), then
  // lane i < NACC adds up sum i: the volume sums, then face f's quantity c at
  // NRED + f NQ + c, stored to accumulator NRED + 4 c + f
  float* s_red = s_r;
  __syncthreads();
  s_red[0 * (kWave + 1) + lane] = t0;
  s_red[1 * (kWave + 1) + lane] = t1;
  if constexpr (PHYS == 1) s_red[2 * (kWave + 1) + lane] = t2;
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int c = 0; c < NQ; ++c) s_red[(NRED + f * NQ + c) * (kWave + 1) + lane] = part[f][c];
  __syncthreads();
  if (lane < NACC) {
    float v = 0.f;
#pragma unroll 8
    for (int i = 0; i < kWave; ++i) v += s_red[lane * (kWave + 1) + i];
    const double Jk = a.J[k];
    if (lane < NRED) {
      s_out[lane] = Jk * v;
    } else {
      const int f = (lane - NRED) / NQ, c = (lane - NRED) - f * NQ;
      float fs = 0.f;
#pragma unroll
      for (int ff = 0; ff < 4; ++ff) fs += (f == ff) ? fsc[ff] : 0.0f;
      s_out[NRED + 4 * c + f] = Jk * static_cast<double>(fs) * v;
    }
  }
  __syncthreads();
  if (lane < NACC) acc[lane] = old + s_out[lane];
}

template <int PHYS>
__global__ void __launch_bounds__(256)
dg_grad_finalize_kernel(int64_t K, const double* __restrict__ gacc, const int32_t* __restrict__ conn,
                        const float* __restrict__ coef, float* __restrict__ grad) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (k >= K) return;
  const double* acc = gacc + k * kGradAccStride;
  if constexpr (PHYS == 0) {
    double dZ = 0.0;
    for (int f = 0; f < 4; ++f) {
      dZ += acc[2 + f];
      const int w = conn[4 * k + f];
      if ((w & 7) == 7) {
        dZ += acc[6 + f];
      } else {
        const int64_t kn = static_cast<int64_t>(w >> 5);
        const int fn = (w >> 3) & 3;
        dZ += gacc[kn * kGradAccStride + 6 + fn];
      }
    }
    const double rho = coef[2 * k], c = coef[2 * k + 1];
    const double ap = acc[0], av = acc[1];
    grad[2 * k] = static_cast<float>(ap / (rho * rho * c * c) + av + c * dZ);
    grad[2 * k + 1] = static_cast<float>(2.0 * ap / (rho * c * c * c) + rho * dZ);
  } else {
    double dZp = 0.0, dZs = 0.0;
    for (int f = 0; f < 4; ++f) {
      dZp += acc[3 + f];
      dZs += acc[7 + f];
      const int w = conn[4 * k + f];
      if ((w & 7) == 7) {
        dZp += acc[11 + f];
        dZs += acc[15 + f];
      } else {
        const int64_t kn = static_cast<int64_t>(w >> 5);
        const int fn = (w >> 3) & 3;
        dZp += gacc[kn * kGradAccStride + 11 + fn];
        dZs += gacc[kn * kGradAccStride + 15 + fn];
      }
    }
    const double rho = coef[3 * k], lam = coef[3 * k + 1], mu = coef[3 * k + 2];
    const double av = acc[0], as = acc[1], at = acc[2];
    const double l2m = lam + 2.0 * mu, d3 = 3.0 * lam + 2.0 * mu;
    const double beta = lam / d3;
    const double Zp = sqrt(rho * l2m), Zs = sqrt(rho * mu);
    grad[3 * k] = static_cast<float>(av + l2m / (2.0 * Zp) * dZp + mu / (2.0 * Zs) * dZs);
    grad[3 * k + 1] = static_cast<float>(at / (d3 * d3) + rho / (2.0 * Zp) * dZp);
    grad[3 * k + 2] = static_cast<float>((as - beta * at) / (2.0 * mu * mu) - lam * at / (mu * d3 * d3) +
                                         rho / Zp * dZp + rho / (2.0 * Zs) * dZs);
  }
}

__global__ void __launch_bounds__(256) dg_fill_f64_kernel(int64_t n, double* __restrict__ p) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void __launch_bounds__(256) dg_fill_f32_kernel(int64_t n, float* __restrict__ p) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

template <int N, int PHYS>
hipError_t inject_impl(const InjectArgs& a, hipStream_t s) {
  if (a.nelem <= 0) return hipSuccess;
  hipLaunchKernelGGL((dg_inject_kernel<N, PHYS>), dim3(static_cast<unsigned>(a.nelem)), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

template <int N, int PHYS>
hipError_t record_impl(int nch, const float* q, const int64_t* elem, const int32_t* field, const float* w,
                       float* out, hipStream_t s) {
  if (nch <= 0) return hipSuccess;
  hipLaunchKernelGGL((dg_record_kernel<N, PHYS>), dim3((nch + 255) / 256), dim3(256), 0, s, nch, q, elem, field, w,
                     out);
  return hipGetLastError();
}

template <int N, int PHYS>
hipError_t grad_impl(const GradArgs& a, hipStream_t s) {
  if (a.K <= 0) return hipSuccess;
  if (a.K > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dg_grad_accum_kernel<N, PHYS>), dim3(static_cast<unsigned>(a.K)), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

}  // namespace

#define DGW_DISPATCH(CALL)                                                                            \
  if (physics == 0) {                                                                                 \
    switch (N) {                                                                                      \
      case 1: return CALL(1, 0); case 2: return CALL(2, 0); case 3: return CALL(3, 0);               \
      case 4: return CALL(4, 0); case 5: return CALL(5, 0); case 6: return CALL(6, 0);               \
      case 7: return CALL(7, 0); case 8: return CALL(8, 0);                                          \
    }                                                                                                 \
  } else {                                                                                            \
    switch (N) {                                                                                      \
      case 1: return CALL(1, 1); case 2: return CALL(2, 1); case 3: return CALL(3, 1);               \
      case 4: return CALL(4, 1); case 5: return CALL(5, 1); case 6: return CALL(6, 1);               \
      case 7: return CALL(7, 1); case 8: return CALL(8, 1);                                          \
    }                                                                                                 \
  }                                                                                                   \
  return hipErrorInvalidValue;

hipError_t launch_inject(int physics, int N, const InjectArgs& a, hipStream_t s) {
#define CALL(n, p) inject_impl<n, p>(a, s)
  DGW_DISPATCH(CALL)
#undef CALL
}

hipError_t launch_record(int physics, int N, int nch, const float* q, const int64_t* elem, const int32_t* field,
                         const float* w, float* out, hipStream_t s) {
#define CALL(n, p) record_impl<n, p>(nch, q, elem, field, w, out, s)
  DGW_DISPATCH(CALL)
#undef CALL
}

hipError_t launch_grad_accum(int physics, int N, const GradArgs& a, hipStream_t s) {
#define CALL(n, p) grad_impl<n, p>(a, s)
  DGW_DISPATCH(CALL)
#undef CALL
}

#undef DGW_DISPATCH

hipError_t launch_grad_finalize(int physics, int64_t K, const double* gacc, const int32_t* conn, const float* coef,
                                float* grad, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  const int64_t blocks = (K + 255) / 256;
  if (physics == 0)
    hipLaunchKernelGGL(dg_grad_finalize_kernel<0>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, K, gacc,
                       conn, coef, grad);
  else
    hipLaunchKernelGGL(dg_grad_finalize_kernel<1>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, K, gacc,
                       conn, coef, grad);
  return hipGetLastError();
}

hipError_t launch_fill_zero_f64(int64_t n, double* p, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dg_fill_f64_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, n, p);
  return hipGetLastError();
}

hipError_t launch_fill_zero_f32(int64_t n, float* p, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dg_fill_f32_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, n, p);
  return hipGetLastError();
}

}  // namespace dgw
