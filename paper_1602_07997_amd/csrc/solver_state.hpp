// Host-side state of a dg_solver (shared by the C ABI translation units).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <sstream>
#include <vector>

#include "dg_internal.hpp"
#include "dgwave.h"
#include "kernels.hpp"

// Return DG_E_HIP with the failing call and HIP's message as the error text.
#define DG_HIP(call)                                   \
  do {                                                 \
    hipError_t err_ = (call);                          \
    if (err_ != hipSuccess) {                          \
      std::ostringstream os_;                          \
      os_ << #call << ": " << hipGetErrorString(err_); \
      dgw::set_error(os_.str());                       \
      return DG_E_HIP;                                 \
    }                                                  \
  } while (0)

// Every device pointer below points into the caller's workspace (see
// dg_workspace_bytes); the solver owns none of them.
struct dg_solver {
  int physics = 0, N = 0, Np = 0, Nfp = 0, NF = 0, NT = 0, CB = 0, ncoef = 0;
  int64_t K = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  float* q = nullptr;
  float* r[3] = {nullptr, nullptr, nullptr};
  float* qf[2] = {nullptr, nullptr};
  float* qf_tmp = nullptr;
  float* geo = nullptr;
  float* cf = nullptr;
  float* coef = nullptr;
  float* DT = nullptr;
  float* LT = nullptr;
  int32_t* conn = nullptr;
  int32_t* fmask = nullptr;
  int32_t* perm = nullptr;
  int32_t* nodeface = nullptr;
  double* J = nullptr;
  double* mass = nullptr;
  double* partial = nullptr;
  double* e_out = nullptr;
  int* flag = nullptr;
  int32_t* iface = nullptr;  // [K] slow elements with a fast neighbour (two-rate stepping)
  int64_t k_fast = 0;        // elements [0, k_fast) take two half steps (0: single rate)
  int64_t n_iface = 0;
  int cur = 0;     // trace buffer holding the traces of q
  int64_t m = 0;   // step index
  bool have_coef = false, have_fields = false;
  uint64_t coef_gen = 0;  // bumped by every dg_set_coefficients
  // energy growth check: the last dg_energy result and the step index it
  // belongs to (-1: none since the fields were set); growth tolerance
  double e_prev = -1.0;
  int64_t e_prev_m = -1;
  double e_tol = 1e-4;
  // tiles in launch order (0), or each XCD given a contiguous range of tiles
  // (1, environment DGWAVE_XCD_REMAP=1): launch order measured 1-5 % faster
  // on the ~2M-node meshes at every degree
  int xcd_remap = 0;
  // a last, partial round of MFMA workgroups split by tile pairs
  // over more compute units (1; environment DGWAVE_TAIL_SPLIT=0 turns it off)
  int tail_split = 1;
  int variant = 0;
  float* Dpack = nullptr;
  float* Lpack = nullptr;
  uint16_t* D16[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [bf16, f16][hi, lo]
  uint16_t* L16[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  std::vector<double> elem_xyz;  // host copy for node coordinates
  std::vector<int32_t> conn_h;   // host copy of the packed face words
};

namespace dgw {

// Step-size coefficients dt*(a1, a2, a3) of eq. (4) for step m, with the
// forward-Euler and two-step Adams-Bashforth start-up.
inline void ab_coefficients(int64_t m, double dt, float* c) {
  double a1, a2, a3;
  if (m == 0) {
    a1 = 1.0; a2 = 0.0; a3 = 0.0;
  } else if (m == 1) {
    a1 = 1.5; a2 = -0.5; a3 = 0.0;
  } else {
    a1 = 23.0 / 12.0; a2 = -16.0 / 12.0; a3 = 5.0 / 12.0;
  }
  c[0] = static_cast<float>(dt * a1);
  c[1] = static_cast<float>(dt * a2);
  c[2] = static_cast<float>(dt * a3);
}

// Arguments shared by every step of a solver (operators, geometry, tables).
StepArgs base_args(const dg_solver* s);

// Arguments of step m of a solver whose trace buffer `cur` holds the traces
// of q^m: ring slot of r^m = m mod 3, traces read from qf[cur], written to
// qf[cur ^ 1].
StepArgs step_args(const dg_solver* s, int64_t m, int cur, double dt);

}  // namespace dgw
