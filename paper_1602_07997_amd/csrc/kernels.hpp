// Launch interface between the C ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace dgw {

// Per-step kernel arguments.  All pointers are device pointers.
struct StepArgs {
  int64_t K;
  const float* q_in;     // fields read this step [K][NF][NP]
  float* q_out;          // fields written (step mode; may equal q_in)
  const float* r1;       // r^{m-1} (read when c1 != 0)
  const float* r2;       // r^{m-2} (read when c2 != 0)
  float* r_out;          // r^m
  const float* qf_in;    // neighbour traces [K][4][NT][NFP]
  float* qf_out;         // own traces of the updated fields (step mode)
  const float* geo;      // [K][9] G[i][j] = d r_j / d x_i
  const float* cf;       // [K][CB] derived coefficients (see coef_prep)
  const int32_t* conn;   // [K][4] packed (neighbour<<5 | face<<3 | orient), orient 7 = wall
  const float* DT;       // [3][NP][NP] DT[j][m][n] = D_j[n][m]
  const float* LT;       // [4*NFP][NP] LT[fm][n] = L[n][fm]
  const int32_t* fmask;  // [4][NFP]
  const int32_t* perm;   // [6][NFP]
  const int32_t* nodeface;  // [NP][3] face slots f*NFP+j containing node n, -1 padded
  const float* Dpack;    // MFMA variant: D_j in 16x4 fragment order [3][MB][KP/4][64]
  const float* Lpack;    // MFMA variant: LIFT, face blocks padded to NFPP, [MB][4*NFPP/4][64]
  float c0, c1, c2;      // dt*a1, dt*a2, dt*a3
  int mode;              // 0: AB3 step, 1: right-hand side only (r_out = r(q_in))
  int xcd_remap;         // map consecutive tiles onto one XCD
};

constexpr int kStepMode = 0;
constexpr int kRhsMode = 1;

// Number of coefficient words per element in `cf`.
int coef_block(int physics);
// Number of traces per face node (2 acoustic, 6 elastic).
int num_traces(int physics);

// Kernel variants of the step.
constexpr int kVariantValu = 0;  // node per thread, VALU contractions
constexpr int kVariantMfma = 1;  // element tiles, FP32 MFMA contractions
bool variant_supported(int physics, int N, int variant);

// Fragment-order packing used by the MFMA variant (host side).
int mfma_mblocks(int N);        // ceil(Np / 16)
int mfma_kpad(int N);           // Np rounded up to a multiple of 4
int mfma_face_pad(int N);       // Nfp rounded up to a multiple of 4

hipError_t launch_step(int physics, int N, int variant, const StepArgs& a, hipStream_t s);

// Batched stepping: per-member arguments for kBatchPhases consecutive steps
// (the ring slot rotates with period 3 and the trace buffer with period 2).
constexpr int kBatchPhases = 6;
int tile_elements(int physics, int N, int variant);  // elements per workgroup tile
int64_t tiles_for(int physics, int N, int variant, int64_t K);
int mfma_tile_elements(int N);
hipError_t launch_step_batch(int physics, int N, int variant, const StepArgs* args, const int2* work,
                             int64_t ntiles, int phase, hipStream_t s);
hipError_t launch_traces(int physics, int N, int64_t K, const float* q, const float* geo,
                         const int32_t* fmask, float* qf, hipStream_t s);
hipError_t launch_coef_prep(int physics, int64_t K, const float* coef, const int32_t* conn,
                            float* cf, hipStream_t s);
// Energy: partial sums per block into `partial` (size energy_blocks), then
// the total into out[0].
int64_t energy_blocks(int physics, int N, int64_t K);
hipError_t launch_energy(int physics, int N, int64_t K, const float* q, const float* coef,
                         const double* J, const double* mass, double* partial, double* out,
                         hipStream_t s);

}  // namespace dgw
