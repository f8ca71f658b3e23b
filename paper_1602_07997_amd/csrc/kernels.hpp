// Launch interface between the C ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace dgw {

// Per-step kernel arguments.  All pointers are device pointers.
struct StepArgs {
  int64_t K;             // end (exclusive) of the element range of the launch
  int64_t e_begin;       // first element of the range (0: the whole mesh)
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
  const float* Dpack;    // FP32 MFMA: D_j in 16x4 fragment order [3][MB][KP/4][64]
  const float* Lpack;    // FP32 MFMA: LIFT [MB][KL/4][64] (acoustic per face, elastic merged)
  const uint16_t* D16h;  // 16-bit MFMA: D_j split hi / lo, [3][MB][KP/KS][64][KS/4] (KS = 32 acoustic, 16 elastic)
  const uint16_t* D16l;
  const uint16_t* L16h;  // 16-bit MFMA: LIFT split hi / lo [MB][KL/KS][64][KS/4], K as in Lpack
  const uint16_t* L16l;
  float c0, c1, c2;      // dt*a1, dt*a2, dt*a3
  int mode;              // 0: AB3 step, 1: right-hand side only (r_out = r(q_in))
  int xcd_remap;         // 1: give each XCD a contiguous range of tiles (0: launch order)
  int tail_split;        // 1: the MFMA launchers may split a last, partial round of tiles
  // set by those launchers: from tile split_from on, each tile is shared by
  // split_parts workgroups, each taking a contiguous range of the tile's
  // (node block, element block) pairs (split_parts <= 1: no split)
  int split_parts;
  int64_t split_from;
};

constexpr int kStepMode = 0;
constexpr int kRhsMode = 1;

// Number of coefficient words per element in `cf`.
int coef_block(int physics);
// Number of caller coefficients per element (2 acoustic, 3 elastic, 22
// anisotropic).
inline int num_coefficients(int physics) { return physics == 0 ? 2 : (physics == 1 ? 3 : 22); }
// Number of traces per face node (2 acoustic, 6 elastic and anisotropic).
int num_traces(int physics);

// Kernel variants of the step.
constexpr int kVariantValu = 0;      // node per thread, VALU contractions
constexpr int kVariantMfma = 1;      // element tiles, FP32 MFMA contractions
constexpr int kVariantMfmaBf16 = 2;  // BF16 MFMA, three split products, FP32 accumulation
constexpr int kVariantMfmaF16 = 3;   // FP16 MFMA, three split products, FP32 accumulation
constexpr int kVariantElem = 4;      // element per thread (acoustic N = 1, 2; elastic N = 1)
constexpr int kVariantMfmaWide = 5;  // FP32 MFMA, the alternative acoustic tile shape
constexpr int kNumVariants = 6;
bool variant_supported(int physics, int N, int variant);

// Fragment packing of the MFMA variants: node blocks MB, padded volume K (KP)
// and LIFT K (KL), k per instruction KS, elements per tile E.
// KF > 0: the LIFT is packed per face, face f's columns at K = f*KF .. (the
// acoustic kernel); KF = 0: merged faces, K = 4 Nfp padded (the elastic kernel).
struct MfmaPacking {
  int MB = 0, KP = 0, KL = 0, KS = 0, E = 0, KF = 0;
};
int mfma_precision(int variant);  // 0 FP32, 1 BF16, 2 FP16, -1 not an MFMA variant
MfmaPacking mfma_packing(int physics, int N, int variant);
MfmaPacking mfma_elastic_packing(int N, int variant);
hipError_t launch_step_mfma(int physics, int N, int variant, const StepArgs& a, hipStream_t s);
// Element-per-thread kernels (N = 1, 2).
bool elem_supported(int physics, int N);
int elem_tile_elements();
hipError_t launch_step_elem(int physics, int N, const StepArgs& a, hipStream_t s);
hipError_t launch_step_batch_elem(int physics, int N, const StepArgs* args, const int2* work, int64_t ntiles,
                                  int phase, hipStream_t s);
// Elastic MFMA kernels (512-thread workgroups); physics 1 isotropic (every
// precision), 2 anisotropic (FP32 products only).
int mfma_elastic_tile_elements(int N, int variant);
hipError_t launch_step_mfma_elastic(int physics, int N, int variant, const StepArgs& a, hipStream_t s);
hipError_t launch_step_batch_mfma_elastic(int physics, int N, int variant, const StepArgs* args, const int2* work,
                                          int64_t ntiles, int phase, hipStream_t s);
hipError_t launch_step_batch_mfma(int physics, int N, int variant, const StepArgs* args, const int2* work,
                                  int64_t ntiles, int phase, hipStream_t s);

hipError_t launch_step(int physics, int N, int variant, const StepArgs& a, hipStream_t s);

// Batched stepping: per-member arguments for kBatchPhases consecutive steps
// (the ring slot rotates with period 3 and the trace buffer with period 2).
constexpr int kBatchPhases = 6;
int tile_elements(int physics, int N, int variant);  // elements per workgroup tile
int64_t tiles_for(int physics, int N, int variant, int64_t K);
hipError_t launch_step_batch(int physics, int N, int variant, const StepArgs* args, const int2* work,
                             int64_t ntiles, int phase, hipStream_t s);
// Point injection: for each distinct element elem[u], entries
// e in [start[u], start[u+1]) add a_e * vec[e][:] to q[elem[u]][field[e]][:],
// a_e = amp when chan[e] < 0, else traces[chan[e]] - data[chan[e]]; the
// element's own traces in qf are then rewritten.
struct InjectArgs {
  int nelem;
  float* q;
  float* qf;
  const float* geo;
  const int32_t* fmask;
  const int64_t* elem;    // [nelem]
  const int32_t* start;   // [nelem + 1]
  const int32_t* field;   // [entries]
  const int32_t* chan;    // [entries]
  const float* vec;       // [entries][Np]
  float amp;
  const float* traces;    // receiver values of this step (chan >= 0 entries)
  const float* data;      // data of this step
};
hipError_t launch_inject(int physics, int N, const InjectArgs& a, hipStream_t s);
// out[ch] = w[ch] . q[elem[ch]][field[ch]][:]
hipError_t launch_record(int physics, int N, int nch, const float* q, const int64_t* elem, const int32_t* field,
                         const float* w, float* out, hipStream_t s);

// Per-step accumulation of the coefficient gradient (see kernels_adjoint.hip).
constexpr int kGradAccStride = 20;  // float64 accumulators per element
struct GradArgs {
  int64_t K;
  const float* phi1;      // phi_{m+1}, phi_{m+2}, phi_{m+3}
  const float* phi2;
  const float* phi3;
  float c0, c1, c2;       // chi_m = c0 phi1 + c1 phi2 + c2 phi3
  const float* r;         // A q_m  [K][NF][Np]
  const float* tr;        // traces of q_m [K][4][NT][Nfp]
  const float* geo;
  const float* cf;
  const int32_t* conn;
  const int32_t* fmask;
  const int32_t* perm;
  const float* mass_pack; // M as 16x4 FP32 fragments [MB][KP/4][64] (MB = ceil(Np/16), KP = Np rounded up to 4)
  const float* face_mass; // [Nfp][Nfp]
  const double* J;        // [K]
  double* gacc;           // [K][kGradAccStride]
};
hipError_t launch_grad_accum(int physics, int N, const GradArgs& a, hipStream_t s);
hipError_t launch_grad_finalize(int physics, int64_t K, const double* gacc, const int32_t* conn, const float* coef,
                                float* grad, hipStream_t s);
hipError_t launch_fill_zero_f64(int64_t n, double* p, hipStream_t s);
// flag[0] = smallest i < n with x[i] not positive and finite, or -1.
hipError_t launch_first_nonpositive(int64_t n, const float* x, int* flag, hipStream_t s);
// Anisotropic coefficients [K][22]: flag[0] = smallest element whose density
// is not positive and finite or whose stiffness is not finite and positive
// definite, or -1.
hipError_t launch_first_bad_stiffness(int64_t K, const float* coef, int* flag, hipStream_t s);
hipError_t launch_fill_zero_f32(int64_t n, float* p, hipStream_t s);

hipError_t launch_traces(int physics, int N, int64_t K, const float* q, const float* geo,
                         const int32_t* fmask, float* qf, hipStream_t s);
// Traces of q + c0 r0 + c1 r1 + c2 r2 for the elements list[0 .. nlist)
// (terms with a zero coefficient are not read).
hipError_t launch_trace_comb(int physics, int N, int64_t nlist, const int32_t* list, const float* q,
                             const float* r0, const float* r1, const float* r2, float c0, float c1, float c2,
                             const float* geo, const int32_t* fmask, float* qf, hipStream_t s);
hipError_t launch_coef_prep(int physics, int64_t K, const float* coef, const int32_t* conn,
                            float* cf, hipStream_t s);
// Energy: partial sums per block into `partial` (size energy_blocks), then
// the total into out[0].
int64_t energy_blocks(int physics, int N, int64_t K);
hipError_t launch_energy(int physics, int N, int64_t K, const float* q, const float* coef,
                         const double* J, const double* mass, double* partial, double* out,
                         hipStream_t s);
// Partial sums of the allocation-free energy entry point live in a static
// device array of this many doubles (one copy per device, in kernels.hip).
constexpr int64_t kStaticEnergyPartials = 16384;
// Device address of that array on `device` (looked up once per device, with
// the device current, and cached).
hipError_t static_energy_partials(int device, double** ptr);

}  // namespace dgw
