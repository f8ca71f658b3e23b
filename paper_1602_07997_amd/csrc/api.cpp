// C ABI of the dgwave library: set-up on the host, hot path on the GPU.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "dg_internal.hpp"
#include "dgwave.h"
#include "kernels.hpp"
#include "mfma_pack.hpp"
#include "solver_state.hpp"

namespace dgw {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }
const char* last_error() { return g_error.c_str(); }

}  // namespace dgw

using dgw::set_error;


namespace {

template <class T>
hipError_t dev_alloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T) + (count == 0 ? 16 : 0));
}

dg_status check_solver(const dg_solver* s) {
  if (!s) {
    set_error("null solver");
    return DG_E_ARG;
  }
  return DG_OK;
}

void free_all(dg_solver* s) {
  void* ptrs[] = {s->q,  s->r[0], s->r[1], s->r[2], s->qf[0], s->qf[1], s->qf_tmp, s->geo,
                  s->cf, s->coef, s->DT,   s->LT,   s->conn,  s->fmask, s->perm,   s->nodeface, s->J,
                  s->mass, s->partial, s->e_out, s->flag, s->Dpack, s->Lpack};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int v = 0; v < 2; ++v)
    for (int h = 0; h < 2; ++h) {
      if (s->D16[v][h]) (void)hipFree(s->D16[v][h]);
      if (s->L16[v][h]) (void)hipFree(s->L16[v][h]);
    }
}

size_t field_count(const dg_solver* s) { return static_cast<size_t>(s->K) * s->NF * s->Np; }
size_t trace_count(const dg_solver* s) { return static_cast<size_t>(s->K) * 4 * s->NT * s->Nfp; }

}  // namespace

namespace dgw {

StepArgs base_args(const dg_solver* s) {
  StepArgs a{};
  a.K = s->K;
  a.geo = s->geo;
  a.cf = s->cf;
  a.conn = s->conn;
  a.DT = s->DT;
  a.LT = s->LT;
  a.fmask = s->fmask;
  a.perm = s->perm;
  a.nodeface = s->nodeface;
  a.Dpack = s->Dpack;
  a.Lpack = s->Lpack;
  const int p16 = s->variant == kVariantMfmaF16 ? 1 : 0;
  a.D16h = s->D16[p16][0];
  a.D16l = s->D16[p16][1];
  a.L16h = s->L16[p16][0];
  a.L16l = s->L16[p16][1];
  a.xcd_remap = s->xcd_remap;
  return a;
}

StepArgs step_args(const dg_solver* s, int64_t m, int cur, double dt) {
  StepArgs a = base_args(s);
  a.mode = kStepMode;
  float c[3];
  ab_coefficients(m, dt, c);
  a.c0 = c[0];
  a.c1 = c[1];
  a.c2 = c[2];
  a.q_in = s->q;
  a.q_out = s->q;
  a.r_out = s->r[m % 3];
  a.r1 = s->r[(m + 2) % 3];
  a.r2 = s->r[(m + 1) % 3];
  a.qf_in = s->qf[cur];
  a.qf_out = s->qf[cur ^ 1];
  return a;
}

}  // namespace dgw

extern "C" {

int dg_abi_version(void) { return 1; }

const char* dg_last_error(void) { return dgw::last_error(); }

int dg_num_fields(int physics) {
  if (physics == DG_ACOUSTIC) return 4;
  if (physics == DG_ELASTIC) return 9;
  return -1;
}

dg_status dg_ref_sizes(int order, int* Np, int* Nfp) {
  if (order < 1 || order > dgw::kMaxOrder) {
    set_error("order must be in [1, 8]");
    return DG_E_UNSUPPORTED;
  }
  if (Np) *Np = dgw::num_nodes(order);
  if (Nfp) *Nfp = dgw::num_face_nodes(order);
  return DG_OK;
}

dg_status dg_reference_operators(int order, double* nodes, double* D, double* mass, double* lift,
                                 int32_t* fmask) {
  const dgw::RefElement* ref = nullptr;
  try {
    ref = dgw::reference_element(order);
  } catch (const std::exception& e) {
    set_error(e.what());
    return DG_E_ARG;
  }
  if (!ref) {
    set_error("order must be in [1, 8]");
    return DG_E_UNSUPPORTED;
  }
  if (nodes) std::memcpy(nodes, ref->nodes.data(), ref->nodes.size() * sizeof(double));
  if (D) std::memcpy(D, ref->D.data(), ref->D.size() * sizeof(double));
  if (mass) std::memcpy(mass, ref->mass.data(), ref->mass.size() * sizeof(double));
  if (lift) std::memcpy(lift, ref->lift.data(), ref->lift.size() * sizeof(double));
  if (fmask) std::memcpy(fmask, ref->fmask.data(), ref->fmask.size() * sizeof(int32_t));
  return DG_OK;
}

dg_status dg_face_permutations(int order, int32_t* perm) {
  const dgw::RefElement* ref = dgw::reference_element(order);
  if (!ref) {
    set_error("order must be in [1, 8]");
    return DG_E_UNSUPPORTED;
  }
  if (!perm) {
    set_error("null perm");
    return DG_E_ARG;
  }
  std::memcpy(perm, ref->perm.data(), ref->perm.size() * sizeof(int32_t));
  return DG_OK;
}

dg_status dg_mesh_connectivity(int64_t K, const int64_t* elem_topo, int64_t* e2e, int32_t* e2f,
                               int32_t* orient) {
  if (K <= 0 || !elem_topo || !e2e || !e2f || !orient) {
    set_error("dg_mesh_connectivity: bad arguments");
    return DG_E_ARG;
  }
  std::string msg = dgw::connect_faces(K, elem_topo, e2e, e2f, orient);
  if (!msg.empty()) {
    set_error(msg);
    return DG_E_MESH;
  }
  return DG_OK;
}

dg_status dg_create(int physics, int order, int64_t K, const double* elem_xyz, const int64_t* elem_topo,
                    void* stream, dg_solver** out) {
  if (!out) {
    set_error("null output handle");
    return DG_E_ARG;
  }
  *out = nullptr;
  if (physics != DG_ACOUSTIC && physics != DG_ELASTIC) {
    set_error("unknown physics");
    return DG_E_ARG;
  }
  const dgw::RefElement* ref = (order >= 1 && order <= dgw::kMaxOrder) ? dgw::reference_element(order) : nullptr;
  if (!ref) {
    set_error("order must be in [1, 8]");
    return DG_E_UNSUPPORTED;
  }
  if (K <= 0 || K >= (int64_t(1) << 26) || !elem_xyz || !elem_topo) {
    set_error("K must be in [1, 2^26) and the mesh arrays non-null");
    return DG_E_ARG;
  }
  const int Np = ref->Np, Nfp = ref->Nfp;

  // ---- host geometry (float64) ----
  std::vector<float> geo(static_cast<size_t>(K) * 9);
  std::vector<double> J(K);
  for (int64_t k = 0; k < K; ++k) {
    const double* x = elem_xyz + 12 * k;
    double F[3][3];  // F[i][j] = d x_i / d r_j
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) F[i][j] = 0.5 * (x[3 * (j + 1) + i] - x[i]);
    const double det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                       F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                       F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    if (!(det > 0.0) || !std::isfinite(det)) {
      std::ostringstream os;
      os << "element " << k << " has non-positive Jacobian " << det;
      set_error(os.str());
      return DG_E_MESH;
    }
    J[k] = det;
    // G = F^{-T}: G[i][j] = d r_j / d x_i = cofactor(F)[i][j] / det
    double C[3][3];
    C[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
    C[0][1] = -(F[1][0] * F[2][2] - F[1][2] * F[2][0]);
    C[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
    C[1][0] = -(F[0][1] * F[2][2] - F[0][2] * F[2][1]);
    C[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
    C[1][2] = -(F[0][0] * F[2][1] - F[0][1] * F[2][0]);
    C[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
    C[2][1] = -(F[0][0] * F[1][2] - F[0][2] * F[1][0]);
    C[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) geo[9 * k + 3 * i + j] = static_cast<float>(C[i][j] / det);
  }

  // ---- connectivity ----
  std::vector<int64_t> e2e(4 * K);
  std::vector<int32_t> e2f(4 * K), orient(4 * K);
  std::string msg = dgw::connect_faces(K, elem_topo, e2e.data(), e2f.data(), orient.data());
  if (!msg.empty()) {
    set_error(msg);
    return DG_E_MESH;
  }
  std::vector<int32_t> conn(4 * K);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int64_t s = 4 * k + f;
      if (e2e[s] < 0) {
        conn[s] = static_cast<int32_t>((k << 5) | 7);
        continue;
      }
      const int64_t kn = e2e[s];
      const int fn = e2f[s], o = orient[s];
      // paired faces must coincide up to a translation (zero, or the period)
      const double* x = elem_xyz + 12 * k;
      const double* xn = elem_xyz + 12 * kn;
      double d0[3];
      for (int p = 0; p < 3; ++p) {
        const int v = dgw::kFaceVerts[f][p];
        const int vn = dgw::kFaceVerts[fn][dgw::kFacePerms[o][p]];
        for (int c = 0; c < 3; ++c) {
          const double d = x[3 * v + c] - xn[3 * vn + c];
          if (p == 0) d0[c] = d;
          else if (std::fabs(d - d0[c]) > 1e-9 * (1.0 + std::fabs(d0[c]))) {
            std::ostringstream os;
            os << "faces " << k << ":" << f << " and " << kn << ":" << fn
               << " share vertex ids but not coordinates";
            set_error(os.str());
            return DG_E_MESH;
          }
        }
      }
      conn[s] = static_cast<int32_t>((kn << 5) | (static_cast<int64_t>(fn) << 3) | o);
    }

  // ---- MFMA fragment packing (FP32, and the BF16 / FP16 hi + lo splits) ----
  std::vector<float> Dpack, Lpack;
  std::vector<uint16_t> D16[2][2], L16[2][2];  // [bf16, f16][hi, lo]
  {
    const dgw::MfmaPacking p32 = dgw::mfma_packing(physics, order, dgw::kVariantMfma);
    const dgw::ColMap c32 = dgw::face_block_columns(Nfp, p32.KF);
    for (int j = 0; j < 3; ++j) dgw::pack_fp32(ref->D.data() + static_cast<size_t>(j) * Np * Np, Np, Np, p32.MB, p32.KP, Dpack);
    dgw::pack_fp32(ref->lift.data(), Np, 4 * Nfp, p32.MB, p32.KL, Lpack, p32.KF > 0 ? &c32 : nullptr);
    const int vars[2] = {dgw::kVariantMfmaBf16, dgw::kVariantMfmaF16};
    for (int v = 0; v < 2; ++v) {
      const dgw::MfmaPacking p16 = dgw::mfma_packing(physics, order, vars[v]);
      const dgw::ColMap c16 = dgw::face_block_columns(Nfp, p16.KF);
      const int kw = p16.KS / 4;  // k per lane group: 4 (16x16x16) or 8 (16x16x32)
      for (int j = 0; j < 3; ++j)
        dgw::pack_split16(ref->D.data() + static_cast<size_t>(j) * Np * Np, Np, Np, p16.MB, p16.KP, kw, v == 0,
                          D16[v][0], D16[v][1]);
      dgw::pack_split16(ref->lift.data(), Np, 4 * Nfp, p16.MB, p16.KL, kw, v == 0, L16[v][0], L16[v][1],
                        p16.KF > 0 ? &c16 : nullptr);
    }
  }

  // ---- operators in the kernels' layouts (float32) ----
  std::vector<float> DT(3 * static_cast<size_t>(Np) * Np), LT(static_cast<size_t>(4) * Nfp * Np);
  for (int j = 0; j < 3; ++j)
    for (int n = 0; n < Np; ++n)
      for (int mm = 0; mm < Np; ++mm)
        DT[(static_cast<size_t>(j) * Np + mm) * Np + n] = static_cast<float>(ref->D[(static_cast<size_t>(j) * Np + n) * Np + mm]);
  for (int n = 0; n < Np; ++n)
    for (int fm = 0; fm < 4 * Nfp; ++fm)
      LT[static_cast<size_t>(fm) * Np + n] = static_cast<float>(ref->lift[static_cast<size_t>(n) * 4 * Nfp + fm]);

  dg_solver* s = new dg_solver();
  s->physics = physics;
  s->N = order;
  s->Np = Np;
  s->Nfp = Nfp;
  s->NF = dg_num_fields(physics);
  s->NT = dgw::num_traces(physics);
  s->CB = dgw::coef_block(physics);
  s->ncoef = physics == DG_ACOUSTIC ? 2 : 3;
  s->K = K;
  s->stream = static_cast<hipStream_t>(stream);
  s->elem_xyz.assign(elem_xyz, elem_xyz + 12 * K);
  (void)hipGetDevice(&s->device);
  if (const char* env = std::getenv("DGWAVE_XCD_REMAP")) s->xcd_remap = (std::atoi(env) != 0);

  auto fail = [&](hipError_t err, const char* what) {
    std::ostringstream os;
    os << what << ": " << hipGetErrorString(err);
    set_error(os.str());
    free_all(s);
    delete s;
    return DG_E_HIP;
  };
  hipError_t err;
  const size_t nq = field_count(s), nt = trace_count(s);
  if ((err = dev_alloc(&s->q, nq)) != hipSuccess) return fail(err, "alloc q");
  for (int i = 0; i < 3; ++i)
    if ((err = dev_alloc(&s->r[i], nq)) != hipSuccess) return fail(err, "alloc r");
  for (int i = 0; i < 2; ++i)
    if ((err = dev_alloc(&s->qf[i], nt)) != hipSuccess) return fail(err, "alloc qf");
  if ((err = dev_alloc(&s->qf_tmp, nt)) != hipSuccess) return fail(err, "alloc qf_tmp");
  if ((err = dev_alloc(&s->geo, geo.size())) != hipSuccess) return fail(err, "alloc geo");
  if ((err = dev_alloc(&s->cf, static_cast<size_t>(K) * s->CB)) != hipSuccess) return fail(err, "alloc cf");
  if ((err = dev_alloc(&s->coef, static_cast<size_t>(K) * s->ncoef)) != hipSuccess) return fail(err, "alloc coef");
  if ((err = dev_alloc(&s->DT, DT.size())) != hipSuccess) return fail(err, "alloc DT");
  if ((err = dev_alloc(&s->LT, LT.size())) != hipSuccess) return fail(err, "alloc LT");
  if ((err = dev_alloc(&s->conn, conn.size())) != hipSuccess) return fail(err, "alloc conn");
  if ((err = dev_alloc(&s->fmask, ref->fmask.size())) != hipSuccess) return fail(err, "alloc fmask");
  if ((err = dev_alloc(&s->perm, ref->perm.size())) != hipSuccess) return fail(err, "alloc perm");
  if ((err = dev_alloc(&s->nodeface, ref->nodeface.size())) != hipSuccess) return fail(err, "alloc nodeface");
  if ((err = dev_alloc(&s->J, J.size())) != hipSuccess) return fail(err, "alloc J");
  if ((err = dev_alloc(&s->mass, ref->mass.size())) != hipSuccess) return fail(err, "alloc mass");
  const int64_t eb = dgw::energy_blocks(physics, order, K);
  if ((err = dev_alloc(&s->partial, static_cast<size_t>(eb))) != hipSuccess) return fail(err, "alloc partial");
  if ((err = dev_alloc(&s->e_out, 1)) != hipSuccess) return fail(err, "alloc e_out");
  if ((err = dev_alloc(&s->flag, 1)) != hipSuccess) return fail(err, "alloc flag");
  if ((err = dev_alloc(&s->Dpack, Dpack.size())) != hipSuccess) return fail(err, "alloc Dpack");
  if ((err = dev_alloc(&s->Lpack, Lpack.size())) != hipSuccess) return fail(err, "alloc Lpack");
  for (int v = 0; v < 2; ++v)
    for (int h = 0; h < 2; ++h) {
      if ((err = dev_alloc(&s->D16[v][h], D16[v][h].size())) != hipSuccess) return fail(err, "alloc D16");
      if ((err = dev_alloc(&s->L16[v][h], L16[v][h].size())) != hipSuccess) return fail(err, "alloc L16");
      if ((err = hipMemcpy(s->D16[v][h], D16[v][h].data(), D16[v][h].size() * sizeof(uint16_t),
                           hipMemcpyHostToDevice)) != hipSuccess)
        return fail(err, "upload D16");
      if ((err = hipMemcpy(s->L16[v][h], L16[v][h].data(), L16[v][h].size() * sizeof(uint16_t),
                           hipMemcpyHostToDevice)) != hipSuccess)
        return fail(err, "upload L16");
    }

  struct Up {
    void* dst;
    const void* src;
    size_t bytes;
  } ups[] = {
      {s->geo, geo.data(), geo.size() * sizeof(float)},
      {s->DT, DT.data(), DT.size() * sizeof(float)},
      {s->LT, LT.data(), LT.size() * sizeof(float)},
      {s->conn, conn.data(), conn.size() * sizeof(int32_t)},
      {s->fmask, ref->fmask.data(), ref->fmask.size() * sizeof(int32_t)},
      {s->perm, ref->perm.data(), ref->perm.size() * sizeof(int32_t)},
      {s->nodeface, ref->nodeface.data(), ref->nodeface.size() * sizeof(int32_t)},
      {s->J, J.data(), J.size() * sizeof(double)},
      {s->mass, ref->mass.data(), ref->mass.size() * sizeof(double)},
      {s->Dpack, Dpack.data(), Dpack.size() * sizeof(float)},
      {s->Lpack, Lpack.data(), Lpack.size() * sizeof(float)},
  };
  for (const auto& u : ups)
    if ((err = hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return fail(err, "upload");
  for (int i = 0; i < 3; ++i)
    if ((err = hipMemset(s->r[i], 0, nq * sizeof(float))) != hipSuccess) return fail(err, "clear r");
  *out = s;
  return DG_OK;
}

void dg_destroy(dg_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  free_all(s);
  delete s;
}

dg_status dg_set_stream(dg_solver* s, void* stream) {
  if (dg_status st = check_solver(s)) return st;
  s->stream = static_cast<hipStream_t>(stream);
  return DG_OK;
}

dg_status dg_set_variant(dg_solver* s, int variant) {
  if (dg_status st = check_solver(s)) return st;
  if (!dgw::variant_supported(s->physics, s->N, variant)) {
    std::ostringstream os;
    os << "kernel variant " << variant << " is not available for this physics and degree";
    set_error(os.str());
    return DG_E_UNSUPPORTED;
  }
  s->variant = variant;
  return DG_OK;
}

dg_status dg_get_variant(dg_solver* s, int* variant) {
  if (dg_status st = check_solver(s)) return st;
  if (!variant) {
    set_error("null output");
    return DG_E_ARG;
  }
  *variant = s->variant;
  return DG_OK;
}

dg_status dg_synchronize(dg_solver* s) {
  if (dg_status st = check_solver(s)) return st;
  DG_HIP(hipStreamSynchronize(s->stream));
  return DG_OK;
}

dg_status dg_node_coordinates(dg_solver* s, double* xyz) {
  if (dg_status st = check_solver(s)) return st;
  if (!xyz) {
    set_error("null output");
    return DG_E_ARG;
  }
  const dgw::RefElement* ref = dgw::reference_element(s->N);
  const int Np = s->Np;
  for (int64_t k = 0; k < s->K; ++k) {
    const double* x = s->elem_xyz.data() + 12 * k;
    for (int n = 0; n < Np; ++n) {
      const double r1 = ref->nodes[3 * n] + 1.0, s1 = ref->nodes[3 * n + 1] + 1.0, t1 = ref->nodes[3 * n + 2] + 1.0;
      for (int c = 0; c < 3; ++c)
        xyz[(k * Np + n) * 3 + c] =
            x[c] + 0.5 * (r1 * (x[3 + c] - x[c]) + s1 * (x[6 + c] - x[c]) + t1 * (x[9 + c] - x[c]));
    }
  }
  return DG_OK;
}

dg_status dg_set_coefficients(dg_solver* s, const float* coef) {
  if (dg_status st = check_solver(s)) return st;
  if (!coef) {
    set_error("null coefficients");
    return DG_E_ARG;
  }
  const size_t n = static_cast<size_t>(s->K) * s->ncoef;
  DG_HIP(hipMemcpyAsync(s->coef, coef, n * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  // validate on the host copy: set-up call, a synchronisation is acceptable
  std::vector<float> h(n);
  DG_HIP(hipMemcpyAsync(h.data(), s->coef, n * sizeof(float), hipMemcpyDeviceToHost, s->stream));
  DG_HIP(hipStreamSynchronize(s->stream));
  for (size_t i = 0; i < n; ++i)
    if (!(h[i] > 0.0f) || !std::isfinite(h[i])) {
      std::ostringstream os;
      os << "coefficient " << i % s->ncoef << " of element " << i / s->ncoef << " is not positive and finite";
      set_error(os.str());
      return DG_E_ARG;
    }
  DG_HIP(dgw::launch_coef_prep(s->physics, s->K, s->coef, s->conn, s->cf, s->stream));
  s->have_coef = true;
  s->coef_gen += 1;
  return DG_OK;
}

dg_status dg_set_fields(dg_solver* s, const float* q) {
  if (dg_status st = check_solver(s)) return st;
  if (!q) {
    set_error("null fields");
    return DG_E_ARG;
  }
  DG_HIP(hipMemcpyAsync(s->q, q, field_count(s) * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  DG_HIP(dgw::launch_traces(s->physics, s->N, s->K, s->q, s->geo, s->fmask, s->qf[0], s->stream));
  s->cur = 0;
  s->m = 0;
  s->have_fields = true;
  s->e_prev = -1.0;
  s->e_prev_m = -1;
  return DG_OK;
}

dg_status dg_get_fields(dg_solver* s, float* q) {
  if (dg_status st = check_solver(s)) return st;
  if (!q) {
    set_error("null output");
    return DG_E_ARG;
  }
  if (!s->have_fields) {
    set_error("fields not set");
    return DG_E_STATE;
  }
  DG_HIP(hipMemcpyAsync(q, s->q, field_count(s) * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  return DG_OK;
}

dg_status dg_set_state(dg_solver* s, const float* q, const float* r1, const float* r2, int64_t step_index) {
  if (dg_status st = check_solver(s)) return st;
  if (!q || step_index < 0 || (step_index >= 1 && !r1) || (step_index >= 2 && !r2)) {
    set_error("dg_set_state: bad arguments");
    return DG_E_ARG;
  }
  const size_t bytes = field_count(s) * sizeof(float);
  DG_HIP(hipMemcpyAsync(s->q, q, bytes, hipMemcpyDeviceToDevice, s->stream));
  if (step_index >= 1)
    DG_HIP(hipMemcpyAsync(s->r[(step_index - 1) % 3], r1, bytes, hipMemcpyDeviceToDevice, s->stream));
  if (step_index >= 2)
    DG_HIP(hipMemcpyAsync(s->r[(step_index - 2) % 3], r2, bytes, hipMemcpyDeviceToDevice, s->stream));
  DG_HIP(dgw::launch_traces(s->physics, s->N, s->K, s->q, s->geo, s->fmask, s->qf[0], s->stream));
  s->cur = 0;
  s->m = step_index;
  s->have_fields = true;
  s->e_prev = -1.0;
  s->e_prev_m = -1;
  return DG_OK;
}

dg_status dg_get_state(dg_solver* s, float* q, float* r1, float* r2, int64_t* step_index) {
  if (dg_status st = check_solver(s)) return st;
  if (!s->have_fields) {
    set_error("fields not set");
    return DG_E_STATE;
  }
  const size_t bytes = field_count(s) * sizeof(float);
  if (q) DG_HIP(hipMemcpyAsync(q, s->q, bytes, hipMemcpyDeviceToDevice, s->stream));
  if (r1 && s->m >= 1)
    DG_HIP(hipMemcpyAsync(r1, s->r[(s->m - 1) % 3], bytes, hipMemcpyDeviceToDevice, s->stream));
  if (r2 && s->m >= 2)
    DG_HIP(hipMemcpyAsync(r2, s->r[(s->m - 2) % 3], bytes, hipMemcpyDeviceToDevice, s->stream));
  if (step_index) *step_index = s->m;
  return DG_OK;
}

dg_status dg_step_index(dg_solver* s, int64_t* m) {
  if (dg_status st = check_solver(s)) return st;
  if (!m) {
    set_error("null output");
    return DG_E_ARG;
  }
  *m = s->m;
  return DG_OK;
}

dg_status dg_step(dg_solver* s, int nsteps, double dt) {
  if (dg_status st = check_solver(s)) return st;
  if (nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) {
    set_error("nsteps must be >= 0 and dt > 0");
    return DG_E_ARG;
  }
  if (!s->have_coef || !s->have_fields) {
    set_error("set coefficients and fields before stepping");
    return DG_E_STATE;
  }
  for (int i = 0; i < nsteps; ++i) {
    const dgw::StepArgs a = dgw::step_args(s, s->m, s->cur, dt);
    DG_HIP(dgw::launch_step(s->physics, s->N, s->variant, a, s->stream));
    s->cur ^= 1;
    s->m += 1;
  }
  return DG_OK;
}

dg_status dg_rhs(dg_solver* s, const float* q, float* r) {
  if (dg_status st = check_solver(s)) return st;
  if (!q || !r) {
    set_error("null array");
    return DG_E_ARG;
  }
  if (!s->have_coef) {
    set_error("set coefficients first");
    return DG_E_STATE;
  }
  DG_HIP(dgw::launch_traces(s->physics, s->N, s->K, q, s->geo, s->fmask, s->qf_tmp, s->stream));
  dgw::StepArgs a = dgw::base_args(s);
  a.mode = dgw::kRhsMode;
  a.q_in = q;
  a.r_out = r;
  a.qf_in = s->qf_tmp;
  DG_HIP(dgw::launch_step(s->physics, s->N, s->variant, a, s->stream));
  return DG_OK;
}

dg_status dg_energy(dg_solver* s, double* e) {
  if (dg_status st = check_solver(s)) return st;
  if (!e) {
    set_error("null output");
    return DG_E_ARG;
  }
  if (!s->have_coef || !s->have_fields) {
    set_error("set coefficients and fields first");
    return DG_E_STATE;
  }
  DG_HIP(dgw::launch_energy(s->physics, s->N, s->K, s->q, s->coef, s->J, s->mass, s->partial, s->e_out,
                            s->stream));
  DG_HIP(hipMemcpyAsync(e, s->e_out, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  DG_HIP(hipStreamSynchronize(s->stream));
  if (!std::isfinite(*e)) {
    set_error("energy is not finite");
    s->e_prev = -1.0;
    return DG_E_UNSTABLE;
  }
  // The upwind flux only removes energy (Sec. 2.1), so in the AB3 regime the
  // energy of one trajectory must not grow between two evaluations; the
  // Euler and two-step start-up steps may raise it slightly and are exempt.
  const double prev = s->e_prev;
  const int64_t prev_m = s->e_prev_m;
  s->e_prev = *e;
  s->e_prev_m = s->m;
  if (s->e_tol >= 0.0 && prev >= 0.0 && prev_m >= 2 && s->m > prev_m && *e > prev * (1.0 + s->e_tol)) {
    std::ostringstream os;
    os << "energy grew from " << prev << " at step " << prev_m << " to " << *e << " at step " << s->m
       << " (tolerance " << s->e_tol << "): the step size is likely above the stability limit";
    set_error(os.str());
    return DG_E_UNSTABLE;
  }
  return DG_OK;
}

dg_status dg_energy_noalloc(dg_solver* s, double* e_dev) {
  if (dg_status st = check_solver(s)) return st;
  if (!e_dev) {
    set_error("null output");
    return DG_E_ARG;
  }
  const int64_t blocks = dgw::energy_blocks(s->physics, s->N, s->K);
  if (blocks < 1 || blocks > dgw::kStaticEnergyPartials) {
    std::ostringstream os;
    os << "dg_energy_noalloc: this mesh needs " << blocks << " partial sums, the static array holds "
       << dgw::kStaticEnergyPartials << " (use dg_energy)";
    set_error(os.str());
    return DG_E_SHAPE;
  }
  if (!s->have_coef || !s->have_fields) {
    set_error("set coefficients and fields first");
    return DG_E_STATE;
  }
  double* partial = nullptr;
  DG_HIP(dgw::static_energy_partials(s->device, &partial));
  // every partial sum the reduction reads is written first by the same
  // launch sequence, so the array needs no clearing
  DG_HIP(dgw::launch_energy(s->physics, s->N, s->K, s->q, s->coef, s->J, s->mass, partial, e_dev, s->stream));
  return DG_OK;
}

dg_status dg_set_energy_tolerance(dg_solver* s, double tol) {
  if (dg_status st = check_solver(s)) return st;
  if (std::isnan(tol)) {
    set_error("tolerance is NaN");
    return DG_E_ARG;
  }
  s->e_tol = tol;
  return DG_OK;
}

dg_status dg_debug_buffer(dg_solver* s, const char* name, void* dst, size_t* bytes) {
  if (dg_status st = check_solver(s)) return st;
  if (!name || !bytes) {
    set_error("null argument");
    return DG_E_ARG;
  }
  const void* src = nullptr;
  size_t n = 0;
  const std::string key(name);
  const size_t K = static_cast<size_t>(s->K);
  if (key == "geo") { src = s->geo; n = K * 9 * sizeof(float); }
  else if (key == "cf") { src = s->cf; n = K * s->CB * sizeof(float); }
  else if (key == "conn") { src = s->conn; n = K * 4 * sizeof(int32_t); }
  else if (key == "fmask") { src = s->fmask; n = 4 * static_cast<size_t>(s->Nfp) * sizeof(int32_t); }
  else if (key == "perm") { src = s->perm; n = 6 * static_cast<size_t>(s->Nfp) * sizeof(int32_t); }
  else if (key == "nodeface") { src = s->nodeface; n = 3 * static_cast<size_t>(s->Np) * sizeof(int32_t); }
  else if (key == "DT") { src = s->DT; n = 3 * static_cast<size_t>(s->Np) * s->Np * sizeof(float); }
  else if (key == "LT") { src = s->LT; n = 4 * static_cast<size_t>(s->Nfp) * s->Np * sizeof(float); }
  else if (key == "traces") { src = s->qf[s->cur]; n = trace_count(s) * sizeof(float); }
  else if (key == "traces_rhs") { src = s->qf_tmp; n = trace_count(s) * sizeof(float); }
  else {
    set_error("unknown buffer name " + key);
    return DG_E_ARG;
  }
  const size_t have = *bytes;
  *bytes = n;
  if (!dst) return DG_OK;
  if (have < n) {
    set_error("destination too small");
    return DG_E_SHAPE;
  }
  DG_HIP(hipStreamSynchronize(s->stream));
  DG_HIP(hipMemcpy(dst, src, n, hipMemcpyDeviceToHost));
  return DG_OK;
}

}  // extern "C"
