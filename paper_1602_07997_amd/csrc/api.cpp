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
#include "workspace.hpp"

namespace dgw {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }
const char* last_error() { return g_error.c_str(); }

}  // namespace dgw

using dgw::set_error;


namespace {

dg_status check_solver(const dg_solver* s) {
  if (!s) {
    set_error("null solver");
    return DG_E_ARG;
  }
  return DG_OK;
}

size_t field_count(const dg_solver* s) { return static_cast<size_t>(s->K) * s->NF * s->Np; }
size_t trace_count(const dg_solver* s) { return static_cast<size_t>(s->K) * 4 * s->NT * s->Nfp; }

// Operator tables of one (physics, degree) in the kernels' layouts, built on
// the host: D_j and LIFT transposed (node-per-thread kernel), in FP32 MFMA
// fragment order, and as BF16 / FP16 hi + lo splits.
struct HostTables {
  std::vector<float> DT, LT, Dpack, Lpack;
  std::vector<uint16_t> D16[2][2], L16[2][2];  // [bf16, f16][hi, lo]
};

HostTables make_tables(int physics, const dgw::RefElement* ref) {
  HostTables t;
  const int order = ref->N, Np = ref->Np, Nfp = ref->Nfp;
  t.DT.resize(3 * static_cast<size_t>(Np) * Np);
  t.LT.resize(static_cast<size_t>(4) * Nfp * Np);
  for (int j = 0; j < 3; ++j)
    for (int n = 0; n < Np; ++n)
      for (int mm = 0; mm < Np; ++mm)
        t.DT[(static_cast<size_t>(j) * Np + mm) * Np + n] =
            static_cast<float>(ref->D[(static_cast<size_t>(j) * Np + n) * Np + mm]);
  for (int n = 0; n < Np; ++n)
    for (int fm = 0; fm < 4 * Nfp; ++fm)
      t.LT[static_cast<size_t>(fm) * Np + n] = static_cast<float>(ref->lift[static_cast<size_t>(n) * 4 * Nfp + fm]);
  const dgw::MfmaPacking p32 = dgw::mfma_packing(physics, order, dgw::kVariantMfma);
  const dgw::ColMap c32 = dgw::face_block_columns(Nfp, p32.KF);
  for (int j = 0; j < 3; ++j)
    dgw::pack_fp32(ref->D.data() + static_cast<size_t>(j) * Np * Np, Np, Np, p32.MB, p32.KP, t.Dpack);
  dgw::pack_fp32(ref->lift.data(), Np, 4 * Nfp, p32.MB, p32.KL, t.Lpack, p32.KF > 0 ? &c32 : nullptr);
  const int vars[2] = {dgw::kVariantMfmaBf16, dgw::kVariantMfmaF16};
  for (int v = 0; v < 2; ++v) {
    const dgw::MfmaPacking p16 = dgw::mfma_packing(physics, order, vars[v]);
    const dgw::ColMap c16 = dgw::face_block_columns(Nfp, p16.KF);
    const int kw = p16.KS / 4;  // k per lane group: 4 (16x16x16) or 8 (16x16x32)
    for (int j = 0; j < 3; ++j)
      dgw::pack_split16(ref->D.data() + static_cast<size_t>(j) * Np * Np, Np, Np, p16.MB, p16.KP, kw, v == 0,
                        t.D16[v][0], t.D16[v][1]);
    dgw::pack_split16(ref->lift.data(), Np, 4 * Nfp, p16.MB, p16.KL, kw, v == 0, t.L16[v][0], t.L16[v][1],
                      p16.KF > 0 ? &c16 : nullptr);
  }
  return t;
}

// Sizes of a solver that do not depend on the mesh's geometry.
void set_sizes(dg_solver* s, int physics, int order, int64_t K, const dgw::RefElement* ref) {
  s->physics = physics;
  s->N = order;
  s->Np = ref->Np;
  s->Nfp = ref->Nfp;
  s->NF = dg_num_fields(physics);
  s->NT = dgw::num_traces(physics);
  s->CB = dgw::coef_block(physics);
  s->ncoef = dgw::num_coefficients(physics);
  s->K = K;
}

// Every device array of a solver, in one workspace (measuring when the arena
// has no base).
void layout(dg_solver* s, const HostTables& t, const dgw::RefElement* ref, dgw::Arena& a) {
  const size_t K = static_cast<size_t>(s->K);
  const size_t nq = K * s->NF * s->Np, nt = K * 4 * s->NT * s->Nfp;
  s->q = a.take<float>(nq);
  for (int i = 0; i < 3; ++i) s->r[i] = a.take<float>(nq);
  for (int i = 0; i < 2; ++i) s->qf[i] = a.take<float>(nt);
  s->qf_tmp = a.take<float>(nt);
  s->geo = a.take<float>(K * 9);
  s->cf = a.take<float>(K * s->CB);
  s->coef = a.take<float>(K * s->ncoef);
  s->DT = a.take<float>(t.DT.size());
  s->LT = a.take<float>(t.LT.size());
  s->conn = a.take<int32_t>(K * 4);
  s->fmask = a.take<int32_t>(ref->fmask.size());
  s->perm = a.take<int32_t>(ref->perm.size());
  s->nodeface = a.take<int32_t>(ref->nodeface.size());
  s->J = a.take<double>(K);
  s->mass = a.take<double>(ref->mass.size());
  s->partial = a.take<double>(static_cast<size_t>(dgw::energy_blocks(s->physics, s->N, s->K)));
  s->e_out = a.take<double>(1);
  s->flag = a.take<int>(1);
  s->iface = a.take<int32_t>(K);
  s->Dpack = a.take<float>(t.Dpack.size());
  s->Lpack = a.take<float>(t.Lpack.size());
  for (int v = 0; v < 2; ++v)
    for (int h = 0; h < 2; ++h) {
      s->D16[v][h] = a.take<uint16_t>(t.D16[v][h].size());
      s->L16[v][h] = a.take<uint16_t>(t.L16[v][h].size());
    }
}

dg_status check_create_args(int physics, int order, int64_t K, const dgw::RefElement** ref) {
  if (physics != DG_ACOUSTIC && physics != DG_ELASTIC && physics != DG_ANISOTROPIC) {
    set_error("unknown physics");
    return DG_E_ARG;
  }
  *ref = (order >= 1 && order <= dgw::kMaxOrder) ? dgw::reference_element(order) : nullptr;
  if (!*ref) {
    set_error("order must be in [1, 8]");
    return DG_E_UNSUPPORTED;
  }
  if (K <= 0 || K >= (int64_t(1) << 26)) {
    set_error("K must be in [1, 2^26)");
    return DG_E_ARG;
  }
  return DG_OK;
}

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
  a.tail_split = s->tail_split;
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

int dg_abi_version(void) { return 2; }

const char* dg_last_error(void) { return dgw::last_error(); }

int dg_num_fields(int physics) {
  if (physics == DG_ACOUSTIC) return 4;
  if (physics == DG_ELASTIC || physics == DG_ANISOTROPIC) return 9;
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

dg_status dg_workspace_bytes(int physics, int order, int64_t K, size_t* bytes) {
  if (!bytes) {
    set_error("null output");
    return DG_E_ARG;
  }
  const dgw::RefElement* ref = nullptr;
  if (dg_status st = check_create_args(physics, order, K, &ref)) return st;
  dg_solver probe;
  set_sizes(&probe, physics, order, K, ref);
  dgw::Arena arena(nullptr, 0);
  layout(&probe, make_tables(physics, ref), ref, arena);
  *bytes = arena.used();
  return DG_OK;
}

dg_status dg_create(int physics, int order, int64_t K, const double* elem_xyz, const int64_t* elem_topo,
                    void* workspace, size_t workspace_bytes, void* stream, dg_solver** out) {
  if (!out) {
    set_error("null output handle");
    return DG_E_ARG;
  }
  *out = nullptr;
  const dgw::RefElement* ref = nullptr;
  if (dg_status st = check_create_args(physics, order, K, &ref)) return st;
  if (!elem_xyz || !elem_topo) {
    set_error("the mesh arrays must be non-null");
    return DG_E_ARG;
  }
  if (!workspace || !dgw::workspace_aligned(workspace)) {
    set_error("the workspace must be a non-null device pointer aligned to 256 bytes");
    return DG_E_ARG;
  }

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

  // ---- operator tables and the layout in the caller's workspace ----
  const HostTables t = make_tables(physics, ref);
  dg_solver* s = new dg_solver();
  set_sizes(s, physics, order, K, ref);
  s->stream = static_cast<hipStream_t>(stream);
  s->elem_xyz.assign(elem_xyz, elem_xyz + 12 * K);
  s->conn_h = conn;
  (void)hipGetDevice(&s->device);
  if (const char* env = std::getenv("DGWAVE_XCD_REMAP")) s->xcd_remap = (std::atoi(env) != 0);
  if (const char* env = std::getenv("DGWAVE_TAIL_SPLIT")) s->tail_split = (std::atoi(env) != 0);
  dgw::Arena arena(workspace, workspace_bytes);
  layout(s, t, ref, arena);
  if (!arena.fits()) {
    std::ostringstream os;
    os << "workspace holds " << workspace_bytes << " bytes, the solver needs " << arena.used()
       << " (dg_workspace_bytes)";
    set_error(os.str());
    delete s;
    return DG_E_SHAPE;
  }

  // uploads on the solver's stream; the host arrays live until the sync below
  struct Up {
    void* dst;
    const void* src;
    size_t bytes;
  } ups[] = {
      {s->geo, geo.data(), geo.size() * sizeof(float)},
      {s->DT, t.DT.data(), t.DT.size() * sizeof(float)},
      {s->LT, t.LT.data(), t.LT.size() * sizeof(float)},
      {s->conn, conn.data(), conn.size() * sizeof(int32_t)},
      {s->fmask, ref->fmask.data(), ref->fmask.size() * sizeof(int32_t)},
      {s->perm, ref->perm.data(), ref->perm.size() * sizeof(int32_t)},
      {s->nodeface, ref->nodeface.data(), ref->nodeface.size() * sizeof(int32_t)},
      {s->J, J.data(), J.size() * sizeof(double)},
      {s->mass, ref->mass.data(), ref->mass.size() * sizeof(double)},
      {s->Dpack, t.Dpack.data(), t.Dpack.size() * sizeof(float)},
      {s->Lpack, t.Lpack.data(), t.Lpack.size() * sizeof(float)},
      {s->D16[0][0], t.D16[0][0].data(), t.D16[0][0].size() * sizeof(uint16_t)},
      {s->D16[0][1], t.D16[0][1].data(), t.D16[0][1].size() * sizeof(uint16_t)},
      {s->D16[1][0], t.D16[1][0].data(), t.D16[1][0].size() * sizeof(uint16_t)},
      {s->D16[1][1], t.D16[1][1].data(), t.D16[1][1].size() * sizeof(uint16_t)},
      {s->L16[0][0], t.L16[0][0].data(), t.L16[0][0].size() * sizeof(uint16_t)},
      {s->L16[0][1], t.L16[0][1].data(), t.L16[0][1].size() * sizeof(uint16_t)},
      {s->L16[1][0], t.L16[1][0].data(), t.L16[1][0].size() * sizeof(uint16_t)},
      {s->L16[1][1], t.L16[1][1].data(), t.L16[1][1].size() * sizeof(uint16_t)},
  };
  hipError_t err = hipSuccess;
  for (const auto& u : ups)
    if (err == hipSuccess && u.bytes > 0)
      err = hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, s->stream);
  // the AB3 ring starts at zero (a fill kernel, so that no memset node ever
  // enters a captured graph)
  const int64_t nq = s->K * s->NF * s->Np;
  for (int i = 0; i < 3 && err == hipSuccess; ++i) err = dgw::launch_fill_zero_f32(nq, s->r[i], s->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(s->stream);
  if (err != hipSuccess) {
    std::ostringstream os;
    os << "dg_create: upload: " << hipGetErrorString(err);
    set_error(os.str());
    delete s;
    return DG_E_HIP;
  }
  *out = s;
  return DG_OK;
}

void dg_destroy(dg_solver* s) {
  if (!s) return;
  // the device arrays belong to the caller's workspace
  (void)hipStreamSynchronize(s->stream);
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
  const int64_t n = s->K * s->ncoef;
  DG_HIP(hipMemcpyAsync(s->coef, coef, static_cast<size_t>(n) * sizeof(float), hipMemcpyDeviceToDevice,
                        s->stream));
  // validated on the device (set-up call: one synchronisation, one int back)
  int bad = -1;
  if (s->physics == DG_ANISOTROPIC)
    DG_HIP(dgw::launch_first_bad_stiffness(s->K, s->coef, s->flag, s->stream));
  else
    DG_HIP(dgw::launch_first_nonpositive(n, s->coef, s->flag, s->stream));
  DG_HIP(hipMemcpyAsync(&bad, s->flag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  DG_HIP(hipStreamSynchronize(s->stream));
  if (bad >= 0) {
    std::ostringstream os;
    if (s->physics == DG_ANISOTROPIC)
      os << "element " << bad << ": density not positive and finite, or stiffness not finite and positive definite";
    else
      os << "coefficient " << bad % s->ncoef << " of element " << bad / s->ncoef << " is not positive and finite";
    set_error(os.str());
    s->have_coef = false;
    return DG_E_ARG;
  }
  DG_HIP(dgw::launch_coef_prep(s->physics, s->K, s->coef, s->conn, s->cf, s->stream));
  s->have_coef = true;
  s->coef_gen += 1;
  return DG_OK;
}

dg_status dg_set_boundary(dg_solver* s, const int32_t* kind) {
  if (dg_status st = check_solver(s)) return st;
  if (!kind) {
    set_error("null boundary kinds");
    return DG_E_ARG;
  }
  std::vector<int32_t> conn = s->conn_h;
  for (int64_t i = 0; i < 4 * s->K; ++i) {
    const bool wall = (conn[i] & 7) == 7;
    if (kind[i] != DG_BC_REFLECT && kind[i] != DG_BC_ABSORB) {
      std::ostringstream os;
      os << "unknown boundary kind " << kind[i] << " at face " << i % 4 << " of element " << i / 4;
      set_error(os.str());
      return DG_E_ARG;
    }
    if (!wall && kind[i] != DG_BC_REFLECT) {
      std::ostringstream os;
      os << "face " << i % 4 << " of element " << i / 4 << " has a neighbour: only unpaired faces absorb";
      set_error(os.str());
      return DG_E_ARG;
    }
    // a wall's word: own index, bit 3 set for an absorbing face
    if (wall) conn[i] = static_cast<int32_t>(((i / 4) << 5) | (kind[i] == DG_BC_ABSORB ? 8 : 0) | 7);
  }
  DG_HIP(hipMemcpyAsync(s->conn, conn.data(), conn.size() * sizeof(int32_t), hipMemcpyHostToDevice, s->stream));
  DG_HIP(hipStreamSynchronize(s->stream));
  s->conn_h.swap(conn);
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
  if (s->k_fast > 0) {
    set_error("the AB3 state of a two-rate solver is per class: dg_set_state is single-rate only");
    return DG_E_UNSUPPORTED;
  }
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
  if (s->k_fast > 0) {
    set_error("the AB3 state of a two-rate solver is per class: dg_get_state is single-rate only");
    return DG_E_UNSUPPORTED;
  }
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
  if (s->k_fast > 0) {
    set_error("this solver has a fast class: step it with dg_step_multirate");
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

dg_status dg_set_rate_classes(dg_solver* s, int64_t k_fast) {
  if (dg_status st = check_solver(s)) return st;
  if (k_fast < 0 || k_fast > s->K) {
    set_error("k_fast must lie in [0, K]");
    return DG_E_ARG;
  }
  // slow elements that read a fast neighbour's traces
  std::vector<int32_t> iface;
  for (int64_t k = k_fast; k < s->K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int32_t w = s->conn_h[4 * k + f];
      if ((w & 7) != 7 && static_cast<int64_t>(w >> 5) < k_fast) {
        iface.push_back(static_cast<int32_t>(k));
        break;
      }
    }
  if (!iface.empty()) {
    DG_HIP(hipMemcpyAsync(s->iface, iface.data(), iface.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          s->stream));
    DG_HIP(hipStreamSynchronize(s->stream));
  }
  s->k_fast = k_fast;
  s->n_iface = static_cast<int64_t>(iface.size());
  s->m = 0;  // both classes restart with the Euler / two-step start-up
  s->e_prev = -1.0;
  s->e_prev_m = -1;
  return DG_OK;
}

dg_status dg_step_multirate(dg_solver* s, int nsteps, double dt) {
  if (dg_status st = check_solver(s)) return st;
  if (nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) {
    set_error("nsteps must be >= 0 and dt > 0");
    return DG_E_ARG;
  }
  if (!s->have_coef || !s->have_fields) {
    set_error("set coefficients and fields before stepping");
    return DG_E_STATE;
  }
  const double h = 0.5 * dt;
  const int64_t K = s->K, KF = s->k_fast;
  for (int i = 0; i < nsteps; ++i) {
    const int64_t ms = s->m, mf = 2 * s->m;  // coarse and fine steps taken so far
    float* A = s->qf[s->cur];                // every trace at t_n
    float* B = s->qf_tmp;                    // traces at t_n + h (fast; slow next to fast)
    float* C = s->qf[s->cur ^ 1];            // every trace at t_n + dt
    // 1. fast elements: first half step, traces at t_n + h into B
    if (KF > 0) {
      dgw::StepArgs a = dgw::step_args(s, mf, s->cur, h);
      a.K = KF;
      a.qf_in = A;
      a.qf_out = B;
      DG_HIP(dgw::launch_step(s->physics, s->N, s->variant, a, s->stream));
    }
    // 2. slow elements: full step, traces at t_n + dt into C
    if (KF < K) {
      dgw::StepArgs a = dgw::step_args(s, ms, s->cur, dt);
      a.e_begin = KF;
      a.qf_in = A;
      a.qf_out = C;
      DG_HIP(dgw::launch_step(s->physics, s->N, s->variant, a, s->stream));
      // 3. slow elements next to fast ones: traces of their state at t_n + h,
      // q(t_n + h) = q(t_n + dt) + dt sum_i (w_half - w_full)_i r^{n-i} with
      // w the integrals of the history polynomial over half and full steps
      if (KF > 0 && s->n_iface > 0) {
        static const double d[3][3] = {{-0.5, 0.0, 0.0},
                                       {5.0 / 8.0 - 1.5, -1.0 / 8.0 + 0.5, 0.0},
                                       {17.0 / 24.0 - 23.0 / 12.0, -7.0 / 24.0 + 16.0 / 12.0,
                                        1.0 / 12.0 - 5.0 / 12.0}};
        const int st = ms < 2 ? static_cast<int>(ms) : 2;
        DG_HIP(dgw::launch_trace_comb(s->physics, s->N, s->n_iface, s->iface, s->q, s->r[ms % 3],
                                      s->r[(ms + 2) % 3], s->r[(ms + 1) % 3], static_cast<float>(dt * d[st][0]),
                                      static_cast<float>(dt * d[st][1]), static_cast<float>(dt * d[st][2]),
                                      s->geo, s->fmask, B, s->stream));
      }
    }
    // 4. fast elements: second half step from B, traces at t_n + dt into C
    if (KF > 0) {
      dgw::StepArgs a = dgw::step_args(s, mf + 1, s->cur, h);
      a.K = KF;
      a.qf_in = B;
      a.qf_out = C;
      DG_HIP(dgw::launch_step(s->physics, s->N, s->variant, a, s->stream));
    }
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
