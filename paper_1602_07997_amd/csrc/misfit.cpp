// Misfit of receiver traces against data and its gradient with respect to
// the per-element coefficients: forward solve with a point source and
// checkpoints, reverse sweep of the adjoint recursion with the forward step
// kernel, per-step gradient accumulation.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "dg_internal.hpp"
#include "dgwave.h"
#include "kernels.hpp"
#include "mfma_pack.hpp"
#include "solver_state.hpp"
#include "workspace.hpp"

using dgw::set_error;

namespace {

// Fields of the point source (acoustic p; elastic the normal stresses, an
// explosive source) and of the receivers (acoustic p; elastic v1, v2, v3).
const int kSrcAcoustic[] = {0};
const int kSrcElastic[] = {3, 4, 5};
const int kRecAcoustic[] = {0};
const int kRecElastic[] = {0, 1, 2};

// A device array carved from the misfit's workspace (not owned).
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void carve(dgw::Arena& a, size_t count) {
    n = count;
    p = a.take<T>(count);
  }
  // Stream-ordered copy of a host array of exactly n entries; the caller
  // keeps `h` alive until the stream has passed the copy.
  hipError_t upload(const std::vector<T>& h, hipStream_t st) {
    if (h.size() != n) return hipErrorInvalidValue;
    if (h.empty()) return hipSuccess;
    return hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st);
  }
};

// Element containing x and the reference coordinates of x in it.
bool locate_point(const dg_solver* s, const double* x, int64_t* elem, double xi[3]) {
  const double tol = 1e-12;
  for (int64_t k = 0; k < s->K; ++k) {
    const double* v = s->elem_xyz.data() + 12 * k;
    double F[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) F[i][j] = 0.5 * (v[3 * (j + 1) + i] - v[i]);
    const double det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                       F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                       F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    if (!(det > 0.0)) continue;
    double inv[3][3];
    inv[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) / det;
    inv[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) / det;
    inv[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) / det;
    inv[1][0] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) / det;
    inv[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) / det;
    inv[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) / det;
    inv[2][0] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) / det;
    inv[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) / det;
    inv[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) / det;
    double r[3];
    for (int i = 0; i < 3; ++i) {
      r[i] = -1.0;
      for (int j = 0; j < 3; ++j) r[i] += inv[i][j] * (x[j] - v[j]);
    }
    const double l0 = -(1.0 + r[0] + r[1] + r[2]) / 2.0;
    if (l0 >= -tol && (1.0 + r[0]) / 2.0 >= -tol && (1.0 + r[1]) / 2.0 >= -tol && (1.0 + r[2]) / 2.0 >= -tol) {
      *elem = k;
      xi[0] = r[0];
      xi[1] = r[1];
      xi[2] = r[2];
      return true;
    }
  }
  return false;
}

// Entries of a point-injection list grouped by element (CSR).
struct HostInject {
  std::vector<int64_t> elem;
  std::vector<int32_t> start{0};
  std::vector<int32_t> field, chan;
  std::vector<float> vec;
};

struct Entry {
  int64_t k;
  int field, chan;
  std::vector<double> v;
};

HostInject group_entries(const std::vector<Entry>& entries) {
  std::map<int64_t, std::vector<const Entry*>> by_elem;
  for (const Entry& e : entries) by_elem[e.k].push_back(&e);
  HostInject h;
  for (const auto& kv : by_elem) {
    h.elem.push_back(kv.first);
    for (const Entry* e : kv.second) {
      h.field.push_back(e->field);
      h.chan.push_back(e->chan);
      for (double x : e->v) h.vec.push_back(static_cast<float>(x));
    }
    h.start.push_back(static_cast<int32_t>(h.field.size()));
  }
  return h;
}

struct DevInject {
  DevBuf<int64_t> elem;
  DevBuf<int32_t> start, field, chan;
  DevBuf<float> vec;
  int nelem = 0;
  // arrays sized for h (an injection list of the same shape may be uploaded
  // later with other values)
  void carve(dgw::Arena& a, const HostInject& h) {
    nelem = static_cast<int>(h.elem.size());
    elem.carve(a, h.elem.size());
    start.carve(a, h.start.size());
    field.carve(a, h.field.size());
    chan.carve(a, h.chan.size());
    vec.carve(a, h.vec.size());
  }
  hipError_t upload(const HostInject& h, hipStream_t st) {
    if (static_cast<int>(h.elem.size()) != nelem) return hipErrorInvalidValue;
    hipError_t e;
    if ((e = elem.upload(h.elem, st)) != hipSuccess) return e;
    if ((e = start.upload(h.start, st)) != hipSuccess) return e;
    if ((e = field.upload(h.field, st)) != hipSuccess) return e;
    if ((e = chan.upload(h.chan, st)) != hipSuccess) return e;
    return vec.upload(h.vec, st);
  }
};

}  // namespace

struct dg_misfit {
  dg_solver* s = nullptr;
  int64_t M = 0;   // steps
  int C = 0;       // checkpoint interval
  double dt = 0.0;
  int nrec = 0, R = 0;  // receivers, channels
  std::vector<double> wavelet;             // f(t_m), m = 0..M
  std::vector<int64_t> rec_elem_h;         // per receiver
  std::vector<std::vector<double>> rec_w;  // per receiver, Np
  DevInject src;
  DevInject adj;
  DevBuf<int64_t> ch_elem;
  DevBuf<int32_t> ch_field;
  DevBuf<float> ch_w;
  DevBuf<float> traces, data;  // [M+1][R]
  bool have_data = false, have_forward = false;
  uint64_t fwd_coef_gen = 0;  // the solver's coefficient generation of the last forward
  // segment of C steps: states, traces and right-hand sides
  DevBuf<float> seg_q, seg_tr, seg_r;
  // checkpoints: q at the segment start and the two previous right-hand sides
  DevBuf<float> ck;
  int64_t seg_loaded = -1;  // segment whose states are in seg_*
  // adjoint
  DevBuf<float> phi, aring, atr;
  DevBuf<double> gacc;
  DevBuf<float> mass_pack_f, face_mass_f;
  size_t nq = 0, ntr = 0;
};

namespace {

double ab(int64_t m, int i) {
  if (m == 0) return i == 0 ? 1.0 : 0.0;
  if (m == 1) return i == 0 ? 1.5 : (i == 1 ? -0.5 : 0.0);
  return i == 0 ? 23.0 / 12.0 : (i == 1 ? -16.0 / 12.0 : 5.0 / 12.0);
}

int64_t num_segments(const dg_misfit* f) { return (f->M + f->C - 1) / f->C; }

float* seg_q(dg_misfit* f, int64_t i) { return f->seg_q.p + i * f->nq; }
float* seg_tr(dg_misfit* f, int64_t i) { return f->seg_tr.p + i * f->ntr; }
float* seg_r(dg_misfit* f, int64_t i) { return f->seg_r.p + i * f->nq; }
float* ck_q(dg_misfit* f, int64_t s) { return f->ck.p + (3 * s) * f->nq; }
float* ck_r1(dg_misfit* f, int64_t s) { return f->ck.p + (3 * s + 1) * f->nq; }
float* ck_r2(dg_misfit* f, int64_t s) { return f->ck.p + (3 * s + 2) * f->nq; }

dgw::InjectArgs inject_args(dg_misfit* f, DevInject& d, float* q, float* qf) {
  dgw::InjectArgs a{};
  a.nelem = d.nelem;
  a.q = q;
  a.qf = qf;
  a.geo = f->s->geo;
  a.fmask = f->s->fmask;
  a.elem = d.elem.p;
  a.start = d.start.p;
  a.field = d.field.p;
  a.chan = d.chan.p;
  a.vec = d.vec.p;
  return a;
}

// Forward steps [ms, me) of segment `seg` starting from the state in
// seg_q[0] / seg_tr[0] with history ck_r1/ck_r2 of that segment; records the
// receivers when `record` is set.
dg_status run_segment(dg_misfit* f, int64_t seg, bool record) {
  dg_solver* s = f->s;
  const int64_t ms = seg * f->C, me = std::min(ms + f->C, f->M);
  for (int64_t m = ms; m < me; ++m) {
    const int64_t i = m - ms;
    dgw::StepArgs a = dgw::step_args(s, m, 0, f->dt);
    a.q_in = seg_q(f, i);
    a.q_out = seg_q(f, i + 1);
    a.r_out = seg_r(f, i);
    a.r1 = i >= 1 ? seg_r(f, i - 1) : ck_r1(f, seg);
    a.r2 = i >= 2 ? seg_r(f, i - 2) : (i == 1 ? ck_r1(f, seg) : ck_r2(f, seg));
    a.qf_in = seg_tr(f, i);
    a.qf_out = seg_tr(f, i + 1);
    DG_HIP(dgw::launch_step(s->physics, s->N, s->variant, a, s->stream));
    // source: dt sum_i a_i f(t_{m-i}), the forcing part of the AB3 update
    double amp = 0.0;
    for (int j = 0; j < 3; ++j)
      if (m - j >= 0) amp += ab(m, j) * f->wavelet[static_cast<size_t>(m - j)];
    dgw::InjectArgs ia = inject_args(f, f->src, seg_q(f, i + 1), seg_tr(f, i + 1));
    ia.amp = static_cast<float>(f->dt * amp);
    DG_HIP(dgw::launch_inject(s->physics, s->N, ia, s->stream));
    if (record)
      DG_HIP(dgw::launch_record(s->physics, s->N, f->R, seg_q(f, i + 1), f->ch_elem.p, f->ch_field.p, f->ch_w.p,
                                f->traces.p + (m + 1) * f->R, s->stream));
  }
  f->seg_loaded = seg;
  return DG_OK;
}

// Segment `seg`'s start state from its checkpoint.
dg_status load_segment_start(dg_misfit* f, int64_t seg) {
  dg_solver* s = f->s;
  DG_HIP(hipMemcpyAsync(seg_q(f, 0), ck_q(f, seg), f->nq * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  DG_HIP(dgw::launch_traces(s->physics, s->N, s->K, seg_q(f, 0), s->geo, s->fmask, seg_tr(f, 0), s->stream));
  return DG_OK;
}

// Adjoint source vectors s = P W^{-1} g per receiver channel:
// dt P_c (C^{-1})_cc / J_k M^{-1} l(xi_r) with the coefficients `coef`
// (host [K][ncoef]).  The list's shape depends only on the receivers.
HostInject adjoint_entries(const dg_misfit* f, const std::vector<float>& coef) {
  const dg_solver* s = f->s;
  const dgw::RefElement* ref = dgw::reference_element(s->N);
  const int Np = ref->Np;
  std::vector<Entry> entries;
  const int* rf = s->physics == DG_ACOUSTIC ? kRecAcoustic : kRecElastic;
  const int nrf = s->physics == DG_ACOUSTIC ? 1 : 3;
  for (int i = 0; i < f->nrec; ++i) {
    const int64_t k = f->rec_elem_h[static_cast<size_t>(i)];
    const double* v = s->elem_xyz.data() + 12 * k;
    double F[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) F[a][b] = 0.5 * (v[3 * (b + 1) + a] - v[a]);
    const double Jk = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                      F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                      F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    std::vector<double> mw(static_cast<size_t>(Np), 0.0);
    for (int n = 0; n < Np; ++n)
      for (int m = 0; m < Np; ++m) mw[n] += ref->minv[n * Np + m] * f->rec_w[static_cast<size_t>(i)][m];
    for (int c = 0; c < nrf; ++c) {
      const int field = rf[c];
      double scale;
      if (s->physics == DG_ACOUSTIC) {
        const double rho = coef[2 * k], cc = coef[2 * k + 1];
        scale = field == 0 ? rho * cc * cc : -1.0 / rho;
      } else {
        scale = -1.0 / coef[3 * k];  // velocity receivers
      }
      std::vector<double> vec(static_cast<size_t>(Np));
      for (int n = 0; n < Np; ++n) vec[n] = f->dt * scale / Jk * mw[n];
      entries.push_back(Entry{k, field, i * nrf + c, vec});
    }
  }
  return group_entries(entries);
}

// Builds a misfit in `workspace` (device, ws_bytes); with a null workspace
// only the bytes it needs are computed (*need), nothing is returned.
dg_status misfit_build(dg_solver* s, int64_t nsteps, double dt, int checkpoint_every, int nsrc,
                       const double* src_xyz, const double* wavelet, int nrec, const double* rec_xyz,
                       void* workspace, size_t ws_bytes, size_t* need, dg_misfit** out);

}  // namespace

extern "C" {

dg_status dg_locate_points(dg_solver* s, int64_t n, const double* xyz, int64_t* elem, double* weights) {
  if (!s || n < 0 || (n > 0 && (!xyz || !elem))) {
    set_error("dg_locate_points: bad arguments");
    return DG_E_ARG;
  }
  const dgw::RefElement* ref = dgw::reference_element(s->N);
  for (int64_t p = 0; p < n; ++p) {
    double xi[3];
    if (!locate_point(s, xyz + 3 * p, elem + p, xi)) {
      std::ostringstream os;
      os << "point " << p << " (" << xyz[3 * p] << ", " << xyz[3 * p + 1] << ", " << xyz[3 * p + 2]
         << ") is outside the mesh";
      set_error(os.str());
      return DG_E_ARG;
    }
    if (weights) dgw::lagrange_weights(ref, xi, weights + p * ref->Np);
  }
  return DG_OK;
}

dg_status dg_misfit_workspace_bytes(dg_solver* s, int64_t nsteps, double dt, int checkpoint_every, int nsrc,
                                    const double* src_xyz, const double* wavelet, int nrec, const double* rec_xyz,
                                    size_t* bytes) {
  if (!bytes) {
    set_error("dg_misfit_workspace_bytes: null output");
    return DG_E_ARG;
  }
  return misfit_build(s, nsteps, dt, checkpoint_every, nsrc, src_xyz, wavelet, nrec, rec_xyz, nullptr, 0, bytes,
                      nullptr);
}

dg_status dg_misfit_create(dg_solver* s, int64_t nsteps, double dt, int checkpoint_every, int nsrc,
                           const double* src_xyz, const double* wavelet, int nrec, const double* rec_xyz,
                           void* workspace, size_t workspace_bytes, dg_misfit** out) {
  if (!out) {
    set_error("dg_misfit_create: null output");
    return DG_E_ARG;
  }
  *out = nullptr;
  if (!workspace || !dgw::workspace_aligned(workspace)) {
    set_error("dg_misfit_create: the workspace must be a non-null device pointer aligned to 256 bytes");
    return DG_E_ARG;
  }
  size_t need = 0;
  return misfit_build(s, nsteps, dt, checkpoint_every, nsrc, src_xyz, wavelet, nrec, rec_xyz, workspace,
                      workspace_bytes, &need, out);
}

void dg_misfit_destroy(dg_misfit* f) {
  if (!f) return;
  (void)hipStreamSynchronize(f->s->stream);
  delete f;
}

int64_t dg_misfit_channels(dg_misfit* f) { return f ? f->R : -1; }

// The projected point source b = (1/J_k) M^-1 l(x_s) grows with the mesh's
// resolution far beyond FP16's range, so the FP16 split products, whose
// operands must stay below 65504, are refused for misfits.
static dg_status check_misfit_variant(const dg_solver* s) {
  if (s->variant == dgw::kVariantMfmaF16) {
    set_error("misfits need a variant with the FP32 exponent range (the FP16 split products overflow on the "
              "projected point source): use DG_VARIANT_VALU, _MFMA, _MFMA_BF16 or _ELEM");
    return DG_E_UNSUPPORTED;
  }
  return DG_OK;
}

dg_status dg_misfit_forward(dg_misfit* f, const float* data, float* traces, double* J) {
  if (!f) {
    set_error("null misfit");
    return DG_E_ARG;
  }
  dg_solver* s = f->s;
  if (!s->have_coef) {
    set_error("set coefficients before the misfit");
    return DG_E_STATE;
  }
  if (dg_status st = check_misfit_variant(s)) return st;
  const size_t ntrace = static_cast<size_t>(f->M + 1) * f->R;
  // zero state, zero history, zero traces
  DG_HIP(dgw::launch_fill_zero_f32(static_cast<int64_t>(f->nq), seg_q(f, 0), s->stream));
  DG_HIP(dgw::launch_fill_zero_f32(static_cast<int64_t>(f->ntr), seg_tr(f, 0), s->stream));
  DG_HIP(dgw::launch_fill_zero_f32(static_cast<int64_t>(3 * f->nq), f->ck.p, s->stream));
  DG_HIP(dgw::launch_fill_zero_f32(static_cast<int64_t>(f->R), f->traces.p, s->stream));
  const int64_t nseg = num_segments(f);
  for (int64_t seg = 0; seg < nseg; ++seg) {
    if (seg > 0) {
      // checkpoint: the state at the segment start and its two previous rhs
      const size_t b = f->nq * sizeof(float);
      DG_HIP(hipMemcpyAsync(ck_q(f, seg), seg_q(f, f->C), b, hipMemcpyDeviceToDevice, s->stream));
      DG_HIP(hipMemcpyAsync(ck_r1(f, seg), seg_r(f, f->C - 1), b, hipMemcpyDeviceToDevice, s->stream));
      if (f->C >= 2)
        DG_HIP(hipMemcpyAsync(ck_r2(f, seg), seg_r(f, f->C - 2), b, hipMemcpyDeviceToDevice, s->stream));
      else
        DG_HIP(hipMemcpyAsync(ck_r2(f, seg), ck_r1(f, seg - 1), b, hipMemcpyDeviceToDevice, s->stream));
      DG_HIP(hipMemcpyAsync(seg_q(f, 0), seg_q(f, f->C), b, hipMemcpyDeviceToDevice, s->stream));
      DG_HIP(hipMemcpyAsync(seg_tr(f, 0), seg_tr(f, f->C), f->ntr * sizeof(float), hipMemcpyDeviceToDevice,
                            s->stream));
    }
    if (dg_status st = run_segment(f, seg, true)) return st;
  }
  f->have_forward = true;
  f->fwd_coef_gen = s->coef_gen;
  if (traces)
    DG_HIP(hipMemcpyAsync(traces, f->traces.p, ntrace * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  f->have_data = data != nullptr;
  if (data) {
    DG_HIP(hipMemcpyAsync(f->data.p, data, ntrace * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
    if (J) {
      std::vector<float> u(ntrace), d(ntrace);
      DG_HIP(hipMemcpyAsync(u.data(), f->traces.p, ntrace * sizeof(float), hipMemcpyDeviceToHost, s->stream));
      DG_HIP(hipMemcpyAsync(d.data(), f->data.p, ntrace * sizeof(float), hipMemcpyDeviceToHost, s->stream));
      DG_HIP(hipStreamSynchronize(s->stream));
      double acc = 0.0;
      for (size_t i = static_cast<size_t>(f->R); i < ntrace; ++i) {
        const double r = static_cast<double>(u[i]) - static_cast<double>(d[i]);
        acc += r * r;
      }
      *J = 0.5 * f->dt * acc;
      if (!std::isfinite(*J)) {
        set_error("dg_misfit_forward: the misfit is not finite");
        return DG_E_UNSTABLE;
      }
    }
  } else if (J) {
    *J = 0.0;
  }
  return DG_OK;
}

dg_status dg_misfit_gradient(dg_misfit* f, float* grad) {
  if (!f || !grad) {
    set_error("dg_misfit_gradient: null argument");
    return DG_E_ARG;
  }
  if (!f->have_forward || !f->have_data) {
    set_error("dg_misfit_gradient needs a preceding dg_misfit_forward with data");
    return DG_E_STATE;
  }
  dg_solver* s = f->s;
  if (dg_status st = check_misfit_variant(s)) return st;
  if (s->coef_gen != f->fwd_coef_gen) {
    set_error("dg_misfit_gradient: the coefficients changed after the last dg_misfit_forward");
    return DG_E_STATE;
  }
  // adjoint source vectors with the current coefficients
  std::vector<float> coef(static_cast<size_t>(s->K) * s->ncoef);
  DG_HIP(hipMemcpyAsync(coef.data(), s->coef, coef.size() * sizeof(float), hipMemcpyDeviceToHost, s->stream));
  DG_HIP(hipStreamSynchronize(s->stream));
  const HostInject adj_h = adjoint_entries(f, coef);
  DG_HIP(f->adj.upload(adj_h, s->stream));
  DG_HIP(hipStreamSynchronize(s->stream));  // adj_h dies at return

  auto phi = [&](int64_t j) { return f->phi.p + (j % 4) * f->nq; };
  auto aring = [&](int64_t j) { return f->aring.p + (j % 3) * f->nq; };
  auto coefs = [&](int64_t j, int i) { return (j >= 0 && j <= f->M - 1) ? ab(j, i) : 0.0; };
  DG_HIP(dgw::launch_fill_zero_f32(static_cast<int64_t>(4 * f->nq), f->phi.p, s->stream));
  DG_HIP(dgw::launch_fill_zero_f32(static_cast<int64_t>(3 * f->nq), f->aring.p, s->stream));
  DG_HIP(dgw::launch_fill_zero_f32(static_cast<int64_t>(2 * f->ntr), f->atr.p, s->stream));
  DG_HIP(dgw::launch_fill_zero_f64(static_cast<int64_t>(s->K) * dgw::kGradAccStride, f->gacc.p, s->stream));
  int cur = 0;
  // phi_M = P W^{-1} g_M
  {
    dgw::InjectArgs ia = inject_args(f, f->adj, phi(f->M), f->atr.p + cur * f->ntr);
    ia.traces = f->traces.p + f->M * f->R;
    ia.data = f->data.p + f->M * f->R;
    DG_HIP(dgw::launch_inject(s->physics, s->N, ia, s->stream));
  }
  const int64_t nseg = num_segments(f);
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t ms = seg * f->C, me = std::min(ms + f->C, f->M);
    if (f->seg_loaded != seg) {
      if (dg_status st = load_segment_start(f, seg)) return st;
      if (dg_status st = run_segment(f, seg, false)) return st;
    }
    for (int64_t m = me - 1; m >= ms; --m) {
      const float c0 = static_cast<float>(f->dt * coefs(m, 0));
      const float c1 = static_cast<float>(f->dt * coefs(m + 1, 1));
      const float c2 = static_cast<float>(f->dt * coefs(m + 2, 2));
      // gradient terms at step m (phi_{m+1..m+3} are all still in the ring)
      dgw::GradArgs g{};
      g.K = s->K;
      g.phi1 = phi(m + 1);
      g.phi2 = phi(m + 2);
      g.phi3 = phi(m + 3);
      g.c0 = c0;
      g.c1 = c1;
      g.c2 = c2;
      g.r = seg_r(f, m - ms);
      g.tr = seg_tr(f, m - ms);
      g.geo = s->geo;
      g.cf = s->cf;
      g.conn = s->conn;
      g.fmask = s->fmask;
      g.perm = s->perm;
      g.mass_pack = f->mass_pack_f.p;
      g.face_mass = f->face_mass_f.p;
      g.J = s->J;
      g.gacc = f->gacc.p;
      DG_HIP(dgw::launch_grad_accum(s->physics, s->N, g, s->stream));
      // phi_m = phi_{m+1} + A(c0 phi_{m+1} + c1 phi_{m+2} + c2 phi_{m+3}) + P W^{-1} g_m
      dgw::StepArgs a = dgw::base_args(s);
      a.mode = dgw::kStepMode;
      a.c0 = c0;
      a.c1 = c1;
      a.c2 = c2;
      a.q_in = phi(m + 1);
      a.q_out = phi(m);
      a.r_out = aring(m + 1);
      a.r1 = aring(m + 2);
      a.r2 = aring(m + 3);
      a.qf_in = f->atr.p + cur * f->ntr;
      a.qf_out = f->atr.p + (cur ^ 1) * f->ntr;
      DG_HIP(dgw::launch_step(s->physics, s->N, s->variant, a, s->stream));
      cur ^= 1;
      if (m >= 1) {
        dgw::InjectArgs ia = inject_args(f, f->adj, phi(m), f->atr.p + cur * f->ntr);
        ia.traces = f->traces.p + m * f->R;
        ia.data = f->data.p + m * f->R;
        DG_HIP(dgw::launch_inject(s->physics, s->N, ia, s->stream));
      }
    }
  }
  f->seg_loaded = -1;
  DG_HIP(dgw::launch_grad_finalize(s->physics, s->K, f->gacc.p, s->conn, s->coef, grad, s->stream));
  return DG_OK;
}

}  // extern "C"

namespace {

dg_status misfit_build(dg_solver* s, int64_t nsteps, double dt, int checkpoint_every, int nsrc,
                       const double* src_xyz, const double* wavelet, int nrec, const double* rec_xyz,
                       void* workspace, size_t ws_bytes, size_t* need, dg_misfit** out) {
  if (!s || nsteps < 1 || !(dt > 0.0) || checkpoint_every < 1 || nsrc < 0 || nrec < 1 ||
      (nsrc > 0 && (!src_xyz || !wavelet)) || !rec_xyz) {
    set_error("dg_misfit_create: bad arguments");
    return DG_E_ARG;
  }
  if (s->physics == DG_ANISOTROPIC) {
    set_error("dg_misfit_create: the adjoint gradient is built for the acoustic and elastic physics only");
    return DG_E_UNSUPPORTED;
  }
  std::unique_ptr<dg_misfit> f(new dg_misfit);
  f->s = s;
  f->M = nsteps;
  f->C = static_cast<int>(std::min<int64_t>(checkpoint_every, nsteps));
  f->dt = dt;
  f->nrec = nrec;
  const dgw::RefElement* ref = dgw::reference_element(s->N);
  const int Np = ref->Np;
  const int* sf = s->physics == DG_ACOUSTIC ? kSrcAcoustic : kSrcElastic;
  const int nsf = s->physics == DG_ACOUSTIC ? 1 : 3;
  const int* rf = s->physics == DG_ACOUSTIC ? kRecAcoustic : kRecElastic;
  const int nrf = s->physics == DG_ACOUSTIC ? 1 : 3;
  f->R = nrec * nrf;
  f->wavelet.assign(static_cast<size_t>(nsteps + 1), 0.0);
  if (nsrc > 0) std::copy(wavelet, wavelet + nsteps + 1, f->wavelet.begin());

  // host geometry for J_k
  auto jac = [&](int64_t k) {
    const double* v = s->elem_xyz.data() + 12 * k;
    double F[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) F[i][j] = 0.5 * (v[3 * (j + 1) + i] - v[i]);
    return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
           F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  };
  // sources: b = (1/J_k) M^{-1} l(xi_s) in every source field
  std::vector<Entry> src_entries;
  std::vector<int64_t> pe(static_cast<size_t>(std::max(nsrc, nrec)));
  std::vector<double> pw(static_cast<size_t>(std::max(nsrc, nrec)) * Np);
  if (nsrc > 0) {
    if (dg_status st = dg_locate_points(s, nsrc, src_xyz, pe.data(), pw.data())) return st;
    for (int i = 0; i < nsrc; ++i) {
      std::vector<double> b(static_cast<size_t>(Np), 0.0);
      const double Jk = jac(pe[i]);
      for (int n = 0; n < Np; ++n)
        for (int m = 0; m < Np; ++m) b[n] += ref->minv[n * Np + m] * pw[i * Np + m] / Jk;
      for (int c = 0; c < nsf; ++c) src_entries.push_back(Entry{pe[i], sf[c], -1, b});
    }
  }
  // receivers: channel ch = (receiver, field)
  if (dg_status st = dg_locate_points(s, nrec, rec_xyz, pe.data(), pw.data())) return st;
  std::vector<int64_t> che;
  std::vector<int32_t> chf;
  std::vector<float> chw;
  for (int i = 0; i < nrec; ++i) {
    f->rec_elem_h.push_back(pe[i]);
    f->rec_w.emplace_back(pw.begin() + i * Np, pw.begin() + (i + 1) * Np);
    for (int c = 0; c < nrf; ++c) {
      che.push_back(pe[i]);
      chf.push_back(rf[c]);
      for (int n = 0; n < Np; ++n) chw.push_back(static_cast<float>(pw[i * Np + n]));
    }
  }
  f->nq = static_cast<size_t>(s->K) * s->NF * s->Np;
  f->ntr = static_cast<size_t>(s->K) * 4 * s->NT * s->Nfp;
  const size_t nseg = static_cast<size_t>(num_segments(f.get()));
  const HostInject src_h = group_entries(src_entries);
  // the adjoint source list has the receivers' shape; its values follow the
  // coefficients and are written by each gradient call
  const HostInject adj_h = adjoint_entries(f.get(), std::vector<float>(static_cast<size_t>(s->K) * s->ncoef, 1.0f));
  // the mass matrix in the fragment order of the gradient kernel's products
  std::vector<float> mf, fmf(ref->face_mass.begin(), ref->face_mass.end());
  dgw::pack_fp32(ref->mass.data(), s->Np, s->Np, (s->Np + 15) / 16, (s->Np + 3) / 4 * 4, mf);

  // ---- layout in the workspace ----
  dgw::Arena arena(workspace, ws_bytes);
  f->src.carve(arena, src_h);
  f->adj.carve(arena, adj_h);
  f->ch_elem.carve(arena, che.size());
  f->ch_field.carve(arena, chf.size());
  f->ch_w.carve(arena, chw.size());
  f->traces.carve(arena, static_cast<size_t>(nsteps + 1) * f->R);
  f->data.carve(arena, static_cast<size_t>(nsteps + 1) * f->R);
  f->seg_q.carve(arena, (f->C + 1) * f->nq);
  f->seg_tr.carve(arena, (f->C + 1) * f->ntr);
  f->seg_r.carve(arena, f->C * f->nq);
  f->ck.carve(arena, 3 * nseg * f->nq);
  f->phi.carve(arena, 4 * f->nq);
  f->aring.carve(arena, 3 * f->nq);
  f->atr.carve(arena, 2 * f->ntr);
  f->gacc.carve(arena, static_cast<size_t>(s->K) * dgw::kGradAccStride);
  f->mass_pack_f.carve(arena, mf.size());
  f->face_mass_f.carve(arena, fmf.size());
  if (need) *need = arena.used();
  if (!workspace) return DG_OK;
  if (!arena.fits()) {
    std::ostringstream os;
    os << "dg_misfit_create: workspace holds " << ws_bytes << " bytes, the misfit needs " << arena.used();
    set_error(os.str());
    return DG_E_SHAPE;
  }
  hipError_t err = f->src.upload(src_h, s->stream);
  if (err == hipSuccess) err = f->adj.upload(adj_h, s->stream);
  if (err == hipSuccess) err = f->ch_elem.upload(che, s->stream);
  if (err == hipSuccess) err = f->ch_field.upload(chf, s->stream);
  if (err == hipSuccess) err = f->ch_w.upload(chw, s->stream);
  if (err == hipSuccess) err = f->mass_pack_f.upload(mf, s->stream);
  if (err == hipSuccess) err = f->face_mass_f.upload(fmf, s->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(s->stream);  // the host arrays die here
  if (err != hipSuccess) {
    set_error(std::string("dg_misfit_create: upload: ") + hipGetErrorString(err));
    return DG_E_HIP;
  }
  *out = f.release();
  return DG_OK;
}

}  // namespace
