// Kernel choice per solver (autotuning) and batches of meshes stepped with
// one launch per (degree, variant) group.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "dg_internal.hpp"
#include "dgwave.h"
#include "kernels.hpp"
#include "solver_state.hpp"
#include "workspace.hpp"

using dgw::set_error;

namespace {

size_t field_floats(const dg_solver* s) { return static_cast<size_t>(s->K) * s->NF * s->Np; }

}  // namespace

struct dg_batch_group {
  int N = 0, variant = 0;
  std::vector<int> members;           // indices into dg_batch::members
  dgw::StepArgs* args = nullptr;      // device [members][kBatchPhases], in the workspace
  int2* work = nullptr;               // device [nwork] (member slot, tile), in the workspace
  int64_t tiles = 0;                  // real work items
  int64_t nwork = 0;                  // launched workgroups (one per work item)
};

struct dg_batch {
  std::vector<dg_solver*> members;
  int physics = 0;
  hipStream_t stream = nullptr;
  void* ws = nullptr;                 // caller-owned device workspace
  size_t ws_bytes = 0;
  std::vector<dg_batch_group> groups;
  std::vector<int> group_variant;     // member variants the groups were built for
  // argument tables: valid for member i at step m0[i] + p with trace buffer
  // cur0[i] ^ (p & 1), for every p >= 0 (the tables have period kBatchPhases)
  bool tables_valid = false;
  std::vector<int64_t> m0;
  std::vector<int> cur0;
  std::vector<double> dt;
  int64_t p = 0;                      // batched steps since the tables were built
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // one side stream per launch group (default priority): the groups' members
  // are independent meshes, so their launches run concurrently, forked from
  // and joined back to the batch's stream
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
};

namespace {

void free_groups(dg_batch* b) { b->groups.clear(); }

// Most work items a member can contribute: its tile count under the variant
// with the most tiles (the groups are rebuilt when a variant changes).
int64_t max_member_tiles(int physics, const dg_solver* s) {
  int64_t most = 0;
  for (int v = 0; v < dgw::kNumVariants; ++v)
    if (dgw::variant_supported(physics, s->N, v)) most = std::max(most, dgw::tiles_for(physics, s->N, v, s->K));
  return most;
}

// Workspace bytes that cover every grouping of the members: at most one group
// per member, each group's work list (rounded up to 8 entries), plus the
// alignment of every array.
size_t batch_bytes(int physics, dg_solver* const* members, int count) {
  size_t bytes = 0;
  for (int i = 0; i < count; ++i) {
    const int64_t t = max_member_tiles(physics, members[i]);
    bytes += dgw::align_up(dgw::kBatchPhases * sizeof(dgw::StepArgs));
    bytes += dgw::align_up(static_cast<size_t>((t + 7) / 8 * 8) * sizeof(int2));
    bytes += 2 * dgw::kWorkspaceAlign;
  }
  return bytes;
}

void drop_graph(dg_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

dg_status build_groups(dg_batch* b) {
  if (b->stream) DG_HIP(hipStreamSynchronize(b->stream));
  else DG_HIP(hipDeviceSynchronize());
  drop_graph(b);
  free_groups(b);
  b->tables_valid = false;
  b->group_variant.clear();
  std::vector<std::pair<int, int>> keys;
  for (dg_solver* s : b->members) {
    b->group_variant.push_back(s->variant);
    const std::pair<int, int> key(s->N, s->variant);
    if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
  }
  std::sort(keys.begin(), keys.end());
  dgw::Arena arena(b->ws, b->ws_bytes);
  for (const auto& key : keys) {
    dg_batch_group g;
    g.N = key.first;
    g.variant = key.second;
    std::vector<int2> items;
    for (int i = 0; i < static_cast<int>(b->members.size()); ++i) {
      const dg_solver* s = b->members[static_cast<size_t>(i)];
      if (s->N != g.N || s->variant != g.variant) continue;
      const int slot = static_cast<int>(g.members.size());
      g.members.push_back(i);
      const int64_t nt = dgw::tiles_for(b->physics, g.N, g.variant, s->K);
      if (nt < 0) {
        set_error("batch member has a kernel variant that is not built");
        return DG_E_UNSUPPORTED;
      }
      for (int64_t t = 0; t < nt; ++t) {
        if (t > 0x7fffffff) {
          set_error("batch member too large");
          return DG_E_SHAPE;
        }
        items.push_back(int2{slot, static_cast<int>(t)});
      }
    }
    g.tiles = static_cast<int64_t>(items.size());
    // launch order = (member, tile) order: the tiles in flight stay one
    // contiguous window of each member's arrays (a per-XCD split of the list
    // measured 1.5 % slower)
    const std::vector<int2>& work = items;
    g.nwork = static_cast<int64_t>(work.size());
    if (g.nwork > 0x7fffffff) {
      set_error("batch launch too large");
      return DG_E_SHAPE;
    }
    b->groups.push_back(g);
    dg_batch_group& gg = b->groups.back();
    gg.args = arena.take<dgw::StepArgs>(gg.members.size() * dgw::kBatchPhases);
    gg.work = arena.take<int2>(work.size());
    if (!arena.fits()) {
      std::ostringstream os;
      os << "batch workspace of " << b->ws_bytes << " bytes is too small (dg_batch_workspace_bytes)";
      set_error(os.str());
      free_groups(b);
      return DG_E_SHAPE;
    }
    if (!work.empty()) {
      DG_HIP(hipMemcpyAsync(gg.work, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
      DG_HIP(hipStreamSynchronize(b->stream));
    }
  }
  return DG_OK;
}

// Fill the argument tables from the members' current state.  Rare (after a
// start-up step, a state change outside the batch or a new dt), so the upload
// synchronises.
dg_status build_tables(dg_batch* b, const double* dt) {
  const size_t n = b->members.size();
  b->m0.resize(n);
  b->cur0.resize(n);
  b->dt.assign(dt, dt + n);
  for (size_t i = 0; i < n; ++i) {
    b->m0[i] = b->members[i]->m;
    b->cur0[i] = b->members[i]->cur;
  }
  for (dg_batch_group& g : b->groups) {
    std::vector<dgw::StepArgs> h(g.members.size() * dgw::kBatchPhases);
    for (size_t slot = 0; slot < g.members.size(); ++slot) {
      const int i = g.members[slot];
      const dg_solver* s = b->members[static_cast<size_t>(i)];
      for (int ph = 0; ph < dgw::kBatchPhases; ++ph)
        h[slot * dgw::kBatchPhases + ph] = dgw::step_args(s, b->m0[i] + ph, b->cur0[i] ^ (ph & 1), b->dt[i]);
    }
    DG_HIP(hipMemcpyAsync(g.args, h.data(), h.size() * sizeof(dgw::StepArgs), hipMemcpyHostToDevice, b->stream));
    DG_HIP(hipStreamSynchronize(b->stream));
  }
  b->p = 0;
  b->tables_valid = true;
  return DG_OK;
}

bool tables_match(const dg_batch* b, const double* dt) {
  if (!b->tables_valid) return false;
  for (size_t i = 0; i < b->members.size(); ++i) {
    const dg_solver* s = b->members[i];
    if (s->m != b->m0[i] + b->p || s->cur != (b->cur0[i] ^ static_cast<int>(b->p & 1))) return false;
    if (dt[i] != b->dt[i]) return false;
  }
  return true;
}

dg_status ensure_side_streams(dg_batch* b) {
  if (!b->fork) DG_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  while (b->side.size() < b->groups.size()) {
    hipStream_t st = nullptr;
    DG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    b->side.push_back(st);
    hipEvent_t ev = nullptr;
    DG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    b->join.push_back(ev);
  }
  return DG_OK;
}

// Phases [ph0, ph1) of every group.  One group launches on the batch's stream;
// several fork onto their own streams (each group's phases in order) and
// join back, so that one group's launch tail overlaps another's work.
dg_status launch_groups(dg_batch* b, int ph0, int ph1) {
  if (b->groups.size() == 1) {
    const dg_batch_group& g = b->groups[0];
    for (int ph = ph0; ph < ph1; ++ph)
      DG_HIP(dgw::launch_step_batch(b->physics, g.N, g.variant, g.args, g.work, g.nwork, ph, b->stream));
    return DG_OK;
  }
  if (dg_status st = ensure_side_streams(b)) return st;
  DG_HIP(hipEventRecord(b->fork, b->stream));
  for (size_t i = 0; i < b->groups.size(); ++i) {
    const dg_batch_group& g = b->groups[i];
    DG_HIP(hipStreamWaitEvent(b->side[i], b->fork, 0));
    for (int ph = ph0; ph < ph1; ++ph)
      DG_HIP(dgw::launch_step_batch(b->physics, g.N, g.variant, g.args, g.work, g.nwork, ph, b->side[i]));
    DG_HIP(hipEventRecord(b->join[i], b->side[i]));
    DG_HIP(hipStreamWaitEvent(b->stream, b->join[i], 0));
  }
  return DG_OK;
}

void release_streams(dg_batch* b) {
  for (hipStream_t st : b->side) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->join) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  b->side.clear();
  b->join.clear();
  b->fork = nullptr;
}

void advance_members(dg_batch* b, int steps) {
  for (dg_solver* s : b->members) {
    s->m += steps;
    s->cur ^= (steps & 1);
  }
  b->p += steps;
}

}  // namespace

extern "C" {

dg_status dg_autotune(dg_solver* s, int steps, double dt, unsigned candidates, void* scratch,
                      size_t scratch_bytes, double* us_per_step) {
  if (!s) {
    set_error("null solver");
    return DG_E_ARG;
  }
  if (steps < 1 || !(dt > 0.0) || !std::isfinite(dt)) {
    set_error("steps must be >= 1 and dt > 0");
    return DG_E_ARG;
  }
  if (!s->have_coef || !s->have_fields) {
    set_error("set coefficients and fields before tuning");
    return DG_E_STATE;
  }
  const size_t need = field_floats(s) * sizeof(float);
  if (!scratch || scratch_bytes < need) {
    std::ostringstream os;
    os << "dg_autotune: scratch must hold one field array (" << need << " bytes)";
    set_error(os.str());
    return DG_E_ARG;
  }
  // Every timed step reads the current state and writes only memory that
  // holds nothing the state needs: the updated fields go to the caller's
  // scratch, r^m to the ring slot of r^{m-3} and the traces to the buffer the
  // next step would overwrite.  The state is untouched, so there is nothing
  // to restore.  Every step uses the AB3 weights (the start-up steps read
  // less history and would time short).
  dgw::StepArgs a = dgw::step_args(s, s->m, s->cur, dt);
  a.q_out = static_cast<float*>(scratch);
  a.c0 = static_cast<float>(dt * 23.0 / 12.0);
  a.c1 = static_cast<float>(dt * -16.0 / 12.0);
  a.c2 = static_cast<float>(dt * 5.0 / 12.0);
  const int variant_saved = s->variant;

  hipEvent_t e0 = nullptr, e1 = nullptr;
  DG_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("dg_autotune: hipEventCreate failed");
    return DG_E_HIP;
  }
  double best = -1.0;
  int best_variant = variant_saved;
  dg_status st = DG_OK;
  for (int v = 0; v < DG_NUM_VARIANTS && st == DG_OK; ++v) {
    double us = -1.0;
    const bool wanted = candidates == 0u || ((candidates >> v) & 1u);
    if (wanted && dgw::variant_supported(s->physics, s->N, v)) {
      s->variant = v;
      const dgw::StepArgs base = dgw::base_args(s);  // the variant's operator tables
      dgw::StepArgs av = a;
      av.D16h = base.D16h;
      av.D16l = base.D16l;
      av.L16h = base.L16h;
      av.L16l = base.L16l;
      hipError_t err = hipSuccess;
      for (int i = 0; i <= steps && err == hipSuccess; ++i) {
        if (i == 1) err = hipEventRecord(e0, s->stream);
        if (err == hipSuccess) err = dgw::launch_step(s->physics, s->N, v, av, s->stream);
      }
      if (err == hipSuccess) err = hipEventRecord(e1, s->stream);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) {
        set_error(std::string("autotune: ") + hipGetErrorString(err));
        st = DG_E_HIP;
      }
      us = 1000.0 * ms / steps;
      if (st == DG_OK && (best < 0.0 || us < best)) {
        best = us;
        best_variant = v;
      }
    }
    if (us_per_step) us_per_step[v] = us;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->variant = st == DG_OK ? best_variant : variant_saved;
  return st;
}

dg_status dg_batch_workspace_bytes(dg_solver* const* members, int count, size_t* bytes) {
  if (!members || !bytes || count < 1) {
    set_error("dg_batch_workspace_bytes: need members, a count >= 1 and an output");
    return DG_E_ARG;
  }
  for (int i = 0; i < count; ++i)
    if (!members[i]) {
      set_error("dg_batch_workspace_bytes: null member");
      return DG_E_ARG;
    }
  *bytes = batch_bytes(members[0]->physics, members, count);
  return DG_OK;
}

dg_status dg_batch_create(dg_solver* const* members, int count, void* workspace, size_t workspace_bytes,
                          void* stream, dg_batch** out) {
  if (!members || !out || count < 1) {
    set_error("dg_batch_create: need an output pointer and at least one member");
    return DG_E_ARG;
  }
  if (!workspace || !dgw::workspace_aligned(workspace)) {
    set_error("dg_batch_create: the workspace must be a non-null device pointer aligned to 256 bytes");
    return DG_E_ARG;
  }
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    if (!members[i]) {
      set_error("dg_batch_create: null member");
      return DG_E_ARG;
    }
    if (members[i]->physics != members[0]->physics || members[i]->device != members[0]->device) {
      set_error("dg_batch_create: members must share physics and device");
      return DG_E_ARG;
    }
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) {
        set_error("dg_batch_create: repeated member");
        return DG_E_ARG;
      }
  }
  const size_t need = batch_bytes(members[0]->physics, members, count);
  if (workspace_bytes < need) {
    std::ostringstream os;
    os << "dg_batch_create: workspace holds " << workspace_bytes << " bytes, the batch needs " << need;
    set_error(os.str());
    return DG_E_SHAPE;
  }
  dg_batch* b = new dg_batch;
  b->members.assign(members, members + count);
  b->physics = members[0]->physics;
  b->stream = static_cast<hipStream_t>(stream);
  b->ws = workspace;
  b->ws_bytes = workspace_bytes;
  if (dg_status st = build_groups(b)) {
    free_groups(b);
    delete b;
    return st;
  }
  *out = b;
  return DG_OK;
}

void dg_batch_destroy(dg_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  free_groups(b);
  release_streams(b);
  delete b;
}

dg_status dg_batch_set_graph(dg_batch* b, int enable) {
  if (!b) {
    set_error("null batch");
    return DG_E_ARG;
  }
  if (enable && !b->stream) {
    set_error("graph replay needs a non-default stream");
    return DG_E_STATE;
  }
  if (!enable) drop_graph(b);
  b->use_graph = enable != 0;
  return DG_OK;
}

dg_status dg_batch_step(dg_batch* b, int nsteps, const double* dt) {
  if (!b || !dt || nsteps < 0) {
    set_error("dg_batch_step: bad arguments");
    return DG_E_ARG;
  }
  const size_t n = b->members.size();
  for (size_t i = 0; i < n; ++i) {
    const dg_solver* s = b->members[i];
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) {
      set_error("dg_batch_step: every dt must be positive and finite");
      return DG_E_ARG;
    }
    if (!s->have_coef || !s->have_fields) {
      set_error("dg_batch_step: a member has no coefficients or fields");
      return DG_E_STATE;
    }
    if (s->k_fast > 0) {
      set_error("dg_batch_step: a member has a fast class (two-rate members step with dg_step_multirate)");
      return DG_E_STATE;
    }
  }
  for (size_t i = 0; i < n; ++i)
    if (b->members[i]->variant != b->group_variant[i]) {
      if (dg_status st = build_groups(b)) return st;
      break;
    }
  int done = 0;
  while (done < nsteps) {
    bool startup = false;
    for (const dg_solver* s : b->members) startup = startup || s->m < 2;
    if (startup) {
      // start-up steps use their own coefficients: one launch per member
      for (size_t i = 0; i < n; ++i) {
        dg_solver* s = b->members[i];
        const dgw::StepArgs a = dgw::step_args(s, s->m, s->cur, dt[i]);
        DG_HIP(dgw::launch_step(s->physics, s->N, s->variant, a, b->stream));
        s->m += 1;
        s->cur ^= 1;
      }
      b->tables_valid = false;
      ++done;
      continue;
    }
    if (!tables_match(b, dt))
      if (dg_status st = build_tables(b, dt)) return st;
    const int phase = static_cast<int>(b->p % dgw::kBatchPhases);
    if (b->use_graph && phase == 0 && nsteps - done >= dgw::kBatchPhases) {
      if (!b->exec) {
        DG_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        dg_status st = DG_OK;
        st = launch_groups(b, 0, dgw::kBatchPhases);
        hipGraph_t graph = nullptr;
        const hipError_t cerr = hipStreamEndCapture(b->stream, &graph);
        if (st != DG_OK) {
          if (graph) (void)hipGraphDestroy(graph);
          return st;
        }
        DG_HIP(cerr);
        b->graph = graph;
        DG_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      }
      DG_HIP(hipGraphLaunch(b->exec, b->stream));
      advance_members(b, dgw::kBatchPhases);
      done += dgw::kBatchPhases;
      continue;
    }
    if (dg_status st = launch_groups(b, phase, phase + 1)) return st;
    advance_members(b, 1);
    ++done;
  }
  return DG_OK;
}

dg_status dg_batch_groups(dg_batch* b, int* ngroups, int32_t* order, int32_t* variant, int64_t* tiles) {
  if (!b || !ngroups) {
    set_error("null argument");
    return DG_E_ARG;
  }
  const int n = static_cast<int>(b->groups.size());
  const bool fill = order || variant || tiles;
  const int cap = *ngroups;
  *ngroups = n;
  if (!fill) return DG_OK;
  if (cap < n) {
    set_error("group arrays too small");
    return DG_E_SHAPE;
  }
  for (int i = 0; i < n; ++i) {
    const dg_batch_group& g = b->groups[static_cast<size_t>(i)];
    if (order) order[i] = g.N;
    if (variant) variant[i] = g.variant;
    if (tiles) tiles[i] = g.nwork;
  }
  return DG_OK;
}

}  // extern "C"
