// Host-side entry points of the dgwave C ABI under AddressSanitizer.
//
// Built by tests/test_asan_host.py: the host C++ sources of the library with
// -fsanitize=address (host code only), linked with the normally built device
// objects.  Every call here returns before any device work: reference
// operators, face permutations, connectivity, workspace sizes, and the
// set-up and validation paths of dg_create (geometry, connectivity, operator
// packing and the workspace layout) with a stand-in workspace that the size
// check refuses.  Exit status 0 when every expectation holds; ASan aborts the
// process on a memory error.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "dgwave.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what, dg_last_error());
    ++failures;
  }
}

// Kuhn box of n^3 subcubes, six tetrahedra each (vertex ids on the (n+1)^3
// grid, positively oriented), coordinates of the unit cube.
static void kuhn_box(int n, std::vector<double>& xyz, std::vector<int64_t>& topo) {
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  static const int odd[6] = {0, 1, 1, 0, 0, 1};
  const double h = 1.0 / n;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        for (int p = 0; p < 6; ++p) {
          int c[4][3];
          c[0][0] = i;
          c[0][1] = j;
          c[0][2] = k;
          for (int s = 0; s < 3; ++s) {
            for (int a = 0; a < 3; ++a) c[s + 1][a] = c[s][a];
            c[s + 1][perms[p][s]] += 1;
          }
          if (odd[p])  // odd axis order: swap the last two vertices (positive orientation)
            for (int a = 0; a < 3; ++a) {
              const int t = c[2][a];
              c[2][a] = c[3][a];
              c[3][a] = t;
            }
          for (int v = 0; v < 4; ++v) {
            for (int a = 0; a < 3; ++a) xyz.push_back(c[v][a] * h);
            topo.push_back((static_cast<int64_t>(c[v][0]) * (n + 1) + c[v][1]) * (n + 1) + c[v][2]);
          }
        }
}

int main() {
  // reference operators and permutations, every degree
  for (int N = 1; N <= 8; ++N) {
    int Np = 0, Nfp = 0;
    expect(dg_ref_sizes(N, &Np, &Nfp) == DG_OK, "ref sizes");
    std::vector<double> nodes(3 * Np), D(3 * Np * Np), mass(Np * Np), lift(Np * 4 * Nfp);
    std::vector<int32_t> fmask(4 * Nfp), perm(6 * Nfp);
    expect(dg_reference_operators(N, nodes.data(), D.data(), mass.data(), lift.data(), fmask.data()) == DG_OK,
           "reference operators");
    expect(dg_face_permutations(N, perm.data()) == DG_OK, "face permutations");
    for (int physics = 0; physics < 3; ++physics) {
      size_t bytes = 0;
      expect(dg_workspace_bytes(physics, N, 1000, &bytes) == DG_OK && bytes > 0, "workspace bytes");
    }
  }
  int a = 0, b = 0;
  expect(dg_ref_sizes(0, &a, &b) == DG_E_UNSUPPORTED, "order 0 refused");
  expect(dg_ref_sizes(9, &a, &b) == DG_E_UNSUPPORTED, "order 9 refused");

  // connectivity of a box, and a face shared three times
  std::vector<double> xyz;
  std::vector<int64_t> topo;
  kuhn_box(3, xyz, topo);
  const int64_t K = static_cast<int64_t>(topo.size() / 4);
  std::vector<int64_t> e2e(4 * K);
  std::vector<int32_t> e2f(4 * K), orient(4 * K);
  expect(dg_mesh_connectivity(K, topo.data(), e2e.data(), e2f.data(), orient.data()) == DG_OK, "connectivity");
  int64_t walls = 0;
  for (int64_t i = 0; i < 4 * K; ++i) walls += e2e[i] < 0;
  expect(walls == 6 * 2 * 9, "boundary face count");
  const int64_t bad3[12] = {0, 1, 2, 3, 0, 1, 2, 4, 0, 1, 2, 5};
  expect(dg_mesh_connectivity(3, bad3, e2e.data(), e2f.data(), orient.data()) == DG_E_MESH, "triple face");

  // dg_create up to the workspace check: host geometry, connectivity,
  // operator packing and layout run; the stand-in buffer is never touched
  void* fake = reinterpret_cast<void*>(uintptr_t(1) << 20);
  for (int physics = 0; physics < 3; ++physics)
    for (int N = 1; N <= 8; ++N) {
      size_t need = 0;
      dg_workspace_bytes(physics, N, K, &need);
      dg_solver* s = nullptr;
      expect(dg_create(physics, N, K, xyz.data(), topo.data(), fake, need - 256, nullptr, &s) == DG_E_SHAPE &&
                 s == nullptr,
             "short workspace refused");
    }
  dg_solver* s = nullptr;
  std::vector<double> inv = xyz;
  for (int c = 0; c < 3; ++c) {  // swap two vertices of element 5: negative Jacobian
    const double t = inv[(5 * 4 + 2) * 3 + c];
    inv[(5 * 4 + 2) * 3 + c] = inv[(5 * 4 + 3) * 3 + c];
    inv[(5 * 4 + 3) * 3 + c] = t;
  }
  expect(dg_create(0, 2, K, inv.data(), topo.data(), fake, size_t(1) << 40, nullptr, &s) == DG_E_MESH,
         "inverted element refused");
  expect(dg_create(0, 2, K, xyz.data(), topo.data(), reinterpret_cast<void*>((uintptr_t(1) << 20) + 64),
                   size_t(1) << 40, nullptr, &s) == DG_E_ARG,
         "misaligned workspace refused");
  expect(dg_create(0, 2, 0, xyz.data(), topo.data(), fake, 0, nullptr, &s) == DG_E_ARG, "K = 0 refused");

  // null-argument paths
  size_t nb = 0;
  expect(dg_batch_create(nullptr, 0, fake, 0, nullptr, nullptr) == DG_E_ARG, "batch null");
  expect(dg_batch_workspace_bytes(nullptr, 0, &nb) == DG_E_ARG, "batch bytes null");
  expect(dg_autotune(nullptr, 1, 1.0, 0, nullptr, 0, nullptr) == DG_E_ARG, "autotune null");
  expect(dg_misfit_workspace_bytes(nullptr, 10, 0.1, 5, 0, nullptr, nullptr, 1, nullptr, &nb) == DG_E_ARG,
         "misfit bytes null");
  expect(dg_set_boundary(nullptr, nullptr) == DG_E_ARG, "boundary null");
  expect(dg_set_rate_classes(nullptr, 0) == DG_E_ARG, "rate classes null");
  expect(dg_energy_noalloc(nullptr, nullptr) == DG_E_ARG, "noalloc energy null");

  if (failures) {
    std::fprintf(stderr, "%d failure(s)\n", failures);
    return 1;
  }
  std::printf("asan host ABI checks passed\n");
  return 0;
}
