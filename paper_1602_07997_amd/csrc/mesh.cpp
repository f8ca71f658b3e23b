// Face connectivity of a tetrahedral mesh from topological vertex ids.
//
// The surface term of eq. (3) needs, at every face node, the neighbour's trace
// (Sec. 3.2).  Faces pair up when they carry the same three vertex ids; the
// relative orientation of the pair (which own face vertex is which neighbour
// face vertex) selects one of six face-node permutations, so the per-node map
// of the paper collapses to one packed word per face.
#include <algorithm>
#include <array>
#include <numeric>
#include <sstream>
#include <vector>

#include "dg_internal.hpp"

namespace dgw {

std::string connect_faces(int64_t K, const int64_t* topo, int64_t* e2e, int32_t* e2f,
                          int32_t* orient) {
  struct FaceKey {
    std::array<int64_t, 3> v;
    int64_t slot;  // k*4 + f
  };
  std::vector<FaceKey> keys(static_cast<size_t>(K) * 4);
  for (int64_t k = 0; k < K; ++k) {
    const int64_t* t = topo + 4 * k;
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (t[a] == t[b]) {
          std::ostringstream os;
          os << "element " << k << " repeats a vertex id";
          return os.str();
        }
    for (int f = 0; f < 4; ++f) {
      std::array<int64_t, 3> v = {t[kFaceVerts[f][0]], t[kFaceVerts[f][1]], t[kFaceVerts[f][2]]};
      std::sort(v.begin(), v.end());
      keys[k * 4 + f] = {v, k * 4 + f};
    }
  }
  std::sort(keys.begin(), keys.end(), [](const FaceKey& x, const FaceKey& y) {
    return x.v != y.v ? x.v < y.v : x.slot < y.slot;
  });
  for (int64_t i = 0; i < 4 * K; ++i) {
    e2e[i] = -1;
    e2f[i] = -1;
    orient[i] = -1;
  }
  const size_t nf = keys.size();
  for (size_t i = 0; i < nf;) {
    size_t j = i + 1;
    while (j < nf && keys[j].v == keys[i].v) ++j;
    if (j - i > 2) {
      std::ostringstream os;
      os << "a face is shared by " << (j - i) << " elements (element " << keys[i].slot / 4 << ")";
      return os.str();
    }
    if (j - i == 2) {
      for (int side = 0; side < 2; ++side) {
        int64_t own = keys[i + side].slot, nb = keys[i + 1 - side].slot;
        int64_t k = own / 4, kn = nb / 4;
        int f = static_cast<int>(own % 4), fn = static_cast<int>(nb % 4);
        e2e[own] = kn;
        e2f[own] = fn;
        const int64_t* t = topo + 4 * k;
        const int64_t* tn = topo + 4 * kn;
        int o = -1;
        for (int c = 0; c < 6 && o < 0; ++c) {
          bool ok = true;
          for (int p = 0; p < 3; ++p)
            ok = ok && t[kFaceVerts[f][p]] == tn[kFaceVerts[fn][kFacePerms[c][p]]];
          if (ok) o = c;
        }
        orient[own] = o;
      }
    }
    i = j;
  }
  return "";
}

}  // namespace dgw
