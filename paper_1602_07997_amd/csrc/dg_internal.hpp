// Internal host-side declarations of the dgwave library (not part of the ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace dgw {

constexpr int kMaxOrder = 8;

inline int num_nodes(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
inline int num_face_nodes(int N) { return (N + 1) * (N + 2) / 2; }

// Vertices of the four faces of the reference tetrahedron (0-based).
extern const int kFaceVerts[4][3];
// The six permutations of a face's three vertices, in orientation-index order.
extern const int kFacePerms[6][3];

// Reference element of degree N, built in long double and stored in double.
struct RefElement {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<double> nodes;   // [Np][3]
  std::vector<double> D;       // [3][Np][Np]
  std::vector<double> mass;    // [Np][Np]
  std::vector<double> minv;    // [Np][Np] inverse mass matrix
  std::vector<double> vinv;    // [Np][Np] inverse Vandermonde of the orthonormal basis
  std::vector<double> face_mass;  // [Nfp][Nfp] face mass in the parameter triangle
  std::vector<double> lift;    // [Np][4*Nfp]
  std::vector<int32_t> fmask;  // [4][Nfp]
  std::vector<int32_t> perm;   // [6][Nfp]
  std::vector<int32_t> nodeface;  // [Np][3] face slots f*Nfp+j holding node n, -1 padded
};

// Builds (and caches) the reference element; returns nullptr for bad N.
const RefElement* reference_element(int N);

// Lagrange weights of the nodal basis at reference point xi: w [Np].
void lagrange_weights(const RefElement* ref, const double xi[3], double* w);

// Face connectivity from topological vertex ids; returns an error message or "".
std::string connect_faces(int64_t K, const int64_t* topo, int64_t* e2e, int32_t* e2f,
                          int32_t* orient);

// Thread-local error message plumbing for the C ABI.
void set_error(const std::string& msg);
const char* last_error();

}  // namespace dgw
