// Reference tetrahedron of the nodal DG scheme (Sec. 2.2 of the paper):
// warp-and-blend nodes, differentiation matrices D_j, mass matrix and the
// merged lift matrix L of eqs. (3), (5)-(6).  Everything is computed once per
// degree on the host in long double and cached.
//
// Route taken here:
//   * nodes: equidistant barycentric lattice on an equilateral tetrahedron,
//     displaced by the blended Gauss-Lobatto warp (alpha = 0), mapped back to
//     the reference tetrahedron;
//   * orthonormal basis psi_m (collapsed-coordinate Jacobi products) for the
//     nodal <-> modal change of basis V;
//   * D_j = V Dhat_j V^{-1}, where Dhat_j[l][m] = int psi_l d psi_m / d r_j is
//     integrated with a conical-product Gauss rule whose points are all
//     interior, and d psi_m / d r_j comes from forward-mode dual numbers;
//   * M^{-1} = V V^T; face mass E = (V2 V2^T)^{-1} with the orthonormal
//     triangle basis on the face nodes; L = M^{-1} [E_0 .. E_3].
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>

#include "dg_internal.hpp"

namespace dgw {

const int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
const int kFacePerms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

namespace {

using real = long double;

// ---------------------------------------------------------------------------
// forward-mode dual number with a 3-vector of partial derivatives
// ---------------------------------------------------------------------------
struct Dual {
  real v;
  real d[3];
  Dual(real x = 0) : v(x), d{0, 0, 0} {}
};
inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline real value(real x) { return x; }
inline real value(const Dual& x) { return x.v; }

template <class T>
T ipow(const T& x, int e) {
  T r(1);
  for (int i = 0; i < e; ++i) r = r * x;
  return r;
}

// ---------------------------------------------------------------------------
// small dense linear algebra (row-major, long double)
// ---------------------------------------------------------------------------
using Mat = std::vector<real>;

Mat matmul(const Mat& A, const Mat& B, int n, int k, int m) {  // (n x k)(k x m)
  Mat C(static_cast<size_t>(n) * m, 0);
  for (int i = 0; i < n; ++i)
    for (int p = 0; p < k; ++p) {
      real a = A[i * k + p];
      if (a == 0) continue;
      for (int j = 0; j < m; ++j) C[i * m + j] += a * B[p * m + j];
    }
  return C;
}

Mat transpose(const Mat& A, int n, int m) {
  Mat T(static_cast<size_t>(n) * m);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) T[j * n + i] = A[i * m + j];
  return T;
}

// Inverse by Gauss-Jordan elimination with partial pivoting.
Mat inverse(Mat A, int n) {
  Mat I(static_cast<size_t>(n) * n, 0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0) throw std::runtime_error("singular matrix in reference element");
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(A[c * n + j], A[piv * n + j]);
        std::swap(I[c * n + j], I[piv * n + j]);
      }
    real inv = 1 / A[c * n + c];
    for (int j = 0; j < n; ++j) {
      A[c * n + j] *= inv;
      I[c * n + j] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      real f = A[r * n + c];
      if (f == 0) continue;
      for (int j = 0; j < n; ++j) {
        A[r * n + j] -= f * A[c * n + j];
        I[r * n + j] -= f * I[c * n + j];
      }
    }
  }
  return I;
}

// ---------------------------------------------------------------------------
// 1D polynomials and quadrature
// ---------------------------------------------------------------------------

// Legendre P_n(x) and P_n'(x), P_n''(x) by the three-term recurrence.
void legendre(int n, real x, real& p, real& dp, real& ddp) {
  real p0 = 1, p1 = x, d0 = 0, d1 = 1, dd0 = 0, dd1 = 0;
  if (n == 0) {
    p = 1; dp = 0; ddp = 0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    real p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    real d2 = ((2 * k + 1) * (p1 + x * d1) - k * d0) / (k + 1);
    real dd2 = ((2 * k + 1) * (2 * d1 + x * dd1) - k * dd0) / (k + 1);
    p0 = p1; p1 = p2; d0 = d1; d1 = d2; dd0 = dd1; dd1 = dd2;
  }
  p = p1; dp = d1; ddp = dd1;
}

// N+1 Gauss-Lobatto-Legendre points: -1, the N-1 zeros of P_N', 1 (Newton).
std::vector<real> gll_points(int N) {
  std::vector<real> x(N + 1);
  x[0] = -1;
  x[N] = 1;
  const real pi = 3.141592653589793238462643383279502884L;
  for (int i = 1; i < N; ++i) {
    real z = -std::cos(pi * i / N);
    for (int it = 0; it < 100; ++it) {
      real p, dp, ddp;
      legendre(N, z, p, dp, ddp);
      real dz = dp / ddp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    x[i] = z;
  }
  std::sort(x.begin(), x.end());
  return x;
}

// q-point Gauss-Legendre rule (Newton on P_q).
void gauss_legendre(int q, std::vector<real>& x, std::vector<real>& w) {
  x.resize(q);
  w.resize(q);
  const real pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < q; ++i) {
    real z = -std::cos(pi * (i + 0.75L) / (q + 0.5L));
    real p = 0, dp = 1, ddp = 0;
    for (int it = 0; it < 100; ++it) {
      legendre(q, z, p, dp, ddp);
      real dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    legendre(q, z, p, dp, ddp);
    x[i] = z;
    w[i] = 2 / ((1 - z * z) * dp * dp);
  }
}

// Orthonormal Jacobi polynomial p_n^{(al,be)} by the orthonormal three-term
// recurrence x p_k = a_{k+1} p_{k+1} + b_k p_k + a_k p_{k-1}.
template <class T>
T jacobi_on(int n, real al, real be, const T& x) {
  real h0 = std::pow(2.0L, al + be + 1) * std::tgamma(al + 1) * std::tgamma(be + 1) /
            std::tgamma(al + be + 2);
  T pkm1(0);
  T pk(1 / std::sqrt(h0));
  if (n == 0) return pk;
  auto a_of = [&](int k) {
    real s = 2 * k + al + be;
    return 2 / s * std::sqrt(k * (k + al + be) * (k + al) * (k + be) / ((s - 1) * (s + 1)));
  };
  auto b_of = [&](int k) {
    if (k == 0) return (be - al) / (al + be + 2);
    real s = 2 * k + al + be;
    return (be * be - al * al) / (s * (s + 2));
  };
  for (int k = 0; k < n; ++k) {
    real ak1 = a_of(k + 1);
    real ak = (k == 0) ? 0 : a_of(k);
    T pkp1 = ((x - T(b_of(k))) * pk - T(ak) * pkm1) / T(ak1);
    pkm1 = pk;
    pk = pkp1;
  }
  return pk;
}

// Orthonormal basis on the reference tetrahedron, in collapsed coordinates.
template <class T>
void tet_basis(int N, const T& r, const T& s, const T& t, std::vector<T>& out) {
  // a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t; singular limits a=b=-1
  T a(-1), b(-1);
  if (std::fabs(value(s) + value(t)) > 1e-16L) a = T(2) * (T(1) + r) / (T(0) - s - t) - T(1);
  if (std::fabs(1 - value(t)) > 1e-16L) b = T(2) * (T(1) + s) / (T(1) - t) - T(1);
  const T& c = t;
  out.clear();
  const real s8 = 2 * std::sqrt(2.0L);
  for (int i = 0; i <= N; ++i)
    for (int j = 0; i + j <= N; ++j)
      for (int k = 0; i + j + k <= N; ++k) {
        T v = jacobi_on<T>(i, 0, 0, a) * jacobi_on<T>(j, 2 * i + 1, 0, b) * ipow(T(1) - b, i) *
              jacobi_on<T>(k, 2 * i + 2 * j + 2, 0, c) * ipow(T(1) - c, i + j);
        out.push_back(T(s8) * v);
      }
}

// Orthonormal basis on the triangle (-1,-1),(1,-1),(-1,1).
void tri_basis(int N, real x, real y, std::vector<real>& out) {
  real a = -1;
  if (std::fabs(1 - y) > 1e-16L) a = 2 * (1 + x) / (1 - y) - 1;
  out.clear();
  for (int i = 0; i <= N; ++i)
    for (int j = 0; i + j <= N; ++j)
      out.push_back(std::sqrt(2.0L) * jacobi_on<real>(i, 0, 0, a) *
                    jacobi_on<real>(j, 2 * i + 1, 0, y) * ipow<real>(1 - y, i));
}

// ---------------------------------------------------------------------------
// lattice and warp-and-blend nodes
// ---------------------------------------------------------------------------
std::vector<std::array<int, 4>> lattice(int N) {
  std::vector<std::array<int, 4>> L;
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j + k <= N; ++j)
      for (int i = 0; i + j + k <= N; ++i) L.push_back({N - i - j - k, i, j, k});
  return L;
}

// Edge displacement w(r) = sum_i (gll_i - equi_i) ell_i(r) on equidistant nodes.
real edge_warp(int N, const std::vector<real>& gll, real r) {
  real w = 0;
  for (int i = 0; i <= N; ++i) {
    real ei = -1 + 2.0L * i / N;
    real li = 1;
    for (int m = 0; m <= N; ++m) {
      if (m == i) continue;
      real em = -1 + 2.0L * m / N;
      li *= (r - em) / (ei - em);
    }
    w += (gll[i] - ei) * li;
  }
  return w;
}

std::vector<real> warp_blend_nodes(int N) {
  const real s3 = std::sqrt(3.0L), s6 = std::sqrt(6.0L);
  const real E[4][3] = {{-1, -1 / s3, -1 / s6}, {1, -1 / s3, -1 / s6}, {0, 2 / s3, -1 / s6},
                        {0, 0, 3 / s6}};
  const real R[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
  auto gll = gll_points(N);
  auto lat = lattice(N);
  std::vector<real> out;
  for (const auto& l : lat) {
    real L[4];
    int nz = 0;
    for (int i = 0; i < 4; ++i) {
      L[i] = real(l[i]) / N;
      nz += (l[i] == 0);
    }
    real X[3] = {0, 0, 0};
    for (int i = 0; i < 4; ++i)
      for (int d = 0; d < 3; ++d) X[d] += L[i] * E[i][d];
    real sh[3] = {0, 0, 0};
    if (nz == 2) {  // edge node: the 1D warp along the edge
      int P = -1, Q = -1;
      for (int i = 0; i < 4; ++i)
        if (l[i] != 0) (P < 0 ? P : Q) = i;
      real w = edge_warp(N, gll, L[Q] - L[P]);
      for (int d = 0; d < 3; ++d) sh[d] = w * (E[Q][d] - E[P][d]) / 2;
    } else if (nz < 2) {  // face or interior node: blended face warps
      for (int f = 0; f < 4; ++f) {
        int A = kFaceVerts[f][0], B = kFaceVerts[f][1], C = kFaceVerts[f][2];
        int D = 6 - A - B - C;
        real num = L[A] * L[B] * L[C];
        if (num == 0) continue;
        real blend = num / ((L[A] + L[D] / 2) * (L[B] + L[D] / 2) * (L[C] + L[D] / 2));
        const int edges[3][2] = {{A, B}, {B, C}, {A, C}};
        for (const auto& e : edges) {
          int P = e[0], Q = e[1];
          real rr = L[Q] - L[P];
          real fac = 4 * L[P] * L[Q] * edge_warp(N, gll, rr) / (1 - rr * rr);
          for (int d = 0; d < 3; ++d) sh[d] += blend * fac * (E[Q][d] - E[P][d]) / 2;
        }
      }
    }
    for (int d = 0; d < 3; ++d) X[d] += sh[d];
    // barycentrics of X in the equilateral tetrahedron (Cramer's rule)
    auto det3 = [](const real a[3], const real b[3], const real c[3]) {
      return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
             a[2] * (b[0] * c[1] - b[1] * c[0]);
    };
    real e1[3], e2[3], e3[3], xv[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = E[1][d] - E[0][d];
      e2[d] = E[2][d] - E[0][d];
      e3[d] = E[3][d] - E[0][d];
      xv[d] = X[d] - E[0][d];
    }
    real vol = det3(e1, e2, e3);
    real b1 = det3(xv, e2, e3) / vol, b2 = det3(e1, xv, e3) / vol, b3 = det3(e1, e2, xv) / vol;
    real b0 = 1 - b1 - b2 - b3;
    real bb[4] = {b0, b1, b2, b3};
    for (int d = 0; d < 3; ++d) {
      real v = 0;
      for (int i = 0; i < 4; ++i) v += bb[i] * R[i][d];
      out.push_back(v);
    }
  }
  return out;
}

std::unique_ptr<RefElement> build(int N) {
  auto ref = std::make_unique<RefElement>();
  const int Np = num_nodes(N), Nfp = num_face_nodes(N);
  ref->N = N;
  ref->Np = Np;
  ref->Nfp = Nfp;
  auto nodes = warp_blend_nodes(N);
  auto lat = lattice(N);

  // Vandermonde of the orthonormal basis at the nodes
  Mat V(static_cast<size_t>(Np) * Np);
  std::vector<real> row;
  for (int n = 0; n < Np; ++n) {
    tet_basis<real>(N, nodes[3 * n], nodes[3 * n + 1], nodes[3 * n + 2], row);
    for (int m = 0; m < Np; ++m) V[n * Np + m] = row[m];
  }
  Mat Vinv = inverse(V, Np);

  // modal derivative matrices by interior conical-product Gauss cubature
  const int q = N + 2;
  std::vector<real> gx, gw;
  gauss_legendre(q, gx, gw);
  std::vector<Mat> Dhat(3, Mat(static_cast<size_t>(Np) * Np, 0));
  std::vector<Dual> db;
  for (int ia = 0; ia < q; ++ia)
    for (int ib = 0; ib < q; ++ib)
      for (int ic = 0; ic < q; ++ic) {
        real a = gx[ia], b = gx[ib], c = gx[ic];
        real r = (1 + a) * (1 - b) * (1 - c) / 4 - 1;
        real s = (1 + b) * (1 - c) / 2 - 1;
        real t = c;
        real w = gw[ia] * gw[ib] * gw[ic] * (1 - b) * (1 - c) * (1 - c) / 8;
        Dual R(r), S(s), T(t);
        R.d[0] = 1;
        S.d[1] = 1;
        T.d[2] = 1;
        tet_basis<Dual>(N, R, S, T, db);
        for (int l = 0; l < Np; ++l) {
          real wl = w * db[l].v;
          for (int m = 0; m < Np; ++m)
            for (int d = 0; d < 3; ++d) Dhat[d][l * Np + m] += wl * db[m].d[d];
        }
      }
  ref->D.resize(3 * static_cast<size_t>(Np) * Np);
  for (int d = 0; d < 3; ++d) {
    Mat Dn = matmul(matmul(V, Dhat[d], Np, Np, Np), Vinv, Np, Np, Np);
    for (size_t i = 0; i < Dn.size(); ++i) ref->D[d * Np * Np + i] = static_cast<double>(Dn[i]);
  }

  // mass matrix M = V^{-T} V^{-1}; M^{-1} = V V^T
  Mat M = matmul(transpose(Vinv, Np, Np), Vinv, Np, Np, Np);
  Mat Minv = matmul(V, transpose(V, Np, Np), Np, Np, Np);
  ref->mass.assign(M.begin(), M.end());
  ref->minv.assign(Minv.begin(), Minv.end());
  ref->vinv.assign(Vinv.begin(), Vinv.end());

  // face masks from the lattice
  std::map<std::array<int, 4>, int> index;
  for (int n = 0; n < Np; ++n) index[lat[n]] = n;
  ref->fmask.resize(4 * Nfp);
  for (int f = 0; f < 4; ++f) {
    int j = 0;
    for (int b = 0; b <= N; ++b)
      for (int a = 0; a + b <= N; ++a) {
        std::array<int, 4> l = {0, 0, 0, 0};
        l[kFaceVerts[f][0]] = N - a - b;
        l[kFaceVerts[f][1]] = a;
        l[kFaceVerts[f][2]] = b;
        ref->fmask[f * Nfp + j++] = index.at(l);
      }
  }

  // face mass in the parameter triangle from face 0 (t = -1: (r, s))
  Mat V2(static_cast<size_t>(Nfp) * Nfp);
  for (int j = 0; j < Nfp; ++j) {
    int n = ref->fmask[j];
    tri_basis(N, nodes[3 * n], nodes[3 * n + 1], row);
    for (int m = 0; m < Nfp; ++m) V2[j * Nfp + m] = row[m];
  }
  Mat V2inv = inverse(V2, Nfp);
  Mat Ef = matmul(transpose(V2inv, Nfp, Nfp), V2inv, Nfp, Nfp, Nfp);
  ref->face_mass.assign(Ef.begin(), Ef.end());
  Mat Emb(static_cast<size_t>(Np) * 4 * Nfp, 0);
  for (int f = 0; f < 4; ++f)
    for (int i = 0; i < Nfp; ++i)
      for (int j = 0; j < Nfp; ++j)
        Emb[ref->fmask[f * Nfp + i] * 4 * Nfp + f * Nfp + j] = Ef[i * Nfp + j];
  Mat Lift = matmul(Minv, Emb, Np, Np, 4 * Nfp);
  ref->lift.assign(Lift.begin(), Lift.end());
  ref->nodes.assign(nodes.begin(), nodes.end());

  // for every volume node, the face slots (f*Nfp + j) it occupies
  ref->nodeface.assign(static_cast<size_t>(Np) * 3, -1);
  for (int f = 0; f < 4; ++f)
    for (int j = 0; j < Nfp; ++j) {
      const int n = ref->fmask[f * Nfp + j];
      int s = 0;
      while (ref->nodeface[3 * n + s] >= 0) ++s;  // a node lies on at most three faces
      ref->nodeface[3 * n + s] = f * Nfp + j;
    }

  // face-node permutations for the six relative orientations
  ref->perm.resize(6 * Nfp);
  std::map<std::pair<int, int>, int> fidx;
  {
    int j = 0;
    for (int b = 0; b <= N; ++b)
      for (int a = 0; a + b <= N; ++a) fidx[{a, b}] = j++;
  }
  for (int o = 0; o < 6; ++o) {
    int j = 0;
    for (int b = 0; b <= N; ++b)
      for (int a = 0; a + b <= N; ++a) {
        int beta[3] = {N - a - b, a, b};  // w.r.t. own face vertices
        int nb[3];
        for (int p = 0; p < 3; ++p) nb[kFacePerms[o][p]] = beta[p];
        ref->perm[o * Nfp + j++] = fidx.at({nb[1], nb[2]});
      }
  }
  return ref;
}

std::mutex g_cache_mutex;
std::unique_ptr<RefElement> g_cache[kMaxOrder + 1];

}  // namespace

void lagrange_weights(const RefElement* ref, const double xi[3], double* w) {
  // u(xi) = psi(xi)^T V^{-1} u_nodes, so l(xi) = V^{-T} psi(xi)
  std::vector<real> psi;
  tet_basis<real>(ref->N, xi[0], xi[1], xi[2], psi);
  const int Np = ref->Np;
  for (int n = 0; n < Np; ++n) {
    real acc = 0;
    for (int m = 0; m < Np; ++m) acc += psi[m] * static_cast<real>(ref->vinv[m * Np + n]);
    w[n] = static_cast<double>(acc);
  }
}

const RefElement* reference_element(int N) {
  if (N < 1 || N > kMaxOrder) return nullptr;
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  if (!g_cache[N]) g_cache[N] = build(N);
  return g_cache[N].get();
}

}  // namespace dgw
