// Modal bases, quadrature and reference matrices for the ADER-DG element
// update (host side, double precision).
//
// Element basis: the Karniadakis-Sherwin (Dubiner) tetrahedral expansion named
// in Sec. III-A (Discrete Formulation), orthonormal on the unit tetrahedron (0,0,0),(1,0,0),(0,1,0),
// (0,0,1) so that the mass matrix is the identity (the paper's "inverse,
// diagonal mass matrix" is then a scalar 1/|det J|).  B(O) = O(O+1)(O+2)/6
// functions ordered by total degree, then i descending, then j descending.
// Face basis: the orthonormal Dubiner triangle basis on the unit triangle,
// F(O) = O(O+1)/2 functions.
//
// Evaluation uses the scaled Jacobi recurrences at points; gradients come from
// forward-mode dual numbers carried through the same recurrences.  Integrals
// use collapsed Gauss-Jacobi (Stroud) rules whose nodes come from a Golub-
// Welsch eigen-solve.
#pragma once

#include <array>
#include <cmath>
#include <cstdint>
#include <vector>

namespace edg {

inline int n_basis(int O) { return O * (O + 1) * (O + 2) / 6; }
inline int n_face_basis(int O) { return O * (O + 1) / 2; }

// value + gradient (3 partials)
struct Dual3 {
  double v, d[3];
  Dual3(double x = 0.0) : v(x), d{0.0, 0.0, 0.0} {}
};
inline Dual3 operator+(const Dual3& a, const Dual3& b) {
  Dual3 r(a.v + b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
inline Dual3 operator-(const Dual3& a, const Dual3& b) {
  Dual3 r(a.v - b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
inline Dual3 operator*(const Dual3& a, const Dual3& b) {
  Dual3 r(a.v * b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
inline Dual3 operator*(double s, const Dual3& a) {
  Dual3 r(s * a.v);
  for (int i = 0; i < 3; ++i) r.d[i] = s * a.d[i];
  return r;
}

// Q_n(x, y) = y^n P_n^{(alpha,0)}(x / y) for n = 0..nmax, by the three-term
// recurrence multiplied through by y^n (no division, so it stays finite at the
// collapsed vertex).
template <class T>
void scaled_jacobi(int nmax, double alpha, const T& x, const T& y, std::vector<T>& out) {
  out.assign(nmax + 1, T(0.0));
  out[0] = T(1.0);
  if (nmax >= 1) out[1] = 0.5 * ((alpha + 2.0) * x + alpha * y);
  for (int n = 2; n <= nmax; ++n) {
    const double a = alpha, N = n;
    const double c1 = 2.0 * N * (N + a) * (2.0 * N + a - 2.0);
    const double c2 = (2.0 * N + a - 1.0) * (2.0 * N + a) * (2.0 * N + a - 2.0);
    const double c3 = (2.0 * N + a - 1.0) * (a * a);
    const double c4 = 2.0 * (N + a - 1.0) * (N - 1.0) * (2.0 * N + a);
    out[n] = (1.0 / c1) * ((c2 * x + c3 * y) * out[n - 1] - c4 * (y * y) * out[n - 2]);
  }
}

struct TetIndex { int i, j, k; };
inline std::vector<TetIndex> tet_indices(int O) {
  std::vector<TetIndex> v;
  for (int n = 0; n < O; ++n)
    for (int i = n; i >= 0; --i)
      for (int j = n - i; j >= 0; --j) v.push_back({i, j, n - i - j});
  return v;
}
inline std::vector<std::array<int, 2>> tri_indices(int O) {
  std::vector<std::array<int, 2>> v;
  for (int n = 0; n < O; ++n)
    for (int i = n; i >= 0; --i) v.push_back({i, n - i});
  return v;
}

// all tetrahedral basis functions at xi = (u, v, w) (unit-tet coordinates)
template <class T>
void tet_basis(int O, const T& u, const T& v, const T& w, std::vector<T>& out) {
  const T one(1.0);
  const T y1 = one - v - w, x1 = 2.0 * u - y1;
  const T y2 = one - w, x2 = 2.0 * v - y2;
  const T z3 = 2.0 * w - one;
  auto idx = tet_indices(O);
  out.assign(idx.size(), T(0.0));
  std::vector<T> qi, qj, pk;
  scaled_jacobi(O - 1, 0.0, x1, y1, qi);
  for (size_t b = 0; b < idx.size(); ++b) {
    const int i = idx[b].i, j = idx[b].j, k = idx[b].k, n = i + j + k;
    scaled_jacobi(j, 2.0 * i + 1.0, x2, y2, qj);
    scaled_jacobi(k, 2.0 * i + 2.0 * j + 2.0, z3, one, pk);
    // orthonormal on the unit tet: int psi^2 = 1/((2i+1)(2i+2j+2)(2n+3))
    const double nrm = std::sqrt((2.0 * i + 1.0) * (2.0 * i + 2.0 * j + 2.0) * (2.0 * n + 3.0));
    out[b] = nrm * (qi[i] * qj[j] * pk[k]);
  }
}

// all triangle basis functions at chi = (a, b) on the unit triangle
inline void tri_basis(int O, double a, double b, std::vector<double>& out) {
  const double y1 = 1.0 - b, x1 = 2.0 * a - y1, z2 = 2.0 * b - 1.0;
  auto idx = tri_indices(O);
  out.assign(idx.size(), 0.0);
  std::vector<double> qi, pj;
  scaled_jacobi(O - 1, 0.0, x1, y1, qi);
  for (size_t f = 0; f < idx.size(); ++f) {
    const int i = idx[f][0], j = idx[f][1];
    scaled_jacobi(j, 2.0 * i + 1.0, z2, 1.0, pj);
    const double nrm = std::sqrt((2.0 * i + 1.0) * (2.0 * i + 2.0 * j + 2.0));
    out[f] = nrm * qi[i] * pj[j];
  }
}

// Gauss-Jacobi rule for weight (1-x)^alpha on [-1,1] by Golub-Welsch: the
// nodes are the eigenvalues of the symmetric Jacobi matrix, the weights the
// squared first eigenvector components times the weight's integral.
void gauss_jacobi(int n, double alpha, std::vector<double>& x, std::vector<double>& w);

struct Rule { std::vector<std::array<double, 3>> pts; std::vector<double> w; };
// Stroud conical rule on the unit tetrahedron / triangle with n points per
// direction (exact for total degree 2n-1)
Rule tet_rule(int n);
Rule tri_rule(int n);

// Reference tet faces: face i is opposite local vertex i, parameterised by its
// three vertices in ascending local index (a0, a1, a2):
// xi(chi) = V[a0] + chi1 (V[a1]-V[a0]) + chi2 (V[a2]-V[a0]).
void face_point(int i, double c1, double c2, double xi[3]);

struct RefMats {
  int O, B, F;
  // K[c][b][bb] = int phi_b d(phi_bb)/d xi_c   (3 x B x B)
  std::vector<double> K;
  // Ft[i][b][f] = int_face_i phi_b psi_f d chi over the unit triangle (4 x B x F)
  std::vector<double> Ft;
};
RefMats reference_matrices(int O);

// Three independent reference directions w_k = sum_c V[k][c] d/dxi_c along
// which this basis's derivative matrices have the fewest non-zeros (entries of
// V in {0, +-1/2, +-1}, largest entry 1, first non-zero positive; ties go to
// the earliest triple in enumeration order).  A gradient taken along them is
// mapped to physical coordinates by G' = V^-T G (G[c][d] = d xi_c / d x_d):
// sum_k G'[k][d] w_k = sum_c G[c][d] d/dxi_c.  The stiffness products then
// cost sum_k nnz(sum_c V[k][c] K_c) FMAs per row instead of sum_c nnz(K_c)
// (O=5: 364 instead of 647).
struct Directions {
  double V[9], Vinv[9];
  int nnz[3];
};
Directions sparse_directions(int O);
// K' [3][B][B] with K'[k] = sum_c V[k][c] K[c] (same layout as RefMats::K)
std::vector<double> direction_matrices(const RefMats& M, const Directions& D);

// Coefficients of the same polynomial after a permutation of the tet's local
// vertices: if new local vertex m is old local vertex perm[m], then
// q_new[b] = sum_bb C[b][bb] q_old[bb].  C is orthogonal (B x B).
std::vector<double> vertex_permutation_matrix(int O, const int perm[4]);

// Basis values at a reference point
std::vector<double> eval_basis(int O, const double xi[3]);

}  // namespace edg
