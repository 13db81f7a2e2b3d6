// Quadrature rules and reference matrices (host, double precision).
#include "basis.hpp"

#include <algorithm>
#include <stdexcept>

namespace edg {

namespace {
// cyclic Jacobi eigenvalue iteration for a small symmetric matrix (row-major)
void sym_eig(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}
}  // namespace

void gauss_jacobi(int n, double alpha, std::vector<double>& x, std::vector<double>& w) {
  // monic recurrence for P^{(alpha, 0)}: diagonal a_k, off-diagonal sqrt(b_k)
  const double a = alpha, b = 0.0;
  std::vector<double> J(n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    const double s = 2.0 * k + a + b;
    double ak;
    if (k == 0) ak = (b - a) / (a + b + 2.0);
    else ak = (b * b - a * a) / (s * (s + 2.0));
    J[k * n + k] = ak;
    if (k + 1 < n) {
      const double kk = k + 1.0, s1 = 2.0 * kk + a + b;
      const double bk = 4.0 * kk * (kk + a) * (kk + b) * (kk + a + b) / (s1 * s1 * (s1 + 1.0) * (s1 - 1.0));
      J[k * n + k + 1] = J[(k + 1) * n + k] = std::sqrt(bk);
    }
  }
  std::vector<double> V;
  sym_eig(n, J, V);
  const double mu0 = std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) / std::tgamma(a + b + 2.0);
  std::vector<std::pair<double, double>> xw(n);
  for (int i = 0; i < n; ++i) xw[i] = {J[i * n + i], mu0 * V[0 * n + i] * V[0 * n + i]};
  std::sort(xw.begin(), xw.end());
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) { x[i] = xw[i].first; w[i] = xw[i].second; }
}

Rule tet_rule(int n) {
  // collapse: xi3 = (1+c)/2, xi2 = (1+b)/2 (1-xi3), xi1 = (1+a)/2 (1-xi2-xi3);
  // Jacobian factors (1-b)/2 and ((1-c)/2)^2 go into Gauss-Jacobi weights
  std::vector<double> xa, wa, xb, wb, xc, wc;
  gauss_jacobi(n, 0.0, xa, wa);
  gauss_jacobi(n, 1.0, xb, wb);
  gauss_jacobi(n, 2.0, xc, wc);
  Rule r;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const double xi3 = 0.5 * (1.0 + xc[k]);
        const double xi2 = 0.5 * (1.0 + xb[j]) * (1.0 - xi3);
        const double xi1 = 0.5 * (1.0 + xa[i]) * (1.0 - xi2 - xi3);
        // d(xi)/d(a,b,c) = (1/2)(1/2)(1/2) * ((1-b)/2) * ((1-c)/2)^2; the
        // (1-b) and (1-c)^2 parts are in the Jacobi weights: factor 1/2*1/4*1/8
        r.pts.push_back({xi1, xi2, xi3});
        r.w.push_back(wa[i] * wb[j] * wc[k] / 64.0);
      }
  return r;
}

Rule tri_rule(int n) {
  std::vector<double> xa, wa, xb, wb;
  gauss_jacobi(n, 0.0, xa, wa);
  gauss_jacobi(n, 1.0, xb, wb);
  Rule r;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double c2 = 0.5 * (1.0 + xb[j]);
      const double c1 = 0.5 * (1.0 + xa[i]) * (1.0 - c2);
      r.pts.push_back({c1, c2, 0.0});
      r.w.push_back(wa[i] * wb[j] / 8.0);
    }
  return r;
}

static const double REFV[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

void face_point(int i, double c1, double c2, double xi[3]) {
  int a[3], m = 0;
  for (int v = 0; v < 4; ++v)
    if (v != i) a[m++] = v;
  for (int d = 0; d < 3; ++d)
    xi[d] = REFV[a[0]][d] + c1 * (REFV[a[1]][d] - REFV[a[0]][d]) + c2 * (REFV[a[2]][d] - REFV[a[0]][d]);
}

std::vector<double> eval_basis(int O, const double xi[3]) {
  std::vector<double> out;
  tet_basis<double>(O, xi[0], xi[1], xi[2], out);
  return out;
}

RefMats reference_matrices(int O) {
  RefMats R;
  R.O = O;
  R.B = n_basis(O);
  R.F = n_face_basis(O);
  const int B = R.B, F = R.F;
  R.K.assign(3 * B * B, 0.0);
  R.Ft.assign(4 * B * F, 0.0);
  Rule vr = tet_rule(O + 1);
  std::vector<Dual3> phi;
  for (size_t p = 0; p < vr.w.size(); ++p) {
    Dual3 u(vr.pts[p][0]), v(vr.pts[p][1]), w(vr.pts[p][2]);
    u.d[0] = 1.0;
    v.d[1] = 1.0;
    w.d[2] = 1.0;
    tet_basis<Dual3>(O, u, v, w, phi);
    for (int c = 0; c < 3; ++c)
      for (int b = 0; b < B; ++b)
        for (int bb = 0; bb < B; ++bb) R.K[(c * B + b) * B + bb] += vr.w[p] * phi[b].v * phi[bb].d[c];
  }
  Rule fr = tri_rule(O + 1);
  std::vector<double> psi, ph;
  for (int i = 0; i < 4; ++i)
    for (size_t p = 0; p < fr.w.size(); ++p) {
      double xi[3];
      face_point(i, fr.pts[p][0], fr.pts[p][1], xi);
      tet_basis<double>(O, xi[0], xi[1], xi[2], ph);
      tri_basis(O, fr.pts[p][0], fr.pts[p][1], psi);
      for (int b = 0; b < B; ++b)
        for (int f = 0; f < F; ++f) R.Ft[(i * B + b) * F + f] += fr.w[p] * ph[b] * psi[f];
    }
  return R;
}

std::vector<double> direction_matrices(const RefMats& M, const Directions& D) {
  const int B = M.B;
  std::vector<double> Kd(3 * B * B, 0.0);
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c)
      if (D.V[3 * k + c] != 0.0)
        for (int i = 0; i < B * B; ++i) Kd[k * B * B + i] += D.V[3 * k + c] * M.K[c * B * B + i];
  return Kd;
}

Directions sparse_directions(int O) {
  const RefMats M = reference_matrices(O);
  const int B = M.B;
  const double vals[5] = {-1.0, -0.5, 0.0, 0.5, 1.0};
  std::vector<std::array<double, 3>> cand;
  std::vector<int> nnz;
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b)
      for (int c = 0; c < 5; ++c) {
        const std::array<double, 3> v = {vals[a], vals[b], vals[c]};
        const double mx = std::max(std::fabs(v[0]), std::max(std::fabs(v[1]), std::fabs(v[2])));
        const double first = v[0] != 0.0 ? v[0] : (v[1] != 0.0 ? v[1] : v[2]);
        if (mx != 1.0 || first <= 0.0) continue;
        int n = 0;
        for (int i = 0; i < B * B; ++i)
          n += std::fabs(v[0] * M.K[i] + v[1] * M.K[B * B + i] + v[2] * M.K[2 * B * B + i]) > 1e-12;
        cand.push_back(v);
        nnz.push_back(n);
      }
  const int n = (int)cand.size();
  int best[3] = {-1, -1, -1}, best_cost = 1 << 30;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      for (int k = j + 1; k < n; ++k) {
        const int cost = nnz[i] + nnz[j] + nnz[k];
        if (cost >= best_cost) continue;
        const auto &x = cand[i], &y = cand[j], &z = cand[k];
        const double det = x[0] * (y[1] * z[2] - y[2] * z[1]) - x[1] * (y[0] * z[2] - y[2] * z[0]) +
                           x[2] * (y[0] * z[1] - y[1] * z[0]);
        if (std::fabs(det) < 1e-9) continue;
        best_cost = cost;
        best[0] = i; best[1] = j; best[2] = k;
      }
  Directions D;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) D.V[3 * r + c] = cand[best[r]][c];
    D.nnz[r] = nnz[best[r]];
  }
  const double* V = D.V;
  const double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                     V[2] * (V[3] * V[7] - V[4] * V[6]);
  const double id = 1.0 / det;
  D.Vinv[0] = (V[4] * V[8] - V[5] * V[7]) * id;
  D.Vinv[1] = (V[2] * V[7] - V[1] * V[8]) * id;
  D.Vinv[2] = (V[1] * V[5] - V[2] * V[4]) * id;
  D.Vinv[3] = (V[5] * V[6] - V[3] * V[8]) * id;
  D.Vinv[4] = (V[0] * V[8] - V[2] * V[6]) * id;
  D.Vinv[5] = (V[2] * V[3] - V[0] * V[5]) * id;
  D.Vinv[6] = (V[3] * V[7] - V[4] * V[6]) * id;
  D.Vinv[7] = (V[1] * V[6] - V[0] * V[7]) * id;
  D.Vinv[8] = (V[0] * V[4] - V[1] * V[3]) * id;
  return D;
}

std::vector<double> vertex_permutation_matrix(int O, const int perm[4]) {
  // q_new(xi_new) is the same polynomial as q_old(xi_old): project
  // phi_bb(xi_old(xi_new)) onto phi_b(xi_new).  Barycentrics: lambda_new[m] =
  // lambda_old[perm[m]].
  const int B = n_basis(O);
  std::vector<double> C(B * B, 0.0);
  Rule vr = tet_rule(O + 1);
  std::vector<double> pn, po;
  for (size_t p = 0; p < vr.w.size(); ++p) {
    const double* xn = vr.pts[p].data();
    double lam_new[4] = {1.0 - xn[0] - xn[1] - xn[2], xn[0], xn[1], xn[2]};
    double lam_old[4];
    for (int m = 0; m < 4; ++m) lam_old[perm[m]] = lam_new[m];
    tet_basis<double>(O, xn[0], xn[1], xn[2], pn);
    tet_basis<double>(O, lam_old[1], lam_old[2], lam_old[3], po);
    for (int b = 0; b < B; ++b)
      for (int bb = 0; bb < B; ++bb) C[b * B + bb] += vr.w[p] * pn[b] * po[bb];
  }
  return C;
}

}  // namespace edg
