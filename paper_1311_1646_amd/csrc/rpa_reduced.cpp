// The reduced DMRG-RPA eigenproblem (Sec. III E, eq. reducedrpa); see the
// header for the formulation.
#include "rpa_reduced.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace dmrg {

void jacobi_eigh(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[i + size_t(i) * n] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[i + size_t(j) * n]; };
  double scale = 0;
  for (double v : A) scale = std::max(scale, std::abs(v));
  for (int sweep = 0; sweep < 100 && scale > 0; ++sweep) {
    double off = 0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < j; ++i) off = std::max(off, std::abs(a(i, j)));
    if (off <= 1e-17 * scale) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::abs(apq) <= 1e-300) continue;
        // rotation that zeroes A[p][q]
        const double theta = 0.5 * (a(q, q) - a(p, p)) / apq;
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::abs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k + size_t(p) * n], vkq = V[k + size_t(q) * n];
          V[k + size_t(p) * n] = c * vkp - s * vkq;
          V[k + size_t(q) * n] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int i, int j) { return a(i, i) < a(j, j); });
  std::vector<double> V2(size_t(n) * n);
  w.resize(n);
  for (int k = 0; k < n; ++k) {
    w[k] = a(ord[k], ord[k]);
    for (int i = 0; i < n; ++i) V2[i + size_t(k) * n] = V[i + size_t(ord[k]) * n];
  }
  V.swap(V2);
}

namespace {

// C = A^T B with A (m x p), B (m x q), column-major
std::vector<double> atb(int m, int p, int q, const double* A, const double* B) {
  std::vector<double> C(size_t(p) * q, 0.0);
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < p; ++i) {
      double s = 0;
      for (int k = 0; k < m; ++k) s += A[k + size_t(i) * m] * B[k + size_t(j) * m];
      C[i + size_t(j) * p] = s;
    }
  return C;
}

// C = A B with A (m x k), B (k x n)
std::vector<double> ab(int m, int k, int n, const double* A, const double* B) {
  std::vector<double> C(size_t(m) * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int t = 0; t < k; ++t) {
      const double b = B[t + size_t(j) * k];
      if (b == 0.0) continue;
      for (int i = 0; i < m; ++i) C[i + size_t(j) * m] += A[i + size_t(t) * m] * b;
    }
  return C;
}

void symmetrize(int n, std::vector<double>& A) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < j; ++i) {
      const double v = 0.5 * (A[i + size_t(j) * n] + A[j + size_t(i) * n]);
      A[i + size_t(j) * n] = A[j + size_t(i) * n] = v;
    }
}

}  // namespace

int rpa_reduced_solve(int l, const double* HR, const double* SR, const double* WR, double e0, double rank_tol,
                      RpaReduced& out) {
  // canonical orthogonalization of S_R
  std::vector<double> s, Vs;
  std::vector<double> S(SR, SR + size_t(l) * l);
  symmetrize(l, S);
  jacobi_eigh(l, S, s, Vs);
  const double smax = l ? std::max(s.back(), 0.0) : 0.0;
  std::vector<int> keep;
  for (int k = 0; k < l; ++k)
    if (s[k] > rank_tol * smax) keep.push_back(k);
  const int r = int(keep.size());
  out.r = r;
  out.T.assign(size_t(l) * r, 0.0);
  for (int j = 0; j < r; ++j) {
    const double f = 1.0 / std::sqrt(s[keep[j]]);
    for (int i = 0; i < l; ++i) out.T[i + size_t(j) * l] = Vs[i + size_t(keep[j]) * l] * f;
  }
  out.omega.clear();
  out.x.clear();
  out.y.clear();
  if (r == 0) return 0;
  // A' = T^T (H_R - E0 S_R) T, W' = T^T W_R T
  std::vector<double> A(size_t(l) * l), W(WR, WR + size_t(l) * l);
  for (size_t e = 0; e < A.size(); ++e) A[e] = HR[e] - e0 * SR[e];
  symmetrize(l, A);
  symmetrize(l, W);
  std::vector<double> AT = ab(l, l, r, A.data(), out.T.data());
  std::vector<double> WT = ab(l, l, r, W.data(), out.T.data());
  std::vector<double> Ap = atb(l, r, r, out.T.data(), AT.data());
  std::vector<double> Wp = atb(l, r, r, out.T.data(), WT.data());
  std::vector<double> P(size_t(r) * r), Q(size_t(r) * r);
  for (size_t e = 0; e < P.size(); ++e) {
    P[e] = Ap[e] + Wp[e];
    Q[e] = Ap[e] - Wp[e];
  }
  symmetrize(r, P);
  symmetrize(r, Q);
  // Q^(1/2) from the eigen-decomposition of Q (positive definite if stable)
  std::vector<double> q, Vq;
  jacobi_eigh(r, Q, q, Vq);
  if (q[0] <= 0.0) return -1;
  std::vector<double> Qh(size_t(r) * r, 0.0);
  for (int k = 0; k < r; ++k) {
    const double f = std::sqrt(q[k]);
    for (int j = 0; j < r; ++j)
      for (int i = 0; i < r; ++i) Qh[i + size_t(j) * r] += Vq[i + size_t(k) * r] * f * Vq[j + size_t(k) * r];
  }
  // M = Q^(1/2) P Q^(1/2): M z = omega^2 z
  std::vector<double> PQh = ab(r, r, r, P.data(), Qh.data());
  std::vector<double> M = ab(r, r, r, Qh.data(), PQh.data());
  symmetrize(r, M);
  std::vector<double> w2, Z;
  jacobi_eigh(r, M, w2, Z);
  if (w2[0] <= 0.0) return -1;
  out.omega.resize(r);
  out.x.assign(size_t(r) * r, 0.0);
  out.y.assign(size_t(r) * r, 0.0);
  // u = X + Y = Q^(1/2) z, v = X - Y = P u / omega (from (A + W)(X + Y) =
  // omega (X - Y)); u . v = omega for unit z, so X, Y scale by 1/sqrt(omega)
  std::vector<double> U = ab(r, r, r, Qh.data(), Z.data());
  std::vector<double> PU = ab(r, r, r, P.data(), U.data());
  for (int k = 0; k < r; ++k) {
    const double om = std::sqrt(w2[k]);
    out.omega[k] = om;
    const double f = 1.0 / std::sqrt(om);
    for (int i = 0; i < r; ++i) {
      const double u = U[i + size_t(k) * r], v = PU[i + size_t(k) * r] / om;
      out.x[i + size_t(k) * r] = 0.5 * (u + v) * f;
      out.y[i + size_t(k) * r] = 0.5 * (u - v) * f;
    }
  }
  return 0;
}

}  // namespace dmrg
