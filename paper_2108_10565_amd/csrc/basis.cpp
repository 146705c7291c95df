// Host construction of the reference matrices; see basis.hpp.
#include "basis.hpp"

#include <cmath>
#include <stdexcept>

namespace stp_host {

namespace {

// Jacobi polynomial P_n^(alpha,beta)(x) by the three-term recurrence.
double jacobi(int n, double alpha, double beta, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0;
  double p1 = 0.5 * (alpha - beta + (alpha + beta + 2.0) * x);
  for (int m = 2; m <= n; ++m) {
    const double ab = alpha + beta;
    const double c = 2.0 * m + ab;
    const double a1 = 2.0 * m * (m + ab) * (c - 2.0);
    const double a2 = (c - 1.0) * (alpha * alpha - beta * beta);
    const double a3 = (c - 2.0) * (c - 1.0) * c;
    const double a4 = 2.0 * (m + alpha - 1.0) * (m + beta - 1.0) * c;
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// d/dx P_n^(alpha,beta)(x) = (n + alpha + beta + 1)/2 P_{n-1}^(alpha+1,beta+1)(x).
double djacobi(int n, double alpha, double beta, double x) {
  if (n == 0) return 0.0;
  return 0.5 * (n + alpha + beta + 1.0) * jacobi(n - 1, alpha + 1.0, beta + 1.0, x);
}

// Gauss-Legendre rule with n points on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double t = std::cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      const double p = jacobi(n, 0, 0, t);
      const double dp = djacobi(n, 0, 0, t);
      const double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    const double dp = djacobi(n, 0, 0, t);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

}  // namespace

void mode_ijk(int N, int m, int* i, int* j, int* k) {
  int idx = 0;
  for (int n = 0; n <= N; ++n)
    for (int kk = 0; kk <= n; ++kk)
      for (int jj = 0; jj <= n - kk; ++jj, ++idx)
        if (idx == m) {
          *i = n - kk - jj;
          *j = jj;
          *k = kk;
          return;
        }
  throw std::out_of_range("mode index");
}

ReferenceMatrices build_reference_matrices(int N) {
  if (N < 0 || N > kMaxDegree) throw std::out_of_range("degree");
  ReferenceMatrices R;
  R.N = N;
  R.B = n_modes(N);
  R.T = N + 1;
  const int B = R.B, T = R.T;

  // ---- temporal: S_rs = delta_rs/(2s+1), W_rs = 1, w_r = (-1)^r,
  //      K^tau_rs = 2 for r > s with r - s odd (Legendre derivative identity)
  R.Z.assign(T * T, 0.0);
  R.Sinv_w.assign(T, 0.0);
  for (int u = 0; u < T; ++u) {
    R.Sinv_w[u] = (2.0 * u + 1.0) * ((u % 2) ? -1.0 : 1.0);
    for (int s = 0; s < T; ++s) {
      const double kt = (u > s && ((u - s) % 2) == 1) ? 2.0 : 0.0;
      R.Z[u * T + s] = (2.0 * u + 1.0) * (1.0 - kt);
    }
  }

  // ---- spatial: collapsed coordinates (a, b, c) in [-1, 1]^3,
  //      x = (1+a)(1-b)(1-c)/8, y = (1+b)(1-c)/4, z = (1+c)/2,
  //      dV = (1-b)(1-c)^2/64 da db dc.
  const int nq = N + 3;  // exact for the polynomial degrees involved
  std::vector<double> qx, qw;
  gauss_legendre(nq, qx, qw);
  const int P = nq * nq * nq;
  std::vector<double> phi(static_cast<size_t>(B) * P), dphi(static_cast<size_t>(3) * B * P), wq(P);
  std::vector<int> mi(B), mj(B), mk(B);
  for (int m = 0; m < B; ++m) mode_ijk(N, m, &mi[m], &mj[m], &mk[m]);
  for (int ia = 0; ia < nq; ++ia)
    for (int ib = 0; ib < nq; ++ib)
      for (int ic = 0; ic < nq; ++ic) {
        const int q = (ia * nq + ib) * nq + ic;
        const double a = qx[ia], b = qx[ib], c = qx[ic];
        const double h1 = 0.25 * (1.0 - b) * (1.0 - c);  // 1 - y - z
        const double h2 = 0.5 * (1.0 - c);                // 1 - z
        wq[q] = qw[ia] * qw[ib] * qw[ic] * (1.0 - b) * (1.0 - c) * (1.0 - c) / 64.0;
        for (int m = 0; m < B; ++m) {
          const int i = mi[m], j = mj[m], k = mk[m];
          const double ab = 2.0 * i + 1.0, ac = 2.0 * i + 2.0 * j + 2.0;
          // factor A = P_i(a) h1^i, Bf = P_j^(2i+1,0)(b) h2^j, C = P_k^(2i+2j+2,0)(c)
          const double Pa = jacobi(i, 0, 0, a), dPa = djacobi(i, 0, 0, a);
          const double Pb = jacobi(j, ab, 0, b), dPb = djacobi(j, ab, 0, b);
          const double Pc = jacobi(k, ac, 0, c), dPc = djacobi(k, ac, 0, c);
          const double h1i = std::pow(h1, i), h2j = std::pow(h2, j);
          const double h1im = i > 0 ? std::pow(h1, i - 1) : 0.0;
          const double h2jm = j > 0 ? std::pow(h2, j - 1) : 0.0;
          const double A = Pa * h1i, Bf = Pb * h2j, C = Pc;
          // dA/dx = 2 P_i'(a) h1^(i-1);  dA/dy = dA/dz = h1^(i-1) (P_i'(a)(a+1) - i P_i(a))
          const double dAx = 2.0 * dPa * h1im;
          const double dAyz = h1im * (dPa * (a + 1.0) - i * Pa);
          // dBf/dy = 2 P_j'(b) h2^(j-1);  dBf/dz = h2^(j-1) (P_j'(b)(b+1) - j P_j(b))
          const double dBy = 2.0 * dPb * h2jm;
          const double dBz = h2jm * (dPb * (b + 1.0) - j * Pb);
          const double dCz = 2.0 * dPc;
          phi[static_cast<size_t>(m) * P + q] = A * Bf * C;
          dphi[(0 * static_cast<size_t>(B) + m) * P + q] = dAx * Bf * C;
          dphi[(1 * static_cast<size_t>(B) + m) * P + q] = dAyz * Bf * C + A * dBy * C;
          dphi[(2 * static_cast<size_t>(B) + m) * P + q] = dAyz * Bf * C + A * dBz * C + A * Bf * dCz;
        }
      }
  R.M.assign(B, 0.0);
  R.K.assign(static_cast<size_t>(3) * B * B, 0.0);
  R.Khat.assign(static_cast<size_t>(3) * B * B, 0.0);
  R.max_mass_offdiag = 0.0;
  for (int k = 0; k < B; ++k)
    for (int l = 0; l < B; ++l) {
      double s = 0.0;
      for (int q = 0; q < P; ++q) s += wq[q] * phi[static_cast<size_t>(k) * P + q] * phi[static_cast<size_t>(l) * P + q];
      if (k == l) R.M[k] = s;
      else R.max_mass_offdiag = std::fmax(R.max_mass_offdiag, std::fabs(s));
    }
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < B; ++k)
      for (int l = 0; l < B; ++l) {
        // exact zeros of the Lemma (deg phi_l <= deg phi_k) are set, not summed
        if (mi[l] + mj[l] + mk[l] <= mi[k] + mj[k] + mk[k]) continue;
        double s = 0.0;
        for (int q = 0; q < P; ++q)
          s += wq[q] * phi[static_cast<size_t>(k) * P + q] * dphi[(static_cast<size_t>(d) * B + l) * P + q];
        R.K[(static_cast<size_t>(d) * B + k) * B + l] = s;
        R.Khat[(static_cast<size_t>(d) * B + k) * B + l] = s / R.M[k];
      }
  // Quadrature leaves ~1e-16 noise where the exact integral vanishes (the
  // smallest true non-zero of Khat at N <= 7 is ~1e-6 of the largest):
  // flush entries below 1e-11 of the largest to exact zeros.
  double kmax = 0.0;
  for (double v : R.Khat) kmax = std::fmax(kmax, std::fabs(v));
  for (size_t t = 0; t < R.Khat.size(); ++t)
    if (std::fabs(R.Khat[t]) < 1e-11 * kmax) {
      R.Khat[t] = 0.0;
      R.K[t] = 0.0;
    }
  return R;
}

}  // namespace stp_host
