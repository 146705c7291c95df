// Host side of the ADER-DG corrector (section "ADER-DG discretisation",
// eq:semi_discrete integrated over one time step): reference volume and
// face tables, the Dubiner basis at arbitrary points, the Godunov (upwind)
// split of a normal Jacobian, and the per-face flux operators of a mesh.
#include "ader_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <unordered_map>
#include <utility>

namespace stp_host {

namespace {

double jac(int n, double alpha, double beta, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * (alpha - beta + (alpha + beta + 2.0) * x);
  for (int m = 2; m <= n; ++m) {
    const double ab = alpha + beta, c = 2.0 * m + ab;
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

// Gauss-Legendre nodes and weights on [-1, 1].
void gauss(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double t = std::cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      const double p = jac(n, 0, 0, t);
      const double dp = 0.5 * (n + 1.0) * jac(n - 1, 1, 1, t);
      const double d = p / dp;
      t -= d;
      if (std::fabs(d) < 1e-16) break;
    }
    const double dp = 0.5 * (n + 1.0) * jac(n - 1, 1, 1, t);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// Quadrature on the reference triangle {s, t >= 0, s + t <= 1} (collapsed
// Gauss rule, exact for polynomials of degree 2n - 2).
void triangle_rule(int n, std::vector<double>& s, std::vector<double>& t, std::vector<double>& w) {
  std::vector<double> x, wx;
  gauss(n, x, wx);
  s.clear();
  t.clear();
  w.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double u = x[i], v = x[j];
      s.push_back(0.25 * (1.0 + u) * (1.0 - v));
      t.push_back(0.5 * (1.0 + v));
      w.push_back(wx[i] * wx[j] * (1.0 - v) / 8.0);
    }
}

constexpr double kRefV[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

void face_point(int f, double s, double t, double* x) {
  const int* v = kFaceVertices[f];
  for (int d = 0; d < 3; ++d)
    x[d] = kRefV[v[0]][d] + s * (kRefV[v[1]][d] - kRefV[v[0]][d]) + t * (kRefV[v[2]][d] - kRefV[v[0]][d]);
}

// ---- eigenvalues of a real matrix with real spectrum ------------------------

// Diagonal similarity by powers of two that equalises row and column norms
// (balancing; the spectrum is unchanged and the QR iteration more accurate).
void balance(int n, std::vector<double>& a) {
  bool done = false;
  while (!done) {
    done = true;
    for (int i = 0; i < n; ++i) {
      double c = 0.0, r = 0.0;
      for (int j = 0; j < n; ++j)
        if (j != i) {
          c += std::fabs(a[j * n + i]);
          r += std::fabs(a[i * n + j]);
        }
      if (c == 0.0 || r == 0.0) continue;
      double f = 1.0;
      const double s = c + r;
      while (c < r / 2.0) {
        c *= 2.0;
        r /= 2.0;
        f *= 2.0;
      }
      while (c >= r * 2.0) {
        c /= 2.0;
        r *= 2.0;
        f /= 2.0;
      }
      if ((c + r) < 0.95 * s) {
        done = false;
        for (int j = 0; j < n; ++j) a[i * n + j] /= f;
        for (int j = 0; j < n; ++j) a[j * n + i] *= f;
      }
    }
  }
}

// Upper Hessenberg form by Householder reflections (similarity).
void hessenberg(int n, std::vector<double>& a) {
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += a[i * n + k] * a[i * n + k];
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    if (a[(k + 1) * n + k] > 0) alpha = -alpha;
    std::vector<double> v(n, 0.0);
    v[k + 1] = a[(k + 1) * n + k] - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = a[i * n + k];
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    // A <- (I - 2 v v^T / vv) A (I - 2 v v^T / vv)
    for (int j = 0; j < n; ++j) {
      double d = 0.0;
      for (int i = k + 1; i < n; ++i) d += v[i] * a[i * n + j];
      d *= 2.0 / vv;
      for (int i = k + 1; i < n; ++i) a[i * n + j] -= d * v[i];
    }
    for (int i = 0; i < n; ++i) {
      double d = 0.0;
      for (int j = k + 1; j < n; ++j) d += a[i * n + j] * v[j];
      d *= 2.0 / vv;
      for (int j = k + 1; j < n; ++j) a[i * n + j] -= d * v[j];
    }
  }
}

// Eigenvalues of an upper Hessenberg matrix by the implicitly shifted
// (Francis double-shift) QR iteration with deflation.  Complex pairs are
// returned with their imaginary parts; false if the iteration stalls.
bool hessenberg_eigenvalues(int n, std::vector<double> h, std::vector<double>& wr, std::vector<double>& wi) {
  wr.assign(n, 0.0);
  wi.assign(n, 0.0);
  auto H = [&](int i, int j) -> double& { return h[i * n + j]; };
  double norm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = std::max(i - 1, 0); j < n; ++j) norm += std::fabs(H(i, j));
  int hi = n - 1;
  int iter = 0;
  double t = 0.0;  // accumulated exceptional shift
  while (hi >= 0) {
    // find a negligible subdiagonal element
    int l = hi;
    for (; l > 0; --l) {
      double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
      if (s == 0.0) s = norm;
      if (std::fabs(H(l, l - 1)) <= 1e-16 * s) {
        H(l, l - 1) = 0.0;
        break;
      }
    }
    double x = H(hi, hi);
    if (l == hi) {  // one root
      wr[hi] = x + t;
      wi[hi] = 0.0;
      --hi;
      iter = 0;
      continue;
    }
    double y = H(hi - 1, hi - 1), w = H(hi, hi - 1) * H(hi - 1, hi);
    if (l == hi - 1) {  // two roots
      const double p = 0.5 * (y - x), q = p * p + w;
      const double z = std::sqrt(std::fabs(q));
      x += t;
      if (q >= 0.0) {
        const double zz = p + (p >= 0 ? z : -z);
        wr[hi - 1] = wr[hi] = x + zz;
        if (zz != 0.0) wr[hi] = x - w / zz;
        wi[hi - 1] = wi[hi] = 0.0;
      } else {
        wr[hi - 1] = wr[hi] = x + p;
        wi[hi - 1] = z;
        wi[hi] = -z;
      }
      hi -= 2;
      iter = 0;
      continue;
    }
    if (iter >= 60) return false;
    if (iter == 10 || iter == 20) {  // exceptional shift
      t += x;
      for (int i = 0; i <= hi; ++i) H(i, i) -= x;
      const double s = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
      x = y = 0.75 * s;
      w = -0.4375 * s * s;
    }
    ++iter;
    // double-shift QR step on rows/columns l..hi
    int m = hi - 2;
    double p = 0.0, q = 0.0, r = 0.0, z;
    for (; m >= l; --m) {
      z = H(m, m);
      const double rr = x - z, ss = y - z;
      p = (rr * ss - w) / H(m + 1, m) + H(m, m + 1);
      q = H(m + 1, m + 1) - z - rr - ss;
      r = H(m + 2, m + 1);
      const double s = std::fabs(p) + std::fabs(q) + std::fabs(r);
      p /= s;
      q /= s;
      r /= s;
      if (m == l) break;
      const double u = std::fabs(H(m, m - 1)) * (std::fabs(q) + std::fabs(r));
      const double v = std::fabs(p) * (std::fabs(H(m - 1, m - 1)) + std::fabs(z) + std::fabs(H(m + 1, m + 1)));
      if (u <= 1e-16 * v) break;
    }
    for (int i = m + 2; i <= hi; ++i) {
      H(i, i - 2) = 0.0;
      if (i != m + 2) H(i, i - 3) = 0.0;
    }
    for (int k = m; k <= hi - 1; ++k) {
      if (k != m) {
        p = H(k, k - 1);
        q = H(k + 1, k - 1);
        r = (k != hi - 1) ? H(k + 2, k - 1) : 0.0;
        x = std::fabs(p) + std::fabs(q) + std::fabs(r);
        if (x != 0.0) {
          p /= x;
          q /= x;
          r /= x;
        }
      }
      const double s0 = std::sqrt(p * p + q * q + r * r);
      const double s = p >= 0 ? s0 : -s0;
      if (s == 0.0) continue;
      if (k == m) {
        if (l != m) H(k, k - 1) = -H(k, k - 1);
      } else {
        H(k, k - 1) = -s * x;
      }
      p += s;
      x = p / s;
      y = q / s;
      z = r / s;
      q /= p;
      r /= p;
      for (int j = k; j <= hi; ++j) {  // rows k, k+1, k+2
        double pp = H(k, j) + q * H(k + 1, j);
        if (k != hi - 1) {
          pp += r * H(k + 2, j);
          H(k + 2, j) -= pp * z;
        }
        H(k + 1, j) -= pp * y;
        H(k, j) -= pp * x;
      }
      const int mmin = hi < k + 3 ? hi : k + 3;
      for (int i = l; i <= mmin; ++i) {  // columns k, k+1, k+2
        double pp = x * H(i, k) + y * H(i, k + 1);
        if (k != hi - 1) {
          pp += z * H(i, k + 2);
          H(i, k + 2) -= pp * r;
        }
        H(i, k + 1) -= pp * q;
        H(i, k) -= pp;
      }
    }
  }
  return true;
}

void matmul(int n, const std::vector<double>& a, const std::vector<double>& b, std::vector<double>& c) {
  c.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double v = a[i * n + k];
      if (v == 0.0) continue;
      for (int j = 0; j < n; ++j) c[i * n + j] += v * b[k * n + j];
    }
}

}  // namespace

void eval_dubiner(int N, double x, double y, double z, double* phi) {
  const double h1 = 1.0 - y - z, h2 = 1.0 - z;
  const double a = h1 > 1e-300 ? 2.0 * x / h1 - 1.0 : -1.0;
  const double b = h2 > 1e-300 ? 2.0 * y / h2 - 1.0 : -1.0;
  const double c = 2.0 * z - 1.0;
  int m = 0;
  for (int n = 0; n <= N; ++n)
    for (int k = 0; k <= n; ++k)
      for (int j = 0; j <= n - k; ++j, ++m) {
        const int i = n - k - j;
        phi[m] = jac(i, 0, 0, a) * std::pow(h1, i) * jac(j, 2.0 * i + 1.0, 0, b) * std::pow(h2, j) *
                 jac(k, 2.0 * i + 2.0 * j + 2.0, 0, c);
      }
}

CorrectorTables build_corrector_tables(int N) {
  const ReferenceMatrices R = build_reference_matrices(N);
  const int B = R.B;
  CorrectorTables C;
  C.N = N;
  C.B = B;
  C.M = R.M;
  const size_t BB = static_cast<size_t>(B) * B;
  C.V.assign(3 * BB, 0.0);
  for (int d = 0; d < 3; ++d)
    for (int l = 0; l < B; ++l)
      for (int k = 0; k < B; ++k) C.V[d * BB + l * B + k] = R.K[d * BB + l * B + k] / R.M[k];
  std::vector<double> s, t, w;
  triangle_rule(N + 2, s, t, w);
  const int P = static_cast<int>(w.size());
  // basis on every face at the rule's points, and at the neighbour's
  // parameters under each of the 6 vertex correspondences
  std::vector<double> own(static_cast<size_t>(4) * P * B), nb(static_cast<size_t>(4) * 6 * P * B);
  for (int f = 0; f < 4; ++f)
    for (int q = 0; q < P; ++q) {
      double x[3];
      face_point(f, s[q], t[q], x);
      eval_dubiner(N, x[0], x[1], x[2], &own[(static_cast<size_t>(f) * P + q) * B]);
      const double wgt[3] = {1.0 - s[q] - t[q], s[q], t[q]};
      for (int h = 0; h < 6; ++h) {
        double wn[3];
        for (int r = 0; r < 3; ++r) wn[kPerm[h][r]] = wgt[r];
        face_point(f, wn[1], wn[2], x);
        eval_dubiner(N, x[0], x[1], x[2], &nb[((static_cast<size_t>(f) * 6 + h) * P + q) * B]);
      }
    }
  C.Fl.assign(4 * BB, 0.0);
  C.Fn.assign(96 * BB, 0.0);
  for (int i = 0; i < 4; ++i)
    for (int l = 0; l < B; ++l)
      for (int k = 0; k < B; ++k) {
        double acc = 0.0;
        for (int q = 0; q < P; ++q)
          acc += w[q] * own[(static_cast<size_t>(i) * P + q) * B + l] * own[(static_cast<size_t>(i) * P + q) * B + k];
        C.Fl[i * BB + l * B + k] = acc / R.M[k];
      }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int h = 0; h < 6; ++h) {
        double* F = &C.Fn[((i * 4 + j) * 6 + h) * BB];
        for (int l = 0; l < B; ++l)
          for (int k = 0; k < B; ++k) {
            double acc = 0.0;
            for (int q = 0; q < P; ++q)
              acc += w[q] * nb[((static_cast<size_t>(j) * 6 + h) * P + q) * B + l] *
                     own[(static_cast<size_t>(i) * P + q) * B + k];
            F[l * B + k] = acc / R.M[k];
          }
      }
  return C;
}

bool upwind_split(int nq, const double* An, double* Ap, double* Am, std::string* err) {
  const int n = nq;
  std::vector<double> a(An, An + static_cast<size_t>(n) * n);
  double scale = 0.0;
  for (double v : a) scale = std::fmax(scale, std::fabs(v));
  if (scale == 0.0) {
    std::fill(Ap, Ap + n * n, 0.0);
    std::fill(Am, Am + n * n, 0.0);
    return true;
  }
  std::vector<double> h = a;
  balance(n, h);
  hessenberg(n, h);
  std::vector<double> wr, wi;
  if (!hessenberg_eigenvalues(n, h, wr, wi)) {
    if (err) *err = "eigenvalue iteration did not converge";
    return false;
  }
  double lmax = 0.0;
  for (int i = 0; i < n; ++i) lmax = std::fmax(lmax, std::hypot(wr[i], wi[i]));
  for (int i = 0; i < n; ++i)
    if (std::fabs(wi[i]) > 1e-8 * lmax) {
      if (err) *err = "the normal Jacobian has complex eigenvalues (not hyperbolic)";
      return false;
    }
  // distinct eigenvalues (clusters within 1e-7 of the spectral radius)
  std::sort(wr.begin(), wr.end());
  std::vector<double> lam;
  for (double v : wr)
    if (lam.empty() || v - lam.back() > 1e-7 * lmax) lam.push_back(v);
    else lam.back() = 0.5 * (lam.back() + v);
  for (double& v : lam)
    if (std::fabs(v) <= 1e-7 * lmax) v = 0.0;
  // A^+ = sum_{lambda > 0} lambda P_lambda with the spectral projectors
  // P_i = prod_{j != i} (A - lambda_j I) / (lambda_i - lambda_j)
  // (A is diagonalisable for a hyperbolic system); A^- = A - A^+.
  std::vector<double> plus(static_cast<size_t>(n) * n, 0.0), prod, tmp, f;
  for (size_t i = 0; i < lam.size(); ++i) {
    if (lam[i] <= 0.0) continue;
    prod.assign(static_cast<size_t>(n) * n, 0.0);
    for (int d = 0; d < n; ++d) prod[d * n + d] = 1.0;
    for (size_t j = 0; j < lam.size(); ++j) {
      if (j == i) continue;
      f = a;
      for (int d = 0; d < n; ++d) f[d * n + d] -= lam[j];
      const double den = lam[i] - lam[j];
      for (double& v : f) v /= den;
      matmul(n, prod, f, tmp);
      prod.swap(tmp);
    }
    for (size_t e = 0; e < plus.size(); ++e) plus[e] += lam[i] * prod[e];
  }
  // check: A^+ A^- = 0 and A^+ has no negative part, within rounding
  std::vector<double> minus(static_cast<size_t>(n) * n);
  for (size_t e = 0; e < minus.size(); ++e) minus[e] = a[e] - plus[e];
  matmul(n, plus, minus, tmp);
  double pm = 0.0;
  for (double v : tmp) pm = std::fmax(pm, std::fabs(v));
  if (pm > 1e-8 * lmax * scale) {
    if (err) *err = "spectral split inaccurate (eigenvalues too close)";
    return false;
  }
  std::copy(plus.begin(), plus.end(), Ap);
  std::copy(minus.begin(), minus.end(), Am);
  return true;
}

bool face_operators(int nq, int64_t n, const double* ABC, const double* verts, double* Gp, double* Gm,
                    std::string* err) {
  const size_t q2 = static_cast<size_t>(nq) * nq;
  std::vector<double> An(q2);
  // meshes of few materials repeat normal Jacobians: split each distinct one once
  std::unordered_map<std::string, std::pair<std::vector<double>, std::vector<double>>> cache;
  for (int64_t e = 0; e < n; ++e) {
    const double* v = verts + e * 12;
    double J[3][3];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) J[d][c] = v[(c + 1) * 3 + d] - v[d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double absJ = std::fabs(det);
    if (!(absJ > 0.0)) {
      if (err) *err = "degenerate element " + std::to_string(e);
      return false;
    }
    for (int f = 0; f < 4; ++f) {
      const int* fv = kFaceVertices[f];
      const int opp = 6 - fv[0] - fv[1] - fv[2];
      double e1[3], e2[3], nrm[3], out[3];
      for (int d = 0; d < 3; ++d) {
        e1[d] = v[fv[1] * 3 + d] - v[fv[0] * 3 + d];
        e2[d] = v[fv[2] * 3 + d] - v[fv[0] * 3 + d];
        out[d] = v[fv[0] * 3 + d] - v[opp * 3 + d];
      }
      nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
      nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
      nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
      const double len = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
      const double sgn = (nrm[0] * out[0] + nrm[1] * out[1] + nrm[2] * out[2]) > 0 ? 1.0 : -1.0;
      for (int d = 0; d < 3; ++d) nrm[d] *= sgn / len;
      const double area = 0.5 * len;
      for (size_t t = 0; t < q2; ++t)
        An[t] = nrm[0] * ABC[(e * 3 + 0) * q2 + t] + nrm[1] * ABC[(e * 3 + 1) * q2 + t] +
                nrm[2] * ABC[(e * 3 + 2) * q2 + t];
      double* gp = Gp + (e * 4 + f) * q2;
      double* gm = Gm + (e * 4 + f) * q2;
      std::string key(reinterpret_cast<const char*>(An.data()), q2 * sizeof(double));
      auto it = cache.find(key);
      if (it == cache.end()) {
        std::vector<double> p(q2), m(q2);
        if (!upwind_split(nq, An.data(), p.data(), m.data(), err)) {
          if (err) *err = "element " + std::to_string(e) + " face " + std::to_string(f) + ": " + *err;
          return false;
        }
        it = cache.emplace(std::move(key), std::make_pair(std::move(p), std::move(m))).first;
      }
      std::memcpy(gp, it->second.first.data(), q2 * sizeof(double));
      std::memcpy(gm, it->second.second.data(), q2 * sizeof(double));
      const double sc = 2.0 * area / absJ;
      for (size_t t = 0; t < q2; ++t) {
        gp[t] *= sc;
        gm[t] *= sc;
      }
    }
  }
  return true;
}

}  // namespace stp_host
