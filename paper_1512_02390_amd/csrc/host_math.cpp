// Host numerics for the set-up phase (see host_math.h).
#include "host_math.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <stdexcept>
#include <thread>
#include <vector>

namespace sem {

// Runs f(i) for i in [0, n) on the host's cores (at most 16 threads).
static void parallel_for(int n, const std::function<void(int)> &f) {
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t)
    pool.emplace_back([&] {
      for (int i = next++; i < n; i = next++) f(i);
    });
  for (std::thread &t : pool) t.join();
}

// Legendre P_n and P_n' by the three-term recurrence.
static void legendre_pd(int n, double x, double &P, double &dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) away from the ends
  dP = (std::fabs(x) < 1.0) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.5 * n * (n + 1) * (x > 0 ? 1 : (n % 2 ? 1 : -1));
}

void gll_rule(int p, Vec &xi, Vec &w) {
  xi.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  xi[0] = -1.0;
  xi[p] = 1.0;
  // interior points: roots of P_p', by Newton on q(x) = P_p'(x) using the
  // Legendre equation for q'(x) = (2 x P' - p (p+1) P) / (1 - x^2);
  // by symmetry only the left half is iterated.
  for (int i = 1; i <= p / 2; ++i) {
    double x = -std::cos(M_PI * i / p);
    for (int it = 0; it < 200; ++it) {
      double P, dP;
      legendre_pd(p, x, P, dP);
      double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
      double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    xi[i] = x;
    xi[p - i] = -x;
  }
  if (p % 2 == 0) xi[p / 2] = 0.0;
  for (int i = 0; i <= p; ++i) {
    double P, dP;
    legendre_pd(p, xi[i], P, dP);
    w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
}

Mat lagrange_derivative(const Vec &xi) {
  const int n = (int)xi.size();
  Vec bw(n, 1.0);  // barycentric weights
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) bw[j] /= (xi[j] - xi[k]);
  Mat D(n, n);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      D(i, j) = bw[j] / bw[i] / (xi[i] - xi[j]);
      s += D(i, j);
    }
    D(i, i) = -s;
  }
  return D;
}

Mat lagrange_eval(const Vec &xi, const Vec &x) {
  const int n = (int)xi.size(), q = (int)x.size();
  Mat E(q, n);
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < n; ++j) {
      double v = 1.0;
      for (int m = 0; m < n; ++m)
        if (m != j) v *= (x[k] - xi[m]) / (xi[j] - xi[m]);
      E(k, j) = v;
    }
  return E;
}

Mat ref_stiffness(int p) {
  Vec xi, w;
  gll_rule(p, xi, w);
  Mat D = lagrange_derivative(xi);
  Mat L(p + 1, p + 1);
  for (int a = 0; a <= p; ++a)
    for (int b = 0; b <= p; ++b) {
      double s = 0.0;
      for (int q = 0; q <= p; ++q) s += D(q, a) * w[q] * D(q, b);
      L(a, b) = s;
    }
  return L;
}

void sym_eig(const Mat &A0, Vec &lam, Mat &Q) {
  const int n = A0.r;
  Mat A = A0;
  Q = Mat(n, n);
  for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A(i, j) * A(i, j);
        if (i != j) off += A(i, j) * A(i, j);
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (apq == 0.0) continue;
        // rotation angle that annihilates A(p, q)
        double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double qkp = Q(k, p), qkq = Q(k, q);
          Q(k, p) = c * qkp - s * qkq;
          Q(k, q) = s * qkp + c * qkq;
        }
      }
  }
  // sort ascending
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A(a, a) < A(b, b); });
  lam.assign(n, 0.0);
  Mat Qs(n, n);
  for (int k = 0; k < n; ++k) {
    lam[k] = A(idx[k], idx[k]);
    for (int i = 0; i < n; ++i) Qs(i, k) = Q(i, idx[k]);
  }
  Q = Qs;
}

void gen_eig_diag(const Mat &L, const Vec &Md, Vec &lam, Mat &S) {
  const int n = L.r;
  Vec d(n);
  for (int i = 0; i < n; ++i) d[i] = 1.0 / std::sqrt(Md[i]);
  Mat C(n, n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C(i, j) = d[i] * L(i, j) * d[j];
  // symmetrise against rounding of the scaling
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) C(i, j) = C(j, i) = 0.5 * (C(i, j) + C(j, i));
  Mat Q;
  sym_eig(C, lam, Q);
  S = Mat(n, n);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) S(i, k) = d[i] * Q(i, k);
}

bool spd_inverse(Mat &A) {
  const int n = A.r;
  // Cholesky A = G G^T (lower G stored in A)
  for (int j = 0; j < n; ++j) {
    double s = A(j, j);
    for (int k = 0; k < j; ++k) s -= A(j, k) * A(j, k);
    if (!(s > 0.0)) return false;
    double g = std::sqrt(s);
    A(j, j) = g;
    for (int i = j + 1; i < n; ++i) {
      double t = A(i, j);
      const double *ri = &A.a[(size_t)i * n], *rj = &A.a[(size_t)j * n];
      for (int k = 0; k < j; ++k) t -= ri[k] * rj[k];
      A(i, j) = t / g;
    }
  }
  // H = G^{-1} (lower triangular), stored transposed (Ht(j, k) = H(k, j)) so
  // that both remaining phases read contiguous rows; the columns of H, and
  // then the rows of the product, are independent and spread over threads
  Mat Ht(n, n);
  parallel_for(n, [&](int j) {
    double *hj = &Ht.a[(size_t)j * n];
    hj[j] = 1.0 / A(j, j);
    for (int i = j + 1; i < n; ++i) {
      const double *gi = &A.a[(size_t)i * n];
      double t = 0.0;
      for (int k = j; k < i; ++k) t -= gi[k] * hj[k];
      hj[i] = t / gi[i];
    }
  });
  // A^{-1}(i, j) = sum_k H(k, i) H(k, j), k >= max(i, j)
  parallel_for(n, [&](int i) {
    const double *hi = &Ht.a[(size_t)i * n];
    for (int j = 0; j <= i; ++j) {
      const double *hj = &Ht.a[(size_t)j * n];
      double t = 0.0;
      for (int k = i; k < n; ++k) t += hi[k] * hj[k];
      A(i, j) = t;
    }
  });
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A(j, i) = A(i, j);
  return true;
}

// phi^ for odd kappa: normalised integral of (1 - t^2)^q, q = (kappa-1)/2,
// written out with the binomial expansion; reproduces the polynomials of
// Table 1 for kappa = 1, 3, 5, 7.
static double phi_hat(int kappa, double x) {
  const int q = (kappa - 1) / 2;
  double num = 0.0, den = 0.0, binom = 1.0;
  for (int k = 0; k <= q; ++k) {
    if (k > 0) binom = binom * (q - k + 1) / k;
    double c = binom * ((k % 2) ? -1.0 : 1.0) / (2.0 * k + 1.0);
    num += c * std::pow(x, 2 * k + 1);
    den += c;
  }
  return num / den;
}

double shape_phi(int kappa, double x) {
  double sgn = (x > 0) - (x < 0);
  if (kappa == -1) return sgn;
  if (std::fabs(x) > 1.0) return sgn;
  return phi_hat(kappa, x);
}

double weight_fn(int kappa, double xi, double dl, double dr, bool sat_l, bool sat_r) {
  double left = sat_l ? 1.0 : shape_phi(kappa, (xi + 1.0) / dl);
  double right = sat_r ? -1.0 : shape_phi(kappa, (xi - 1.0) / dr);
  return 0.5 * (left - right);
}

}  // namespace sem
