// Host-side numerics for the set-up phase: GLL rules, Lagrange operators,
// symmetric eigen-solver, dense Cholesky, and the paper's weight function.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace sem {

using Vec = std::vector<double>;

// Dense row-major square/rectangular matrix.
struct Mat {
  int r = 0, c = 0;
  Vec a;
  Mat() = default;
  Mat(int rows, int cols) : r(rows), c(cols), a((size_t)rows * cols, 0.0) {}
  double &operator()(int i, int j) { return a[(size_t)i * c + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

// GLL points and weights of order p (p+1 points on [-1, 1]).
void gll_rule(int p, Vec &xi, Vec &w);
// D(i, j) = derivative of the j-th Lagrange polynomial through xi at xi_i.
Mat lagrange_derivative(const Vec &xi);
// E(q, j) = j-th Lagrange polynomial through xi evaluated at x_q.
Mat lagrange_eval(const Vec &xi, const Vec &x);
// Reference stiffness D^T W D.
Mat ref_stiffness(int p);

// Symmetric eigen-decomposition A = Q diag(lam) Q^T by cyclic Jacobi
// rotations; Q stored column-wise (Q(i, k) = component i of vector k),
// eigenvalues ascending.
void sym_eig(const Mat &A, Vec &lam, Mat &Q);
// Generalised problem L s = lam M s, M diagonal positive, S^T M S = I.
void gen_eig_diag(const Mat &L, const Vec &Mdiag, Vec &lam, Mat &S);

// In-place inverse of a symmetric positive definite matrix (Cholesky).
bool spd_inverse(Mat &A);

// Shape function phi_kappa on the real line (odd kappa, or -1 top hat).
double shape_phi(int kappa, double x);
// w = 1/2 [phi((xi+1)/dl) - phi((xi-1)/dr)], saturated sides held at +1/-1.
double weight_fn(int kappa, double xi, double dl, double dr, bool sat_l, bool sat_r);

}  // namespace sem
