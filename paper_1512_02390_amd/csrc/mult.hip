// Multiplicative Schwarz method (Section 3.1, Algorithm 1) for the Poisson
// operator: the extended-element subproblems are solved one after the
// other, each on the residual left by all corrections before it, without
// weights; odd sweeps visit the elements in row-major order e = ey nx + ex,
// even sweeps in reverse (the symmetrised form).
//
// The method is sequential over subdomains, and any parallel ordering (a
// colouring) would be a different smoother, so one workgroup walks the
// subdomains in the paper's order.  Per subdomain:
//   1. r_s = R_s (f - A u) on the window, node by node from the assembled
//      1-D operators: (A u)(row, col) = M_y(row) (L_x u_row)(col) +
//      M_x(col) (L_y u_col)(row), each 1-D product summed over the (one or
//      two) elements that contain the node;
//   2. du_s = A_ss^{-1} r_s by fast diagonalisation with the unweighted
//      factors of the subdomain's type pair: four m x m products in LDS;
//   3. u += R_s^T du_s.
// Every thread of the workgroup sees the previous subdomain's update after
// the barrier that ends it (one compute unit, one L1).
#include "common.h"
#include "kernels.h"

#include <stdexcept>

namespace sem {
namespace {

constexpr int kMultThreads = 256;

// (L_1d v)(node c) along one direction of the level: sum over the elements
// that contain node c of s_E * Lhat row (local index of c in E) . v(E nodes).
// v(k) reads node k of that direction (wrapped when periodic).
template <typename V>
__device__ __forceinline__ double op1d(int c, int p, int ne, int N, int per, const double *Lhat,
                                       const double *s, V v) {
  double acc = 0.0;
  const int e = c / p, a = c - e * p;
  // element e with local index a (for a == 0 also the element on the left,
  // local index p); the last node of a Dirichlet line belongs to e - 1 only
  for (int side = 0; side < 2; ++side) {
    int E, al;
    if (side == 0) {
      E = e;
      al = a;
      if (!per && E >= ne) continue;
    } else {
      if (a != 0) break;
      E = e - 1;
      al = p;
      if (E < 0) {
        if (!per) continue;
        E += ne;
      }
    }
    const double *row = Lhat + al * (p + 1);
    double t = 0.0;
    for (int b = 0; b <= p; ++b) {
      int k = E * p + b;
      if (per && k >= N) k -= N;
      t = fma(row[b], v(k), t);
    }
    acc = fma(s[E], t, acc);
  }
  return acc;
}

// Lumped mass of node c along one direction: sum over its elements of h/2 w.
__device__ __forceinline__ double mass1d(int c, int p, int ne, int per, const double *w,
                                         const double *mh) {
  const int e = c / p, a = c - e * p;
  double m = 0.0;
  if (per || e < ne) m += mh[per ? e % ne : e] * w[a];
  if (a == 0) {
    int E = e - 1;
    if (E < 0 && per) E += ne;
    if (E >= 0) m += mh[E] * w[p];
  }
  return m;
}

__global__ __launch_bounds__(kMultThreads) void k_mult(MultArgs A) {
  extern __shared__ double sm[];
  const int m = A.m, mm = m * m;
  double *R = sm;        // m x m
  double *T = sm + mm;   // m x m
  const Grid g = A.g;
  const int per = g.periodic, p = g.p;
  const int tid = threadIdx.x;
  const long ne = (long)g.nx * g.ny;
  for (int it = 1; it <= A.n_it; ++it) {
    const bool fwd = it % 2 == 1;
    for (long q = 0; q < ne; ++q) {
      const long e = fwd ? q : ne - 1 - q;
      const int ey = (int)(e / g.nx), ex = (int)(e - (long)ey * g.nx);
      const int row0 = ey * p - A.n_o, col0 = ex * p - A.n_o;
      const int ty = A.ty_of[ey], tx = A.tx_of[ex];
      // 1. residual on the window
      for (int t = tid; t < mm; t += kMultThreads) {
        const int i = t / m, j = t - (t / m) * m;
        int gr = row0 + i, gc = col0 + j;
        bool ok;
        if (per) {
          gr = wrap(gr, g.rows);
          gc = wrap(gc, g.cols);
          ok = true;
        } else {
          ok = gr >= 1 && gr <= g.rows - 2 && gc >= 1 && gc <= g.cols - 2;
        }
        double r = 0.0;
        if (ok) {
          const double *urow = A.u + (long)gr * g.cols;
          const double xpart = op1d(gc, p, g.nx, g.cols, per, A.Lhat, A.sx,
                                    [&](int k) { return urow[k]; });
          const double ypart = op1d(gr, p, g.ny, g.rows, per, A.Lhat, A.sy,
                                    [&](int k) { return A.u[(long)k * g.cols + gc]; });
          const double au = mass1d(gr, p, g.ny, per, A.w, A.my) * xpart +
                            mass1d(gc, p, g.nx, per, A.w, A.mx) * ypart;
          r = A.f[(long)gr * g.cols + gc] - au;
        }
        R[t] = r;
      }
      __syncthreads();
      // 2. du = S_y [ D .* (S_y^T R S_x) ] S_x^T (unweighted factors)
      const double *SyT = A.SyT + (long)ty * mm, *Sy = A.Sy + (long)ty * mm;
      const double *Sx = A.Sx + (long)tx * mm, *SxT = A.SxT + (long)tx * mm;
      const double *D = A.dinv + ((long)ty * A.ntx + tx) * mm;
      for (int t = tid; t < mm; t += kMultThreads) {   // T = S_y^T R
        const int i = t / m, j = t - (t / m) * m;
        double s = 0.0;
        for (int k = 0; k < m; ++k) s = fma(SyT[i * m + k], R[k * m + j], s);
        T[t] = s;
      }
      __syncthreads();
      for (int t = tid; t < mm; t += kMultThreads) {   // R = (T S_x) .* D
        const int i = t / m, j = t - (t / m) * m;
        double s = 0.0;
        for (int k = 0; k < m; ++k) s = fma(T[i * m + k], Sx[k * m + j], s);
        R[t] = s * D[t];
      }
      __syncthreads();
      for (int t = tid; t < mm; t += kMultThreads) {   // T = S_y R
        const int i = t / m, j = t - (t / m) * m;
        double s = 0.0;
        for (int k = 0; k < m; ++k) s = fma(Sy[i * m + k], R[k * m + j], s);
        T[t] = s;
      }
      __syncthreads();
      // 3. u += du on the window's unknowns (du = T S_x^T)
      for (int t = tid; t < mm; t += kMultThreads) {
        const int i = t / m, j = t - (t / m) * m;
        int gr = row0 + i, gc = col0 + j;
        bool ok;
        if (per) {
          gr = wrap(gr, g.rows);
          gc = wrap(gc, g.cols);
          ok = true;
        } else {
          ok = gr >= 1 && gr <= g.rows - 2 && gc >= 1 && gc <= g.cols - 2;
        }
        if (ok) {
          double s = 0.0;
          for (int k = 0; k < m; ++k) s = fma(T[i * m + k], SxT[k * m + j], s);
          A.u[(long)gr * g.cols + gc] += s;
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

void launch_mult(const MultArgs &a, hipStream_t s) {
  if (a.n_it <= 0) return;
  if (a.m > kMaxTile) throw std::runtime_error("multiplicative Schwarz: tile wider than 48");
  const unsigned shm = 2u * a.m * a.m * sizeof(double);
  klaunch(k_mult, dim3(1), dim3(kMultThreads), shm, s, a);
}

}  // namespace sem
