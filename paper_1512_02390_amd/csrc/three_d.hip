// Kernels of the 3-D Poisson extension (Section 5 names three dimensions as
// the method's next step): the tensor-product operator in three directions,
// the weighted additive Schwarz step with 3-D fast diagonalisation, and the
// one-axis transforms that carry the transfers and the coarse solve.
// Node arrays are u[z][y][x] (x fastest), Dirichlet boundary nodes kept and
// zero.  FP64.
#include "common.h"
#include "kernels3.h"

#include <stdexcept>

namespace sem {
namespace {

// (L_1d v)(c) along one direction: sum over the (one or two) elements that
// contain node c of (2/h_E) Lhat row (local index of c in E) . v(E's nodes);
// v(k) reads node k.  Dirichlet lines: node n p belongs to element n-1 only.
template <typename V>
__device__ __forceinline__ double line_op(int c, int p, int ne, const double *Lhat, const double *s,
                                          V v) {
  const int e = c / p, a = c - e * p;
  double acc = 0.0;
  if (e < ne) {
    const double *row = Lhat + a * (p + 1);
    double t = 0.0;
    for (int b = 0; b <= p; ++b) t = fma(row[b], v(e * p + b), t);
    acc = s[e] * t;
  }
  if (a == 0 && e > 0) {
    const double *row = Lhat + p * (p + 1);
    double t = 0.0;
    for (int b = 0; b <= p; ++b) t = fma(row[b], v((e - 1) * p + b), t);
    acc = fma(s[e - 1], t, acc);
  }
  return acc;
}

// Lumped 1-D mass of node c: sum over its elements of (h/2) w.
__device__ __forceinline__ double line_mass(int c, int p, int ne, const double *w, const double *mh) {
  const int e = c / p, a = c - e * p;
  double m = e < ne ? mh[e] * w[a] : 0.0;
  if (a == 0 && e > 0) m += mh[e - 1] * w[p];
  return m;
}

// r = f - A u (f null: r = A u), one thread per node:
//   (A u)(k, j, i) = m_z m_y (L_x u) + m_z m_x (L_y u) + m_y m_x (L_z u).
__global__ void k3_residual(Res3Args A) {
  const long n = (long)A.NX * A.NY * A.NZ;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = (int)(t % A.NX);
  const int j = (int)((t / A.NX) % A.NY);
  const int k = (int)(t / ((long)A.NX * A.NY));
  if (i == 0 || j == 0 || k == 0 || i == A.NX - 1 || j == A.NY - 1 || k == A.NZ - 1) {
    A.r[t] = 0.0;
    return;
  }
  const long sy = A.NX, sz = (long)A.NX * A.NY;
  const double *u = A.u;
  const long base = t;
  const double lx = line_op(i, A.p, A.nx, A.Lhat, A.sx, [&](int b) { return u[base - i + b]; });
  const double ly = line_op(j, A.p, A.ny, A.Lhat, A.sy,
                            [&](int b) { return u[base + (long)(b - j) * sy]; });
  const double lz = line_op(k, A.p, A.nz, A.Lhat, A.sz,
                            [&](int b) { return u[base + (long)(b - k) * sz]; });
  const double mx = line_mass(i, A.p, A.nx, A.w, A.mx);
  const double my = line_mass(j, A.p, A.ny, A.w, A.my);
  const double mz = line_mass(k, A.p, A.nz, A.w, A.mz);
  const double au = mz * my * lx + mz * mx * ly + my * mx * lz;
  A.r[t] = A.f ? A.f[t] - au : au;
}

// Weighted additive Schwarz correction (Algorithm 2 in 3-D): one workgroup
// per subdomain.  The m^3 tile of r goes to LDS, the six 1-D transforms of
// the fast diagonalisation
//   du = (S_z (x) S_y (x) S_x) [ (S_z (x) S_y (x) S_x)^T R / (l_z + l_y + l_x) ]
// run along x, y, z with the subdomain type's factors, and the weighted
// result w_z w_y w_x du is added into u (atomics: overlapping subdomains).
constexpr int kFdm3Threads = 256;

// out(k, j, i) = sum_a M(idx, a) in(... a along axis ...), M row-major m x m,
// where idx is the output's index along the axis.
__device__ __forceinline__ void axis_apply(const double *__restrict__ in, double *__restrict__ out,
                                           const double *__restrict__ M, int m, int axis) {
  const int mm = m * m, mmm = mm * m;
  for (int t = threadIdx.x; t < mmm; t += kFdm3Threads) {
    const int k = t / mm, j = (t / m) % m, i = t % m;
    const int idx = axis == 0 ? i : axis == 1 ? j : k;
    const int stride = axis == 0 ? 1 : axis == 1 ? m : mm;
    const int base = t - idx * stride;
    const double *row = M + idx * m;
    double s = 0.0;
    for (int a = 0; a < m; ++a) s = fma(row[a], in[base + a * stride], s);
    out[t] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kFdm3Threads) void k3_fdm(Fdm3Args A) {
  extern __shared__ double sm3[];
  const int m = A.m, mm = m * m, mmm = mm * m;
  double *X = sm3, *Y = sm3 + mmm;
  const long s = blockIdx.x;
  const int ex = (int)(s % A.nx), ey = (int)((s / A.nx) % A.ny), ez = (int)(s / ((long)A.nx * A.ny));
  const int tx = A.tx_of[ex], ty = A.ty_of[ey], tz = A.tz_of[ez];
  const int i0 = ex * A.p - A.n_o, j0 = ey * A.p - A.n_o, k0 = ez * A.p - A.n_o;
  // gather (positions that are not unknowns read zero)
  for (int t = threadIdx.x; t < mmm; t += kFdm3Threads) {
    const int k = t / mm, j = (t / m) % m, i = t % m;
    const int gi = i0 + i, gj = j0 + j, gk = k0 + k;
    const bool ok = gi >= 1 && gi <= A.NX - 2 && gj >= 1 && gj <= A.NY - 2 && gk >= 1 &&
                    gk <= A.NZ - 2;
    X[t] = ok ? A.r[((long)gk * A.NY + gj) * A.NX + gi] : 0.0;
  }
  __syncthreads();
  const long t2 = (long)m * m;
  axis_apply(X, Y, A.SxT + tx * t2, m, 0);   // S_x^T along x
  axis_apply(Y, X, A.SyT + ty * t2, m, 1);   // S_y^T along y
  axis_apply(X, Y, A.SzT + tz * t2, m, 2);   // S_z^T along z
  const double *lx = A.lx + (long)tx * m, *ly = A.ly + (long)ty * m, *lz = A.lz + (long)tz * m;
  for (int t = threadIdx.x; t < mmm; t += kFdm3Threads) {
    const int k = t / mm, j = (t / m) % m, i = t % m;
    Y[t] /= lz[k] + ly[j] + lx[i];
  }
  __syncthreads();
  axis_apply(Y, X, A.Sx + tx * t2, m, 0);    // S_x along x
  axis_apply(X, Y, A.Sy + ty * t2, m, 1);    // S_y along y
  axis_apply(Y, X, A.Sz + tz * t2, m, 2);    // S_z along z
  const double *wx = A.wx + (long)ex * m, *wy = A.wy + (long)ey * m, *wz = A.wz + (long)ez * m;
  for (int t = threadIdx.x; t < mmm; t += kFdm3Threads) {
    const int k = t / mm, j = (t / m) % m, i = t % m;
    const int gi = i0 + i, gj = j0 + j, gk = k0 + k;
    const bool ok = gi >= 1 && gi <= A.NX - 2 && gj >= 1 && gj <= A.NY - 2 && gk >= 1 &&
                    gk <= A.NZ - 2;
    if (ok) atomic_add(&A.u[((long)gk * A.NY + gj) * A.NX + gi], wz[k] * wy[j] * wx[i] * X[t]);
  }
}

// out = (accumulate ? out : 0) + band-matrix product along one axis:
//   out[.. o ..] = sum_{t < cnt[o]} val[o * B + t] in[.. start[o] + t ..],
// dims of out (o0 slowest .. o2 fastest), axis 0 = z, 1 = y, 2 = x; in has
// the same dims except nin along the axis.  zero_bnd: the output's boundary
// nodes (first and last index along any axis of a node array) are set to 0.
__global__ void k3_axis(Axis3Args A) {
  const long n = (long)A.d0 * A.d1 * A.d2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int o2 = (int)(t % A.d2), o1 = (int)((t / A.d2) % A.d1), o0 = (int)(t / ((long)A.d1 * A.d2));
  const int o = A.axis == 0 ? o0 : A.axis == 1 ? o1 : o2;
  // strides of in
  const long in_d0 = A.axis == 0 ? A.nin : A.d0;
  const long in_d1 = A.axis == 1 ? A.nin : A.d1;
  const long in_d2 = A.axis == 2 ? A.nin : A.d2;
  (void)in_d0;
  const long s2 = 1, s1 = in_d2, s0 = in_d1 * in_d2;
  const long stride = A.axis == 0 ? s0 : A.axis == 1 ? s1 : s2;
  const long base = (A.axis == 0 ? 0 : (long)o0 * s0) + (A.axis == 1 ? 0 : (long)o1 * s1) +
                    (A.axis == 2 ? 0 : (long)o2 * s2);
  const int st = A.start[o], cn = A.cnt[o];
  const double *v = A.val + (long)o * A.B;
  double s = 0.0;
  for (int q = 0; q < cn; ++q) s = fma(v[q], A.in[base + (long)(st + q) * stride], s);
  if (A.zero_bnd && (o0 == 0 || o1 == 0 || o2 == 0 || o0 == A.d0 - 1 || o1 == A.d1 - 1 ||
                     o2 == A.d2 - 1))
    s = 0.0;
  A.out[t] = A.accumulate ? A.out[t] + s : s;
}

// x /= (l_z + l_y + l_x) on the coarse unknowns' grid (n0 x n1 x n2).
__global__ void k3_eig_divide(double *x, int n0, int n1, int n2, const double *lz, const double *ly,
                              const double *lx) {
  const long n = (long)n0 * n1 * n2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = (int)(t % n2), j = (int)((t / n2) % n1), k = (int)(t / ((long)n1 * n2));
  x[t] /= lz[k] + ly[j] + lx[i];
}

__global__ void k3_axpy(double *y, const double *x, double a, long n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = fma(a, x[t], y[t]);
}

// p = z + beta p
__global__ void k3_xpby(double *p, const double *z, double beta, long n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = fma(beta, p[t], z[t]);
}

inline unsigned blocks_for(long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch3_residual(const Res3Args &a, hipStream_t s) {
  const long n = (long)a.NX * a.NY * a.NZ;
  if (n <= 0) return;
  klaunch(k3_residual, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
}

void launch3_fdm(const Fdm3Args &a, hipStream_t s) {
  if (a.m > kMaxTile3) throw std::runtime_error("3-D Schwarz kernel: tile wider than 15");
  const long ns = (long)a.nx * a.ny * a.nz;
  if (ns <= 0) return;
  const unsigned shm = 2u * a.m * a.m * a.m * sizeof(double);
  klaunch(k3_fdm, dim3((unsigned)ns), dim3(kFdm3Threads), shm, s, a);
}

void launch3_axis(const Axis3Args &a, hipStream_t s) {
  const long n = (long)a.d0 * a.d1 * a.d2;
  if (n <= 0) return;   // an empty axis (no coarse unknowns)
  klaunch(k3_axis, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
}

void launch3_eig_divide(double *x, int n0, int n1, int n2, const double *lz, const double *ly,
                        const double *lx, hipStream_t s) {
  const long n = (long)n0 * n1 * n2;
  if (n <= 0) return;
  klaunch(k3_eig_divide, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n0, n1, n2, lz, ly, lx);
}

void launch3_axpy(double *y, const double *x, double a, long n, hipStream_t s) {
  if (n <= 0) return;
  klaunch(k3_axpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, y, x, a, n);
}

void launch3_xpby(double *p, const double *z, double beta, long n, hipStream_t s) {
  if (n <= 0) return;
  klaunch(k3_xpby, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, z, beta, n);
}

}  // namespace sem
