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

// r = f - A u (f null: r = A u) by elements.  The assembled operator is the
// sum of the element operators, each the tensor product of 1-D element
// matrices (the 1-D assembly sums factor element by element):
//   A_e u_e = M_z M_y (s_x Lhat) u + M_z (s_y Lhat) M_x u + (s_z Lhat) M_y M_x u
// on the element's (p+1)^3 nodes, with the element masses (h/2) w.
// k3_res_init sets r = f on the unknowns (0 elsewhere); k3_res_elem stages an
// element's u in LDS and subtracts A_e u_e with atomics (adds it when f is
// null; elements that share a node add in any order).  Lane (j, i) of the element's (p+1)^2 pencils
// keeps its x and y operator rows and its z pencil in registers and walks the
// pencil's layers: the x and y sums read LDS, the z sum uses the layer's
// operator row (one row for the whole wavefront).
__global__ void k3_res_init(Res3Args A) {
  const long n = (long)A.NX * A.NY * A.NZ;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = (int)(t % A.NX);
  const int j = (int)((t / A.NX) % A.NY);
  const int k = (int)(t / ((long)A.NX * A.NY));
  const bool in = i > 0 && j > 0 && k > 0 && i < A.NX - 1 && j < A.NY - 1 && k < A.NZ - 1;
  A.r[t] = (in && A.f) ? A.f[t] : 0.0;
}

template <int P>
constexpr int res3_threads() { return (P + 1) * (P + 1) <= 64 ? 64 : (P + 1) * (P + 1) <= 128 ? 128 : 256; }

template <int P>
__global__ __launch_bounds__(res3_threads<P>()) void k3_res_elem(Res3Args A) {
  constexpr int N = P + 1, NN = N * N;
  __shared__ double U[N * NN];
  const long e = blockIdx.x;
  const int ex = (int)(e % A.nx), ey = (int)((e / A.nx) % A.ny), ez = (int)(e / ((long)A.nx * A.ny));
  const int i0 = ex * P, j0 = ey * P, k0 = ez * P;
  for (int q = threadIdx.x; q < N * NN; q += blockDim.x) {
    const int kk = q / NN, jj = (q / N) % N, ii = q % N;
    const int gi = i0 + ii, gj = j0 + jj, gk = k0 + kk;
    const bool in = gi > 0 && gj > 0 && gk > 0 && gi < A.NX - 1 && gj < A.NY - 1 && gk < A.NZ - 1;
    U[q] = in ? A.u[((long)gk * A.NY + gj) * A.NX + gi] : 0.0;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= NN) return;   // no barrier below
  const int jj = t / N, ii = t - (t / N) * N;
  const int gi = i0 + ii, gj = j0 + jj;
  const bool in_ji = gi > 0 && gj > 0 && gi < A.NX - 1 && gj < A.NY - 1;
  double lx[N], ly[N], pz[N];
#pragma unroll
  for (int b = 0; b < N; ++b) {
    lx[b] = A.Lhat[ii * N + b];
    ly[b] = A.Lhat[jj * N + b];
    pz[b] = U[(b * N + jj) * N + ii];
  }
  const double sx = A.sx[ex], sy = A.sy[ey], sz = A.sz[ez];
  const double mxi = A.mx[ex] * A.w[ii], myj = A.my[ey] * A.w[jj], mz = A.mz[ez];
  const cptr<double> Lc = as_const(A.Lhat);
#pragma unroll
  for (int kk = 0; kk < N; ++kk) {
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      ax = fma(lx[b], U[(kk * N + jj) * N + b], ax);
      ay = fma(ly[b], U[(kk * N + b) * N + ii], ay);
      az = fma(Lc[kk * N + b], pz[b], az);
    }
    const double mzk = mz * A.w[kk];
    const double v = mzk * myj * sx * ax + mzk * mxi * sy * ay + myj * mxi * sz * az;
    const int gk = k0 + kk;
    if (in_ji && gk > 0 && gk < A.NZ - 1)
      atomic_add(&A.r[((long)gk * A.NY + gj) * A.NX + gi], A.f ? -v : v);
  }
}

// Weighted additive Schwarz correction (Algorithm 2 in 3-D): one workgroup
// of two wavefronts per subdomain, the fast diagonalisation
//   du = (S_z (x) S_y (x) S_x) [ (S_z (x) S_y (x) S_x)^T R / (l_z + l_y + l_x) ]
// as six one-axis transforms of the m^3 tile.  In each transform a lane owns
// one pencil along the axis (m^2 pencils): it reads the pencil's m values
// from LDS into registers and forms the m outputs as dot products with the
// rows of the factor, which every lane of the wavefront reads at the same
// time (scalar loads of the subdomain type's matrix).  The divide by the
// eigenvalue sum is fused into the third transform, and the weighted result
// w_z w_y w_x du of the sixth goes straight to u with atomics (overlapping
// subdomains).
constexpr int kFdm3Threads = 128;

template <int M>
__device__ __forceinline__ double pdot(cptr<double> row, const double (&v)[M]) {
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int i = 0; i + 1 < M; i += 2) {
    a0 = fma(row[i], v[i], a0);
    a1 = fma(row[i + 1], v[i + 1], a1);
  }
  if constexpr (M % 2) a0 = fma(row[M - 1], v[M - 1], a0);
  return a0 + a1;
}

// Element offset of tile position (k, j, i) and the pencil of lane t along
// axis (0 x, 1 y, 2 z): base offset and stride.
template <int M>
__device__ __forceinline__ void pencil(int t, int axis, int &base, int &stride, int &p0, int &p1) {
  const int hi = t / M, lo = t - (t / M) * M;
  if (axis == 0) {          // pencil (k, j), along i
    base = (hi * M + lo) * M;
    stride = 1;
  } else if (axis == 1) {   // pencil (k, i), along j
    base = hi * M * M + lo;
    stride = M;
  } else {                  // pencil (j, i), along k
    base = hi * M + lo;
    stride = M * M;
  }
  p0 = hi;
  p1 = lo;
}

template <int M>
__global__ __launch_bounds__(kFdm3Threads) void k3_fdm(Fdm3Args A) {
  constexpr int MM = M * M, MMM = MM * M;
  __shared__ double X[MMM], Y[MMM];
  const long s = blockIdx.x;
  const int ex = (int)(s % A.nx), ey = (int)((s / A.nx) % A.ny), ez = (int)(s / ((long)A.nx * A.ny));
  const int tx = A.tx_of[ex], ty = A.ty_of[ey], tz = A.tz_of[ez];
  const int i0 = ex * A.p - A.n_o, j0 = ey * A.p - A.n_o, k0 = ez * A.p - A.n_o;
  const int t = threadIdx.x;
  // gather (positions that are not unknowns read zero)
  for (int q = t; q < MMM; q += kFdm3Threads) {
    const int k = q / MM, j = (q / M) % M, i = q % M;
    const int gi = i0 + i, gj = j0 + j, gk = k0 + k;
    const bool ok = gi >= 1 && gi <= A.NX - 2 && gj >= 1 && gj <= A.NY - 2 && gk >= 1 &&
                    gk <= A.NZ - 2;
    X[q] = ok ? A.r[((long)gk * A.NY + gj) * A.NX + gi] : 0.0;
  }
  __syncthreads();
  // one transform: out(pencil, o) = post(sum_a F(o, a) in(pencil, a)); the
  // m^2 pencils over the block's lanes (more than one per lane from m = 12)
  auto transform = [&](const double *in, double *out, const double *F, int axis, auto post) {
    const cptr<double> Fc = as_const(F);
    for (int q = t; q < MM; q += kFdm3Threads) {
      int base, stride, p0, p1;
      pencil<M>(q, axis, base, stride, p0, p1);
      double v[M];
#pragma unroll
      for (int a = 0; a < M; ++a) v[a] = in[base + a * stride];
#pragma unroll 1
      for (int o = 0; o < M; ++o) post(base + o * stride, p0, p1, o, pdot<M>(Fc + o * M, v));
    }
    __syncthreads();
  };
  const long t2 = (long)MM;
  auto store = [](double *dst) {
    return [dst](int at, int, int, int, double v) { dst[at] = v; };
  };
  transform(X, Y, A.SxT + tx * t2, 0, store(Y));   // S_x^T along x
  transform(Y, X, A.SyT + ty * t2, 1, store(X));   // S_y^T along y
  const double *lx = A.lx + (long)tx * M, *ly = A.ly + (long)ty * M, *lz = A.lz + (long)tz * M;
  transform(X, Y, A.SzT + tz * t2, 2, [&](int at, int j, int i, int k, double v) {
    Y[at] = v / (lz[k] + ly[j] + lx[i]);           // S_z^T along z, / eigenvalue sum
  });
  transform(Y, X, A.Sx + tx * t2, 0, store(X));    // S_x along x
  transform(X, Y, A.Sy + ty * t2, 1, store(Y));    // S_y along y
  const double *wx = A.wx + (long)ex * M, *wy = A.wy + (long)ey * M, *wz = A.wz + (long)ez * M;
  transform(Y, X, A.Sz + tz * t2, 2, [&](int, int j, int i, int k, double v) {
    const int gi = i0 + i, gj = j0 + j, gk = k0 + k;   // S_z along z, weighted, into u
    if (gi >= 1 && gi <= A.NX - 2 && gj >= 1 && gj <= A.NY - 2 && gk >= 1 && gk <= A.NZ - 2)
      atomic_add(&A.u[((long)gk * A.NY + gj) * A.NX + gi], wz[k] * wy[j] * wx[i] * v);
  });
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

// Restriction f_c = I^T r_f by elements (Transfer3Args): the element's
// pf^3 fine nodes go to LDS and are contracted with E along x, y, z (three
// passes through LDS, one output per thread and step); the (pc+1)^3 results
// are added into f_c with atomics (coarse nodes on element faces are shared).
// A fine node on a face contributes only to the coarse nodes on that face
// (the coarse basis vanishes there otherwise), which the element holds too.
template <int PF>
__global__ __launch_bounds__(256) void k3_restrict(Transfer3Args A) {
  constexpr int PC = (PF + 1) / 2, NC = PC + 1;
  __shared__ double R[PF * PF * PF], T1[PF * PF * NC], T2[PF * NC * NC];
  __shared__ double E[(PF + 1) * NC];
  const long e = blockIdx.x;
  const int ex = (int)(e % A.nx), ey = (int)((e / A.nx) % A.ny), ez = (int)(e / ((long)A.nx * A.ny));
  const int t = threadIdx.x;
  for (int q = t; q < (PF + 1) * NC; q += blockDim.x) E[q] = A.E[q];
  for (int q = t; q < PF * PF * PF; q += blockDim.x) {
    const int a = q / (PF * PF), b = (q / PF) % PF, c = q % PF;
    R[q] = A.in[((long)(ez * PF + a) * A.NY + ey * PF + b) * A.NX + ex * PF + c];
  }
  __syncthreads();
  for (int q = t; q < PF * PF * NC; q += blockDim.x) {   // along x
    const int ab = q / NC, cx = q % NC;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < PF; ++c) s = fma(E[c * NC + cx], R[ab * PF + c], s);
    T1[q] = s;
  }
  __syncthreads();
  for (int q = t; q < PF * NC * NC; q += blockDim.x) {   // along y
    const int a = q / (NC * NC), cy = (q / NC) % NC, cx = q % NC;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < PF; ++b) s = fma(E[b * NC + cy], T1[(a * PF + b) * NC + cx], s);
    T2[q] = s;
  }
  __syncthreads();
  for (int q = t; q < NC * NC * NC; q += blockDim.x) {   // along z, into f_c
    const int cz = q / (NC * NC), cy = (q / NC) % NC, cx = q % NC;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < PF; ++a) s = fma(E[a * NC + cz], T2[(a * NC + cy) * NC + cx], s);
    const int gx = ex * PC + cx, gy = ey * PC + cy, gz = ez * PC + cz;
    if (gx > 0 && gy > 0 && gz > 0 && gx < A.CX - 1 && gy < A.CY - 1 && gz < A.CZ - 1)
      atomic_add(&A.out[((long)gz * A.CY + gy) * A.CX + gx], s);
  }
}

// Prolongation u_f += I u_c by elements: the element's (pc+1)^3 coarse
// values go to LDS and are interpolated along z, y, x onto the pf^3 fine
// nodes the element holds, each written by exactly one element (no atomics).
template <int PF>
__global__ __launch_bounds__(256) void k3_prolong(Transfer3Args A) {
  constexpr int PC = (PF + 1) / 2, NC = PC + 1;
  __shared__ double UC[NC * NC * NC], T1[PF * NC * NC], T2[PF * PF * NC];
  __shared__ double E[(PF + 1) * NC];
  const long e = blockIdx.x;
  const int ex = (int)(e % A.nx), ey = (int)((e / A.nx) % A.ny), ez = (int)(e / ((long)A.nx * A.ny));
  const int t = threadIdx.x;
  for (int q = t; q < (PF + 1) * NC; q += blockDim.x) E[q] = A.E[q];
  for (int q = t; q < NC * NC * NC; q += blockDim.x) {
    const int cz = q / (NC * NC), cy = (q / NC) % NC, cx = q % NC;
    UC[q] = A.in[((long)(ez * PC + cz) * A.CY + ey * PC + cy) * A.CX + ex * PC + cx];
  }
  __syncthreads();
  for (int q = t; q < PF * NC * NC; q += blockDim.x) {   // along z
    const int a = q / (NC * NC), r = q % (NC * NC);
    double s = 0.0;
#pragma unroll
    for (int cz = 0; cz < NC; ++cz) s = fma(E[a * NC + cz], UC[cz * NC * NC + r], s);
    T1[q] = s;
  }
  __syncthreads();
  for (int q = t; q < PF * PF * NC; q += blockDim.x) {   // along y
    const int a = q / (PF * NC), b = (q / NC) % PF, cx = q % NC;
    double s = 0.0;
#pragma unroll
    for (int cy = 0; cy < NC; ++cy) s = fma(E[b * NC + cy], T1[(a * NC + cy) * NC + cx], s);
    T2[q] = s;
  }
  __syncthreads();
  for (int q = t; q < PF * PF * PF; q += blockDim.x) {   // along x, into u_f
    const int a = q / (PF * PF), b = (q / PF) % PF, c = q % PF;
    double s = 0.0;
#pragma unroll
    for (int cx = 0; cx < NC; ++cx) s = fma(E[c * NC + cx], T2[(a * PF + b) * NC + cx], s);
    const int gx = ex * PF + c, gy = ey * PF + b, gz = ez * PF + a;
    if (gx > 0 && gy > 0 && gz > 0) {
      const long node = ((long)gz * A.NY + gy) * A.NX + gx;
      A.out[node] += s;
    }
  }
}

// Coarse fast diagonalisation in one workgroup (Coarse3Args): the unknowns of
// f0 go to LDS, then three forward transforms S^T along x, y, z (the third
// divides by l_z + l_y + l_x), and three backward transforms S along x, y, z,
// the last one writing u0.  One output per thread and step, operands in LDS.
__global__ __launch_bounds__(1024) void k3_coarse(Coarse3Args A) {
  constexpr int C3 = kCoarse3Max * kCoarse3Max * kCoarse3Max;
  __shared__ double X[C3], Y[C3];
  __shared__ double S[3][kCoarse3Max * kCoarse3Max], lam[3][kCoarse3Max];
  const int nx = A.nu[0], ny = A.nu[1], nz = A.nu[2];
  const int NX = A.N[0], NY = A.N[1], NZ = A.N[2];
  const int n = nx * ny * nz, t = threadIdx.x, nt = blockDim.x;
  for (int d = 0; d < 3; ++d) {
    const int m = A.nu[d];
    for (int q = t; q < m * m; q += nt) S[d][q] = A.S[d][q];
    for (int q = t; q < m; q += nt) lam[d][q] = A.lam[d][q];
  }
  for (int q = t; q < n; q += nt) {
    const int i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
    X[q] = A.f0[((long)(k + 1) * NY + (j + 1)) * NX + (i + 1)];
  }
  __syncthreads();
  // out(k, j, i) = sum_a F(a, idx) in(.. a ..) (forward, F = S^T) or
  // sum_a F(idx, a) in(.. a ..) (backward, F = S), idx the output's index along axis
  auto step = [&](const double *in, double *out, int axis, bool fwd, bool divide) {
    const int m = A.nu[axis];
    const double *F = S[axis];
    for (int q = t; q < n; q += nt) {
      const int i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
      const int idx = axis == 0 ? i : axis == 1 ? j : k;
      const int stride = axis == 0 ? 1 : axis == 1 ? nx : nx * ny;
      const int base = q - idx * stride;
      double s = 0.0;
      for (int a = 0; a < m; ++a)
        s = fma(fwd ? F[a * m + idx] : F[idx * m + a], in[base + a * stride], s);
      if (divide) s /= lam[2][k] + lam[1][j] + lam[0][i];
      out[q] = s;
    }
    __syncthreads();
  };
  step(X, Y, 0, true, false);
  step(Y, X, 1, true, false);
  step(X, Y, 2, true, true);
  step(Y, X, 0, false, false);
  step(X, Y, 1, false, false);
  step(Y, X, 2, false, false);
  const long N3 = (long)NX * NY * NZ;
  for (long q = t; q < N3; q += nt) {
    const int i = (int)(q % NX), j = (int)((q / NX) % NY), k = (int)(q / ((long)NX * NY));
    const bool in = i > 0 && j > 0 && k > 0 && i < NX - 1 && j < NY - 1 && k < NZ - 1;
    A.u0[q] = in ? X[((k - 1) * ny + (j - 1)) * nx + (i - 1)] : 0.0;
  }
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
  if (a.p < 1 || a.p > kMaxTile3 - 1) throw std::runtime_error("3-D residual: order not in [1, 14]");
  klaunch(k3_res_init, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
  const unsigned ne = (unsigned)((long)a.nx * a.ny * a.nz);
  switch (a.p) {
#define SEM3_RCASE(P) \
  case P:             \
    klaunch(k3_res_elem<P>, dim3(ne), dim3(res3_threads<P>()), 0, s, a); \
    break;
    SEM3_RCASE(1) SEM3_RCASE(2) SEM3_RCASE(3) SEM3_RCASE(4) SEM3_RCASE(5) SEM3_RCASE(6)
    SEM3_RCASE(7) SEM3_RCASE(8) SEM3_RCASE(9) SEM3_RCASE(10) SEM3_RCASE(11) SEM3_RCASE(12)
    SEM3_RCASE(13) SEM3_RCASE(14)
#undef SEM3_RCASE
    default:
      break;
  }
}

void launch3_fdm(const Fdm3Args &a, hipStream_t s) {
  if (a.m > kMaxTile3 || a.m < 2) throw std::runtime_error("3-D Schwarz kernel: tile width not in [2, 15]");
  const long ns = (long)a.nx * a.ny * a.nz;
  if (ns <= 0) return;
  switch (a.m) {
#define SEM3_CASE(M) \
  case M:            \
    klaunch(k3_fdm<M>, dim3((unsigned)ns), dim3(kFdm3Threads), 0, s, a); \
    break;
    SEM3_CASE(2) SEM3_CASE(3) SEM3_CASE(4) SEM3_CASE(5) SEM3_CASE(6) SEM3_CASE(7) SEM3_CASE(8)
    SEM3_CASE(9) SEM3_CASE(10) SEM3_CASE(11) SEM3_CASE(12) SEM3_CASE(13) SEM3_CASE(14)
    SEM3_CASE(15)
#undef SEM3_CASE
    default:
      break;
  }
}

void launch3_axis(const Axis3Args &a, hipStream_t s) {
  const long n = (long)a.d0 * a.d1 * a.d2;
  if (n <= 0) return;   // an empty axis (no coarse unknowns)
  klaunch(k3_axis, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
}

void launch3_coarse(const Coarse3Args &a, hipStream_t s) {
  for (int d = 0; d < 3; ++d)
    if (a.nu[d] < 1 || a.nu[d] > kCoarse3Max)
      throw std::runtime_error("3-D coarse solve: unknowns per direction not in [1, 18]");
  klaunch(k3_coarse, dim3(1), dim3(1024), 0, s, a);
}

void launch3_restrict(const Transfer3Args &a, hipStream_t s) {
  const unsigned ne = (unsigned)((long)a.nx * a.ny * a.nz);
  if (ne == 0) return;
  switch (a.pf) {
#define SEM3_TCASE(P) \
  case P:             \
    klaunch(k3_restrict<P>, dim3(ne), dim3(256), 0, s, a); \
    break;
    SEM3_TCASE(2) SEM3_TCASE(3) SEM3_TCASE(4) SEM3_TCASE(5) SEM3_TCASE(6) SEM3_TCASE(7)
    SEM3_TCASE(8) SEM3_TCASE(9) SEM3_TCASE(10) SEM3_TCASE(11) SEM3_TCASE(12) SEM3_TCASE(13)
    SEM3_TCASE(14)
#undef SEM3_TCASE
    default:
      throw std::runtime_error("3-D restriction: fine order not in [2, 14]");
  }
}

void launch3_prolong(const Transfer3Args &a, hipStream_t s) {
  const unsigned ne = (unsigned)((long)a.nx * a.ny * a.nz);
  if (ne == 0) return;
  switch (a.pf) {
#define SEM3_TCASE(P) \
  case P:             \
    klaunch(k3_prolong<P>, dim3(ne), dim3(256), 0, s, a); \
    break;
    SEM3_TCASE(2) SEM3_TCASE(3) SEM3_TCASE(4) SEM3_TCASE(5) SEM3_TCASE(6) SEM3_TCASE(7)
    SEM3_TCASE(8) SEM3_TCASE(9) SEM3_TCASE(10) SEM3_TCASE(11) SEM3_TCASE(12) SEM3_TCASE(13)
    SEM3_TCASE(14)
#undef SEM3_TCASE
    default:
      throw std::runtime_error("3-D prolongation: fine order not in [2, 14]");
  }
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
