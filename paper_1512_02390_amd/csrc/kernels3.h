// Launch interface of the 3-D kernels (three_d.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sem {

constexpr int kMaxTile3 = 15;   // largest 3-D subdomain width (two m^3 FP64 tiles in LDS)

// r = f - A u on one level (f null: r = A u); node array NZ x NY x NX.
struct Res3Args {
  int32_t nx, ny, nz, p;          // elements per direction, order
  int32_t NX, NY, NZ;             // nodes per direction (n p + 1)
  const double *u, *f;
  double *r;
  const double *Lhat, *w;         // (p+1)^2 reference stiffness, GLL weights
  const double *sx, *sy, *sz;     // per element 2/h
  const double *mx, *my, *mz;     // per element h/2
};

// One Schwarz correction: every subdomain of the level, added into u.
struct Fdm3Args {
  int32_t nx, ny, nz, p, n_o, m;
  int32_t NX, NY, NZ;
  const double *r;
  double *u;
  const double *Sx, *SxT, *lx;    // per x type: S, S^T (m x m), eigenvalues (m)
  const double *Sy, *SyT, *ly;
  const double *Sz, *SzT, *lz;
  const int32_t *tx_of, *ty_of, *tz_of;   // type per element column / row / layer
  const double *wx, *wy, *wz;     // per element m weights
};

// Band-matrix product along one axis (see k3_axis).
struct Axis3Args {
  int32_t d0, d1, d2;             // output dims (z, y, x)
  int32_t axis;                   // 0 z, 1 y, 2 x
  int32_t nin;                    // input length along the axis
  const double *in;
  double *out;
  const int32_t *start, *cnt;     // per output index along the axis
  const double *val;              // per output index, B values
  int32_t B;
  int32_t accumulate, zero_bnd;
};

// Coarse solve u0 = A_0^{-1} f0 (level 0, p = 1) by global fast
// diagonalisation in one workgroup, for nu_d <= kCoarse3Max unknowns per
// direction: S_d (nu_d x nu_d row-major, S_d(a, o)) with S_d^T M_d S_d = I and
// L_d S_d = M_d S_d diag(lam_d).  N[d] = nu_d + 2 nodes; u0's boundary is set
// to zero.
constexpr int kCoarse3Max = 18;
struct Coarse3Args {
  int32_t nu[3], N[3];   // x, y, z
  const double *f0;
  double *u0;
  const double *S[3], *lam[3];
};

// Transfers between level l (order pf, nodes NX x NY x NZ) and level l-1
// (order pc = ceil(pf / 2)), element by element with the reference
// interpolation E ((pf+1) x (pc+1), E(a, c) = l_c(xi_a)).  Each fine node is
// taken by the element that holds it at local index 0..pf-1 in every
// direction (the last node plane of a direction is Dirichlet boundary).
struct Transfer3Args {
  int32_t nx, ny, nz, pf;         // elements per direction, fine order
  int32_t NX, NY, NZ;             // fine nodes per direction
  int32_t CX, CY, CZ;             // coarse nodes per direction
  const double *E;
  const double *in;               // restriction: fine r; prolongation: coarse u
  double *out;                    // restriction: coarse f (zeroed before); prolongation: fine u (+=)
};

// First stage of the deterministic dot product x.y: the per-block partial
// sums (their count is returned), added in a fixed order by the consumer.
int launch_dot_partials(const double *x, const double *y, long n, double *partial,
                        hipStream_t s);

void launch3_residual(const Res3Args &a, hipStream_t s);
void launch3_coarse(const Coarse3Args &a, hipStream_t s);
void launch3_restrict(const Transfer3Args &a, hipStream_t s);
void launch3_prolong(const Transfer3Args &a, hipStream_t s);
void launch3_fdm(const Fdm3Args &a, hipStream_t s);
void launch3_axis(const Axis3Args &a, hipStream_t s);
void launch3_eig_divide(double *x, int n0, int n1, int n2, const double *lz, const double *ly,
                        const double *lx, hipStream_t s);
void launch3_axpy(double *y, const double *x, double a, long n, hipStream_t s);
void launch3_xpby(double *p, const double *z, double beta, long n, hipStream_t s);

}  // namespace sem
